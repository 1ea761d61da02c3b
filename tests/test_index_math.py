"""CPU replay of the kernels' index arithmetic (no GPU needed).

Re-derives, for every supported (d, n), the launch geometry that the host code
chooses (threads per line G, lines per workgroup L, dynamic LDS, workgroups)
and the addresses the fused axis-pass kernel forms, then checks that every
global access lies inside its vector, every LDS access inside the
workgroup's allocation, that each unknown is loaded and stored exactly once
per pass, and that the Stockham stages / sine-transform pairs / twiddle
indices stay inside their line buffers and tables.  A mismatch here is a
memory fault on the GPU, so this runs before any kernel change is tried.
"""
import numpy as np
import pytest

MAX_LDS_BLOCK = 163840      # MI355X: maximum LDS per workgroup
STATIC_LDS = 12 * 1024      # budget the host reserves for the kernel's static LDS
MAX_EPT_LINE = 16
KEPT = 8
STREAM_THREADS = 256


def pass_geo(d, n, axis, fp64, max_dyn):
    m = n + 1
    G = max(1, min(64, m // 16))
    elem = 16 if fp64 else 8
    perline = (2 * m + 2) * elem
    L = 256 // G
    while L > 1 and L * perline > max_dyn:
        L //= 2
    while G * L < 64:
        L *= 2
    stride = n ** (d - 1 - axis)
    nlines = n ** (d - 1)
    blocks = (nlines + L - 1) // L
    return dict(G=G, L=L, lds=L * perline, stride=stride, nlines=nlines, blocks=blocks)


def magic(n):
    return ((1 << 32) + n - 1) // n if n >= 2 else 0


def emap(e, n, L, contiguous, mg):
    if contiguous:
        l = e if n == 1 else (e * mg) >> 32
        j = e - l * n
    else:
        j = e >> int(np.log2(L))
        l = e & (L - 1)
    return l, j


SIZES = [(d, n) for d in (1, 2, 3) for n in (1, 3, 7, 15, 31, 63, 127, 255, 511, 1023)
         if n ** d <= 1023 ** 2 or (d == 3 and n <= 255)]


@pytest.mark.parametrize("max_dyn", [MAX_LDS_BLOCK - STATIC_LDS, 64 * 1024 - STATIC_LDS])
@pytest.mark.parametrize("d,n", SIZES)
def test_pass_addresses(d, n, max_dyn):
    N = n ** d
    m = n + 1
    for axis in range(d):
        for fp64 in (True, False):
            g = pass_geo(d, n, axis, fp64, max_dyn)
            G, L, stride = g["G"], g["L"], g["stride"]
            T = G * L
            assert 64 <= T <= 256 and T % 64 == 0
            assert g["lds"] <= max_dyn
            assert L <= 256 and (L & (L - 1)) == 0 and (G & (G - 1)) == 0
            assert G >= m // 16          # per-thread register arrays of the stages
            assert -(-n // G) <= MAX_EPT_LINE
            LS = 2 * m + 2
            contiguous = stride == 1
            mg = magic(n)
            # all blocks for small grids, a sample for large ones
            blocks = range(g["blocks"]) if g["blocks"] <= 64 else \
                sorted(set([0, 1, g["blocks"] // 2, g["blocks"] - 2, g["blocks"] - 1]))
            seen = np.zeros(N, dtype=np.int64) if g["blocks"] <= 64 else None
            E = L * n
            e = np.arange(E)
            for blk in blocks:
                ls, js = [], []
                for ee in e:
                    l, j = emap(int(ee), n, L, contiguous, mg)
                    ls.append(l)
                    js.append(j)
                ls = np.array(ls)
                js = np.array(js)
                assert ls.min() >= 0 and ls.max() < L and js.min() >= 0 and js.max() < n
                # each (line, unknown) exactly once
                assert len(set(zip(ls.tolist(), js.tolist()))) == E
                # LDS slot of the element
                assert (ls * LS + js + 1).max() < L * LS
                lg = blk * L + ls
                valid = lg < g["nlines"]
                o = lg // stride
                i = lg - o * stride
                base = o * n * stride + i
                gi = base + js * stride
                assert gi[valid].min() >= 0 and gi[valid].max() < N
                if seen is not None:
                    np.add.at(seen, gi[valid], 1)
                # each thread handles at most MAX_EPT_LINE elements
                assert -(-E // T) <= MAX_EPT_LINE
            if seen is not None:
                assert np.all(seen == 1), (axis, fp64)


def stage_plan(m):
    plan, ns = [], 1
    while ns < m:
        rem = m // ns
        r = 16 if rem >= 16 else rem
        plan.append((r, ns))
        ns *= r
    return plan


@pytest.mark.parametrize("m", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
def test_line_fft_and_line_ops_indices(m):
    G = max(1, min(64, m // 16))
    for R, Ns in stage_plan(m):
        nb = m // R
        per = 16 // R
        touched_in, touched_out = [], []
        for lt in range(G):
            for q in range(per):
                b = lt + q * G
                if b >= nb:
                    continue
                k = b & (Ns - 1)
                step = k * ((2 * m) // (Ns * R))
                for r in range(R):
                    touched_in.append(b + r * nb)
                    touched_out.append((b - k) * R + k + r * Ns)
                    assert r * step < 2 * m          # twiddle table W_{2m}
        assert sorted(touched_in) == list(range(m))   # every slot read once
        assert sorted(touched_out) == list(range(m))  # and written once
    # sine-transform pairs (j, m-j), j <= m/2, and the output pass p < m/2
    half = m // 2
    slots = set()
    for lt in range(G):
        for j in range(lt, half + 1, G):
            for s in ([0] if j == 0 else ([j] if j == half else [j, m - j])):
                assert 0 <= s < m
                slots.add(s)
        for q in range(8):
            p = lt + q * G
            if p < half:
                assert 2 * p + 1 < m
    assert slots == set(range(m))
    assert half // G <= 8 or G == 1 and half <= 8


@pytest.mark.parametrize("d,n", [(1, 1023), (2, 1023), (3, 255), (2, 7)])
def test_stream_kernels_and_partials(d, n):
    N = n ** d
    blocks = max(1, -(-N // (STREAM_THREADS * KEPT)))
    assert blocks * STREAM_THREADS * KEPT >= N
    pmax = blocks
    for axis in range(d):
        for fp64 in (True, False):
            pmax = max(pmax, pass_geo(d, n, axis, fp64, MAX_LDS_BLOCK - STATIC_LDS)["blocks"])
    # reductions use at most pstride workgroups
    assert min(1024, blocks) <= pmax
    # FP32 basis (restart + 1 vectors of 8N bytes) fits the FP64 basis region
    for restart in (1, 2, 30, 64):
        assert (restart + 1) * 8 * N <= restart * 16 * N
