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
STATIC_LDS = 8 * 1024       # budget the host reserves for the kernel's static LDS
KEPT = 8
STREAM_THREADS = 512


DEFAULT_CFG = {"rmax": (4, 4), "lines": (1, 4)}   # (contiguous axis, strided axes)
PASS_CONFIGS = [DEFAULT_CFG,
           {"rmax": (4, 8), "lines": (2, 4)},
           {"rmax": (4, 4), "lines": (2, 2)},       # FP64 default
           {"rmax": (4, 8), "lines": (1, 4)},       # FP32 default
           {"rmax": (8, 8), "lines": (1, 4)},
           {"rmax": (16, 16), "lines": (1, 4)},
           {"rmax": (8, 8), "lines": (2, 4)},
           {"rmax": (4, 8), "lines": (1, 2)},
           {"rmax": (16, 4), "lines": (4, 1)}]


def line_layout(m, L, fp64, two):
    """Line buffer slots pa >= m and line stride ls (host rule): with L >= 2
    interleaved lines, ls * size = 128 / L mod 256 / L bytes when reachable;
    ls is the smallest such stride >= k m (k buffers), and with two buffers B
    starts pa = m + (ls - 2 m) // 2 slots after A."""
    elem = 16 if fp64 else 8
    k = 2 if two else 1
    extra = 0
    if L >= 2 and 128 // L >= elem:
        target, mod = 128 // L // elem, 256 // L // elem
        for dd in range(mod):
            if (k * m + dd) % mod == target:
                extra = dd
                break
    ls = k * m + extra
    return (m + extra // 2 if two else ls), ls


def par(x):
    return bin(x).count("1") & 1


def lds_extra_cycles(slots, elem, kind="r"):
    """gfx950 LDS model fitted to its bank-conflict counter: a 64-lane
    ds_read_b128 is served in four cycles of 16 lanes keyed by (lane bit 5,
    parity of lane bits 2..4) from 64 banks of 4 B, ds_read_b64 in two cycles
    of 32 lanes (bit 5); ds_write_b128 in eight cycles of 8 consecutive lanes,
    ds_write_b64 in four of 16, from 32 banks.  Returns the cycles beyond the
    conflict-free count (None = inactive lane)."""
    cyc = {}
    for l, sl in enumerate(slots):
        if sl is None:
            continue
        if kind == "r":
            key = ((l >> 5) & 1, par(l & 28)) if elem == 16 else ((l >> 5) & 1,)
        else:
            key = (l >> 3) if elem == 16 else (l >> 4)
        cyc.setdefault(key, []).append(sl)
    nb = 64 if kind == "r" else 32
    extra = 0
    for ss in cyc.values():
        banks = {}
        for sl in ss:
            for w in range(elem // 4):
                dw = sl * (elem // 4) + w
                banks.setdefault(dw % nb, set()).add(dw)
        extra += max(len(v) for v in banks.values()) - 1
    return extra


def out_rot(lane, fp64=True):
    if fp64:
        return ((lane >> 2) & 1) | (((lane >> 1) & 1) << 1)
    return ((lane >> 2) & 1) | (((lane >> 3) & 1) << 1)


def scan_rot(lane, fp64=True):
    return (lane >> 3) & 1 if fp64 else (lane >> 4) & 1


def threads_max(rmax):
    return 256 if rmax == 16 else 4096 // rmax


def pass_geo(d, n, axis, fp64, max_dyn, cfg=DEFAULT_CFG):
    m = n + 1
    col = 0 if axis == d - 1 else 1
    rmax = cfg["rmax"][col]
    G = max(1, m // rmax)
    tmax = threads_max(rmax)
    elem = 16 if fp64 else 8
    table = (m // 4 if m >= 4 else 1) * elem

    def lds_of(L):
        return L * line_layout(m, L, fp64, True)[1] * elem + table + L * (8 + elem // 2)
    gref = 1024 // rmax
    L = cfg["lines"][col] * max(1, gref // G)
    L = max(1, min(L, tmax // G))
    while L > 1 and lds_of(L) > max_dyn:
        L //= 2
    while G * L < 64:
        L *= 2
    stride = n ** (d - 1 - axis)
    nlines = n ** (d - 1)
    blocks = (nlines + L - 1) // L
    lds = lds_of(L)
    return dict(G=G, L=L, lds=lds, stride=stride, nlines=nlines, blocks=blocks, rmax=rmax, tmax=tmax)


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


@pytest.mark.parametrize("cfg", range(len(PASS_CONFIGS)))
@pytest.mark.parametrize("max_dyn", [MAX_LDS_BLOCK - STATIC_LDS, 64 * 1024 - STATIC_LDS])
@pytest.mark.parametrize("d,n", SIZES)
def test_pass_addresses(d, n, max_dyn, cfg):
    N = n ** d
    m = n + 1
    for axis in range(d):
        for fp64 in (True, False):
            g = pass_geo(d, n, axis, fp64, max_dyn, PASS_CONFIGS[cfg])
            G, L, stride = g["G"], g["L"], g["stride"]
            T = G * L
            assert 64 <= T <= g["tmax"] and T % 64 == 0
            assert g["lds"] <= max_dyn
            assert (L & (L - 1)) == 0 and (G & (G - 1)) == 0
            assert G >= m // g["rmax"]      # per-thread register arrays of the stages
            MAX_EPT_LINE = g["rmax"]
            assert -(-n // G) <= MAX_EPT_LINE
            elem = 16 if fp64 else 8
            table = (m // 4 if m >= 4 else 1) * elem
            layouts = [line_layout(m, L, fp64, two) for two in (True, False)]
            for pa, ls in layouts:
                assert pa >= m and ls >= pa + (m if ls != pa else 0)
                # what the launch allocates (reduction sums included) fits
                lds = max(L * ls * elem + table + L * (8 + elem // 2), 66 * (T // 64) * 16, 4096)
                assert L * ls * elem + table + L * (8 + elem // 2) <= g["lds"]
                assert lds <= max_dyn or lds <= 4096 + 66 * 16 * 16
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
                # LDS slot of the element, with two buffers per line (Toeplitz
                # passes) and with one (sine-transform passes)
                slots = js + 1
                for pa, LSb in layouts:
                    assert slots.max() < pa
                    assert (ls * LSb + slots).max() < L * LSb
                    assert (ls * LSb + pa + slots).max() < L * LSb or pa == LSb   # buffer B
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


@pytest.mark.parametrize("d", [1, 2, 3])
def test_direct_line_base_fits_32_bits(d):
    """Before the per-line set-up, a pass thread forms its line's base offset
    from 32-bit unsigned line indices and strides (lg = blk L + l, o = lg /
    stride); at every size the library accepts they stay below 2^32."""
    for n in (1, 3, 7, 15, 31, 63, 127, 255, 511, 1023):
        for axis in range(d):
            for fp64 in (True, False):
                g = pass_geo(d, n, axis, fp64, MAX_LDS_BLOCK - STATIC_LDS)
                assert g["blocks"] * g["L"] < 2 ** 32
                assert g["stride"] < 2 ** 32 and g["nlines"] <= g["blocks"] * g["L"]


def xcd_block(i, nb, xcd=8):
    x, q = i % xcd, i // xcd
    base, rem = nb // xcd, nb % xcd
    return x * base + min(x, rem) + q


@pytest.mark.parametrize("nb", [1, 2, 7, 8, 9, 15, 16, 17, 63, 64, 255, 256, 257, 1023, 4097, 65025])
def test_xcd_block_remap_is_a_permutation(nb):
    """The workgroup -> line-block remap covers every block exactly once, and
    the blocks of one XCD (workgroups i = x mod 8) are one contiguous range."""
    lb = np.array([xcd_block(i, nb) for i in range(nb)])
    assert sorted(lb.tolist()) == list(range(nb))
    for x in range(min(8, nb)):
        own = lb[x::8]
        assert np.all(np.diff(own) == 1)


def stage_plan(m, rmax):
    plan, ns = [], 1
    while ns < m:
        rem = m // ns
        r = rmax if rem >= rmax else rem
        plan.append((r, ns))
        ns *= r
    return plan


@pytest.mark.parametrize("rmax", [4, 8, 16])
@pytest.mark.parametrize("m", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
def test_line_fft_and_line_ops_indices(m, rmax):
    G = max(1, m // rmax)
    lgm = m.bit_length() - 1
    for R, Ns in stage_plan(m, rmax):
        nb = m // R
        per = rmax // R
        touched_in, touched_out = [], []
        for lt in range(G):
            for q in range(per):
                b = lt + q * G
                if b >= nb:
                    continue
                k = b & (Ns - 1)
                step = k * ((2 * m) // (Ns * R))
                tsh = lgm - (Ns.bit_length() - 1) - (R.bit_length() - 1)
                if R == 8:
                    rot = (lt & 63) & 7 if Ns < 8 else 0
                else:
                    rot = out_rot(lt & 63) & (R - 1 if R <= 4 else 0) if Ns < 16 else 0
                # store i writes output i ^ rot: still every output once
                assert sorted(i ^ rot for i in range(R)) == list(range(R))
                for r in range(R):
                    touched_in.append(b + r * nb)
                    touched_out.append((b - k) * R + k + (r ^ rot) * Ns)
                    assert r * step < 2 * m          # twiddle table W_{2m}
                    q = (r * k) << tsh               # W_{Ns R}^{r k} = W_m^q
                    assert q < m
                    if k and r:
                        assert lgm >= 2 and (q & ((1 << (lgm - 2)) - 1)) < max(1, m // 4)
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
    # one-FFT sine transform: thread lt owns p in [lt E, lt E + E), E = half / G
    E = half // G if half >= G else 1
    assert E <= max(1, rmax // 2)
    owned, outs = [], []
    for lt in range(G):
        for e in range(E):
            p = lt * E + e
            if p < half:
                assert 2 * p + 1 < m and m - p <= m
                owned.append(p)
        if rmax // 2 == 2 and E == 2:
            # rotated path: reads p0 + (e ^ sr), m - (p0 + (e ^ sr)) (slot 0
            # for p = 0), writes 2 p0 + (i ^ rot)
            sr = scan_rot(lt & 63)
            for e in range(2):
                q = lt * 2 + (e ^ sr)
                assert 0 <= q < half and 0 <= (m - q if q > 0 else 0) < m
            rot = out_rot(lt & 63)
            outs += [2 * lt * 2 + (i ^ rot) for i in range(4)]
    assert sorted(owned) == list(range(half))
    if outs:
        assert sorted(outs) == list(range(m))
    assert slots == set(range(m))
    # scan segments: G lanes of a line inside a wavefront, or whole wavefronts
    sw = min(G, 64)
    assert 64 % sw == 0 and (G <= 64 or G % 64 == 0)
    assert (1024 // 64) <= 16   # wavefront totals of one workgroup fit the scan's LDS array


MAX_RESTART = 64
REDUNDANT_MAX = 1024


@pytest.mark.parametrize("cfg", range(len(PASS_CONFIGS)))
@pytest.mark.parametrize("d,n", SIZES)
def test_partial_buffers(d, n, cfg):
    """Every per-workgroup partial written, and every one read back, lies in
    its buffer: p1, p2 hold (restart max + 2) values x pstride, p3 and pr one
    value x pstride, px (the pre-summed totals when a producer had more than
    1024 workgroups) restart max + 2 contiguous values."""
    N = n ** d
    sblocks = max(1, -(-N // (STREAM_THREADS * KEPT)))
    pstride = max(sblocks, n ** (d - 1))
    size = {"p1": (MAX_RESTART + 2) * pstride, "p2": (MAX_RESTART + 2) * pstride,
            "p3": pstride, "pr": pstride, "px": MAX_RESTART + 2}
    for fp64 in (True, False):
        nb0 = pass_geo(d, n, 0, fp64, MAX_LDS_BLOCK - STATIC_LDS, PASS_CONFIGS[cfg])["blocks"]
        for restart in (1, 30, MAX_RESTART):
            for j in range(restart):
                # producer -> buffer, number of values, producer workgroups
                chain = [("p1", j + 2, nb0),        # pass with the first dot products and ||w||^2
                         ("p2", j + 1, sblocks),    # first update: second-round dots
                         ("p3", 1, sblocks)]        # second update: ||w||^2
                for buf, nv, nbp in chain:
                    assert nbp <= pstride
                    assert (nv - 1) * pstride + (nbp - 1) < size[buf]
                    if nbp > REDUNDANT_MAX:
                        # pre-sum kernel reads [i][pstride], writes px[i]
                        assert nv <= size["px"]
            for buf, nbp in (("pr", nb0), ("pr", sblocks)):  # residual, prepare
                assert nbp <= pstride and nbp - 1 < size[buf]


@pytest.mark.parametrize("d,n", [(1, 1023), (2, 1023), (3, 255), (2, 7)])
def test_stream_kernels_and_partials(d, n):
    N = n ** d
    blocks = max(1, -(-N // (STREAM_THREADS * KEPT)))
    assert blocks * STREAM_THREADS * KEPT >= N
    pmax = blocks
    for axis in range(d):
        for fp64 in (True, False):
            for cfg in PASS_CONFIGS:
                assert pass_geo(d, n, axis, fp64, MAX_LDS_BLOCK - STATIC_LDS, cfg)["blocks"] <= n ** (d - 1)
    pmax = max(blocks, n ** (d - 1))
    # reductions use at most pstride workgroups
    assert blocks <= pmax
    # FP32 basis (restart + 1 vectors of 8N bytes) fits the FP64 basis region
    for restart in (1, 2, 30, 64):
        assert (restart + 1) * 8 * N <= restart * 16 * N


@pytest.mark.parametrize("fp64", [True, False])
def test_lds_layout_is_conflict_free_at_m1024(fp64):
    """Under the gfx950 bank model, the LDS accesses of a radix-4 line of
    m = 1024 (G = 256 threads) are free of bank conflicts: stage loads,
    lane-rotated stage stores (cyclic rotation (i + s) mod 4), the last two stages' twiddle reads, the
    sine-transform pre-pass pairs, rotated scan reads and output writes, the
    element phases of rows at any offset, and the element writes of 2 and 4
    interleaved strided lines at the host's line stride (whose reads cost at
    most one extra cycle per cycle group)."""
    elem = 16 if fp64 else 8
    m, G = 1024, 256
    bad = []
    for wave in range(G // 64):
        lt = [64 * wave + l for l in range(64)]
        for lgNs in (0, 2, 4, 6, 8):
            Ns = 1 << lgNs
            for i in range(4):
                bad.append(lds_extra_cycles([t + i * 256 for t in lt], elem, "r"))
                st = []
                for l, b in zip(range(64), lt):
                    k = b & (Ns - 1)
                    st.append(((b - k) << 2) + k + ((i + (out_rot(l, fp64) if Ns < 16 else 0)) & 3) * Ns)
                bad.append(lds_extra_cycles(st, elem, "w"))
        for tsh in (0, 2):   # stages 4 and 3: q = k << tsh, table slot q ^ ((q >> 4 or 5) & 3)
            q = [(t & (255 >> tsh)) << tsh for t in lt]
            sh = 4 if fp64 else 5
            bad.append(lds_extra_cycles([x ^ ((x >> sh) & 3) for x in q], elem, "r"))
        for i in range(3):
            js = [t + i * G if t + i * G <= m // 2 else None for t in lt]
            mj = [m - j if j is not None else None for j in js]
            for kind in "rw":
                bad.append(lds_extra_cycles(js, elem, kind))
                bad.append(lds_extra_cycles(mj, elem, kind))
        for e in range(2):
            ps = [2 * t + (e ^ scan_rot(l, fp64)) for l, t in zip(range(64), lt)]
            bad.append(lds_extra_cycles(ps, elem, "r"))
            bad.append(lds_extra_cycles([m - p if p > 0 else 0 for p in ps], elem, "r"))
        for i in range(4):
            bad.append(lds_extra_cycles([4 * t + (i ^ out_rot(l, fp64)) for l, t in zip(range(64), lt)], elem, "w"))
    for L in (1, 2, 4):
        lgL = L.bit_length() - 1
        for two in (True, False):
            pa, ls = line_layout(m, L, fp64, two)
            for start in range(0, 64):
                sl = [((start * 64 + l) & (L - 1)) * ls + ((start * 64 + l) >> lgL) + 1 for l in range(64)]
                bad.append(lds_extra_cycles(sl, elem, "w"))
                assert lds_extra_cycles(sl, elem, "r") <= 4 * (L > 1) * (4 if fp64 else 2)
    for start in range(0, 2000, 37):
        for kind in "rw":
            bad.append(lds_extra_cycles([start + l + 1 for l in range(64)], elem, kind))
    assert max(bad) == 0


@pytest.mark.parametrize("fp64", [True, False])
def test_interleaved_element_writes_are_conflict_free_at_m256(fp64):
    """The element writes of 8 and 16 interleaved strided lines of m = 256
    (the d = 3, n = 255 strided passes) are free of bank conflicts at the
    host's line stride, for one and for two buffers per line (the two-buffer
    stride may be odd, with the spare slot after buffer B)."""
    elem = 16 if fp64 else 8
    m = 256
    for L in (8, 16):
        if 128 // L < elem:
            continue
        lgL = L.bit_length() - 1
        for two in (True, False):
            pa, ls = line_layout(m, L, fp64, two)
            assert pa >= m and (not two or ls >= pa + m)
            for start in range(0, 64):
                sl = [((start * 64 + l) & (L - 1)) * ls + ((start * 64 + l) >> lgL) + 1 for l in range(64)]
                assert lds_extra_cycles(sl, elem, "w") == 0, (L, two, start)


def mul_ipow(v, e):
    """v i^e for e mod 4, as the kernels form it: a swap of the parts for odd
    e, and sign flips."""
    odd = e & 1
    a, b = (v.imag, v.real) if odd else (v.real, v.imag)
    return complex(-a if (e + 1) & 2 else a, -b if e & 2 else b)


@pytest.mark.parametrize("m", [16, 64, 256, 1024])
@pytest.mark.parametrize("inv", [False, True])
@pytest.mark.parametrize("fp64", [True, False])
def test_rotated_radix4_stockham_is_the_dft(m, inv, fp64):
    """Replay of the compile-time radix-4 Stockham plan with the cyclic output
    rotation: stages with Ns < 16 store output register i at slot position
    (i + s) mod 4 (s = out_rot of the lane), the twiddle-free first stage
    multiplies input q by W_4^{+-q s} (part swaps and sign flips), the next
    stage folds W_4^{+-s} into its twiddle W^k (whose powers then carry
    W_4^{+-q s}).  The result in natural order must be the DFT (inverse:
    unnormalised inverse DFT) of the line."""
    rng = np.random.default_rng(m)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    sgn = 1.0 if inv else -1.0
    G = m // 4
    X = x.copy()
    Ns = 1
    while Ns < m:
        Y = np.zeros(m, dtype=complex)
        for b in range(G):
            s = out_rot(b & 63, fp64) if Ns < 16 else 0
            k = b % Ns
            v = [X[b + r * G] for r in range(4)]
            if Ns == 1:
                e1 = s if inv else -s
                v = [v[0], mul_ipow(v[1], e1), mul_ipow(v[2], 2 * s), mul_ipow(v[3], -e1)]
            else:
                w = np.exp(sgn * 2j * np.pi * k / (4 * Ns))
                if Ns < 16:
                    w = mul_ipow(w, s if inv else -s)
                v = [v[r] * w ** r for r in range(4)]
            y = [sum(v[q] * np.exp(sgn * 2j * np.pi * r * q / 4) for q in range(4)) for r in range(4)]
            base = (b - k) * 4 + k
            for i in range(4):
                Y[base + ((i + s) & 3) * Ns] = y[i]
        X = Y
        Ns *= 4
    ref = np.fft.ifft(x) * m if inv else np.fft.fft(x)
    assert np.abs(X - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("cfg", range(len(PASS_CONFIGS)))
def test_mirror_matches_the_library_geometry(cfg):
    """The host geometry rules replayed above (pass_geo, line_layout) are the
    library's own: fnls_pass_geometry (host arithmetic of libfnls, no device)
    gives the same G, L, workgroups, LDS bytes, stride, line count and line
    layouts for every supported size, axis, precision and schedule."""
    import ctypes
    from paper_2410_03643_amd import fnls
    L = fnls.lib()
    out = (ctypes.c_longlong * 10)()
    max_dyn = MAX_LDS_BLOCK - STATIC_LDS
    checked = 0
    for d, n in SIZES:
        for axis in range(d):
            for fp64 in (True, False):
                c = PASS_CONFIGS[cfg]
                col = 0 if axis == d - 1 else 1
                prec = fnls.FP64 if fp64 else fnls.FP32_IR
                rc = L.fnls_pass_geometry(d, n, axis, prec, c["rmax"][col], c["lines"][col], max_dyn, out)
                assert rc == 0
                g = pass_geo(d, n, axis, fp64, max_dyn, c)
                m = n + 1
                pa2, ls2 = line_layout(m, g["L"], fp64, True)
                pa1, ls1 = line_layout(m, g["L"], fp64, False)
                want = [g["G"], g["L"], g["blocks"], g["lds"], g["stride"], g["nlines"], pa2, ls2, pa1, ls1]
                assert list(out) == want, (d, n, axis, fp64, list(out), want)
                checked += 1
    assert checked > 100
    # unsupported settings are rejected
    assert L.fnls_pass_geometry(2, 1000, 0, fnls.FP64, 4, 1, max_dyn, out) != 0
    assert L.fnls_pass_geometry(2, 1023, 2, fnls.FP64, 4, 1, max_dyn, out) != 0
    assert L.fnls_pass_geometry(2, 1023, 0, fnls.FP64, 5, 1, max_dyn, out) != 0
