"""Seeded synthetic inputs for the Riesz fractional NLS linear systems.

This module is the only code shared by the CPU oracle's tests and the GPU
path's tests and benchmark.  It holds no arithmetic of the method itself
(no coefficients, operators, transforms or solver steps): it only lays out the
uniform interior grid of Sec. 2 (x_j = a + j h, h = (b - a)/(M + 1)) and
evaluates analytic initial data of the kind used in Sec. 5 (a sech-shaped
soliton with a plane-wave phase, optional Gaussian modulation), plus seeded
complex Gaussian noise.

Array convention: a d-dimensional field is a C-ordered complex128 array of
shape (n,)*d.  The LAST axis is the first coordinate x_1 (it is the fastest
running index, as in the column-stacking vec() of Sec. 2.2), the first axis is
the last coordinate.

The named workloads below fix sizes, domains, alpha, rho and the time step;
the paper's own experiments (Sec. 5.1, 5.2) use the same kind of data:
u0 = sech(x) exp(2 i x) on [-20, 20] and a Gaussian on [-5, 5]^2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Problem:
    """One linear-system workload: grid, physical parameters and a field u."""

    name: str
    d: int
    n: int
    lo: float
    hi: float
    alpha: float
    rho: float
    tau: float
    u: np.ndarray = field(repr=False)
    steps: int = 1

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / (self.n + 1)

    @property
    def N(self) -> int:
        return self.n ** self.d


def grid_1d(lo: float, hi: float, n: int) -> np.ndarray:
    """Interior grid points x_j = lo + j h, j = 1..n, h = (hi - lo)/(n + 1)."""
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(1, n + 1, dtype=np.float64)


def mesh(d: int, n: int, lo: float, hi: float):
    """Coordinate arrays (x_1, ..., x_d), each of shape (n,)*d.

    x_1 varies along the last axis, x_d along the first axis.
    """
    g = grid_1d(lo, hi, n)
    axes = np.meshgrid(*([g] * d), indexing="ij")  # axes[k] varies along axis k
    return [axes[d - 1 - k] for k in range(d)]


def complex_noise(shape, amplitude: float, seed: int) -> np.ndarray:
    """amplitude * (N(0,1) + i N(0,1)); real block drawn before imaginary, C order."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return amplitude * (re + 1j * im)


def soliton(d: int, n: int, lo: float, hi: float, *, center=None, phase: float = 0.0,
            kx: float = 1.0, gauss_width2: float | None = None,
            noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """sech(|x - c|) * exp(i (kx * x_1 + phase)) [* exp(-|x|^2 / w2)] + noise."""
    xs = mesh(d, n, lo, hi)
    if center is None:
        center = [0.0] * d
    r2 = sum((x - c) ** 2 for x, c in zip(xs, center))
    r = np.sqrt(r2)
    u = (1.0 / np.cosh(r)) * np.exp(1j * (kx * xs[0] + phase))
    if gauss_width2 is not None:
        u = u * np.exp(-r2 / gauss_width2)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    if noise:
        u = u + complex_noise(u.shape, noise, seed)
    return np.ascontiguousarray(u)


def gaussian(d: int, n: int, lo: float, hi: float, *, amplitude: float = 1.0,
             width2: float = 1.0) -> np.ndarray:
    """amplitude * exp(-|x|^2 / width2) on the interior grid (Sec. 5.2 uses
    amplitude 2/sqrt(pi), width2 1 on [-5, 5]^2)."""
    xs = mesh(d, n, lo, hi)
    r2 = sum(x * x for x in xs)
    return np.ascontiguousarray(amplitude * np.exp(-r2 / width2), dtype=np.complex128)


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """A dense random complex field (for operator-level parity tests)."""
    return np.ascontiguousarray(complex_noise(shape, scale, seed))


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def metric_case(n: int = 1023) -> Problem:
    """d=2, n=1023 on [-10,10]^2, alpha 1.5, rho 2, dt 0.01,
    u = sech(|x|) exp(i x_1) + 1e-3 complex noise (seed 0)."""
    u = soliton(2, n, -10.0, 10.0, noise=1e-3, seed=0)
    return Problem("d2_n%d_alpha1.5" % n, 2, n, -10.0, 10.0, 1.5, 2.0, 0.01, u)


def one_dim_case(n: int = 1023) -> Problem:
    """d=1, n=1023 on [-20,20], alpha 1.5, rho 2, dt 0.01,
    u = sech(x) exp(i x) + 1e-3 complex noise (seed 0)."""
    u = soliton(1, n, -20.0, 20.0, noise=1e-3, seed=0)
    return Problem("d1_n%d_alpha1.5" % n, 1, n, -20.0, 20.0, 1.5, 2.0, 0.01, u)


def stepping_case(alpha: float, n: int = 511, steps: int = 100) -> Problem:
    """d=2, n=511 on [-10,10]^2, rho 2, dt 0.005, u0 = sech(|x|) exp(i x_1)."""
    u = soliton(2, n, -10.0, 10.0)
    return Problem("d2_n%d_alpha%g_steps" % (n, alpha), 2, n, -10.0, 10.0, alpha, 2.0,
                   0.005, u, steps=steps)


def three_dim_case(n: int = 255, steps: int = 10) -> Problem:
    """d=3, n=255 on [-8,8]^3, alpha 1.6, rho 1, dt 0.01,
    u0 = sech(|x|) exp(-|x|^2/8) exp(i x_1) + 1e-3 noise (seed 0)."""
    u = soliton(3, n, -8.0, 8.0, gauss_width2=8.0, noise=1e-3, seed=0)
    return Problem("d3_n%d_alpha1.6" % n, 3, n, -8.0, 8.0, 1.6, 1.0, 0.01, u, steps=steps)


def batched_cases(count: int = 64, sizes=(127, 255, 511, 1023), seed: int = 0):
    """Independent d=2 instances on [-10,10]^2 with dt 0.01: per instance, in
    order, n uniform from `sizes`, alpha ~ U[1.1,1.9], rho ~ U[0.5,3],
    centre ~ U[-5,5]^2, phase ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(sizes[rng.integers(len(sizes))])
        alpha = float(rng.uniform(1.1, 1.9))
        rho = float(rng.uniform(0.5, 3.0))
        c = rng.uniform(-5.0, 5.0, size=2)
        phase = float(rng.uniform(0.0, 2 * np.pi))
        u = soliton(2, n, -10.0, 10.0, center=list(c), phase=phase)
        out.append(Problem("batch%02d_n%d" % (k, n), 2, n, -10.0, 10.0, alpha, rho, 0.01, u))
    return out


def paper_1d_mass_case(alpha: float) -> Problem:
    """Sec. 5.1 mass-conservation protocol: [-20,20], h = 0.2 (M = 199),
    dt = 0.05, rho = 2, u0 = sech(x) exp(2 i x)."""
    n = 199
    u = soliton(1, n, -20.0, 20.0, kx=2.0)
    return Problem("paper1d_mass_alpha%g" % alpha, 1, n, -20.0, 20.0, alpha, 2.0, 0.05, u,
                   steps=80)
