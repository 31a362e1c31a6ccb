"""Seeded synthetic inputs shared by the GPU path, the oracle and the bench.

This module holds no arithmetic of the eigensolver: it only draws the
potentials V, start blocks X0, loss weights and perturbation directions, and
states the workload shapes.  Every array is float64 (complex128 for complex
start blocks) and generated on the host.

Grid convention: a periodic N^3 grid with spacing h; the flat index of grid
point (i, j, l) is i + N*(j + N*l), so x varies fastest.  Point (i, j, l) sits
at r = h*(i, j, l) and the box side is L = N*h.

Block convention: an n x K block is column-major with leading dimension n.  In
numpy it is carried as an (n, K) array; ``to_colmajor`` gives the (K, n)
C-contiguous buffer the C ABI expects and ``from_colmajor`` undoes it.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    """Periodic finite-difference grid and stencil choice.

    order 2 = 7-point Laplacian, order 4 = 13-point (fourth-order) Laplacian.
    kpt = Bloch wave vector kappa in 1/length units; all zero means a real
    operator.
    """

    N: int
    h: float = 0.5
    order: int = 2
    kpt: tuple = (0.0, 0.0, 0.0)

    @property
    def n(self) -> int:
        return self.N ** 3

    @property
    def L(self) -> float:
        return self.N * self.h

    @property
    def is_complex(self) -> bool:
        return any(float(c) != 0.0 for c in self.kpt)


def default_nbuf(k: int, q: int) -> int:
    """Buffer-vector count: about 2% of k (at least 2), rounded so that
    K = k + nbuf is a multiple of the sub-block width q.  The paper suggests
    1-5% of k (section on buffer vectors)."""
    extra = max(2, math.ceil(0.02 * k))
    return q * math.ceil((k + extra) / q) - k


def grid_coords(N: int, h: float):
    """x, y, z coordinates of every grid point, flattened in grid order."""
    ax = np.arange(N, dtype=np.float64) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def gaussian_wells(N: int, h: float, nwells: int, seed: int) -> np.ndarray:
    """V(r) = -sum_w d_w exp(-|r - c_w|^2 / (2 sigma_w^2)) with the periodic
    minimum-image distance, c_w ~ U[0, L)^3, d_w ~ U(1, 3),
    sigma_w ~ U(0.5, 1.5).  Draw order: all centres, then depths, then widths,
    from numpy's PCG64 generator seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    L = N * h
    centres = rng.uniform(0.0, L, size=(nwells, 3))
    depths = rng.uniform(1.0, 3.0, size=nwells)
    widths = rng.uniform(0.5, 1.5, size=nwells)
    x, y, z = grid_coords(N, h)
    V = np.zeros(N ** 3, dtype=np.float64)
    for c, d, s in zip(centres, depths, widths):
        r2 = np.zeros_like(V)
        for coord, cc in ((x, c[0]), (y, c[1]), (z, c[2])):
            dd = np.abs(coord - cc)
            dd = np.minimum(dd, L - dd)
            r2 += dd * dd
        V -= d * np.exp(-r2 / (2.0 * s * s))
    return V


def smoothed_field(N: int, h: float, seed: int, lo: float = -2.0, hi: float = 0.0) -> np.ndarray:
    """g ~ N(0,1) on the grid, smoothed periodically with a Gaussian of
    width 2h (applied in Fourier space), then mapped affinely onto [lo, hi]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((N, N, N))
    sigma = 2.0 * h
    f = np.fft.fftfreq(N, d=h) * 2.0 * np.pi
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    filt = np.exp(-0.5 * sigma * sigma * (kx * kx + ky * ky + kz * kz))
    gs = np.real(np.fft.ifftn(np.fft.fftn(g) * filt))
    gmin, gmax = gs.min(), gs.max()
    return (lo + (hi - lo) * (gs - gmin) / (gmax - gmin)).ravel().astype(np.float64)


def start_block(n: int, K: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Random start block X0 (n, K): N(0,1) entries; complex entries have
    independent real and imaginary parts ~ N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    if not complex_:
        return rng.standard_normal((n, K))
    s = math.sqrt(0.5)
    re = rng.standard_normal((n, K)) * s
    im = rng.standard_normal((n, K)) * s
    return re + 1j * im


def start_block_device(n: int, K: int, seed: int, complex_: bool, device="cuda"):
    """Random start block generated on the device, as a (K, n) torch tensor
    (column-major n x K): N(0,1) entries, or complex entries with independent
    real and imaginary parts ~ N(0, 1/2), from torch's seeded generator of
    that device.  Used for the 96^3 Bloch workload, whose 29.9 GB block would
    take minutes through the numpy stream of start_block; the values differ
    from start_block's, the distribution is the same."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    dt = torch.complex128 if complex_ else torch.float64
    return torch.randn((K, n), generator=g, device=device, dtype=dt)


def loss_weights(n: int, seed: int) -> np.ndarray:
    """Density weights w ~ N(0,1) of the loss sum_r w_r rho_r."""
    return np.random.default_rng(seed).standard_normal(n)


def unit_directions(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` directions d ~ N(0, I) in R^n, each scaled to unit 2-norm;
    returned as a (count, n) array."""
    d = np.random.default_rng(seed).standard_normal((count, n))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def to_colmajor(X: np.ndarray) -> np.ndarray:
    """(n, K) array -> (K, n) C-contiguous buffer (column-major n x K)."""
    return np.ascontiguousarray(X.T)


def from_colmajor(B: np.ndarray) -> np.ndarray:
    """(K, n) column-major buffer -> (n, K) array view."""
    return B.T


# ----------------------------------------------------------------------------
# Workloads.  h = 0.5 throughout; the Bloch vector of the complex workload is
# (2 pi * 0.25 / L, 0, 0).
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Problem:
    name: str
    grid: Grid
    V: np.ndarray
    k: int
    q: int
    nbuf: int
    rr_period: int
    tol: float
    x0_seed: int

    @property
    def K(self) -> int:
        return self.k + self.nbuf

    def start(self) -> np.ndarray:
        return start_block(self.grid.n, self.K, self.x0_seed, self.grid.is_complex)


def wells16(seed: int = 101) -> Problem:
    """7-point, 16^3, 4 wells, k = 64, q = 8, rr_period 5, tol 1e-6."""
    g = Grid(16, 0.5, 2)
    return Problem("wells16_k64", g, gaussian_wells(16, 0.5, 4, seed), 64, 8,
                   default_nbuf(64, 8), 5, 1e-6, 201)


def wells48(seed: int = 102) -> Problem:
    """13-point, 48^3, 32 wells, k = 512, q = 16, rr_period 5, tol 1e-6."""
    g = Grid(48, 0.5, 4)
    return Problem("wells48_k512", g, gaussian_wells(48, 0.5, 32, seed), 512, 16,
                   default_nbuf(512, 16), 5, 1e-6, 202)


def bloch96(seed: int = 103, N: int = 96, k: int = 2048, q: int = 32) -> Problem:
    """13-point, N^3 with Bloch vector (2 pi 0.25 / L, 0, 0), smoothed random
    potential in [-2, 0], k = 2048, q = 32 (smaller N/k give reduced
    versions of the same operator family)."""
    L = N * 0.5
    g = Grid(N, 0.5, 4, (2.0 * math.pi * 0.25 / L, 0.0, 0.0))
    nbuf = 64 if (N, k, q) == (96, 2048, 32) else default_nbuf(k, q)
    return Problem(f"bloch{N}_k{k}", g, smoothed_field(N, 0.5, seed), k, q, nbuf, 5, 1e-6, 203)


def batch64(seed: int = 104, count: int = 64) -> list:
    """64 independent 7-point problems: N_b ~ U{24..40}, k_b ~ U{32..256},
    wells ~ U{1..8} drawn from one stream in that order (all N, then all k,
    then all well counts); the wells of problem b use seed 104000 + b and its
    start block seed 204 + b.  q = 8, rr_period 5, tol 1e-6."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(24, 41, size=count)
    ks = rng.integers(32, 257, size=count)
    nw = rng.integers(1, 9, size=count)
    out = []
    for b in range(count):
        N, k = int(Ns[b]), int(ks[b])
        g = Grid(N, 0.5, 2)
        out.append(Problem(f"batch{b}_N{N}_k{k}", g, gaussian_wells(N, 0.5, int(nw[b]), 104000 + b),
                           k, 8, default_nbuf(k, 8), 5, 1e-6, 204 + b))
    return out


def wells32(seed: int = 105) -> Problem:
    """7-point, 32^3, 8 wells, k = 128, q = 8, rr_period 5, tol 1e-6; the
    loss weights use seed 305 and the FD directions seed 405."""
    g = Grid(32, 0.5, 2)
    return Problem("wells32_k128", g, gaussian_wells(32, 0.5, 8, seed), 128, 8,
                   default_nbuf(128, 8), 5, 1e-6, 205)


def small_problem(N: int = 10, k: int = 12, q: int = 4, order: int = 2, nwells: int = 3,
                  seed: int = 7, kpt=(0.0, 0.0, 0.0), rr_period: int = 5, tol: float = 1e-8,
                  nbuf: int | None = None) -> Problem:
    """A small problem of the same family for tests."""
    g = Grid(N, 0.5, order, tuple(kpt))
    V = gaussian_wells(N, 0.5, nwells, seed) if nwells > 0 else np.zeros(N ** 3)
    nb = default_nbuf(k, q) if nbuf is None else nbuf
    return Problem(f"small{N}_k{k}_q{q}_o{order}", g, V, k, q, nb, rr_period, tol, seed + 1000)


def scf_potentials(base: Problem, steps: int = 14, amp: float = 0.5, decay: float = 0.7,
                   seed: int = 106) -> list:
    """A slowly converging sequence of potentials standing in for the
    self-consistent-field iterations of the paper's section 6 (no density
    functional here): V_s = V + amp * decay^s * dV for s = 0..steps, with dV
    a smoothed N(0,1) field (width 2h) mapped onto [-1, 1] from its own seed.
    V_0 is the first SCF potential; V_s -> V."""
    g = base.grid
    dV = smoothed_field(g.N, g.h, seed, -1.0, 1.0)
    return [base.V + amp * decay ** s * dV for s in range(steps + 1)]


def mass_weights(N: int, h: float, seed: int, lo: float = 0.8, hi: float = 1.25) -> np.ndarray:
    """Positive diagonal B of a generalized problem H x = lambda B x (a
    position-dependent weight, e.g. a lumped overlap or metric): a smoothed
    N(0,1) field (width 2h) mapped onto [lo, hi] from its own seed."""
    return smoothed_field(N, h, seed, lo, hi)
