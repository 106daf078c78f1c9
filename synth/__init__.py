"""Seeded synthetic inputs shared by the oracle-based tests, the GPU tests and the benchmark.

This module holds no arithmetic of the eigenvalue method itself: it only produces the
problem data that the paper's problem statement takes as input (Section 1 and Section 3):
the permittivity epsilon sampled per mesh cell, Bloch parameters k, and random start
blocks.  Both the CPU oracle and the GPU path receive identical bits from here.

Conventions (0-based, used everywhere in this repository):
  * cell (c1, c2) is [c1*h1, (c1+1)*h1] x [c2*h2, (c2+1)*h2], flat index c2*n + c1;
    epsilon is piecewise constant per cell, sampled at the cell centre.
  * edge dof order: x-edges (j1, j2) at index j2*n + j1, then y-edges at n*m + j2*n + j1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "cell_centres", "eps_disc", "eps_disc_lattice", "eps_random_field", "start_block",
    "path_gxmg", "uniform_k", "Problem", "config_c1", "config_c2", "config_c3", "config_c4_small",
    "config_c4_problems", "config_c5_requests", "paper_z2_eps", "paper_z1_eps",
]


def cell_centres(n: int, m: int, a: float = 1.0, b: float = 1.0):
    """Cell-centre coordinates (x1, x2), each of shape (m, n) (row c2, column c1)."""
    h1, h2 = a / n, b / m
    x1 = (np.arange(n) + 0.5) * h1
    x2 = (np.arange(m) + 0.5) * h2
    return np.meshgrid(x1, x2, indexing="xy")


def eps_disc(n: int, m: int, a: float, b: float, eps_in: float, radius: float,
             centre=None, eps_out: float = 1.0) -> np.ndarray:
    """One disc of permittivity eps_in (closed disc, distance <= radius) on eps_out.

    Returns a float64 array of n*m cell values in cell order c2*n + c1.
    """
    if centre is None:
        centre = (0.5 * a, 0.5 * b)
    X1, X2 = cell_centres(n, m, a, b)
    d2 = (X1 - centre[0]) ** 2 + (X2 - centre[1]) ** 2
    out = np.where(d2 <= radius * radius, float(eps_in), float(eps_out))
    return np.ascontiguousarray(out.reshape(-1), dtype=np.float64)


def eps_disc_lattice(n: int, m: int, a: float, b: float, eps_in: float, radius: float,
                     eps_out: float = 1.0) -> np.ndarray:
    """Square lattice of discs: one disc centred in every lattice cell of size a x b.

    The unit cell is one lattice period, so this is a single centred disc; the distance
    is taken periodically so radii above half the period overlap their images.
    """
    X1, X2 = cell_centres(n, m, a, b)
    d1 = np.abs(X1 - 0.5 * a)
    d1 = np.minimum(d1, a - d1)
    d2 = np.abs(X2 - 0.5 * b)
    d2 = np.minimum(d2, b - d2)
    out = np.where(d1 * d1 + d2 * d2 <= radius * radius, float(eps_in), float(eps_out))
    return np.ascontiguousarray(out.reshape(-1), dtype=np.float64)


def eps_random_field(n: int, m: int, a: float, b: float, seed: int, sigma: float = 0.05,
                     lo: float = 1.0, hi: float = 11.4, level: float = 0.0) -> np.ndarray:
    """Seeded smoothed random two-phase field.

    i.i.d. N(0,1) samples at the cell centres are blurred with a periodic Gaussian of
    standard deviation sigma (in units of a and b), then thresholded at `level`:
    cells above get `hi`, the rest `lo`.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, n))
    f1 = np.fft.fftfreq(n, d=a / n)
    f2 = np.fft.fftfreq(m, d=b / m)
    F1, F2 = np.meshgrid(f1, f2, indexing="xy")
    kernel_hat = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * (F1 * F1 + F2 * F2))
    smooth = np.real(np.fft.ifft2(np.fft.fft2(g) * kernel_hat))
    out = np.where(smooth > level, float(hi), float(lo))
    return np.ascontiguousarray(out.reshape(-1), dtype=np.float64)


def paper_z1_eps(n: int) -> np.ndarray:
    """The throw-away study's permittivity: 100 in the disc of radius 1/3 at the centre."""
    return eps_disc(n, n, 1.0, 1.0, 100.0, 1.0 / 3.0)


def paper_z2_eps(n: int) -> np.ndarray:
    """The band-structure experiment's permittivity: 11.56 in the disc of radius 0.18."""
    return eps_disc(n, n, 1.0, 1.0, 11.56, 0.18)


def start_block(n_edges: int, p: int, seed: int) -> np.ndarray:
    """Random complex Gaussian start block (X + iY)/sqrt(2), shape (n_edges, p).

    Generated with NumPy's PCG64 (default_rng) in canonical dof order.
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_edges, p))
    y = rng.standard_normal((n_edges, p))
    return (x + 1j * y) / math.sqrt(2.0)


def path_gxmg(per_segment: int, a: float = 1.0, b: float = 1.0) -> np.ndarray:
    """Bloch parameters along Gamma(0,0) -> X(pi/a,0) -> M(pi/a,pi/b) -> Gamma.

    `per_segment` intervals per segment; 3*per_segment + 1 points, Gamma at both ends.
    Returns an array of shape (npts, 2).
    """
    s = per_segment
    pts = []
    for t in range(s):
        pts.append((math.pi / a * t / s, 0.0))
    for t in range(s):
        pts.append((math.pi / a, math.pi / b * t / s))
    for t in range(s + 1):
        f = 1.0 - t / s
        pts.append((math.pi / a * f, math.pi / b * f))
    k = np.array(pts, dtype=np.float64)
    k[-1] = (0.0, 0.0)
    return k


def uniform_k(rng: np.random.Generator, a: float = 1.0, b: float = 1.0) -> tuple:
    """One Bloch parameter uniform in the first Brillouin zone [-pi/a,pi/a] x [-pi/b,pi/b]."""
    return (float(rng.uniform(-math.pi / a, math.pi / a)),
            float(rng.uniform(-math.pi / b, math.pi / b)))


@dataclass
class Problem:
    """One band problem: grid, permittivity samples, Bloch parameters and block sizes."""
    n: int
    m: int
    a: float
    b: float
    eps: np.ndarray
    ks: np.ndarray
    nev: int
    nthrow: int
    seed: int
    tol: float = 1e-8
    levels: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def p(self) -> int:
        return self.nev + self.nthrow

    @property
    def n_edges(self) -> int:
        return 2 * self.n * self.m

    def start(self) -> np.ndarray:
        return start_block(self.n_edges, self.p, self.seed)


def config_c1(eps_one: bool = False) -> Problem:
    """32 x 32 grid, eps = 8.9 in the centred disc of radius 0.2 (or eps = 1), k = (pi/2, 0),
    8 eigenpairs, block size 8, 3 multigrid levels, start seed 0."""
    n = 32
    eps = np.ones(n * n) if eps_one else eps_disc(n, n, 1.0, 1.0, 8.9, 0.2)
    return Problem(n, n, 1.0, 1.0, eps, np.array([[math.pi / 2, 0.0]]), 8, 0, 0,
                   tol=1e-8, levels=3, name="c1-eps1" if eps_one else "c1-disc8.9")


def config_c2(per_segment: int = 10) -> Problem:
    """256 x 256 grid, square lattice of eps = 12 discs of radius 0.3 on eps = 1,
    16 eigenpairs (+8 throw-away) along Gamma-X-M-Gamma (31 points), 6 levels."""
    n = 256
    eps = eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    return Problem(n, n, 1.0, 1.0, eps, path_gxmg(per_segment), 16, 8, 1,
                   tol=1e-8, levels=6, name="c2-lattice12")


def config_c3(per_segment: int = 20) -> Problem:
    """1024 x 1024 grid, smoothed random two-phase field {1, 11.4}, 32 eigenpairs
    (+16 throw-away) at 61 points along Gamma-X-M-Gamma.  Relative residual tolerance 1e-6:
    next to Gamma the FP64 residual of the acoustic band bottoms out near
    u ||A|| / lambda_1 ~ 2e-7 at this mesh width, so 1e-8 cannot be reached by any FP64 run."""
    n = 1024
    eps = eps_random_field(n, n, 1.0, 1.0, seed=2, sigma=0.05, lo=1.0, hi=11.4)
    return Problem(n, n, 1.0, 1.0, eps, path_gxmg(per_segment), 32, 16, 2,
                   tol=1e-6, levels=0, name="c3-randfield")


def config_c4_problems(count: int = 64, master_seed: int = 3) -> list:
    """Independent single-k problems: n in {128,192,256,384,512}, disc lattices with radius
    in [0.1,0.45] and contrast in [2,13], nev in {4,8,16}, k uniform in the Brillouin zone."""
    ss = np.random.SeedSequence(master_seed)
    out = []
    for i, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        n = int(rng.choice([128, 192, 256, 384, 512]))
        r = float(rng.uniform(0.1, 0.45))
        c = float(rng.uniform(2.0, 13.0))
        nev = int(rng.choice([4, 8, 16]))
        k = uniform_k(rng)
        eps = eps_disc_lattice(n, n, 1.0, 1.0, c, r)
        seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(Problem(n, n, 1.0, 1.0, eps, np.array([k]), nev, nev // 2, seed,
                           tol=1e-8, name=f"c4-{i}", meta={"radius": r, "contrast": c}))
    return out


def config_c4_small() -> list:
    """A reduced batch of the C4 kind for parity tests against the oracle: six single-k
    problems, n in {64, 96, 128} and nev in {4, 8, 16} (each n with two nev), disc lattices
    with seeded radius and contrast, k uniform in the Brillouin zone."""
    ss = np.random.SeedSequence(31)
    out = []
    specs = [(64, 4), (96, 8), (128, 16), (64, 16), (96, 4), (128, 8)]
    for i, (child, (n, nev)) in enumerate(zip(ss.spawn(len(specs)), specs)):
        rng = np.random.default_rng(child)
        r = float(rng.uniform(0.1, 0.45))
        c = float(rng.uniform(2.0, 13.0))
        k = uniform_k(rng)
        eps = eps_disc_lattice(n, n, 1.0, 1.0, c, r)
        seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(Problem(n, n, 1.0, 1.0, eps, np.array([k]), nev, nev // 2, seed,
                           tol=1e-8, name=f"c4small-{i}", meta={"radius": r, "contrast": c}))
    return out


def round_grid(n: int) -> int:
    """Round a grid size to n0 * 2**l with n0 in [8, 15], so the hierarchy reaches 8..15."""
    l = 0
    while n >= 16:
        n //= 2
        l += 1
    return n << l


def config_c5_requests(count: int, master_seed: int = 4, n_lo: int = 64, n_hi: int = 2048,
                       nev_lo: int = 4, nev_hi: int = 32, nk_lo: int = 11, nk_hi: int = 61) -> list:
    """Band-path requests for the serving loop: n log-uniform in [n_lo, n_hi] (rounded so the
    hierarchy ends between 8 and 15 cells), nev uniform, path length uniform, eps from the
    disc-lattice or the random-field generator."""
    ss = np.random.SeedSequence(master_seed)
    out = []
    for i, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        n = round_grid(int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))))
        nev = int(rng.integers(nev_lo, nev_hi + 1))
        nk = int(rng.integers(nk_lo, nk_hi + 1))
        seg = max(1, (nk - 1) // 3)
        ks = path_gxmg(seg)[:nk] if nk <= 3 * seg + 1 else path_gxmg(seg)
        if rng.uniform() < 0.5:
            eps = eps_disc_lattice(n, n, 1.0, 1.0, float(rng.uniform(2, 13)),
                                   float(rng.uniform(0.1, 0.45)))
            kind = "disc"
        else:
            eps = eps_random_field(n, n, 1.0, 1.0, int(rng.integers(0, 2 ** 31 - 1)),
                                   hi=float(rng.uniform(2, 13)))
            kind = "field"
        seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(Problem(n, n, 1.0, 1.0, eps, ks, nev, max(2, nev // 2), seed, tol=1e-8,
                           name=f"c5-{i}", meta={"kind": kind}))
    return out
