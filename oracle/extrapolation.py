"""Section 6: starting blocks across Bloch parameters.

For every Bloch parameter after the first, the starting block is the set of the p smallest
non-zero minima of the Rayleigh quotient of the new pencil (A(k), M(k)) on the span of the
eigenvector blocks computed for up to three preceding parameters (quadratic
one-dimensional extrapolation in the paper's terms).  The span is first cleared of the new
gradient space (the null-space elimination of Section 4), M-orthonormalised by the
generalized Householder factorisation, and then a Ritz step selects the vectors.  Ritz
values below `zero_rel` times the smallest eigenvalue of the preceding parameter count as
zero (left-over gradient content) and are skipped.

The first parameter of a path starts from a seeded random block (the nested iteration of
Section 6 is not used here).

On the kappa x kappa grid of Bloch parameters (Section 6) the sources of each point follow
the raster the paper describes: the first row left to right from its predecessors, the
first three columns upward from the points below, and every other point from the three
points to its left in its row.  The paper lists the horizontal rule for rows j >= 3 only;
rows 1 and 2 beyond the third column are read the same way (the three points to the left
exist there too).

Pinned by: Courant-Fischer (extrapolated Ritz values are upper bounds of the true
eigenvalues; with the exact eigenvectors of the same k in the span they are reproduced),
and the end-to-end path results against dense solves (tests).
"""
from __future__ import annotations

import numpy as np

from .dense import dense_eigs
from .fem import Discretization, phases
from .householder import m_householder, reference_columns
from .multigrid import Hierarchy, edge_prolongation, level_sizes
from .pinvit import Projector, initial_block, pinvit, ritz

__all__ = ["extrapolate", "solve_path", "raster_k", "raster_sources", "solve_grid", "level_kappas",
           "nested_start"]


def extrapolate(disc, proj, history, p: int, zero_thr: float):
    """Rayleigh-quotient extrapolation from the blocks in `history` (most recent first)."""
    S = proj(np.hstack(history))
    Q, _ = m_householder(S, disc.M, reference_columns(disc.n, disc.m, S.shape[1]))
    return ritz(Q, disc.A, p, zero_thr)


def solve_path(n, m, a, b, eps, ks, nev, nthrow, start, tol=1e-8, max_iter=200, mu=None,
               nodal_cycles=2, max_levels=0, coarsest_min=8, depth=3, zero_rel=1e-2,
               variant="gradient", nu_pre=1, nu_post=1, on_point=None):
    """Band path: eigenpairs for every Bloch parameter in ks (shape (nk, 2)).

    Returns a list of dicts with lam (nev), relres (nev), iterations and converged flags."""
    p = nev + nthrow
    history = []
    out = []
    prev_lam1 = None
    for t, (k1, k2) in enumerate(ks):
        disc = Discretization(n, m, a, b, eps, float(k1), float(k2))
        hier = Hierarchy(disc, mu=mu, max_levels=max_levels, coarsest_min=coarsest_min,
                         nu_pre=nu_pre, nu_post=nu_post)
        proj = Projector(disc, hier, nodal_cycles)
        if t == 0:
            lam, E = initial_block(disc, proj, start, p)
        else:
            lam, E = extrapolate(disc, proj, history[:depth], p, zero_rel * prev_lam1)
        lam, E, rel, it, conv = pinvit(disc, hier, proj, E, lam, nev, tol, max_iter,
                                       variant=variant)
        history.insert(0, E)
        history = history[:depth]
        prev_lam1 = float(lam[0])
        rec = {"k": (float(k1), float(k2)), "lam": lam[:nev].copy(), "relres": rel[:nev].copy(),
               "iterations": it, "converged": conv}
        out.append(rec)
        if on_point is not None:
            on_point(t, rec, E)
    return out


def raster_k(kappa: int, i: int, j: int, a: float = 1.0, b: float = 1.0):
    """Section 6: the Bloch parameter k_ij = (pi/a (2 i/(kappa-1) - 1), pi/b (2 j/(kappa-1) - 1))."""
    return (np.pi / a * (2.0 * i / (kappa - 1) - 1.0), np.pi / b * (2.0 * j / (kappa - 1) - 1.0))


def raster_sources(kappa: int, i: int, j: int):
    """Section 6: the grid points (i', j') whose eigenvector blocks give the start block of
    point (i, j), oldest first: none for (0, 0); along the first row the up to three points to
    the left; in the first three columns the up to three points below; elsewhere the three
    points to the left."""
    if not (0 <= i < kappa and 0 <= j < kappa):
        raise ValueError("point outside the grid")
    if j == 0:
        return [(s, 0) for s in range(max(0, i - 3), i)]
    if i <= 2:
        return [(i, s) for s in range(max(0, j - 3), j)]
    return [(s, j) for s in range(i - 3, i)]


def solve_grid(n, m, a, b, eps, kappa, nev, nthrow, start, tol=1e-8, max_iter=200, mu=None,
               nodal_cycles=2, max_levels=0, coarsest_min=8, zero_rel=1e-2, absolute=False,
               nu_pre=1, nu_post=1):
    """Every point of the kappa x kappa grid in raster order (row j = 0 .. kappa-1, within a
    row i = 0 .. kappa-1), (0, 0) from `start`, every other point extrapolated from the blocks
    of raster_sources (most recent first) with the zero threshold zero_rel times the smallest
    eigenvalue of the most recent source.  Returns a list of dicts in raster order."""
    p = nev + nthrow
    blocks = {}
    out = []
    for j in range(kappa):
        for i in range(kappa):
            k1, k2 = raster_k(kappa, i, j, a, b)
            disc = Discretization(n, m, a, b, eps, k1, k2)
            hier = Hierarchy(disc, mu=mu, max_levels=max_levels, coarsest_min=coarsest_min,
                             nu_pre=nu_pre, nu_post=nu_post)
            proj = Projector(disc, hier, nodal_cycles)
            src = raster_sources(kappa, i, j)
            if not src:
                lam, E = initial_block(disc, proj, start, p)
            else:
                hist = [blocks[q][0] for q in reversed(src)]
                lam, E = extrapolate(disc, proj, hist, p, zero_rel * blocks[src[-1]][1])
            lam, E, rel, it, conv = pinvit(disc, hier, proj, E, lam, nev, tol, max_iter,
                                           absolute=absolute)
            blocks[(i, j)] = (E, float(lam[0]))
            out.append({"ij": (i, j), "k": (k1, k2), "lam": lam[:nev].copy(),
                        "relres": rel[:nev].copy(), "iterations": it, "converged": conv})
    return out


def level_kappas(n: int, m: int, eps, sizes):
    """kappa = 1/eps on every level of the hierarchy: each coarse cell takes the mean of its
    2 x 2 children (the rediscretisation that equals the Galerkin coarse operators)."""
    kap = [1.0 / np.asarray(eps, dtype=np.float64).reshape(m, n)]
    for (cn, cm) in sizes[1:]:
        f = kap[-1]
        kap.append(0.25 * (f[0::2, 0::2] + f[0::2, 1::2] + f[1::2, 0::2] + f[1::2, 1::2]))
    return [k.reshape(-1) for k in kap]


def nested_start(n, m, a, b, eps, k1, k2, nev, nthrow, tol_levels=1e-3, max_iter=200, mu=None,
                 nodal_cycles=2, max_levels=0, coarsest_min=8, nu_pre=1, nu_post=1):
    """Section 6, first Bloch parameter: the p = nev + nthrow smallest non-zero eigenpairs of
    the coarsest level by a dense generalized eigensolve; then for each finer level the block
    is prolongated (the embedding of the coarse edge space) and, below the finest level,
    iterated on that level to the relative residual tol_levels.  Returns the block
    prolongated to the finest level and the iterations per level (finest first; 0 for the
    finest and the coarsest)."""
    p = nev + nthrow
    sizes = level_sizes(n, m, max_levels, coarsest_min)
    kap = level_kappas(n, m, eps, sizes)
    L = len(sizes)
    al, be = phases(k1, k2, a, b)
    nc, mc = sizes[-1]
    _, E, _ = dense_eigs(Discretization(nc, mc, a, b, 1.0 / kap[-1], k1, k2), p)
    iters = [0] * L
    for l in range(L - 2, -1, -1):
        nf, mf = sizes[l]
        E = edge_prolongation(nf, mf, a, b, al, be) @ E
        if l == 0:
            break
        disc = Discretization(nf, mf, a, b, 1.0 / kap[l], k1, k2)
        hier = Hierarchy(disc, mu=mu, max_levels=L - l, coarsest_min=coarsest_min,
                         nu_pre=nu_pre, nu_post=nu_post)
        proj = Projector(disc, hier, nodal_cycles)
        lam, E = initial_block(disc, proj, E, p)
        lam, E, _, it, _ = pinvit(disc, hier, proj, E, lam, nev, tol_levels, max_iter)
        iters[l] = it
    return E, iters
