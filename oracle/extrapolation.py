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

Pinned by: Courant-Fischer (extrapolated Ritz values are upper bounds of the true
eigenvalues; with the exact eigenvectors of the same k in the span they are reproduced),
and the end-to-end path results against dense solves (tests).
"""
from __future__ import annotations

import numpy as np

from .fem import Discretization
from .householder import m_householder, reference_columns
from .multigrid import Hierarchy
from .pinvit import Projector, initial_block, pinvit, ritz

__all__ = ["extrapolate", "solve_path"]


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
