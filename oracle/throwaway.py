"""Section 7: the throw-away study -- how the rate of convergence of the wanted eigenpairs
changes with the number t of additional ("throw-away") vectors carried in the block.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The analysis of Section 7 is for the unpreconditioned block inverse iteration
E <- A^{-1} E: column i of the block converges to the i-th eigenvector with the tangent of
its angle shrinking by lambda_i / lambda_{p+1} per step, p = nev + t, so a wider block
converges faster.  For the iteration that is actually run (one preconditioner application
per step, Rayleigh-Ritz over the block and its correction) the paper measures the rate
instead; this module measures it the same way: from the per-iteration relative residuals
of the iteration in `pinvit`, a residual being proportional to the tangent of the
eigenvector's angle once the eigenvalue is separated.

  observed_rate     -- geometric rate of a residual sequence: least-squares slope of
                       log(residual) against the iteration index over the asymptotic window
  inverse_iteration_rate -- the Section 7 bound lambda_i / lambda_{p+1}, and its shifted
                       form (lambda_i + mu) / (lambda_{p+1} + mu) for the exact inverse of
                       A + mu M used as preconditioner
  study             -- runs the iteration for each t from the first p columns of one start
                       block and returns, per t, the iteration count and the observed rates of
                       the chosen eigenpairs

Pinned by (tests): exact geometric sequences (the rate is recovered to rounding); the
textbook block inverse iteration on a diagonal pencil, whose observed rates approach
lambda_i / lambda_{p+1} as Section 7 derives; the iteration with the exact inverse of
A + mu M as preconditioner and the exact null-space projection, whose observed rates stay
below the shifted inverse-iteration bound and shrink as t grows.
"""
from __future__ import annotations

import numpy as np

from .pinvit import initial_block, pinvit

__all__ = ["observed_rate", "inverse_iteration_rate", "study"]


def observed_rate(res, upper: float = 1e-2, lower: float = 0.0, min_points: int = 3) -> float:
    """Geometric convergence rate of the residual sequence res[0], res[1], ... (one entry
    per iteration): exp of the least-squares slope of log(res[j]) over the window that
    starts at the first j with res[j] <= upper and ends at the last j with res[j] > lower
    (the pre-asymptotic phase and a floor set by rounding are left out).  NaN when the
    window holds fewer than min_points entries."""
    r = np.asarray(res, dtype=np.float64)
    below = np.nonzero(r <= upper)[0]
    if below.size == 0:
        return float("nan")
    j0 = int(below[0])
    above = np.nonzero(r > lower)[0]
    j1 = int(above[-1]) if above.size else -1
    if j1 - j0 + 1 < min_points:
        return float("nan")
    j = np.arange(j0, j1 + 1, dtype=np.float64)
    slope = np.polyfit(j, np.log(r[j0:j1 + 1]), 1)[0]
    return float(np.exp(slope))


def inverse_iteration_rate(lam, i: int, p: int, mu: float = 0.0) -> float:
    """Section 7: rate (lambda_i + mu) / (lambda_{p+1} + mu) of column i (1-based) of the block
    inverse iteration with p columns for the pencil shifted by mu (mu = 0: the paper's
    lambda_i / lambda_{p+1}); lam holds the smallest non-zero eigenvalues ascending, at least
    p + 1 of them."""
    return float((lam[i - 1] + mu) / (lam[p] + mu))


def study(disc, hier, proj, E0, nev: int, ts, indices, tol: float, max_iter: int,
          upper: float = 1e-2, lower: float = 0.0, ortho: str = "householder"):
    """For each t in ts: p = nev + t, the iteration started from the first p columns of E0
    (null-space projected, M-orthonormalised and Ritz-rotated), run to the relative
    residual tol for the first nev pairs; returns a list of dicts with t, p, iterations,
    converged, and the observed rate of each eigenpair in `indices` (1-based, <= nev).
    ortho selects the orthonormalisation of the iteration (pinvit)."""
    out = []
    for t in ts:
        p = nev + t
        lam0, E = initial_block(disc, proj, E0[:, :p], p, ortho=ortho)
        log = []
        lam, _, _, it, conv = pinvit(disc, hier, proj, E, lam0, nev, tol, max_iter, log=log, ortho=ortho)
        hist = np.array([rel[:nev] for (_, _, rel) in log])
        rates = {i: observed_rate(hist[:, i - 1], upper, lower) for i in indices}
        out.append({"t": int(t), "p": int(p), "iterations": int(it), "converged": bool(conv),
                    "lam": lam[:nev].copy(), "rates": rates, "history": hist})
    return out
