"""Section 4: generalized Householder factorisation in the M inner product.

Given a block X (N x q) and a prescribed M-orthonormal basis P of canonical M-unit vectors
with disjoint supports, reflections Q_i = I - 2 v_i (v_i^* M) / (v_i^* M v_i) are chosen so
that Q_q ... Q_1 X = P R with R upper triangular; then E = Q_1 ... Q_q P is M-orthonormal
and range(E) contains range(X) (if R is singular the basis is extended by the P-directions).

Pinned by: Q_i^2 = I, M-self-adjointness of Q_i, E^* M E = I, X = E R and
range(X) in range(E) (tests), which are the properties the paper states.
"""
from __future__ import annotations

import numpy as np

__all__ = ["reference_columns", "m_householder"]


def reference_columns(n: int, m: int, q: int) -> np.ndarray:
    """Indices of q pairwise M-uncoupled x-edges: x-edges couple in M only to the x-edges
    directly above and below, so x-edges in even rows 0, 2, ..., (excluding the last row
    when m is odd, which touches row 0 through the wrap) are mutually uncoupled.  They are
    taken in row-major order."""
    rows = list(range(0, m - 1 if m % 2 else m, 2))
    idx = [r * n + c for r in rows for c in range(n)]
    if q > len(idx):
        raise ValueError("block too wide for the reference basis of this grid")
    # spread the chosen edges over the grid
    step = max(1, len(idx) // q)
    return np.array(idx[::step][:q], dtype=np.int64)


def m_householder(X: np.ndarray, M, ref_idx: np.ndarray, keep_reflectors: bool = False):
    """Generalized Householder factorisation of X (N x q) with respect to M.

    Returns (E, R) with E = Q_1 ... Q_q P (M-orthonormal, N x q) and Q_q ... Q_1 X = P R.
    With keep_reflectors=True also returns the list of (v_i, v_i^* M v_i)."""
    N, q = X.shape
    d = np.real(M.diagonal())
    P = np.zeros((N, q), dtype=np.complex128)
    P[ref_idx, np.arange(q)] = 1.0 / np.sqrt(d[ref_idx])
    MP = M @ P
    W = np.array(X, dtype=np.complex128, copy=True)
    R = np.zeros((q, q), dtype=np.complex128)
    refl = []
    for j in range(q):
        z = W[:, j]
        znrm = np.sqrt(max(np.real(np.vdot(z, M @ z)), 0.0))
        c = MP[:, :j].conj().T @ z                      # <P_i, M z>, i < j
        z_rest = z - P[:, :j] @ c
        # The components along P_1..P_{j-1} belong to R; a second pass removes what the
        # first left behind in rounding, so that the reflection below leaves P_i (i < j)
        # fixed to working precision relative to z_rest itself.
        c2 = MP[:, :j].conj().T @ z_rest
        z_rest = z_rest - P[:, :j] @ c2
        R[:j, j] = c + c2
        nrm = np.sqrt(max(np.real(np.vdot(z_rest, M @ z_rest)), 0.0))
        if nrm <= 1e-14 * znrm or nrm == 0.0:
            # column dependent on the previous ones: R_jj = 0 and Q_j = I; the basis is
            # extended by the (reflected) P_j, as the paper describes.
            refl.append(None)
            continue
        pz = np.vdot(MP[:, j], z_rest)                  # <P_j, M z_rest>
        phase = pz / abs(pz) if abs(pz) > 0 else 1.0
        r = -phase * nrm
        R[j, j] = r
        v = z_rest - r * P[:, j]
        Mv = M @ v
        vMv = np.real(np.vdot(v, Mv))
        refl.append((v, Mv, vMv))
        W[:, j:] = W[:, j:] - np.outer(v, (Mv.conj() @ W[:, j:]) * (2.0 / vMv))
    E = P.copy()
    for j in range(q - 1, -1, -1):
        if refl[j] is None:
            continue
        v, Mv, vMv = refl[j]
        E = E - np.outer(v, (Mv.conj() @ E) * (2.0 / vMv))
    if keep_reflectors:
        return E, R, [(t[0], t[2]) if t is not None else None for t in refl]
    return E, R
