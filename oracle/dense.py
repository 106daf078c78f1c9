"""The plain definition the iteration converges to (Section 1 and Section 4): the smallest
non-zero eigenvalues, with multiplicity, of the Hermitian pencil A e = lambda M e, and an
M-orthonormal basis of their invariant subspace.

Two references:
  * dense_eigs: scipy.linalg.eigh on the assembled dense pencil (small grids only); the
    null space (dimension nm, or nm + 1 at k = 0) is removed by count.
  * shift_invert_eigs: ARPACK shift-invert around a positive shift, for larger grids.

Pinned by: the closed-form spectrum for constant epsilon and the kernel-dimension count.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

__all__ = ["dense_eigs", "kernel_dimension", "shift_invert_eigs"]


def kernel_dimension(n: int, m: int, gamma: bool) -> int:
    """Dimension of the null space of A: the nm gradients of the Bloch nodal space, plus
    the remaining constant field at k = 0 (where the constant potential has zero gradient
    and both constant edge fields are curl-free): nm + 1."""
    return n * m + (1 if gamma else 0)


def dense_eigs(disc, count: int):
    """Smallest `count` non-zero eigenpairs of (A, M) by a dense generalized eigensolve.

    Returns (lam, E, all_lam) with E M-orthonormal (columns = eigenvectors)."""
    A = disc.A.toarray()
    M = disc.M.toarray()
    lam, V = sla.eigh(A, M)
    kd = kernel_dimension(disc.n, disc.m, disc.gamma)
    return lam[kd:kd + count], V[:, kd:kd + count], lam


def shift_invert_eigs(disc, count: int, sigma: float, extra: int = 8):
    """Eigenvalues of (A, M) nearest to sigma by ARPACK shift-invert, returned ascending
    with those below `1e-8 * sigma` (the kernel) removed.

    If the returned set reaches the kernel cluster, every eigenvalue in (0, 2 sigma) has
    been found: each of them is closer to sigma than the zero eigenvalues are."""
    A = disc.A.tocsc()
    M = disc.M.tocsc()
    k = count + extra
    lam, V = spla.eigsh(A, k=k, M=M, sigma=sigma, which="LM", tol=1e-13)
    order = np.argsort(lam)
    lam = lam[order]
    V = V[:, order]
    reached_kernel = bool(np.any(np.abs(lam) < 1e-8 * sigma))
    keep = lam > 1e-8 * sigma
    return lam[keep], V[:, keep], reached_kernel
