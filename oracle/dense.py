"""The plain definition the iteration converges to (Section 1 and Section 4): the smallest
non-zero eigenvalues, with multiplicity, of the Hermitian pencil A e = lambda M e, and an
M-orthonormal basis of their invariant subspace.

Three references:
  * dense_eigs: scipy.linalg.eigh on the assembled dense pencil (small grids only); the
    null space (dimension nm, or nm + 1 at k = 0) is removed by count.
  * shift_invert_eigs: ARPACK shift-invert around a positive shift, for larger grids.
  * gradient_free_eigs: ARPACK on the pencil restricted to the M-orthogonal complement of
    the null space (exact projection by sparse direct solves), for large grids, where the
    kernel cluster of dimension nm defeats the shift-invert certificate.

Pinned by: the closed-form spectrum for constant epsilon and the kernel-dimension count
(tests); gradient_free_eigs also against dense_eigs, including degenerate spectra.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

__all__ = ["dense_eigs", "kernel_dimension", "shift_invert_eigs", "gradient_free_eigs"]


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


def gradient_free_eigs(disc, count: int, shift: float = 1.0, extra: int = 8, tol: float = 1e-13):
    """Smallest `count` non-zero eigenvalues of (A, M), ascending, by ARPACK on the operator
    Pi (A + shift M)^{-1} M, Pi the exact M-orthogonal projection onto the complement of the
    null space (u - L P^{-1} L^* M u, P = L^* M L by a sparse direct solve; at k = 0 also the
    two constant edge fields).

    (A + shift M)^{-1} M maps the gradients into themselves (A L = 0), so it commutes with Pi
    and the restricted operator is M-self-adjoint with eigenvalues 1 / (lambda + shift) on the
    non-zero spectrum and 0 on the null space: the largest `count + extra` are the wanted
    smallest eigenvalues, and no zero cluster competes.  Returns (lam, V); within a
    degenerate cluster ARPACK's vectors span the eigenspace but need not be M-orthogonal.
    """
    import scipy.sparse as sp

    n, m = disc.n, disc.m
    A, M, L = disc.A.tocsc(), disc.M.tocsc(), disc.L.tocsc()
    K = spla.splu((A + shift * M).tocsc())
    P = disc.P.tocsc()
    if disc.gamma:   # P has the constants as kernel; the right-hand sides are orthogonal to them
        Pr = spla.splu(P[1:, 1:].tocsc())

        def psolve(b):
            x = np.zeros_like(b)
            x[1:] = Pr.solve(b[1:])
            return x
        X = disc.constant_fields()
        X = X / np.sqrt(np.real(np.einsum("ij,ij->j", X.conj(), M @ X)))
    else:
        Pf = spla.splu(P)
        psolve = Pf.solve
        X = None
    LhM = (L.conj().T @ M).tocsc()

    def project(u):
        u = u - L @ psolve(LhM @ u)
        if X is not None:
            u = u - X @ (X.conj().T @ (M @ u))
        return u

    N = 2 * n * m
    opinv = spla.LinearOperator((N, N), matvec=lambda x: project(K.solve(np.asarray(x).reshape(-1))),
                                dtype=np.complex128)
    k = count + extra
    rng = np.random.default_rng(0)
    v0 = project(rng.standard_normal(N) + 1j * rng.standard_normal(N))
    lam, V = spla.eigsh(A, k=k, M=M, sigma=-shift, which="LM", OPinv=opinv, v0=v0, tol=tol,
                        ncv=max(2 * k + 1, 40))
    order = np.argsort(lam)
    return lam[order][:count], V[:, order][:, :count]
