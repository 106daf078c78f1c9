"""Section 4 and Section 7: modified block preconditioned inverse iteration (PINVIT) with
null-space elimination, Ritz step, and throw-away vectors.

One step of the iteration (the Ritz version of the block method, gradient variant):
    R      = A E - M E Lambda                         (Lambda diagonal after the Ritz step)
    E_hat  = E - B R,  B = one V-cycle for A + mu M   (Section 5)
    solve  L^* M L Phi = L^* M E_hat  by nodal V-cycles,  E_hat <- E_hat - L Phi
    (k = 0: also remove the two constant edge fields, M-orthogonally)
    generalized Householder on a basis of span[E_hat, E] (LOBPCG: also E_prev)
    Ritz: (Q^* A Q) = U D U^*, ascending; E <- (Q U)[:, :p], Lambda <- D[:p]
The iteration works with p = nev + nthrow vectors and stops when the first nev relative
residuals ||A e_i - lambda_i M e_i||_2 / (lambda_i ||M e_i||_2) are at most tol.

Pinned by: convergence to the dense generalized eigensolve and to the constant-epsilon
closed form (tests).  Iteration counts of the paper's experiments are parity unpinned
(its figures are not available).
"""
from __future__ import annotations

import numpy as np

from .householder import m_householder, reference_columns

__all__ = ["Projector", "ritz", "initial_block", "pinvit", "residuals", "gram_orthonormalize"]


class Projector:
    """Null-space elimination (Section 4): u <- u - L Phi with L^* M L Phi = L^* M u solved
    approximately by `cycles` nodal V-cycles; at k = 0 additionally the constant edge
    fields (the explicitly known remainder of the kernel) are removed M-orthogonally.

    Plane-wave deflation (deflate=True, the default; a reading of Sections 4-5): P = L^* M L
    has the exact eigenvector w = fem.plane_wave (lambda_w = fem.plane_wave_eigenvalue),
    whose eigenvalue shrinks like |k|^2 h^2 next to the Gamma point, where P turns singular
    (Section 3 notes the k = 0 kernel).  The nodal solve splits along it: the component of
    Phi along w is solved exactly, c = (w^* b) / (w^* w lambda_w) (zero at Gamma, where
    w^* b = 0), and the V-cycles act on the orthogonal complement (right-hand side and
    result orthogonalised against w).  With exact nodal solves this is the same
    projection; with V-cycles it removes the near-singular mode exactly, which a
    single-precision nodal cycle cannot do (its residual loses that mode to rounding).
    deflate=False is the unsplit form."""

    def __init__(self, disc, hier, cycles: int, deflate: bool = True):
        self.disc, self.hier, self.cycles = disc, hier, cycles
        self.X = None
        if disc.gamma:
            X = disc.constant_fields()
            nrm = np.sqrt(np.real(np.einsum("ij,ij->j", X.conj(), disc.M @ X)))
            self.X = X / nrm
        self.w = None
        if deflate:
            self.w, self.lam_w = disc.plane_wave()

    def __call__(self, U):
        d = self.disc
        b = d.L.conj().T @ (d.M @ U)
        if self.w is None:
            phi = self.hier.nodal_solve(b, self.cycles)
        else:
            w, ww = self.w, np.real(np.vdot(self.w, self.w))
            s = (w.conj() @ b) / ww
            c = s / self.lam_w if self.lam_w > 0 else np.zeros_like(s)
            phi = self.hier.nodal_solve(b - np.outer(w, s), self.cycles)
            phi = phi - np.outer(w, (w.conj() @ phi) / ww) + np.outer(w, c)
        U = U - d.L @ phi
        if self.X is not None:
            U = U - self.X @ (self.X.conj().T @ (d.M @ U))
        return U


def gram_orthonormalize(S, M):
    """An M-orthonormal basis of range(S) through the Gram matrix (not the paper's
    Householder route; for comparison with implementations that orthonormalise this way):
    G = S^* M S scaled to unit diagonal by D, Cholesky D G D = L L^*, Q = S D L^{-*}.  Same
    span as the Householder factorisation when S has full rank; the rounding differs, which
    shows in the iteration counts of ill-conditioned cases (p = nev + 1)."""
    G = S.conj().T @ (M @ S)
    dsc = 1.0 / np.sqrt(np.real(np.diag(G)))
    L = np.linalg.cholesky(G * np.outer(dsc, dsc))
    return (S * dsc) @ np.linalg.inv(L).conj().T


def ritz(Q, A, p: int, zero_thr: float = None):
    """Ritz step on the M-orthonormal basis Q: eigen-decomposition of Q^* A Q (ascending);
    returns the p smallest pairs, skipping Ritz values below zero_thr if given."""
    H = Q.conj().T @ (A @ Q)
    H = 0.5 * (H + H.conj().T)
    theta, U = np.linalg.eigh(H)
    sel = np.arange(len(theta))
    if zero_thr is not None:
        sel = sel[theta > zero_thr]
    sel = sel[:p]
    return theta[sel], Q @ U[:, sel]


def residuals(disc, E, lam, absolute: bool = False):
    """R = A E - M E diag(lam) and the relative residual norms, or with absolute=True the
    defects ||A e_i - lambda_i M e_i||_2 of the M-normalised columns (the stopping measure
    of the paper's band-structure experiment, Section 8)."""
    AE = disc.A @ E
    ME = disc.M @ E
    R = AE - ME * lam[None, :]
    if absolute:
        return R, np.linalg.norm(R, axis=0)
    rel = np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(ME, axis=0))
    return R, rel


def initial_block(disc, proj, E0, p: int, zero_thr: float = None, ortho: str = "householder"):
    """Start block: eliminate the null space, M-orthonormalise by generalized Householder
    (or through the Gram matrix, ortho="gram"), and rotate to Ritz vectors."""
    S = proj(np.asarray(E0, dtype=np.complex128))
    if ortho == "gram":
        Q = gram_orthonormalize(S, disc.M)
    else:
        Q, _ = m_householder(S, disc.M, reference_columns(disc.n, disc.m, S.shape[1]))
    return ritz(Q, disc.A, p, zero_thr)


def pinvit(disc, hier, proj, E, lam, nev: int, tol: float, max_iter: int,
           variant: str = "gradient", log=None, absolute: bool = False, ortho: str = "householder"):
    """Run the iteration from an M-orthonormal Ritz block (E, lam).

    The gradient variant minimises the Rayleigh quotient over span[E_hat, E].  The same
    span is factorised through the basis [E, E - E_hat]: near convergence E_hat and E
    agree to the size of the correction, and a Householder factorisation of [E_hat, E]
    then determines the new directions only to u/||C|| (residuals stall near 1e-7 at the
    32 x 32 workload).  The null-space elimination is linear, so with C = B R the projected
    block is [Pi E, Pi C] and E - E_hat = Pi C; the whole block entering the factorisation
    is projected, so that every iteration vector stays (approximately) orthogonal to the
    gradients.  LOBPCG adds the previous block the same way, as the direction
    E_prev - E (E^* M E_prev) removed of its E part.

    absolute=True stops on the defects ||A e_i - lambda_i M e_i||_2 instead of the relative
    residuals.  ortho="gram" orthonormalises through the Gram matrix instead of Householder
    (gram_orthonormalize).  Returns (lam, E, relres, iterations, converged)."""
    p = E.shape[1]
    ref = reference_columns(disc.n, disc.m, 3 * p if variant == "lobpcg" else 2 * p)
    E_prev = None
    it = 0
    while True:
        R, rel = residuals(disc, E, lam, absolute)
        if log is not None:
            log.append((it, lam.copy(), rel.copy()))
        if np.all(rel[:nev] <= tol):
            return lam, E, rel, it, True
        if it >= max_iter:
            return lam, E, rel, it, False
        C = hier.edge_vcycle(R)
        if variant == "lobpcg" and E_prev is not None:
            D = E_prev - E @ (E.conj().T @ (disc.M @ E_prev))
            S = proj(np.hstack([E, C, D]))
        else:
            S = proj(np.hstack([E, C]))
        if ortho == "gram":
            Q = gram_orthonormalize(S, disc.M)
        else:
            Q, _ = m_householder(S, disc.M, ref[:S.shape[1]])
        E_prev = E
        lam, E = ritz(Q, disc.A, p)
        it += 1
