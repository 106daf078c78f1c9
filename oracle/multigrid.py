"""Section 5 (Geometric multigrid method), written plainly in FP64.

* Hierarchy by bisection: level 0 is the finest n x m grid; level l+1 halves both
  directions.  Coarsening continues while both sizes are even and their halves are at
  least `coarsest_min` (8 by default), up to `max_levels` levels (0 = no limit).
* Prolongations are the natural embeddings of the nested coarse spaces into the fine ones:
  the fine edge degrees of freedom of a coarse edge function are its line integrals along
  the fine edges, and the fine nodal values of a coarse Q1 function are its point values.
  Both are evaluated from the coarse cell's local shape functions and the Bloch phase map.
* Coarse matrices by the Galerkin approach: A_c = P^H A P, M_c = P^H M P, and for the
  nodal Laplacian P_c = Pn^H P Pn.
* Edge smoother: block Gauss-Seidel over overlapping node patches (the four edges that
  touch a node, with periodic wrap) for K = A + mu M.  The 4x4 patch systems are solved in
  the stabilised way the paper describes: with D the (diagonal) patch mass matrix and g the
  node's gradient on its four edges, T = D^{-1/2} Q with Q unitary and Q e1 parallel to
  D^{1/2} g splits T^H K T into the 1x1 gradient block (= mu) and a 3x3 Hermitian positive
  definite block, which is solved by Cholesky.
* Nodal smoother: point Gauss-Seidel for P.
* Gauss-Seidel ordering: nodes are coloured (p1 mod 2) + 2 (p2 mod 2); nodes of one colour
  have uncoupled patches (even grid sizes), so all nodes of a colour are relaxed together.
  Pre-smoothing visits colours 0,1,2,3, post-smoothing 3,2,1,0 (symmetric V-cycle).
* Coarsest level: direct solve (Cholesky of K_c; for P_c at k = 0, where it is singular
  with the constants as kernel, the pseudo-inverse).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem

__all__ = ["edge_prolongation", "nodal_prolongation", "level_sizes", "Hierarchy"]


def level_sizes(n: int, m: int, max_levels: int = 0, coarsest_min: int = 8):
    """Grid sizes of the bisection hierarchy, finest first."""
    sizes = [(n, m)]
    while True:
        cn, cm = sizes[-1]
        if max_levels and len(sizes) >= max_levels:
            break
        if cn % 2 or cm % 2 or cn // 2 < coarsest_min or cm // 2 < coarsest_min:
            break
        sizes.append((cn // 2, cm // 2))
    return sizes


def edge_prolongation(nf: int, mf: int, a: float, b: float, alpha: complex, beta: complex):
    """Embedding of the coarse (nf/2 x mf/2) Bloch edge space into the fine one.

    Column g holds the line integrals of coarse basis function g along every fine edge.
    For a fine edge, the coarse cell containing its midpoint (the upper/right one when the
    edge lies on a coarse grid line; tangential continuity makes the choice irrelevant)
    carries the coarse function as phase * local shape function; the tangential component
    of the local shapes is constant along the fine edge."""
    nc, mc = nf // 2, mf // 2
    h1, h2 = a / nf, b / mf
    H1, H2 = a / nc, b / mc
    idx_c, ph_c = fem.cell_local_map(nc, mc, alpha, beta)
    rows, cols, vals = [], [], []
    f1, f2 = np.meshgrid(np.arange(nf), np.arange(mf), indexing="xy")
    f1 = f1.reshape(-1)
    f2 = f2.reshape(-1)
    # fine x-edges: midpoint ((f1 + 1/2) h1, f2 h2)
    mx1, mx2 = (f1 + 0.5) * h1, f2 * h2
    C1 = np.floor(mx1 / H1 + 1e-12).astype(int) % nc
    C2 = np.floor(mx2 / H2 + 1e-12).astype(int) % mc
    t2 = mx2 / H2 - np.floor(mx2 / H2 + 1e-12)
    cell = C2 * nc + C1
    fine = fem.x_index(f1, f2, nf, mf)
    for loc, shape in ((0, (1 - t2) / H1), (1, t2 / H1)):      # bottom, top
        rows.append(fine)
        cols.append(idx_c[cell, loc])
        vals.append(ph_c[cell, loc] * shape * h1)
    # fine y-edges: midpoint (f1 h1, (f2 + 1/2) h2)
    my1, my2 = f1 * h1, (f2 + 0.5) * h2
    C1 = np.floor(my1 / H1 + 1e-12).astype(int) % nc
    C2 = np.floor(my2 / H2 + 1e-12).astype(int) % mc
    t1 = my1 / H1 - np.floor(my1 / H1 + 1e-12)
    cell = C2 * nc + C1
    fine = fem.y_index(f1, f2, nf, mf)
    for loc, shape in ((2, (1 - t1) / H2), (3, t1 / H2)):      # left, right
        rows.append(fine)
        cols.append(idx_c[cell, loc])
        vals.append(ph_c[cell, loc] * shape * h2)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    keep = np.abs(v) > 0
    P = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(2 * nf * mf, 2 * nc * mc))
    P.sum_duplicates()
    return P


def nodal_prolongation(nf: int, mf: int, a: float, b: float, alpha: complex, beta: complex):
    """Embedding of the coarse Bloch Q1 space into the fine one: fine nodal values of each
    coarse basis function, from the coarse cell's bilinear shapes and corner phases."""
    nc, mc = nf // 2, mf // 2
    h1, h2 = a / nf, b / mf
    H1, H2 = a / nc, b / mc
    f1, f2 = np.meshgrid(np.arange(nf), np.arange(mf), indexing="xy")
    f1 = f1.reshape(-1)
    f2 = f2.reshape(-1)
    x1, x2 = f1 * h1, f2 * h2
    C1 = np.floor(x1 / H1 + 1e-12).astype(int)
    C2 = np.floor(x2 / H2 + 1e-12).astype(int)
    t1 = x1 / H1 - C1
    t2 = x2 / H2 - C2
    fine = fem.node_index(f1, f2, nf, mf)
    rows, cols, vals = [], [], []
    for d1, d2, w in ((0, 0, (1 - t1) * (1 - t2)), (1, 0, t1 * (1 - t2)),
                      (0, 1, (1 - t1) * t2), (1, 1, t1 * t2)):
        cn1, cn2 = C1 + d1, C2 + d2
        ph = np.ones(fine.shape, dtype=np.complex128)
        ph = np.where(cn1 == nc, ph * alpha, ph)
        ph = np.where(cn2 == mc, ph * beta, ph)
        rows.append(fine)
        cols.append(fem.node_index(cn1, cn2, nc, mc))
        vals.append(ph * w)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    keep = np.abs(v) > 0
    P = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(nf * mf, nc * mc))
    P.sum_duplicates()
    return P


def _extract(S, rows, cols):
    """Entries S[rows[i,j], cols[i,j]] of a sparse matrix as a dense array."""
    S = S.tocsr()
    flat = np.asarray(S[rows.reshape(-1), cols.reshape(-1)]).reshape(rows.shape)
    return flat


class _EdgeLevel:
    """One level of the edge hierarchy with its patch smoother data."""

    def __init__(self, n, m, a, b, A, M, mu, alpha, beta):
        self.n, self.m = n, m
        self.A, self.M = A.tocsr(), M.tocsr()
        self.K = (A + mu * M).tocsr()
        self.mu = mu
        p1, p2 = np.meshgrid(np.arange(n), np.arange(m), indexing="xy")
        p1 = p1.reshape(-1)
        p2 = p2.reshape(-1)
        self.colour = (p1 % 2) + 2 * (p2 % 2)
        self.patch = np.stack([fem.x_index(p1, p2, n, m), fem.x_index(p1 - 1, p2, n, m),
                               fem.y_index(p1, p2, n, m), fem.y_index(p1, p2 - 1, n, m)], axis=1)
        self.smoothable = (n % 2 == 0) and (m % 2 == 0)
        if not self.smoothable:
            return
        L = fem.lifting(n, m, alpha, beta, a, b)
        nodes = fem.node_index(p1, p2, n, m)
        g = _extract(L, self.patch, np.repeat(nodes[:, None], 4, axis=1))      # (nm, 4)
        rr = np.repeat(self.patch[:, :, None], 4, axis=2)
        cc = np.repeat(self.patch[:, None, :], 4, axis=1)
        Kloc = _extract(self.K, rr, cc)                                          # (nm,4,4)
        Mloc = _extract(self.M, rr, cc)
        self.mloc_offdiag = np.abs(Mloc - np.einsum("nii->ni", Mloc)[:, :, None] * np.eye(4)).max()
        d = np.real(np.einsum("nii->ni", Mloc))                                 # (nm, 4)
        z = np.sqrt(d) * g
        z = z / np.linalg.norm(z, axis=1, keepdims=True)
        theta = np.angle(z[:, 0])
        zp = z * np.exp(-1j * theta)[:, None]
        w = -zp
        w[:, 0] += 1.0
        ww = np.real(np.einsum("ni,ni->n", np.conj(w), w))
        Hh = np.eye(4)[None] - 2.0 * w[:, :, None] * np.conj(w)[:, None, :] / ww[:, None, None]
        Q = np.exp(1j * theta)[:, None, None] * Hh                              # Q e1 = z
        T = Q / np.sqrt(d)[:, :, None]                                           # D^{-1/2} Q
        Kt = np.einsum("nji,njk,nkl->nil", np.conj(T), Kloc, T)
        self.T = T
        self.Kt = Kt
        self.kt00 = np.real(Kt[:, 0, 0])
        self.chol = np.linalg.cholesky(Kt[:, 1:, 1:])                            # lower

    def patch_solve(self, nodes, r_loc):
        """Solve K_loc delta = r_loc for the given nodes, r_loc of shape (len, 4, p)."""
        T = self.T[nodes]
        y = np.einsum("nji,njp->nip", np.conj(T), r_loc)
        z = np.empty_like(y)
        z[:, 0, :] = y[:, 0, :] / self.kt00[nodes][:, None]
        Lc = self.chol[nodes]
        # forward substitution Lc w = y[1:], then back substitution Lc^H z = w
        yb = y[:, 1:, :]
        wv = np.empty_like(yb)
        for i in range(3):
            s = yb[:, i, :].copy()
            for j in range(i):
                s -= Lc[:, i, j][:, None] * wv[:, j, :]
            wv[:, i, :] = s / Lc[:, i, i][:, None]
        zb = np.empty_like(yb)
        for i in (2, 1, 0):
            s = wv[:, i, :].copy()
            for j in range(i + 1, 3):
                s -= np.conj(Lc[:, j, i])[:, None] * zb[:, j, :]
            zb[:, i, :] = s / np.conj(Lc[:, i, i])[:, None]
        z[:, 1:, :] = zb
        return np.einsum("nij,njp->nip", T, z)

    def gs_colour(self, x, b, c):
        nodes = np.nonzero(self.colour == c)[0]
        r = b - self.K @ x
        pidx = self.patch[nodes]
        delta = self.patch_solve(nodes, r[pidx])
        x[pidx] += delta
        return x


class _NodalLevel:
    def __init__(self, n, m, P):
        self.n, self.m = n, m
        self.P = P.tocsr()
        self.diag = np.real(self.P.diagonal())
        p1, p2 = np.meshgrid(np.arange(n), np.arange(m), indexing="xy")
        self.colour = ((p1 % 2) + 2 * (p2 % 2)).reshape(-1)

    def gs_colour(self, x, b, c):
        nodes = np.nonzero(self.colour == c)[0]
        r = b - self.P @ x
        x[nodes] += r[nodes] / self.diag[nodes][:, None]
        return x


class Hierarchy:
    """Edge and nodal multigrid hierarchies for one grid, permittivity and Bloch parameter.

    The finest-level matrices are the Section-3 assembly; every coarser level is Galerkin."""

    def __init__(self, disc, mu: float, max_levels: int = 0, coarsest_min: int = 8,
                 nu_pre: int = 1, nu_post: int = 1):
        self.disc = disc
        self.mu = mu
        self.nu_pre, self.nu_post = nu_pre, nu_post
        a, b = disc.a, disc.b
        al, be = disc.alpha, disc.beta
        self.sizes = level_sizes(disc.n, disc.m, max_levels, coarsest_min)
        self.Pe, self.Pn = [], []
        A, M, P = disc.A, disc.M, disc.P
        self.edge, self.nodal = [], []
        for li, (n, m) in enumerate(self.sizes):
            last = li == len(self.sizes) - 1
            if last:
                self.edge.append(None)
                self.nodal.append(None)
                self._coarse_edge = (A + mu * M).toarray()
                self._coarse_P = P.toarray()
                self.coarse_A, self.coarse_M = A, M
                break
            self.edge.append(_EdgeLevel(n, m, a, b, A, M, mu, al, be))
            self.nodal.append(_NodalLevel(n, m, P))
            Pe = edge_prolongation(n, m, a, b, al, be)
            Pn = nodal_prolongation(n, m, a, b, al, be)
            self.Pe.append(Pe)
            self.Pn.append(Pn)
            A = (Pe.conj().T @ A @ Pe).tocsr()
            M = (Pe.conj().T @ M @ Pe).tocsr()
            P = (Pn.conj().T @ P @ Pn).tocsr()
        self._ce_factor = sla.cho_factor(self._coarse_edge, lower=True)
        lam, V = np.linalg.eigh(self._coarse_P)
        keep = lam > 1e-12 * lam.max()
        self._cp_pinv = (V[:, keep] / lam[keep]) @ V[:, keep].conj().T

    @property
    def nlevels(self):
        return len(self.sizes)

    # ---- edge V-cycle for K = A + mu M -------------------------------------------------
    def edge_vcycle(self, b, level: int = 0):
        """One V(nu_pre, nu_post) cycle with zero initial guess: returns x ~ K_level^{-1} b."""
        if level == self.nlevels - 1:
            return sla.cho_solve(self._ce_factor, b)
        lv = self.edge[level]
        x = np.zeros_like(b)
        for _ in range(self.nu_pre):
            for c in (0, 1, 2, 3):
                x = lv.gs_colour(x, b, c)
        r = b - lv.K @ x
        Pe = self.Pe[level]
        x = x + Pe @ self.edge_vcycle(Pe.conj().T @ r, level + 1)
        for _ in range(self.nu_post):
            for c in (3, 2, 1, 0):
                x = lv.gs_colour(x, b, c)
        return x

    def edge_operator(self, level: int):
        if level == self.nlevels - 1:
            return sp.csr_matrix(self._coarse_edge)
        return self.edge[level].K

    # ---- nodal V-cycle for P -------------------------------------------------------------
    def nodal_vcycle(self, b, level: int = 0):
        if level == self.nlevels - 1:
            return self._cp_pinv @ b
        lv = self.nodal[level]
        x = np.zeros_like(b)
        for _ in range(self.nu_pre):
            for c in (0, 1, 2, 3):
                x = lv.gs_colour(x, b, c)
        r = b - lv.P @ x
        Pn = self.Pn[level]
        x = x + Pn @ self.nodal_vcycle(Pn.conj().T @ r, level + 1)
        for _ in range(self.nu_post):
            for c in (3, 2, 1, 0):
                x = lv.gs_colour(x, b, c)
        return x

    def nodal_solve(self, b, cycles: int):
        """`cycles` V-cycles for P phi = b starting from zero (Section 5: a few multigrid
        steps approximate the null-space projection)."""
        phi = self.nodal_vcycle(b)
        P = self.disc.P if self.nlevels > 1 else sp.csr_matrix(self._coarse_P)
        for _ in range(cycles - 1):
            phi = phi + self.nodal_vcycle(b - P @ phi)
        return phi
