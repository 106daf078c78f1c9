"""Section 3 (Discretization): Bloch-modified lowest-order Nedelec edge elements on an
n x m rectangular mesh of the cell [0,a] x [0,b], the Bloch nodal Q1 space, the Galerkin
matrices A (curl-curl with 1/epsilon) and M (mass), and the lifting matrix L with
grad(phi_j) = sum_i L_ij b_i.

Storage order (0-based) and its relation to the paper's 1-based indices:
  * cell Omega_(i1,i2)            <-> cell (i1-1, i2-1),       flat c2*n + c1
  * b_{x,(i1,i2)} (edge at height i2*h2 over the i1-th column)
                                   <-> x-edge (i1-1, i2 mod m),  flat j2*n + j1
  * b_{y,(i1,i2)} (edge at x1 = i1*h1 over the i2-th row)
                                   <-> y-edge (i1 mod n, i2-1),  flat n*m + j2*n + j1
  * phi_(i1,i2) (node at (i1*h1, i2*h2))
                                   <-> node (i1 mod n, i2 mod m), flat j2*n + j1
The Bloch phases are alpha = exp(i k1 a) and beta = exp(i k2 b).  A basis function whose
support wraps over the top (right) boundary carries the factor beta (alpha) on the cells
of the last row (column), exactly as in the paper's piecewise definitions.

Pinned by: brute-force quadrature of the paper's piecewise basis functions (tests), the
closed-form spectrum for constant epsilon, A L = 0, Hermitian symmetry and the kernel
dimension.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import scipy.sparse as sp

__all__ = ["phases", "is_gamma", "x_index", "y_index", "node_index", "cell_local_map",
           "element_matrices", "assemble", "lifting", "nodal_laplacian", "reduced_k",
           "plane_wave", "plane_wave_eigenvalue", "Discretization"]


def phases(k1: float, k2: float, a: float, b: float):
    """alpha = exp(i k1 a), beta = exp(i k2 b) (Section 1, Bloch boundary conditions).

    At the Gamma point (k1 a and k2 b both multiples of 2 pi up to 1e-14) the phases are
    returned as exactly 1, which selects the k = 0 treatment of the null space."""
    if is_gamma(k1, k2, a, b):
        return 1.0 + 0j, 1.0 + 0j
    return cmath.exp(1j * k1 * a), cmath.exp(1j * k2 * b)


def is_gamma(k1: float, k2: float, a: float, b: float) -> bool:
    """True when k is congruent to 0 modulo the reciprocal lattice (within 1e-14)."""
    t1 = k1 * a - 2 * math.pi * round(k1 * a / (2 * math.pi))
    t2 = k2 * b - 2 * math.pi * round(k2 * b / (2 * math.pi))
    return abs(t1) <= 1e-14 and abs(t2) <= 1e-14


def x_index(j1, j2, n, m):
    return (np.asarray(j2) % m) * n + (np.asarray(j1) % n)


def y_index(j1, j2, n, m):
    return n * m + (np.asarray(j2) % m) * n + (np.asarray(j1) % n)


def node_index(j1, j2, n, m):
    return (np.asarray(j2) % m) * n + (np.asarray(j1) % n)


def cell_local_map(n: int, m: int, alpha: complex, beta: complex):
    """For every cell, the global indices and phase factors of its four local edge shape
    functions, ordered (bottom, top, left, right).

    On cell (c1, c2) the global basis function of a local edge equals phase * (local shape
    function).  Only the top edge of the last row (which is the bottom edge of row 0,
    carrying beta on this row) and the right edge of the last column (carrying alpha)
    have phases different from 1.  Returns (idx, ph), each of shape (n*m, 4)."""
    c1, c2 = np.meshgrid(np.arange(n), np.arange(m), indexing="xy")
    c1 = c1.reshape(-1)
    c2 = c2.reshape(-1)
    idx = np.stack([x_index(c1, c2, n, m), x_index(c1, c2 + 1, n, m),
                    y_index(c1, c2, n, m), y_index(c1 + 1, c2, n, m)], axis=1)
    ph = np.ones((n * m, 4), dtype=np.complex128)
    ph[c2 == m - 1, 1] = beta
    ph[c1 == n - 1, 3] = alpha
    return idx, ph


def element_matrices(h1: float, h2: float):
    """Local 4x4 matrices on one cell for the shape functions
    bottom = ((1-t2)/h1, 0), top = (t2/h1, 0), left = (0, (1-t1)/h2), right = (0, t1/h2)
    with t = local coordinates in [0,1]^2.

    The scalar curl d2 u1 - d1 u2 of these is (-1, +1, +1, -1)/(h1 h2), constant on the
    cell, so a_K = kappa/(h1 h2) c c^T.  The mass integrals of the hat products give the
    1/3, 1/6 pattern; x- and y-components are orthogonal."""
    c = np.array([-1.0, 1.0, 1.0, -1.0])
    a_unit = np.outer(c, c) / (h1 * h2)
    mx = h2 / h1
    my = h1 / h2
    m_loc = np.array([[mx / 3, mx / 6, 0, 0],
                      [mx / 6, mx / 3, 0, 0],
                      [0, 0, my / 3, my / 6],
                      [0, 0, my / 6, my / 3]])
    return a_unit, m_loc


def assemble(n: int, m: int, a: float, b: float, kappa: np.ndarray, alpha: complex,
             beta: complex):
    """Galerkin matrices A (a(b_i, b_j), rows = test functions) and M (m(b_i, b_j)).

    A = sum_K T_K^H (kappa_K a_unit) T_K and M = sum_K T_K^H m_loc T_K, where T_K maps
    the global coefficients to the local shape-function coefficients of cell K including
    the Bloch phases.  kappa = 1/epsilon per cell in cell order.  Returns CSR complex128."""
    h1, h2 = a / n, b / m
    a_unit, m_loc = element_matrices(h1, h2)
    idx, ph = cell_local_map(n, m, alpha, beta)
    ncell = n * m
    rows = np.repeat(idx, 4, axis=1).reshape(-1)
    cols = np.tile(idx, (1, 4)).reshape(-1)
    phase = (np.conj(ph)[:, :, None] * ph[:, None, :]).reshape(ncell, 16)
    va = (kappa[:, None] * a_unit.reshape(1, 16)) * phase
    vm = m_loc.reshape(1, 16) * phase
    N = 2 * n * m
    A = sp.csr_matrix((va.reshape(-1), (rows, cols)), shape=(N, N))
    M = sp.csr_matrix((vm.reshape(-1), (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    M.sum_duplicates()
    return A, M


def paper_hat(x, i, nh: int, h: float, ph: complex):
    """The paper's one-dimensional Bloch hat phi_{x,i} (or phi_{y,j}) of Section 3,
    evaluated at points x in [0, nh*h]; i is 1-based (array-valued allowed, broadcast
    against x), ph is exp(i k1 a) (or exp(i k2 b)).

    For i < nh it is the usual hat on [(i-1)h, (i+1)h]; for i = nh the rising half on the
    last interval carries the phase and the falling half wraps to [0, h]."""
    x = np.asarray(x, dtype=np.float64)
    i = np.asarray(i)
    t = x / h
    inner = i < nh
    rise = (t >= i - 1) & (t <= i)
    fall_inner = (t >= i) & (t <= i + 1)
    fall_wrap = (t >= 0) & (t <= 1)
    val_rise = np.where(inner, t - i + 1, ph * (t - nh + 1))
    out = np.where(rise, val_rise, 0.0 + 0j)
    out = np.where(inner & fall_inner, i + 1 - t, out)
    out = np.where((~inner) & fall_wrap, 1 - t, out)
    return out


def paper_nodal(x1, x2, i1, i2, n: int, m: int, h1: float, h2: float,
                alpha: complex, beta: complex):
    """phi_i(x) = phi_{x,i1}(x1) phi_{y,i2}(x2), the Bloch Q1 nodal basis of Section 3."""
    return paper_hat(x1, i1, n, h1, alpha) * paper_hat(x2, i2, m, h2, beta)


def lifting(n: int, m: int, alpha: complex, beta: complex, a: float = 1.0, b: float = 1.0):
    """Lifting matrix L (2nm x nm) with grad(phi_i) = sum_e L[e, i] b_e (Section 3).

    The degrees of freedom of the edge space are the line integrals along the stored edges
    (each b_e has unit line integral along its own edge and zero along the others), so
    L[e, i] is the line integral of grad(phi_i) along edge e, i.e. phi_i(end) - phi_i(start),
    evaluated with the paper's piecewise nodal basis on [0,a] x [0,b].  Stored x-edge
    (j1, j2) runs from (j1 h1, j2 h2) to ((j1+1) h1, j2 h2); y-edge (j1, j2) from
    (j1 h1, j2 h2) to (j1 h1, (j2+1) h2).  This reproduces the gradient identity
    grad phi_i = b_{x,i} - b_{x,(i1+1,i2)} + b_{y,i} - b_{y,(i1,i2+1)}, whose printed form
    swaps the two shifted indices.

    Every edge within two cells of the node is evaluated (a superset of the support);
    entries that evaluate to zero are dropped."""
    h1, h2 = a / n, b / m
    N = 2 * n * m
    i1, i2 = np.meshgrid(np.arange(1, n + 1), np.arange(1, m + 1), indexing="xy")
    i1 = i1.reshape(-1)
    i2 = i2.reshape(-1)
    p1 = i1 % n          # 0-based node column / row
    p2 = i2 % m
    col = node_index(p1, p2, n, m)
    rows, cols, vals = [], [], []
    for d2 in (-2, -1, 0, 1):
        for d1 in (-2, -1, 0, 1):
            j1 = (p1 + d1) % n
            j2 = (p2 + d2) % m
            for kind in ("x", "y"):
                xs1, xs2 = j1 * h1, j2 * h2
                if kind == "x":
                    xe1, xe2 = (j1 + 1) * h1, j2 * h2
                    eidx = x_index(j1, j2, n, m)
                else:
                    xe1, xe2 = j1 * h1, (j2 + 1) * h2
                    eidx = y_index(j1, j2, n, m)
                v = (paper_nodal(xe1, xe2, i1, i2, n, m, h1, h2, alpha, beta)
                     - paper_nodal(xs1, xs2, i1, i2, n, m, h1, h2, alpha, beta))
                nz = np.abs(v) > 1e-14
                rows.append(eidx[nz])
                cols.append(col[nz])
                vals.append(v[nz])
    # Small grids visit some edges from several offsets; keep one entry per (edge, node).
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    key = r.astype(np.int64) * (n * m) + c
    _, first = np.unique(key, return_index=True)
    L = sp.csr_matrix((v[first], (r[first], c[first])), shape=(N, n * m))
    return L


def nodal_laplacian(L, M):
    """P = L^* M L, the Bloch Q1 Laplacian g_ij = m(grad phi_i, grad phi_j) (Section 3/5)."""
    return (L.conj().T @ M @ L).tocsr()


def reduced_k(k1: float, k2: float, a: float, b: float):
    """The representative of k in the first Brillouin zone: k - 2 pi (p/a, r/b) with the
    integers p, r nearest to k1 a / (2 pi) and k2 b / (2 pi) (ties to even).  Bloch phases
    only depend on k modulo the reciprocal lattice; this representative is the one whose
    nodal plane wave has the smallest energy."""
    return (k1 - 2 * math.pi * round(k1 * a / (2 * math.pi)) / a,
            k2 - 2 * math.pi * round(k2 * b / (2 * math.pi)) / b)


def plane_wave(n: int, m: int, a: float, b: float, k1: float, k2: float) -> np.ndarray:
    """Nodal vector w_j = exp(i (k1' j1 h1 + k2' j2 h2)) with k' = reduced_k(k) (all ones at
    the Gamma point).  It satisfies the Bloch condition of the nodal space (Section 3: a
    node beyond the right/top boundary carries the factor alpha/beta), and since
    P = L^* M L is a constant-coefficient stencil it is an exact eigenvector of P
    (checked in the tests against the assembled P).  Its eigenvalue tends to zero as
    k -> 0, where P becomes singular."""
    if is_gamma(k1, k2, a, b):
        return np.ones(n * m, dtype=np.complex128)
    r1, r2 = reduced_k(k1, k2, a, b)
    j1, j2 = np.meshgrid(np.arange(n), np.arange(m), indexing="xy")
    return np.exp(1j * (r1 * j1 * (a / n) + r2 * j2 * (b / m))).reshape(-1)


def plane_wave_eigenvalue(n: int, m: int, a: float, b: float, k1: float, k2: float) -> float:
    """P w = lambda_w w for w = plane_wave(...), in a cancellation-free closed form.

    Derivation: the gradient of w on x-edge (j1, j2) is w_j (exp(i t1) - 1), t1 = k1' h1,
    with |exp(i t1) - 1|^2 = 4 sin^2(t1/2); the mass matrix couples an x-edge to the x-edges
    directly above and below with (h2/h1)(2/3, 1/6, 1/6), whose symbol is
    (h2/h1)(1 - 2/3 sin^2(t2/2)); y-edges likewise with the roles swapped.  Zero at the
    Gamma point."""
    if is_gamma(k1, k2, a, b):
        return 0.0
    r1, r2 = reduced_k(k1, k2, a, b)
    h1, h2 = a / n, b / m
    s1 = math.sin(r1 * h1 / 2) ** 2
    s2 = math.sin(r2 * h2 / 2) ** 2
    return 4 * s1 * (h2 / h1) * (1 - 2.0 / 3.0 * s2) + 4 * s2 * (h1 / h2) * (1 - 2.0 / 3.0 * s1)


class Discretization:
    """All Section-3 objects for one grid, permittivity and Bloch parameter."""

    def __init__(self, n: int, m: int, a: float, b: float, eps: np.ndarray, k1: float,
                 k2: float):
        eps = np.asarray(eps, dtype=np.float64)
        if eps.shape != (n * m,):
            raise ValueError("eps must hold n*m cell values")
        self.n, self.m, self.a, self.b = n, m, a, b
        self.h1, self.h2 = a / n, b / m
        self.k1, self.k2 = k1, k2
        self.gamma = is_gamma(k1, k2, a, b)
        self.alpha, self.beta = phases(k1, k2, a, b)
        self.kappa = 1.0 / eps
        self.A, self.M = assemble(n, m, a, b, self.kappa, self.alpha, self.beta)
        self.L = lifting(n, m, self.alpha, self.beta, a, b)
        self.P = nodal_laplacian(self.L, self.M)

    @property
    def n_edges(self):
        return 2 * self.n * self.m

    @property
    def n_nodes(self):
        return self.n * self.m

    def plane_wave(self):
        """The lowest eigenvector of P and its eigenvalue (plane_wave, plane_wave_eigenvalue)."""
        args = (self.n, self.m, self.a, self.b, self.k1, self.k2)
        return plane_wave(*args), plane_wave_eigenvalue(*args)

    def constant_fields(self):
        """The two constant edge fields x-hat (all x-edges 1) and y-hat: at k = 0 they are
        curl-free but not gradients of periodic potentials (the explicitly known remainder
        of the null space, Section 3 and Section 4)."""
        N = self.n_edges
        nm = self.n * self.m
        X = np.zeros((N, 2), dtype=np.complex128)
        X[:nm, 0] = 1.0
        X[nm:, 1] = 1.0
        return X
