"""Pins of the oracle's Section-3 discretization against facts that do not come from it.

* brute-force quadrature of the paper's piecewise global basis functions (1-based, with
  their wrap rules exactly as printed) reproduces the assembled A and M;
* the constant-epsilon discrete spectrum (Fourier analysis) and its O(h^2) approach to
  |k+G|^2 / eps;
* Hermitian symmetry, A L = 0, the null-space dimension nm (nm + 1 at k = 0) and rank L;
* symmetries of the spectrum: k -> -k, k -> k + 2 pi / a, eps -> c eps, cell shifts.
"""
import math

import numpy as np
import pytest

from oracle import fem
from oracle.closed_form import continuum, discrete_nonzero
from oracle.dense import dense_eigs

def _paper_bx(i1, i2, x1, x2, n, m, h1, h2, beta):
    """b_{x,i}(x) from the paper's piecewise definition (1-based i), x-component only."""
    c1 = int(math.floor(x1 / h1)) + 1       # 1-based cell containing the (interior) point
    c2 = int(math.floor(x2 / h2)) + 1
    if i2 < m:
        if (c1, c2) == (i1, i2):
            return (x2 / h2 - i2 + 1) / h1
        if (c1, c2) == (i1, i2 + 1):
            return (i2 + 1 - x2 / h2) / h1
        return 0.0
    if (c1, c2) == (i1, i2):
        return beta * (x2 / h2 - i2 + 1) / h1
    if (c1, c2) == (i1, 1):
        return (1 - x2 / h2) / h1
    return 0.0


def _paper_by(i1, i2, x1, x2, n, m, h1, h2, alpha):
    """b_{y,i}(x) from the paper's piecewise definition (1-based i), y-component only."""
    c1 = int(math.floor(x1 / h1)) + 1
    c2 = int(math.floor(x2 / h2)) + 1
    if i1 < n:
        if (c1, c2) == (i1, i2):
            return (x1 / h1 - i1 + 1) / h2
        if (c1, c2) == (i1 + 1, i2):
            return (i1 + 1 - x1 / h1) / h2
        return 0.0
    if (c1, c2) == (i1, i2):
        return alpha * (x1 / h1 - i1 + 1) / h2
    if (c1, c2) == (1, i2):
        return (1 - x1 / h1) / h2
    return 0.0


def _brute_force_exact(n, m, a, b, kappa, k1, k2):
    """Dense A, M by 3x3 Gauss quadrature per cell of the paper's basis functions (exact
    for the quadratic integrands); the scalar curl d2 u1 - d1 u2 by central differences
    inside the cell (the functions are linear there)."""
    h1, h2 = a / n, b / m
    alpha, beta = fem.phases(k1, k2, a, b)
    g, w = np.polynomial.legendre.leggauss(3)
    N = 2 * n * m
    A = np.zeros((N, N), dtype=complex)
    M = np.zeros((N, N), dtype=complex)
    d = 1e-7
    basis = []
    for i2 in range(1, m + 1):
        for i1 in range(1, n + 1):
            basis.append((int(fem.x_index(i1 - 1, i2 % m, n, m)), "x", i1, i2))
            basis.append((int(fem.y_index(i1 % n, i2 - 1, n, m)), "y", i1, i2))

    def ev(kind, i1, i2, x1, x2):
        if kind == "x":
            return np.array([_paper_bx(i1, i2, x1, x2, n, m, h1, h2, beta), 0.0], dtype=complex)
        return np.array([0.0, _paper_by(i1, i2, x1, x2, n, m, h1, h2, alpha)], dtype=complex)

    for c2 in range(m):
        for c1 in range(n):
            kap = kappa[c2 * n + c1]
            for gi, wi in zip(g, w):
                for gj, wj in zip(g, w):
                    x1 = (c1 + 0.5 + 0.5 * gi) * h1
                    x2 = (c2 + 0.5 + 0.5 * gj) * h2
                    wt = wi * wj * 0.25 * h1 * h2
                    idxs, U, cu = [], [], []
                    for (idx, kind, i1, i2) in basis:
                        u = ev(kind, i1, i2, x1, x2)
                        if not np.any(u):
                            continue
                        du1 = (ev(kind, i1, i2, x1, x2 + d * h2)[0] - ev(kind, i1, i2, x1, x2 - d * h2)[0]) / (2 * d * h2)
                        du2 = (ev(kind, i1, i2, x1 + d * h1, x2)[1] - ev(kind, i1, i2, x1 - d * h1, x2)[1]) / (2 * d * h1)
                        idxs.append(idx)
                        U.append(u)
                        cu.append(du1 - du2)
                    idxs = np.array(idxs)
                    U = np.array(U)
                    cu = np.array(cu)
                    A[np.ix_(idxs, idxs)] += wt * kap * np.outer(np.conj(cu), cu)
                    M[np.ix_(idxs, idxs)] += wt * (np.conj(U) @ U.T)
    return A, M


@pytest.mark.parametrize("n,m,a,b,k1,k2", [(3, 4, 1.0, 1.3, 0.7, -1.9), (4, 3, 0.8, 1.0, 2.5, 1.1),
                                           (2, 2, 1.0, 1.0, 0.4, 0.9)])
def test_assembly_equals_quadrature_of_paper_basis(n, m, a, b, k1, k2):
    rng = np.random.default_rng(7)
    kappa = 1.0 / rng.uniform(1.0, 12.0, n * m)
    A_ref, M_ref = _brute_force_exact(n, m, a, b, kappa, k1, k2)
    al, be = fem.phases(k1, k2, a, b)
    A, M = fem.assemble(n, m, a, b, kappa, al, be)
    scale_a = np.abs(A_ref).max()
    assert np.abs(A.toarray() - A_ref).max() <= 1e-6 * scale_a   # finite-difference curl
    assert np.abs(M.toarray() - M_ref).max() <= 1e-13 * np.abs(M_ref).max()


def test_lifting_is_gradient_of_paper_nodal_basis():
    """L[:, i] integrates grad(phi_i) along each edge; check a(., L x) = 0 and that
    L x reproduces phi(end) - phi(start) of a random nodal field evaluated pointwise."""
    n, m, a, b = 4, 3, 1.1, 0.9
    k1, k2 = 0.6, -2.0
    al, be = fem.phases(k1, k2, a, b)
    L = fem.lifting(n, m, al, be, a, b).toarray()
    rng = np.random.default_rng(3)
    c = rng.standard_normal(n * m) + 1j * rng.standard_normal(n * m)
    h1, h2 = a / n, b / m

    def field(x1, x2):
        s = 0.0
        for i2 in range(1, m + 1):
            for i1 in range(1, n + 1):
                s = s + c[int(fem.node_index(i1, i2, n, m))] * fem.paper_nodal(
                    x1, x2, i1, i2, n, m, h1, h2, al, be)
        return complex(s)

    u = L @ c
    for j2 in range(m):
        for j1 in range(n):
            ex = field((j1 + 1) * h1, j2 * h2) - field(j1 * h1, j2 * h2)
            ey = field(j1 * h1, (j2 + 1) * h2) - field(j1 * h1, j2 * h2)
            assert abs(u[int(fem.x_index(j1, j2, n, m))] - ex) < 1e-12
            assert abs(u[int(fem.y_index(j1, j2, n, m))] - ey) < 1e-12


@pytest.mark.parametrize("k", [(math.pi / 2, 0.0), (0.7, -1.9), (math.pi, math.pi), (0.0, 0.0),
                               (2 * math.pi, 0.0)])
def test_invariants_and_kernel_dimension(k):
    n, m, a, b = 6, 4, 1.0, 1.2
    rng = np.random.default_rng(11)
    eps = rng.uniform(1.0, 10.0, n * m)
    d = fem.Discretization(n, m, a, b, eps, *k)
    A = d.A.toarray()
    M = d.M.toarray()
    L = d.L.toarray()
    assert np.abs(A - A.conj().T).max() <= 1e-14 * np.abs(A).max()
    assert np.abs(M - M.conj().T).max() <= 1e-15
    assert np.linalg.eigvalsh(M).min() > 0
    assert np.abs(A @ L).max() <= 1e-13 * np.abs(A).max()
    gamma = fem.is_gamma(*k, a, b)
    assert np.linalg.matrix_rank(L) == n * m - (1 if gamma else 0)
    lam, _, all_lam = dense_eigs(d, 3)
    nzero = int(np.sum(np.abs(all_lam) < 1e-9 * all_lam.max()))
    assert nzero == n * m + (1 if gamma else 0)
    assert lam[0] > 1e-6 * all_lam.max()


@pytest.mark.parametrize("n,m,a,b,k1,k2,e0", [(6, 4, 1.0, 1.3, 0.7, -1.9, 2.0),
                                              (8, 8, 1.0, 1.0, 0.0, 0.0, 1.0),
                                              (5, 7, 1.2, 0.8, math.pi / 1.2, math.pi / 0.8, 3.0)])
def test_constant_eps_closed_form(n, m, a, b, k1, k2, e0):
    d = fem.Discretization(n, m, a, b, np.full(n * m, e0), k1, k2)
    cf = discrete_nonzero(n, m, a, b, e0, k1, k2)
    lam, _, _ = dense_eigs(d, len(cf))
    assert np.max(np.abs(lam - cf) / cf) < 1e-12


def test_closed_form_second_order_convergence():
    k1, k2 = 0.3, 0.7
    exact = continuum(1.0, 1.0, 1.0, k1, k2, 6)
    errs = []
    for n in (16, 32, 64, 128):
        errs.append(np.abs(discrete_nonzero(n, n, 1.0, 1.0, 1.0, k1, k2, 6) - exact) / exact)
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.9) and np.all(ratios < 4.1)


def test_c1_eps_one_against_continuum():
    lam = discrete_nonzero(32, 32, 1.0, 1.0, 1.0, math.pi / 2, 0.0, 9)
    cont = continuum(1.0, 1.0, 1.0, math.pi / 2, 0.0, 9)
    assert np.all(np.abs(lam - cont) / cont < 0.05)
    assert np.allclose(cont / math.pi ** 2, [0.25, 2.25, 4.25, 4.25, 6.25, 6.25, 6.25, 10.25, 10.25])


def test_spectral_symmetries():
    n, m, a, b = 6, 6, 1.0, 1.0
    rng = np.random.default_rng(5)
    eps = rng.uniform(1.0, 8.0, n * m)
    k = (0.9, -0.4)

    def spec(eps_, k_):
        d = fem.Discretization(n, m, a, b, eps_, *k_)
        return dense_eigs(d, 10)[0]

    base = spec(eps, k)
    assert np.allclose(spec(eps, (-k[0], -k[1])), base, rtol=1e-11)
    assert np.allclose(spec(eps, (k[0] + 2 * math.pi / a, k[1])), base, rtol=1e-10)
    assert np.allclose(spec(3.0 * eps, k), base / 3.0, rtol=1e-11)
    rolled = np.roll(eps.reshape(m, n), (2, 1), axis=(0, 1)).reshape(-1)
    assert np.allclose(spec(rolled, k), base, rtol=1e-10)
