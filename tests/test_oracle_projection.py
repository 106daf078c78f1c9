"""Pins of the oracle's null-space elimination (Section 4) and its plane-wave deflation.

* the nodal plane wave of the first-zone representative of k is an exact eigenvector of the
  assembled P = L^* M L, with the closed-form eigenvalue, and it is the lowest one (dense
  eigensolve of P on small grids, k also given outside the first zone);
* with exact nodal solves the deflated projection is the undeflated one, and both are the
  exact M-orthogonal projection onto the complement of the gradients (sparse direct solve);
* with V-cycles the deflated projection removes gradient content along the plane wave to
  rounding, and the result stays within the V-cycle's accuracy of the exact projection.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spl

import synth
from oracle import fem
from oracle.multigrid import Hierarchy
from oracle.pinvit import Projector

KS = [(0.1, 0.0), (0.108, -0.108), (1.2, 0.5), (math.pi, 0.3), (math.pi, math.pi),
      (2 * math.pi + 0.3, -7.0), (0.0, 0.0), (1e-3, 2e-3)]


@pytest.mark.parametrize("n,m,a,b", [(8, 8, 1.0, 1.0), (6, 10, 1.3, 0.8), (12, 8, 0.9, 1.1)])
@pytest.mark.parametrize("k", KS)
def test_plane_wave_is_lowest_eigenvector_of_P(n, m, a, b, k):
    d = fem.Discretization(n, m, a, b, np.ones(n * m), *k)
    w, lw = d.plane_wave()
    Pd = d.P.toarray()
    norm_p = np.linalg.norm(Pd, 2)
    assert np.linalg.norm(Pd @ w - lw * w) <= 1e-13 * norm_p * np.linalg.norm(w)
    ev = sla.eigvalsh(Pd)
    assert abs(ev[0] - lw) <= 1e-12 * norm_p
    assert lw >= 0.0
    if d.gamma:
        assert lw == 0.0 and np.all(w == 1.0)


def test_plane_wave_eigenvalue_near_gamma_is_cancellation_free():
    # P carries the scale h^2 (square cells): lambda_w / (|k| h)^2 -> 1 as k -> 0, with
    # relative deviation O((|k| h)^2); the product form keeps every digit down to tiny |k|
    n = 1024
    h = 1.0 / n
    for t in (1e-2, 1e-4, 1e-6, 1e-9):
        lw = fem.plane_wave_eigenvalue(n, n, 1.0, 1.0, t, 0.0)
        assert abs(lw / (t * h) ** 2 - 1.0) < 1e-12 + (t * h) ** 2


class _ExactNodal:
    """A hierarchy stand-in whose nodal solve is exact (direct solve; the pseudo-inverse
    at the Gamma point, where P has the constants as kernel)."""

    def __init__(self, d):
        self.P = d.P.toarray()
        self.pinv = np.linalg.pinv(self.P, rcond=1e-12, hermitian=True)

    def nodal_solve(self, b, cycles):
        return self.pinv @ b


@pytest.mark.parametrize("k", [(0.05, -0.02), (1.2, 0.5), (0.0, 0.0)])
def test_deflation_is_exact_with_exact_nodal_solves(k):
    n, m, a, b = 8, 6, 1.0, 0.9
    eps = synth.eps_disc(n, m, a, b, 8.9, 0.3)
    d = fem.Discretization(n, m, a, b, eps, *k)
    ex = _ExactNodal(d)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((2 * n * m, 3)) + 1j * rng.standard_normal((2 * n * m, 3))
    out_d = Projector(d, ex, 1, deflate=True)(U)
    out_u = Projector(d, ex, 1, deflate=False)(U)
    # the exact projection: the M-orthogonal complement of range(L) (and, at Gamma, also
    # of the two constant fields), from an independent dense least-squares solve
    Md = d.M.toarray()
    Ld = d.L.toarray()
    G = Ld
    if d.gamma:
        G = np.hstack([Ld, d.constant_fields()])
    coef = np.linalg.lstsq(G.conj().T @ Md @ G, G.conj().T @ Md @ U, rcond=1e-12)[0]
    ref = U - G @ coef
    scale = np.linalg.norm(U)
    assert np.linalg.norm(out_d - ref) <= 1e-10 * scale
    assert np.linalg.norm(out_u - ref) <= 1e-10 * scale


@pytest.mark.parametrize("k", [(0.108, -0.108), (0.05, 0.0), (1.2, 0.5)])
def test_deflation_removes_plane_wave_gradient_with_vcycles(k):
    n = m = 32
    eps = synth.eps_disc_lattice(n, m, 1.0, 1.0, 12.0, 0.3)
    d = fem.Discretization(n, m, 1.0, 1.0, eps, *k)
    H = Hierarchy(d, 1.0)
    w, lw = d.plane_wave()
    Pf = spl.splu(d.P.tocsc())
    LhM = d.L.conj().T @ d.M
    rng = np.random.default_rng(5)
    U = rng.standard_normal((2 * n * m, 2)) + 1j * rng.standard_normal((2 * n * m, 2))
    U0 = U - d.L @ Pf.solve(LhM @ U)                 # gradient free
    Ug = U0 + d.L @ np.outer(w, [1.0, 2.0 - 1.0j])   # plus plane-wave gradients
    out = Projector(d, H, 2)(Ug)
    left = d.L @ Pf.solve(LhM @ out)                 # remaining gradient content
    mn = lambda v: np.sqrt(np.real(np.einsum("ij,ij->j", v.conj(), d.M @ v)))
    assert np.all(mn(left) <= 1e-12 * mn(Ug))
    # generic content: the deflated and undeflated V-cycle projections agree to the
    # V-cycles' accuracy and both approach the exact projection
    V = rng.standard_normal((2 * n * m, 2)) + 1j * rng.standard_normal((2 * n * m, 2))
    exact = V - d.L @ Pf.solve(LhM @ V)
    for defl in (True, False):
        got = Projector(d, H, 2, deflate=defl)(V)
        assert np.all(mn(got - exact) <= 2e-2 * mn(V - exact))


@pytest.mark.parametrize("n,m,a,b,k,eps_kind", [
    (8, 8, 1.0, 1.0, (0.7, -1.3), "disc"),
    (6, 10, 1.3, 0.8, (0.0, 0.0), "disc"),
    (8, 8, 1.0, 1.0, (0.0, 0.0), "one"),          # degenerate: multiplicities 2 and 4
    (8, 8, 1.0, 1.0, (math.pi, math.pi), "one"),
])
def test_gradient_free_eigs_against_dense(n, m, a, b, k, eps_kind):
    from oracle.dense import dense_eigs, gradient_free_eigs
    eps = np.ones(n * m) if eps_kind == "one" else synth.eps_disc(n, m, a, b, 8.9, 0.3)
    d = fem.Discretization(n, m, a, b, eps, *k)
    ref, _, _ = dense_eigs(d, 12)
    lam, V = gradient_free_eigs(d, 12)
    assert np.max(np.abs(lam - ref) / ref) < 1e-10
    # eigenvectors (within a degenerate cluster ARPACK's are not mutually orthogonal)
    R = d.A @ V - (d.M @ V) * lam[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / (lam * np.linalg.norm(d.M @ V, axis=0))) < 1e-9


def test_gradient_free_eigs_closed_form_and_golden():
    from oracle.closed_form import discrete_nonzero
    from oracle.dense import gradient_free_eigs
    n = 48
    for k in ((0.0, 0.0), (0.4, 0.2)):
        d = fem.Discretization(n, n, 1.0, 1.0, np.ones(n * n), *k)
        lam, _ = gradient_free_eigs(d, 20)
        ref = discrete_nonzero(n, n, 1.0, 1.0, 1.0, *k, count=20)
        assert np.max(np.abs(lam - ref) / ref) < 1e-10
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_dense.json")) as f:
        gold = json.load(f)
    prob = synth.config_c1()
    d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, *prob.ks[0])
    lam, _ = gradient_free_eigs(d, 12)
    assert np.max(np.abs(lam - np.array(gold["disc"][:12])) / lam) < 1e-10
