"""Pins of the oracle's Section-4/6/7 iteration.

* generalized Householder: Q_i^2 = I, Q_i M-self-adjoint, E^* M E = I, Q...Q X = P R,
  range(X) in range(E), rank-deficient input extended to a full M-orthonormal basis;
* the iteration reaches the dense generalized eigensolve (disc permittivity, k = 0
  included) and the constant-epsilon closed form;
* the stored 32 x 32 values (written by tests/golden/make_golden.py with the dense solve);
* extrapolation: Ritz values are upper bounds (Courant-Fischer) and exact eigenvectors of
  the same k are reproduced; a short path matches dense solves at every point.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.closed_form import discrete_nonzero
from oracle.dense import dense_eigs, shift_invert_eigs
from oracle.extrapolation import extrapolate, raster_k, raster_sources, solve_grid, solve_path
from oracle.householder import m_householder, reference_columns
from oracle.multigrid import Hierarchy
from oracle.pinvit import Projector, initial_block, pinvit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _disc(n, k, seed=3, eps=None):
    if eps is None:
        eps = synth.eps_disc(n, n, 1.0, 1.0, 8.9, 0.3)
    return fem.Discretization(n, n, 1.0, 1.0, eps, *k)


def test_householder_properties():
    d = _disc(8, (0.5, 1.0))
    rng = np.random.default_rng(0)
    X = rng.standard_normal((d.n_edges, 6)) + 1j * rng.standard_normal((d.n_edges, 6))
    ref = reference_columns(d.n, d.m, 6)
    E, R, refl = m_householder(X, d.M, ref, keep_reflectors=True)
    M = d.M.toarray()
    assert np.abs(E.conj().T @ M @ E - np.eye(6)).max() < 1e-13
    assert np.abs(E @ R - X).max() < 1e-12 * np.abs(X).max()
    assert np.abs(np.tril(R, -1)).max() == 0.0
    x = rng.standard_normal(d.n_edges) + 1j * rng.standard_normal(d.n_edges)
    y = rng.standard_normal(d.n_edges) + 1j * rng.standard_normal(d.n_edges)
    for v, vMv in (r for r in refl if r is not None):
        def Q(z):
            return z - 2.0 * v * (np.vdot(v, M @ z) / vMv)
        assert np.abs(Q(Q(x)) - x).max() < 1e-12 * np.abs(x).max()
        assert abs(np.vdot(x, M @ Q(y)) - np.vdot(Q(x), M @ y)) < 1e-11 * np.abs(x).max() ** 2


def test_householder_rank_deficient_extends_basis():
    d = _disc(8, (0.5, 1.0))
    rng = np.random.default_rng(1)
    X = rng.standard_normal((d.n_edges, 3)) + 1j * rng.standard_normal((d.n_edges, 3))
    X = np.hstack([X, X[:, :1] * 2.0 - X[:, 1:2]])          # dependent 4th column
    E, R = m_householder(X, d.M, reference_columns(d.n, d.m, 4))
    M = d.M.toarray()
    assert np.abs(E.conj().T @ M @ E - np.eye(4)).max() < 1e-12
    # range(X) is contained in range(E)
    coef = E.conj().T @ (M @ X)
    assert np.abs(E @ coef - X).max() < 1e-11 * np.abs(X).max()


def _run(d, nev, nthrow, mu, cycles=2, variant="gradient", tol=1e-10, coarsest_min=4, seed=0):
    H = Hierarchy(d, mu=mu, coarsest_min=coarsest_min)
    pr = Projector(d, H, cycles)
    E0 = synth.start_block(d.n_edges, nev + nthrow, seed)
    lam, E = initial_block(d, pr, E0, nev + nthrow)
    return pinvit(d, H, pr, E, lam, nev, tol, 150, variant=variant), H, pr


@pytest.mark.parametrize("k,variant", [((0.9, -0.6), "gradient"), ((0.0, 0.0), "gradient"),
                                       ((0.9, -0.6), "lobpcg")])
def test_iteration_reaches_dense_solution(k, variant):
    d = _disc(16, k)
    ref, V, _ = dense_eigs(d, 8)
    # cut the wanted set at a spectral gap so that the subspace is well defined
    nev = max(j for j in range(3, 7) if ref[j] / ref[j - 1] - 1 > 1e-3)
    (lam, E, rel, it, conv), _, _ = _run(d, nev, 3, mu=10.0, variant=variant)
    assert conv
    assert np.max(np.abs(lam[:nev] - ref[:nev]) / ref[:nev]) < 1e-11
    # subspace of the wanted vectors: M-principal angles against the dense eigenvectors
    s = np.linalg.svd(E[:, :nev].conj().T @ (d.M @ V[:, :nev]), compute_uv=False)
    assert np.min(s) > 1 - 1e-10
    # E is M-orthonormal and gradient-free to solver accuracy
    assert np.abs(E.conj().T @ (d.M @ E) - np.eye(E.shape[1])).max() < 1e-12


def test_iteration_constant_eps_closed_form():
    n = 16
    d = fem.Discretization(n, n, 1.0, 1.0, np.full(n * n, 2.0), math.pi / 2, 0.3)
    (lam, E, rel, it, conv), _, _ = _run(d, 5, 3, mu=20.0)
    assert conv
    cf = discrete_nonzero(n, n, 1.0, 1.0, 2.0, math.pi / 2, 0.3, 5)
    assert np.max(np.abs(lam[:5] - cf) / cf) < 1e-11


def test_golden_c1_32x32():
    """The 32 x 32 disc workload (eps = 8.9, r = 0.2, k = (pi/2, 0)): the iteration from the
    seeded random start reproduces the stored dense-solve values."""
    with open(os.path.join(GOLDEN, "c1_dense.json")) as f:
        gold = json.load(f)
    prob = synth.config_c1()
    d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, *prob.ks[0])
    H = Hierarchy(d, mu=15.79, coarsest_min=8)
    assert H.nlevels == 3
    pr = Projector(d, H, 2)
    lam, E = initial_block(d, pr, synth.start_block(d.n_edges, 12, 0), 12)
    lam, E, rel, it, conv = pinvit(d, H, pr, E, lam, 8, 1e-8, 100)
    assert conv
    ref = np.array(gold["disc"][:8])
    assert np.max(np.abs(lam[:8] - ref) / ref) < 1e-11


def test_extrapolation_courant_fischer_and_reproduction():
    n = 12
    k0, k1 = (0.5, 0.2), (0.6, 0.25)
    d0 = _disc(n, k0)
    d1 = _disc(n, k1)
    lam0, V0, _ = dense_eigs(d0, 8)
    lam1, V1, _ = dense_eigs(d1, 8)
    H1 = Hierarchy(d1, mu=10.0, coarsest_min=3)
    pr1 = Projector(d1, H1, 6)
    th, E = extrapolate(d1, pr1, [V0], 6, 1e-2 * lam0[0])
    assert np.all(th >= lam1[:6] * (1 - 1e-10))
    assert np.all(th - lam1[:6] <= 0.05 * lam1[5])     # a good start, not a proof
    # with the exact eigenvectors of the same k in the span they are reproduced
    th2, _ = extrapolate(d1, pr1, [V1, V0], 6, 1e-2 * lam0[0])
    assert np.max(np.abs(th2 - lam1[:6]) / lam1[:6]) < 1e-9


def test_short_path_matches_dense():
    n = 12
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 6.0, 0.3)
    ks = synth.path_gxmg(2)[:5]        # Gamma, half way, X, half way, M
    start = synth.start_block(2 * n * n, 6, 0)
    res = solve_path(n, n, 1.0, 1.0, eps, ks, 4, 2, start, tol=1e-9, mu=10.0,
                     coarsest_min=3)
    for rec, k in zip(res, ks):
        assert rec["converged"]
        d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
        ref, _, _ = dense_eigs(d, 4)
        assert np.max(np.abs(rec["lam"] - ref) / ref) < 1e-10


def test_shift_invert_reference_certifies_completeness():
    n = 24
    d = _disc(n, (1.0, 0.4))
    lam_d, _, _ = dense_eigs(d, 5)
    lam_s, _, reached = shift_invert_eigs(d, 5, sigma=0.75 * 1.1 * lam_d[4], extra=40)
    assert reached
    assert np.max(np.abs(lam_s[:5] - lam_d) / lam_d) < 1e-10


def test_raster_sources_follow_section_6():
    """The raster as Section 6 lists it: k10 from k00; k20 from k00, k10; k_i0 from the three
    to its left; k01, k11, k21 from k00, k10, k20; k02 .. k22 from the two below; k0j .. k2j
    from the three below (j >= 3); k_ij from the three to its left (i, j >= 3).  Every source
    precedes its point in raster order and lies on one axis within distance 3."""
    K = 9
    assert raster_sources(K, 0, 0) == []
    assert raster_sources(K, 1, 0) == [(0, 0)]
    assert raster_sources(K, 2, 0) == [(0, 0), (1, 0)]
    assert raster_sources(K, 6, 0) == [(3, 0), (4, 0), (5, 0)]
    for i in range(3):
        assert raster_sources(K, i, 1) == [(i, 0)]
        assert raster_sources(K, i, 2) == [(i, 0), (i, 1)]
        assert raster_sources(K, i, 5) == [(i, 2), (i, 3), (i, 4)]
    assert raster_sources(K, 5, 4) == [(2, 4), (3, 4), (4, 4)]
    assert raster_sources(K, 3, 3) == [(0, 3), (1, 3), (2, 3)]
    for j in range(K):
        for i in range(K):
            src = raster_sources(K, i, j)
            assert (len(src) == 0) == (i == 0 and j == 0) and len(src) <= 3
            for (a, b) in src:
                assert b * K + a < j * K + i
                assert (a == i and 0 < j - b <= 3) or (b == j and 0 < i - a <= 3)
    k = raster_k(K, 0, K - 1, 2.0, 0.5)
    assert np.allclose(k, (-np.pi / 2.0, np.pi / 0.5))


def test_grid_raster_matches_dense_and_warm_starts():
    """The raster on the 16 x 16 mesh with the band-structure permittivity (11.56 in the disc
    of radius 0.18).  kappa = 3: every point (Gamma at the centre included) converges to the
    dense eigenvalues, and k_20 = k_00 + (2 pi, 0) carries the same pencil, so its start
    extrapolated from k_00 and k_10 is already converged (Courant-Fischer reproduction).
    kappa = 5: the extrapolated points need fewer iterations than the random start.  With
    the absolute defect as stopping measure the reported defects are below the tolerance."""
    n, nev, nthrow = 16, 4, 2
    eps = synth.paper_z2_eps(n)
    start = synth.start_block(2 * n * n, nev + nthrow, 7)
    kw = dict(tol=1e-9, mu=5.0, coarsest_min=4)
    res = solve_grid(n, n, 1.0, 1.0, eps, 3, nev, nthrow, start, **kw)
    assert [r["ij"] for r in res] == [(i, j) for j in range(3) for i in range(3)]
    for r in res:
        assert r["converged"]
        d = fem.Discretization(n, n, 1.0, 1.0, eps, *r["k"])
        lam, _, _ = dense_eigs(d, nev)
        assert np.max(np.abs(r["lam"] - lam) / lam) < 1e-8
    assert res[2]["iterations"] == 0 and np.allclose(res[2]["lam"], res[0]["lam"], rtol=1e-9)
    res5 = solve_grid(n, n, 1.0, 1.0, eps, 5, nev, nthrow, start, **kw)
    assert all(r["converged"] for r in res5)
    assert np.median([r["iterations"] for r in res5[1:]]) < res5[0]["iterations"]
    ab = solve_grid(n, n, 1.0, 1.0, eps, 2, nev, nthrow, start, tol=1e-3, mu=5.0,
                    coarsest_min=4, absolute=True)
    for r in ab:
        assert r["converged"] and np.all(r["relres"] <= 1e-3)
        d = fem.Discretization(n, n, 1.0, 1.0, eps, *r["k"])
        lam, _, _ = dense_eigs(d, nev)
        assert np.max(np.abs(r["lam"] - lam) / lam) < 1e-3


def test_nested_start_follows_section_6():
    """Nested iteration (Section 6): the coarsest block is the dense solution of the coarsest
    pencil; the prolongation is the embedding, so the prolongated coarse eigenvectors keep
    their Rayleigh quotients on the finer mesh's Galerkin hierarchy; the start block needs
    fewer fine iterations than a random one and the iteration from it reaches the dense values."""
    from oracle.extrapolation import level_kappas, nested_start
    from oracle.multigrid import edge_prolongation, level_sizes
    n = 16
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    k = (0.7, -1.3)
    sizes = level_sizes(n, n, 0, 4)
    kap = level_kappas(n, n, eps, sizes)
    dc = fem.Discretization(8, 8, 1.0, 1.0, 1.0 / kap[1], *k)
    lam_c, E_c, _ = dense_eigs(fem.Discretization(4, 4, 1.0, 1.0, 1.0 / kap[2], *k), 5)
    P = edge_prolongation(8, 8, 1.0, 1.0, dc.alpha, dc.beta)
    F = P @ E_c
    rq = np.real(np.einsum("ij,ij->j", F.conj(), dc.A @ F) / np.einsum("ij,ij->j", F.conj(), dc.M @ F))
    assert np.allclose(rq, lam_c, rtol=1e-11)
    E, its = nested_start(n, n, 1.0, 1.0, eps, *k, 4, 2, tol_levels=1e-3, mu=10.0, coarsest_min=4)
    assert its[0] == 0 and its[-1] == 0 and its[1] > 0
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    H = Hierarchy(d, mu=10.0, coarsest_min=4)
    pr = Projector(d, H, 2)
    lam0, E0 = initial_block(d, pr, E, 6)
    lam, _, _, it, conv = pinvit(d, H, pr, E0, lam0, 4, 1e-9, 200)
    lam1, E1 = initial_block(d, pr, synth.start_block(d.n_edges, 6, 5), 6)
    it_random = pinvit(d, H, pr, E1, lam1, 4, 1e-9, 200)[3]
    ref, _, _ = dense_eigs(d, 4)
    assert conv and np.max(np.abs(lam[:4] - ref) / ref) < 1e-8
    assert it < it_random


def test_gram_orthonormalisation_same_span_and_limit():
    """The Gram (Cholesky) orthonormalisation spans the same space as the Householder one,
    is M-orthonormal, and the iteration run with it reaches the dense eigenvalues."""
    from oracle.householder import m_householder, reference_columns
    from oracle.pinvit import gram_orthonormalize
    n = 12
    eps = synth.eps_disc(n, n, 1.0, 1.0, 8.9, 0.3)
    d = fem.Discretization(n, n, 1.0, 1.0, eps, 0.7, -0.2)
    rng = np.random.default_rng(4)
    S = rng.standard_normal((d.n_edges, 9)) + 1j * rng.standard_normal((d.n_edges, 9))
    Qg = gram_orthonormalize(S, d.M)
    Qh, _ = m_householder(S, d.M, reference_columns(n, n, 9))
    assert np.abs(Qg.conj().T @ (d.M @ Qg) - np.eye(9)).max() < 1e-12
    # equal spans: the M-orthogonal projectors agree
    Pg = Qg @ (Qg.conj().T @ d.M.toarray())
    Ph = Qh @ (Qh.conj().T @ d.M.toarray())
    assert np.abs(Pg - Ph).max() < 1e-10
    H = Hierarchy(d, mu=5.0, coarsest_min=3)
    pr = Projector(d, H, 2)
    E0 = synth.start_block(d.n_edges, 6, 2)
    lam0, E = initial_block(d, pr, E0, 6, ortho="gram")
    lam, _, _, it, conv = pinvit(d, H, pr, E, lam0, 4, 1e-10, 200, ortho="gram")
    ref, _, _ = dense_eigs(d, 4)
    assert conv and np.max(np.abs(lam[:4] - ref) / ref) < 1e-9
