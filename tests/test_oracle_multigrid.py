"""Pins of the oracle's Section-5 multigrid against independent facts.

* the edge and nodal prolongations are the embeddings: a coarse function evaluated
  pointwise (paper's piecewise basis) equals its prolongation evaluated on the fine grid;
* they commute with the gradient: L_f Pn = Pe L_c;
* Galerkin coarse matrices equal the rediscretisation with 2x2-averaged 1/eps (A), the
  plain coarse mass matrix (M) and the coarse nodal Laplacian (P);
* patch data: diagonal patch mass matrices, the stabilised split T^* K T = mu (+) HPD 3x3,
  uncoupled same-colour patches;
* colour-batched Gauss-Seidel equals node-by-node Gauss-Seidel (pure Python loop), and a
  patch update zeroes the residual on its four edges;
* the symmetric V-cycle is a Hermitian positive definite contraction.
"""
import math

import numpy as np
import pytest

from oracle import fem
from oracle.multigrid import Hierarchy, edge_prolongation, nodal_prolongation


def _edge_field(u, n, m, a, b, alpha, beta, x1, x2):
    """Pointwise value of the discrete edge field u on the n x m grid at an interior point,
    from the cell's local shape functions and phase map."""
    h1, h2 = a / n, b / m
    c1 = int(math.floor(x1 / h1))
    c2 = int(math.floor(x2 / h2))
    t1 = x1 / h1 - c1
    t2 = x2 / h2 - c2
    idx, ph = fem.cell_local_map(n, m, alpha, beta)
    cell = c2 * n + c1
    co = ph[cell] * u[idx[cell]]
    return np.array([(co[0] * (1 - t2) + co[1] * t2) / h1, (co[2] * (1 - t1) + co[3] * t1) / h2])


@pytest.mark.parametrize("k", [(0.7, -1.3), (0.0, 0.0), (math.pi, 2.0)])
def test_edge_prolongation_is_embedding(k):
    nf, mf, a, b = 8, 4, 1.0, 0.7
    al, be = fem.phases(*k, a, b)
    Pe = edge_prolongation(nf, mf, a, b, al, be)
    rng = np.random.default_rng(1)
    uc = rng.standard_normal(Pe.shape[1]) + 1j * rng.standard_normal(Pe.shape[1])
    uf = Pe @ uc
    for _ in range(40):
        x1 = rng.uniform(0, a)
        x2 = rng.uniform(0, b)
        vc = _edge_field(uc, nf // 2, mf // 2, a, b, al, be, x1, x2)
        vf = _edge_field(uf, nf, mf, a, b, al, be, x1, x2)
        assert np.abs(vc - vf).max() < 1e-12 * max(1.0, np.abs(vc).max())


@pytest.mark.parametrize("k", [(0.7, -1.3), (0.0, 0.0)])
def test_nodal_prolongation_is_embedding_and_commutes(k):
    nf, mf, a, b = 8, 6, 1.0, 0.9
    al, be = fem.phases(*k, a, b)
    Pn = nodal_prolongation(nf, mf, a, b, al, be)
    Pe = edge_prolongation(nf, mf, a, b, al, be)
    rng = np.random.default_rng(2)
    c = rng.standard_normal(Pn.shape[1]) + 1j * rng.standard_normal(Pn.shape[1])
    f = Pn @ c
    hf1, hf2 = a / nf, b / mf
    hc1, hc2 = 2 * hf1, 2 * hf2
    for _ in range(30):
        x1 = rng.uniform(0, a)
        x2 = rng.uniform(0, b)
        vc = sum(c[int(fem.node_index(i1, i2, nf // 2, mf // 2))] * complex(fem.paper_nodal(
            x1, x2, i1, i2, nf // 2, mf // 2, hc1, hc2, al, be))
            for i1 in range(1, nf // 2 + 1) for i2 in range(1, mf // 2 + 1))
        vf = sum(f[int(fem.node_index(i1, i2, nf, mf))] * complex(fem.paper_nodal(
            x1, x2, i1, i2, nf, mf, hf1, hf2, al, be))
            for i1 in range(1, nf + 1) for i2 in range(1, mf + 1))
        assert abs(vc - vf) < 1e-12 * max(1.0, abs(vc))
    Lf = fem.lifting(nf, mf, al, be, a, b)
    Lc = fem.lifting(nf // 2, mf // 2, al, be, a, b)
    assert np.abs((Lf @ Pn - Pe @ Lc).toarray()).max() < 1e-14


@pytest.mark.parametrize("k", [(0.4, 1.1), (0.0, 0.0)])
def test_galerkin_equals_rediscretisation(k):
    n, m, a, b = 16, 8, 1.0, 0.6
    rng = np.random.default_rng(4)
    eps = rng.uniform(1.0, 12.0, n * m)
    d = fem.Discretization(n, m, a, b, eps, *k)
    H = Hierarchy(d, mu=2.0, coarsest_min=2)
    kap = d.kappa.reshape(m, n)
    for lvl in range(1, H.nlevels - 1):
        kap = 0.25 * (kap[0::2, 0::2] + kap[1::2, 0::2] + kap[0::2, 1::2] + kap[1::2, 1::2])
        cn, cm = H.sizes[lvl]
        Ac, Mc = fem.assemble(cn, cm, a, b, kap.reshape(-1), d.alpha, d.beta)
        lv = H.edge[lvl]
        assert np.abs((lv.A - Ac).toarray()).max() <= 1e-13 * np.abs(Ac).max()
        assert np.abs((lv.M - Mc).toarray()).max() <= 1e-14
        Lc = fem.lifting(cn, cm, d.alpha, d.beta, a, b)
        Pc = (Lc.conj().T @ Mc @ Lc)
        assert np.abs((H.nodal[lvl].P - Pc).toarray()).max() <= 1e-13


def test_patch_structure_and_stabilised_split():
    n, m = 8, 8
    rng = np.random.default_rng(6)
    d = fem.Discretization(n, m, 1.0, 1.0, rng.uniform(1, 12, n * m), 1.0, -0.5)
    mu = 3.0
    H = Hierarchy(d, mu=mu, coarsest_min=2)
    for lv in H.edge[:-1]:
        assert lv.mloc_offdiag == 0.0
        assert np.abs(lv.kt00 - mu).max() <= 1e-12 * np.abs(lv.Kt).max()
        assert np.abs(lv.Kt[:, 0, 1:]).max() <= 1e-12 * np.abs(lv.Kt).max()
        # same-colour patches are uncoupled in K
        K = lv.K.toarray()
        for c in range(4):
            nodes = np.nonzero(lv.colour == c)[0]
            for i in nodes:
                for j in nodes:
                    if i != j:
                        assert np.abs(K[np.ix_(lv.patch[i], lv.patch[j])]).max() == 0.0


def test_colour_batched_gs_equals_sequential_gs():
    n, m = 4, 4
    rng = np.random.default_rng(8)
    d = fem.Discretization(n, m, 1.0, 1.0, rng.uniform(1, 12, n * m), 0.8, 0.3)
    H = Hierarchy(d, mu=2.0, coarsest_min=2)
    lv = H.edge[0]
    K = lv.K.toarray()
    b = rng.standard_normal((2 * n * m, 1)) + 1j * rng.standard_normal((2 * n * m, 1))
    x0 = rng.standard_normal((2 * n * m, 1)) + 1j * rng.standard_normal((2 * n * m, 1))
    xb = x0.copy()
    for c in range(4):
        xb = lv.gs_colour(xb, b, c)
    xs = x0.copy()
    for c in range(4):
        for node in np.nonzero(lv.colour == c)[0]:      # one node at a time
            pidx = lv.patch[node]
            r = b[pidx, 0] - K[pidx] @ xs[:, 0]
            xs[pidx, 0] += np.linalg.solve(K[np.ix_(pidx, pidx)], r)
            # the local residual on the patch vanishes after its update
            assert np.abs(b[pidx, 0] - K[pidx] @ xs[:, 0]).max() < 1e-10 * np.abs(b).max()
    assert np.abs(xb - xs).max() < 1e-12 * np.abs(xs).max()


@pytest.mark.parametrize("k", [(0.9, -0.2), (0.0, 0.0)])
def test_vcycle_hermitian_contraction(k):
    n, m = 8, 8
    rng = np.random.default_rng(9)
    d = fem.Discretization(n, m, 1.0, 1.0, rng.uniform(1, 12, n * m), *k)
    H = Hierarchy(d, mu=2.0, coarsest_min=2)
    assert H.nlevels == 3
    N = 2 * n * m
    B = H.edge_vcycle(np.eye(N, dtype=complex))
    assert np.abs(B - B.conj().T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.conj().T)).min() > 0
    K = H.edge[0].K.toarray()
    # error propagation I - B K has spectral radius < 1 (energy-norm contraction)
    rho = np.abs(np.linalg.eigvals(np.eye(N) - B @ K)).max()
    assert rho < 0.6
    Bn = H.nodal_vcycle(np.eye(n * m, dtype=complex))
    assert np.abs(Bn - Bn.conj().T).max() <= 1e-12 * np.abs(Bn).max()
    P = d.P.toarray()
    ev = np.abs(np.linalg.eigvals(np.eye(n * m) - Bn @ P))
    if d.gamma:
        ev = np.sort(ev)[:-1]     # the constant potential is the kernel of P
    assert ev.max() < 0.6
