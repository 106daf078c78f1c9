"""Operator-level parity of the gfx950 kernels (through bl_apply) against the oracle's
sparse matrices and multigrid, element by element on seeded inputs: FP64 to 1e-12
relative (norm-wise), FP32 to 2e-5.  Grids with ragged tails (edge counts not multiples of
the 256-thread blocks), rectangular cells, and k generic / Gamma / zone corner."""
import math

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.multigrid import Hierarchy
from oracle.pinvit import Projector

pytestmark = pytest.mark.gpu

CASES = [
    # n, m, a, b, coarsest_min, k
    (20, 12, 1.0, 0.8, 3, (0.7, -1.3)),
    (20, 12, 1.0, 0.8, 3, (0.0, 0.0)),
    (32, 32, 1.0, 1.0, 8, (math.pi, math.pi)),
    (24, 16, 1.3, 1.0, 4, (math.pi / 2, 0.4)),
]
MU = 5.0


def _setup(case, nodal_cycles=2):
    import torch  # noqa: F401
    from paper_2304_00337_amd import Solver
    n, m, a, b, cmin, k = case
    rng = np.random.default_rng(n * 100 + m)
    eps = rng.uniform(1.0, 12.0, n * m)
    d = fem.Discretization(n, m, a, b, eps, *k)
    H = Hierarchy(d, mu=MU, coarsest_min=cmin)
    s = Solver(n, m, a, b, eps, nev=4, nthrow=2, mu=MU, coarsest_min=cmin, nodal_cycles=nodal_cycles)
    assert s.info()["levels"] == H.nlevels
    assert s.info()["sizes"] == [tuple(x) for x in H.sizes]
    s.set_k(*k)
    return d, H, s, rng


def _rand(rng, N, c):
    return rng.standard_normal((N, c)) + 1j * rng.standard_normal((N, c))


def _gpu(s, op, X, level=0, Y=None, out_rows=None, fp32=False, init=None):
    import torch
    from paper_2304_00337_amd import from_device_block, to_device_block
    dt = torch.float32 if fp32 else torch.float64
    x = to_device_block(X, dtype=dt)
    y = to_device_block(Y, dtype=dt) if Y is not None else None
    c = X.shape[1]
    if init is not None:
        out = to_device_block(init, dtype=dt)
    else:
        out = torch.zeros((c, 2, out_rows), dtype=dt, device="cuda")
    s.apply(op, x, y=y, out=out, level=level)
    return from_device_block(out)


def _close(got, ref, tol):
    err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert err <= tol, f"relative error {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("fp32", [False, True])
def test_edge_and_nodal_operators(case, fp32):
    d, H, s, rng = _setup(case)
    tol = 2e-5 if fp32 else 1e-12
    Ne, Nv = d.n_edges, d.n_nodes
    X = _rand(rng, Ne, 3)
    F = _rand(rng, Nv, 3)
    _close(_gpu(s, "A", X, out_rows=Ne, fp32=fp32), d.A @ X, tol)
    _close(_gpu(s, "M", X, out_rows=Ne, fp32=fp32), d.M @ X, tol)
    _close(_gpu(s, "K", X, out_rows=Ne, fp32=fp32), (d.A + MU * d.M) @ X, tol)
    _close(_gpu(s, "LIFT", F, out_rows=Ne, fp32=fp32), d.L @ F, tol)
    _close(_gpu(s, "LHM", X, out_rows=Nv, fp32=fp32), d.L.conj().T @ (d.M @ X), tol)
    _close(_gpu(s, "P", F, out_rows=Nv, fp32=fp32), d.P @ F, tol)


@pytest.mark.parametrize("case", CASES)
def test_every_level_operators_and_transfers(case):
    d, H, s, rng = _setup(case)
    for lvl in range(H.nlevels - 1):
        lv, nl = H.edge[lvl], H.nodal[lvl]
        Ne = 2 * lv.n * lv.m
        Nv = lv.n * lv.m
        X = _rand(rng, Ne, 2)
        _close(_gpu(s, "K", X, level=lvl, out_rows=Ne), lv.K @ X, 1e-12)
        F = _rand(rng, Nv, 2)
        _close(_gpu(s, "P", F, level=lvl, out_rows=Nv), nl.P @ F, 1e-12)
        Pe, Pn = H.Pe[lvl], H.Pn[lvl]
        Xc = _rand(rng, Pe.shape[1], 2)
        _close(_gpu(s, "EDGE_PROLONG", Xc, level=lvl, out_rows=Ne), Pe @ Xc, 1e-13)
        _close(_gpu(s, "EDGE_RESTRICT", X, level=lvl, out_rows=Pe.shape[1]), Pe.conj().T @ X, 1e-13)
        Fc = _rand(rng, Pn.shape[1], 2)
        _close(_gpu(s, "NODAL_PROLONG", Fc, level=lvl, out_rows=Nv), Pn @ Fc, 1e-13)
        _close(_gpu(s, "NODAL_RESTRICT", F, level=lvl, out_rows=Pn.shape[1]), Pn.conj().T @ F, 1e-13)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("fp32", [False, True])
def test_smoothers_match_oracle_gauss_seidel(case, fp32):
    d, H, s, rng = _setup(case)
    tol = 5e-5 if fp32 else 1e-11
    lv = H.edge[0]
    Ne = d.n_edges
    B = _rand(rng, Ne, 2)
    X0 = _rand(rng, Ne, 2)
    ref = X0.copy()
    for c in (0, 1, 2, 3):
        ref = lv.gs_colour(ref, B, c)
    got = _gpu(s, "EDGE_SMOOTH", B, Y=B, init=X0, fp32=fp32)
    _close(got, ref, tol)
    ref = X0.copy()
    for c in (3, 2, 1, 0):
        ref = lv.gs_colour(ref, B, c)
    _close(_gpu(s, "EDGE_SMOOTH_BACK", B, Y=B, init=X0, fp32=fp32), ref, tol)
    nl = H.nodal[0]
    Bn = _rand(rng, d.n_nodes, 2)
    F0 = _rand(rng, d.n_nodes, 2)
    ref = F0.copy()
    for c in (0, 1, 2, 3):
        ref = nl.gs_colour(ref, Bn, c)
    _close(_gpu(s, "NODAL_SMOOTH", Bn, Y=Bn, init=F0, fp32=fp32), ref, tol)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("fp32", [False, True])
def test_vcycles_coarse_solves_and_projection(case, fp32):
    d, H, s, rng = _setup(case)
    tol = 5e-5 if fp32 else 1e-11
    B = _rand(rng, d.n_edges, 3)
    _close(_gpu(s, "EDGE_VCYCLE", B, out_rows=d.n_edges, fp32=fp32), H.edge_vcycle(B), tol)
    Bn = _rand(rng, d.n_nodes, 3)
    if d.gamma:
        Bn = Bn - Bn.mean(axis=0, keepdims=True)     # consistent right-hand side
    ref = H.nodal_vcycle(Bn)
    got = _gpu(s, "NODAL_VCYCLE", Bn, out_rows=d.n_nodes, fp32=fp32)
    if d.gamma:   # the solution is defined up to a constant potential
        ref = ref - ref.mean(axis=0, keepdims=True)
        got = got - got.mean(axis=0, keepdims=True)
    _close(got, ref, tol)
    lc = H.nlevels - 1
    nc, mc = H.sizes[lc]
    Bc = _rand(rng, 2 * nc * mc, 2)
    _close(_gpu(s, "COARSE_EDGE", Bc, level=lc, out_rows=2 * nc * mc, fp32=fp32),
           np.linalg.solve(H._coarse_edge, Bc), tol)
    if not fp32:
        U = _rand(rng, d.n_edges, 4)
        ref = Projector(d, H, 2)(U)
        _close(_gpu(s, "PROJECT", U, out_rows=d.n_edges), ref, 1e-11)


def test_gram_and_ritz_small():
    import torch  # noqa: F401
    from paper_2304_00337_amd import to_device_block
    d, H, s, rng = _setup(CASES[0])
    X = _rand(rng, 3001, 37)
    W = _rand(rng, 3001, 70)
    G = s.gram(to_device_block(X), to_device_block(W))
    _close(G, X.conj().T @ W, 1e-13)
    # generalized Hermitian eigenproblem with a nearly dependent, badly scaled G
    q = 30
    Z = _rand(rng, 200, q)
    Z[:, 7] = Z[:, 3] * 1e3 + 1e-9 * Z[:, 8]
    Gm = Z.conj().T @ Z
    A0 = _rand(rng, 200, 200)
    A0 = A0 @ A0.conj().T
    Hm = Z.conj().T @ A0 @ Z
    th, Y = s.ritz_small(Gm, Hm, 10)
    assert len(th) == 10
    # reference: the same pencil restricted to the well-determined directions
    w, V = np.linalg.eigh(Gm / np.sqrt(np.outer(np.diag(Gm).real, np.diag(Gm).real)))
    assert np.all(np.diff(th) >= -1e-12)
    # Y is G-orthonormal and H-diagonal
    assert np.abs(Y.conj().T @ Gm @ Y - np.eye(10)).max() < 1e-8
    HY = Y.conj().T @ Hm @ Y
    assert np.abs(HY - np.diag(th)).max() < 1e-8 * np.abs(th).max()
    # with a well-conditioned G the values are the generalized eigenvalues
    Z2 = _rand(rng, 200, 12)
    G2 = Z2.conj().T @ Z2
    H2 = Z2.conj().T @ A0 @ Z2
    import scipy.linalg as sla
    ref = sla.eigh(H2, G2, eigvals_only=True)
    th2, _ = s.ritz_small(G2, H2, 12)
    _close(th2, ref, 1e-12)
    th3, _ = s.ritz_small(G2, H2, 5, zero_thr=ref[2] * 1.0000001)
    _close(th3, ref[3:8], 1e-12)


@pytest.mark.parametrize("q", [49, 72, 96, 120, 144, 450])
def test_ritz_small_wide(q):
    """The Ritz step for bases wider than 48 columns (the 2p = 96 of 32 + 16 vectors, the 3p
    of LOBPCG): generalized eigenvalues against scipy, Y G-orthonormal and H-diagonal, with a
    well-conditioned G, with a nearly dependent column (dropped), and with a four-fold
    eigenvalue (the cluster path)."""
    import scipy.linalg as sla
    d, H, s, rng = _setup(CASES[0])
    want = min(q, 48)
    rows = max(400, q + 50)
    Z = _rand(rng, rows, q)
    G = Z.conj().T @ Z
    A0 = _rand(rng, rows, rows)
    A0 = A0 @ A0.conj().T
    Hm = Z.conj().T @ A0 @ Z
    ref = sla.eigh(Hm, G, eigvals_only=True)
    th, Y = s.ritz_small(G, Hm, want)
    assert len(th) == want
    assert np.abs(th - ref[:want]).max() <= 1e-11 * np.abs(ref[:want]).max()
    assert np.abs(Y.conj().T @ G @ Y - np.eye(want)).max() < 1e-9
    assert np.abs(Y.conj().T @ Hm @ Y - np.diag(th)).max() < 1e-9 * np.abs(th).max()
    # a nearly dependent column is dropped: the rest of the pencil's values remain
    Z2 = Z.copy()
    Z2[:, 5] = 2.0 * Z2[:, 9] + 1e-10 * Z2[:, 11]
    G2 = Z2.conj().T @ Z2
    H2 = Z2.conj().T @ A0 @ Z2
    keep = [j for j in range(q) if j != 5]
    ref2 = sla.eigh(H2[np.ix_(keep, keep)], G2[np.ix_(keep, keep)], eigvals_only=True)
    th2, Y2 = s.ritz_small(G2, H2, want)
    assert np.abs(th2 - ref2[:want]).max() <= 1e-7 * np.abs(ref2[:want]).max()
    assert np.abs(Y2.conj().T @ G2 @ Y2 - np.eye(want)).max() < 1e-7
    # a four-fold eigenvalue inside the wanted range
    L = np.linalg.cholesky(G)
    Q, _ = np.linalg.qr(_rand(rng, q, q))
    lam = np.sort(rng.uniform(0.5, 40.0, q))
    lam[10:14] = lam[10]
    H3 = L @ (Q * lam) @ Q.conj().T @ L.conj().T
    H3 = 0.5 * (H3 + H3.conj().T)
    th3, Y3 = s.ritz_small(G, H3, want)
    assert np.abs(th3 - lam[:want]).max() <= 1e-10 * lam.max()
    assert np.abs(Y3.conj().T @ G @ Y3 - np.eye(want)).max() < 1e-9
    assert np.abs(Y3.conj().T @ H3 @ Y3 - np.diag(th3)).max() < 1e-9 * lam.max()


@pytest.mark.parametrize("case", CASES)
def test_rayleigh_ritz_products(case):
    """G = S^* M S and H = S^* A S formed straight from S (bl_rr_products) against the
    oracle's assembled matrices, for block widths inside one column group of the matrix-core
    path, spanning two and three groups (diagonal and cross blocks) and with ragged tails."""
    import torch  # noqa: F401
    from paper_2304_00337_amd import Solver, to_device_block
    n, m, a, b, cmin, k = case
    rng = np.random.default_rng(7 + n)
    eps = rng.uniform(1.0, 12.0, n * m)
    d = fem.Discretization(n, m, a, b, eps, *k)
    s = Solver(n, m, a, b, eps, nev=40, nthrow=8, mu=MU, coarsest_min=cmin)
    s.set_k(*k)
    for q in (1, 5, 48, 60, 72, 96, 121, 144):
        S = _rand(rng, d.n_edges, q)
        G, Hm = s.rr_products(to_device_block(S))
        _close(G, S.conj().T @ (d.M @ S), 1e-13)
        _close(Hm, S.conj().T @ (d.A @ S), 1e-13)


@pytest.mark.parametrize("n,levels", [(20, 0), (64, 0), (128, 5), (80, 3)])
@pytest.mark.parametrize("fp32", [False, True])
def test_fused_and_tiled_cycles_equal_per_level_cycles(n, levels, fp32):
    """The coarse levels of a V-cycle run fused in one workgroup per column when they fit
    LDS, each smoothing sweep of the other levels runs as one launch over LDS tiles with
    halos, and the transfers may ride in the sweeps; all perform the per-level, per-colour
    operations in the same order, so every combination gives the same bits, for the edge
    and the nodal cycle, the projection (two nodal cycles) and through a whole solve
    (80 x 48: tiles with ragged edges)."""
    import torch  # noqa: F401
    from paper_2304_00337_amd import Solver
    rng = np.random.default_rng(n)
    m = {20: 12, 80: 48}.get(n, n)
    eps = rng.uniform(1.0, 12.0, n * m)
    k = (0.7, -1.3)
    kw = dict(nev=4, nthrow=2, mu=MU, levels=levels, coarsest_min=3, max_iter=40,
              precision="mixed" if fp32 else "fp64")
    variants = [(0, 0), (1, 0), (0, 1), (1, 1), (0, 2), (1, 2)]
    sv = [Solver(n, m, 1.0, 1.0, eps, coarse_fuse=f, tiled_sweeps=t, **kw) for f, t in variants]
    infos = [s.info() for s in sv]
    assert infos[0]["fused_edge_level"] == -1 and infos[0]["fused_nodal_level"] == -1
    assert infos[1]["fused_edge_level"] >= 0 and infos[1]["fused_nodal_level"] >= 0
    assert all(i["sizes"] == infos[0]["sizes"] for i in infos)
    for s in sv:
        s.set_k(*k)
    B = _rand(rng, 2 * n * m, 5)
    Bn = _rand(rng, n * m, 5)
    E0 = synth.start_block(2 * n * m, 6, 1)
    ref = None
    for s, var in zip(sv, variants):
        got = [_gpu(s, "EDGE_VCYCLE", B, out_rows=2 * n * m, fp32=fp32),
               _gpu(s, "NODAL_VCYCLE", Bn, out_rows=n * m, fp32=fp32),
               _gpu(s, "PROJECT", B, out_rows=2 * n * m)]
        r = s.solve_k(*k, start=E0, allow_noconv=True)
        if ref is None:
            ref = (got, r)
            continue
        assert np.array_equal(got[0], ref[0][0]), ("edge V-cycle", var)
        assert np.array_equal(got[1], ref[0][1]), ("nodal V-cycle", var)
        assert np.array_equal(got[2], ref[0][2]), ("projection (two nodal cycles)", var)
        assert np.array_equal(r["evals"], ref[1]["evals"]) and r["iterations"] == ref[1]["iterations"], var


@pytest.mark.parametrize("fp32", [False, True])
def test_tiled_sweeps_with_many_workgroups(fp32):
    """A 256 x 256 grid with 24 columns launches more tile workgroups than the device holds
    at once, so tiles run in several waves: the tiled V-cycles must still equal the
    per-colour ones bit for bit (the sweeps read and write different buffers)."""
    import torch  # noqa: F401
    from paper_2304_00337_amd import Solver
    n = 256
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    rng = np.random.default_rng(11)
    kw = dict(nev=16, nthrow=8, mu=MU, levels=6, precision="mixed" if fp32 else "fp64")
    B = _rand(rng, 2 * n * n, 24)
    Bn = _rand(rng, n * n, 24)
    outs = []
    for tiled in (0, 1, 2):
        s = Solver(n, n, 1.0, 1.0, eps, tiled_sweeps=tiled, **kw)
        s.set_k(0.9, 0.4)
        outs.append([_gpu(s, "EDGE_VCYCLE", B, out_rows=2 * n * n, fp32=fp32) for _ in range(2)] +
                    [_gpu(s, "NODAL_VCYCLE", Bn, out_rows=n * n, fp32=fp32) for _ in range(2)])
        s.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
