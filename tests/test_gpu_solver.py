"""Solver-level parity of the GPU path (bl_solve_k / bl_solve_path through the C ABI)
against the oracle: eigenvalues to 1e-9 relative in FP64 and 1e-6 in mixed precision,
eigenvector subspaces (cluster-wise M-principal angles) to 1e-5, iteration counts close to
the oracle's iteration with the same options."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.closed_form import discrete_nonzero
from oracle.dense import dense_eigs
from oracle.extrapolation import solve_path
from oracle.multigrid import Hierarchy
from oracle.pinvit import Projector, initial_block, pinvit

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solver(prob, precision="fp64", **kw):
    from paper_2304_00337_amd import Solver
    opts = dict(nthrow=prob.nthrow, precision=precision, tol=prob.tol)
    opts.update(kw)
    return Solver(prob.n, prob.m, prob.a, prob.b, prob.eps, nev=prob.nev, **opts)


def _clusters(lam, gap=1e-3):
    """Split ascending values into clusters at relative gaps > gap."""
    cl, cur = [], [0]
    for j in range(1, len(lam)):
        if (lam[j] - lam[j - 1]) / lam[j - 1] > gap:
            cl.append(cur)
            cur = [j]
        else:
            cur.append(j)
    cl.append(cur)
    return cl


def _subspace_check(E_gpu, V_ref, M, lam_ref, nev, tol=1e-5):
    """Cluster-wise M-principal angles; clusters straddling nev are skipped."""
    for cl in _clusters(lam_ref):
        if cl[-1] >= nev:
            break
        s = np.linalg.svd(E_gpu[:, cl].conj().T @ (M @ V_ref[:, cl]), compute_uv=False)
        ang = np.arccos(np.clip(s.min(), -1, 1))
        assert ang < tol, f"cluster {cl}: angle {ang:.2e}"


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c1_disc_against_dense(precision):
    from paper_2304_00337_amd import from_device_block
    prob = synth.config_c1()
    with open(os.path.join(GOLDEN, "c1_dense.json")) as f:
        gold = np.array(json.load(f)["disc"])
    s = _solver(prob, precision, levels=3, max_iter=400)
    assert s.info()["levels"] == 3
    r = s.solve_k(*prob.ks[0], start=prob.start(), want_vectors=True)
    assert r["converged"]
    tol = 1e-9 if precision == "fp64" else 1e-6
    rel = np.abs(r["evals"] - gold[:8]) / gold[:8]
    assert rel.max() < tol, rel
    d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, *prob.ks[0])
    lam, V, _ = dense_eigs(d, 9)
    _subspace_check(from_device_block(r["evecs"]), V, d.M, lam, 8)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_wide_block_against_arpack(precision):
    """32 eigenpairs with 16 throw-away vectors, the block width of the 1024 x 1024 path (a
    96-column Rayleigh-Ritz basis), on a 48 x 48 random two-phase field next to Gamma, against
    the oracle's ARPACK solve: 1e-9 relative in FP64, 1e-6 in mixed precision."""
    from oracle.dense import gradient_free_eigs
    from paper_2304_00337_amd import Solver
    n = 48
    eps = synth.eps_random_field(n, n, 1.0, 1.0, seed=2, sigma=0.05, lo=1.0, hi=11.4)
    k = (math.pi / 20, 0.0)
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    ref = gradient_free_eigs(d, 32)[0]
    s = Solver(n, n, 1.0, 1.0, eps, nev=32, nthrow=16, precision=precision, tol=1e-8, max_iter=300)
    r = s.solve_k(*k, start=synth.start_block(d.n_edges, 48, 5))
    assert r["converged"], r["iterations"]
    rel = np.abs(r["evals"] - ref) / ref
    assert rel.max() < (1e-9 if precision == "fp64" else 1e-6), rel.max()


def test_c1_eps_one_closed_form():
    prob = synth.config_c1(eps_one=True)
    s = _solver(prob, "fp64", levels=3, max_iter=400)
    r = s.solve_k(*prob.ks[0], start=prob.start())
    assert r["converged"]
    cf = discrete_nonzero(32, 32, 1.0, 1.0, 1.0, math.pi / 2, 0.0, 8)
    assert np.max(np.abs(r["evals"] - cf) / cf) < 1e-9


@pytest.mark.parametrize("k", [(0.9, -0.6), (0.0, 0.0), (math.pi, math.pi)])
def test_iteration_matches_oracle_iteration(k):
    """Same start block, same options: eigenvalues, residual decrease and iteration count."""
    n = 32
    eps = synth.eps_disc(n, n, 1.0, 1.0, 8.9, 0.3)
    nev, nthrow, mu = 6, 4, 10.0
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    H = Hierarchy(d, mu=mu, coarsest_min=4)
    pr = Projector(d, H, 2)
    E0 = synth.start_block(d.n_edges, nev + nthrow, 5)
    lam0, Eo = initial_block(d, pr, E0, nev + nthrow)
    lam_o, E_o, rel_o, it_o, conv_o = pinvit(d, H, pr, Eo, lam0, nev, 1e-9, 200)
    assert conv_o
    from paper_2304_00337_amd import Solver
    s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9,
               max_iter=200)
    r = s.solve_k(*k, start=E0)
    assert r["converged"]
    assert np.max(np.abs(r["evals"] - lam_o[:nev]) / lam_o[:nev]) < 1e-9
    # The GPU orthonormalises through the Gram matrix, the oracle by generalized
    # Householder.  Below relative residuals of about 1e-6 the Householder route converges
    # slightly faster (reproduced on the CPU with scipy.linalg.eigh on the same Gram
    # matrices, which matches the GPU count), so the counts agree to about 15%.
    assert abs(r["iterations"] - it_o) <= max(3, int(0.15 * it_o)), (r["iterations"], it_o)


@pytest.mark.parametrize("k", [(0.7, -1.3), (math.pi, 0.0)])
def test_lobpcg_matches_oracle_lobpcg(k):
    """The LOBPCG variant (Section 4: the previous block joins the basis as the direction
    E_prev - E (E^* M E_prev)) against the oracle's LOBPCG from the same start block:
    eigenvalues, convergence and iteration count (which it cuts against the gradient
    variant)."""
    n = 32
    eps = synth.eps_disc(n, n, 1.0, 1.0, 8.9, 0.3)
    nev, nthrow, mu = 6, 4, 10.0
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    H = Hierarchy(d, mu=mu, coarsest_min=4)
    pr = Projector(d, H, 2)
    E0 = synth.start_block(d.n_edges, nev + nthrow, 5)
    lam0, Eo = initial_block(d, pr, E0, nev + nthrow)
    lam_o, E_o, rel_o, it_o, conv_o = pinvit(d, H, pr, Eo, lam0, nev, 1e-9, 200, variant="lobpcg")
    assert conv_o
    from paper_2304_00337_amd import Solver
    kw = dict(nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9, max_iter=200)
    r = Solver(n, n, 1.0, 1.0, eps, variant="lobpcg", **kw).solve_k(*k, start=E0)
    g = Solver(n, n, 1.0, 1.0, eps, **kw).solve_k(*k, start=E0)
    assert r["converged"] and g["converged"]
    assert np.max(np.abs(r["evals"] - lam_o[:nev]) / lam_o[:nev]) < 1e-9
    assert np.max(np.abs(r["evals"] - g["evals"]) / g["evals"]) < 1e-9
    assert abs(r["iterations"] - it_o) <= max(3, int(0.15 * it_o)), (r["iterations"], it_o)
    assert r["iterations"] < g["iterations"], (r["iterations"], g["iterations"])


def test_throwaway_rates_match_oracle():
    """The throw-away study (Section 7) through the C ABI: permittivity 100 in the disc of
    radius 1/3, the same start block and options on both sides.  Per t the residual records
    agree to 1e-5 while the wanted pairs are above 1e-2 (t = 1: the first ten iterations), the
    observed rates of the last two wanted
    pairs over the window 1e-2 .. 1e-6 and the iteration counts agree with the oracle's, and
    both rates fall as t grows.  With t = 4 and 8 the rates are well determined (the oracle's
    own rates move by < 0.5% when its start block is perturbed at the rounding level,
    tests/test_oracle_throwaway.py), so the GPU's must agree to 3%.  With t = 1 (p = nev + 1)
    they are not: the same perturbations move the oracle's rates over 0.67 .. 0.72 and its
    iteration count over 63 .. 70, and the route of the orthonormalisation matters: the
    oracle run with the Gram (Cholesky) orthonormalisation the GPU uses instead of
    Householder takes 73 .. 74 iterations at rates 0.72 .. 0.75.  The GPU's t = 1 count is
    held to 25% of the Gram-route oracle's and its rates to the two routes' envelope widened
    by 10%."""
    from oracle.throwaway import observed_rate, study
    from paper_2304_00337_amd import Solver
    n, nev, ts, mu = 32, 8, (1, 4, 8), 0.5
    k = (0.5 * math.pi, 0.25 * math.pi)
    eps = synth.paper_z1_eps(n)
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    H = Hierarchy(d, mu=mu, coarsest_min=4)
    E0 = synth.start_block(d.n_edges, nev + max(ts), 3)
    ref = study(d, H, Projector(d, H, 2), E0, nev, ts, (nev - 1, nev), tol=1e-9, max_iter=300,
                lower=1e-6)
    ref_gram = study(d, H, Projector(d, H, 2), E0, nev, (1,), (nev - 1, nev), tol=1e-9, max_iter=300,
                     lower=1e-6, ortho="gram")[0]
    gpu = []
    for r in ref:
        s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=r["t"], mu=mu, coarsest_min=4, tol=1e-9,
                   max_iter=300)
        out = s.solve_k(*k, start=np.ascontiguousarray(E0[:, :r["p"]]))
        hist = s.residual_history()
        assert out["converged"] and r["converged"]
        assert hist.shape[0] == out["iterations"] + 1
        assert np.max(np.abs(out["evals"] - r["lam"]) / r["lam"]) < 1e-9
        if r["t"] == 1:
            it_ref = ref_gram["iterations"]
            assert abs(out["iterations"] - it_ref) <= max(3, int(0.25 * it_ref)), (out["iterations"], it_ref)
        else:
            assert abs(out["iterations"] - r["iterations"]) <= max(3, int(0.15 * r["iterations"])), (
                r["t"], out["iterations"], r["iterations"])
        # the residual records while the last wanted pairs are above 1e-2: with t >= 4 the
        # oracle's own record moves by < 3e-8 under rounding-level perturbations there, with
        # t = 1 its deviation grows about threefold per iteration (6e-3 by the 19th), so
        # only the first ten rows are determined well enough to compare
        h = r["history"]
        rows = min(len(h), len(hist))
        early = np.all(h[:rows, nev - 2:] >= 1e-2, axis=1)
        if r["t"] == 1:
            early[10:] = False
        assert early.sum() >= 3
        dev = np.abs(hist[:rows][early] - h[:rows][early]) / h[:rows][early]
        assert np.max(dev) < 1e-5, (r["t"], np.max(dev))
        rates = {i: observed_rate(hist[:, i - 1], 1e-2, 1e-6) for i in (nev - 1, nev)}
        for i, v in rates.items():
            if r["t"] == 1:
                lo = 0.9 * min(r["rates"][i], ref_gram["rates"][i])
                hi = 1.1 * max(r["rates"][i], ref_gram["rates"][i])
                assert lo <= v <= hi, (i, v, r["rates"][i], ref_gram["rates"][i])
            else:
                assert abs(v - r["rates"][i]) < 0.03 * r["rates"][i], (r["t"], i, v, r["rates"][i])
        gpu.append(rates)
    for i in (nev - 1, nev):
        assert gpu[2][i] < gpu[1][i] < gpu[0][i]
        assert ref[2]["rates"][i] < ref[1]["rates"][i] < ref[0]["rates"][i]


@pytest.mark.parametrize("k", [(0.7, -1.3), (0.0, 0.0)])
def test_nested_start_matches_oracle(k):
    """Nested iteration for a first Bloch parameter (Section 6) through the C ABI: the dense
    coarsest solve, prolongation and per-level iterations give a start block from which the
    finest solve reaches the dense eigenvalues in about as many iterations as the oracle's
    nested start (and fewer than from a random block); per-level counts agree."""
    from oracle.extrapolation import nested_start
    from paper_2304_00337_amd import Solver
    n, nev, nthrow, mu = 32, 6, 3, 10.0
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
    E, its_o = nested_start(n, n, 1.0, 1.0, eps, *k, nev, nthrow, tol_levels=1e-3, mu=mu, coarsest_min=4)
    H = Hierarchy(d, mu=mu, coarsest_min=4)
    pr = Projector(d, H, 2)
    lam0, E0 = initial_block(d, pr, E, nev + nthrow)
    it_o = pinvit(d, H, pr, E0, lam0, nev, 1e-9, 200)[3]
    s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9, max_iter=200)
    start, its = s.nested_start(*k, tol_levels=1e-3)
    assert len(its) == len(its_o)
    for a, b in zip(its, its_o):
        assert abs(int(a) - b) <= max(2, int(0.2 * b)), (list(its), its_o)
    r = s.solve_k(*k, start=start)
    ref, _, _ = dense_eigs(d, nev)
    assert r["converged"] and np.max(np.abs(r["evals"] - ref) / ref) < 1e-9
    assert abs(r["iterations"] - it_o) <= max(3, int(0.2 * it_o)), (r["iterations"], it_o)
    rnd = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9,
                 max_iter=200).solve_k(*k, start=synth.start_block(d.n_edges, nev + nthrow, 5))
    assert r["iterations"] < rnd["iterations"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nested_start_option_in_the_engine(precision):
    """The nested_start option: a path's first point without a start block starts from the
    nested iteration inside the engine, and gives to the last bit what the same point gives
    from the block bl_nested_start returns; every point of the path matches the dense
    eigenvalues, and the first point needs fewer iterations than from a random block."""
    from paper_2304_00337_amd import Solver
    n, nev, nthrow, mu = 32, 6, 3, 10.0
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    ks = np.array([(0.7, -1.3), (0.8, -1.2), (0.9, -1.1)])
    kw = dict(nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9, max_iter=200, precision=precision)
    block, its = Solver(n, n, 1.0, 1.0, eps, **kw).nested_start(*ks[0], tol_levels=1e-3)
    assert its[1:-1].min() > 0
    a = Solver(n, n, 1.0, 1.0, eps, nested_start=1, nested_tol=1e-3, **kw).solve_path(ks)
    b = Solver(n, n, 1.0, 1.0, eps, **kw).solve_path(ks, start=block)
    assert np.array_equal(a["evals"], b["evals"]) and np.array_equal(a["iterations"], b["iterations"])
    tol = 1e-9 if precision == "fp64" else 1e-6
    for t in range(len(ks)):
        d = fem.Discretization(n, n, 1.0, 1.0, eps, *ks[t])
        ref = dense_eigs(d, nev)[0]
        assert np.max(np.abs(a["evals"][t] - ref) / ref) < tol
    rnd = Solver(n, n, 1.0, 1.0, eps, **kw).solve_k(*ks[0], start=synth.start_block(2 * n * n, nev + nthrow, 5))
    assert a["iterations"][0] < rnd["iterations"]


def test_kgrid_raster_matches_oracle():
    """The Section 6 raster through the C ABI (bl_solve_kgrid) on a 4 x 4 Bloch grid of the
    32 x 32 mesh with the band-structure permittivity: per point the eigenvalues equal the
    oracle's raster run to 1e-9 and its iteration counts agree; with the absolute defect as
    stopping measure (tol_abs) the reported defects are below the tolerance and the
    eigenvalues match the dense solve to it."""
    from oracle.extrapolation import solve_grid
    from paper_2304_00337_amd import Solver
    n, kappa, nev, nthrow, mu = 32, 4, 6, 3, 5.0
    eps = synth.paper_z2_eps(n)
    start = synth.start_block(2 * n * n, nev + nthrow, 8)
    ref = solve_grid(n, n, 1.0, 1.0, eps, kappa, nev, nthrow, start, tol=1e-9, mu=mu, coarsest_min=4)
    s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-9, max_iter=300)
    out = s.solve_kgrid(kappa, start)
    assert out["converged"]
    its_o = []
    for r in ref:
        i, j = r["ij"]
        assert r["converged"]
        assert np.max(np.abs(out["evals"][j, i] - r["lam"]) / r["lam"]) < 1e-9, (i, j)
        it = int(out["iterations"][j, i])
        assert abs(it - r["iterations"]) <= max(3, int(0.2 * r["iterations"])), (i, j, it, r["iterations"])
        its_o.append(r["iterations"])
    assert abs(int(out["iterations"].sum()) - sum(its_o)) <= 0.1 * sum(its_o)
    sa = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=mu, coarsest_min=4, tol=1e-3, tol_abs=1,
                max_iter=300)
    oa = sa.solve_kgrid(2, start)
    assert oa["converged"] and np.all(oa["relres"] <= 1e-3)
    for j in range(2):
        for i in range(2):
            d = fem.Discretization(n, n, 1.0, 1.0, eps, *((2 * i - 1) * math.pi, (2 * j - 1) * math.pi))
            lam, _, _ = dense_eigs(d, nev)
            assert np.max(np.abs(oa["evals"][j, i] - lam) / lam) < 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_short_path_matches_oracle_path(precision):
    n = 32
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    ks = synth.path_gxmg(3)[:7]      # Gamma .. X .. toward M
    nev, nthrow = 6, 3
    start = synth.start_block(2 * n * n, nev + nthrow, 1)
    from paper_2304_00337_amd import Solver
    s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=10.0, precision=precision,
               tol=1e-9, max_iter=300)
    r = s.solve_path(ks, start=start)
    assert r["converged"]
    for t, k in enumerate(ks):
        d = fem.Discretization(n, n, 1.0, 1.0, eps, *k)
        ref, _, _ = dense_eigs(d, nev)
        tol = 1e-9 if precision == "fp64" else 1e-6
        assert np.max(np.abs(r["evals"][t] - ref) / ref) < tol, (t, r["evals"][t], ref)
    # warm starts by extrapolation need fewer iterations than the cold first point
    assert np.median(r["iterations"][2:]) < r["iterations"][0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_soft_locking_keeps_the_results(precision):
    """Soft locking (no V-cycle direction for the converged pairs: a leading run skipped by
    the column offset, pairs further in squeezed out of the residual block in place) changes
    the basis of later iterations only: the path's eigenvalues still match the dense solve at the
    stated tolerance, the locked run takes about as many iterations (within 10%: the dropped
    directions of a pair locked just below tol can cost it an extra iteration), and it did
    lock."""
    n = 32
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    ks = synth.path_gxmg(3)[:5]
    nev, nthrow = 8, 4
    start = synth.start_block(2 * n * n, nev + nthrow, 2)
    from paper_2304_00337_amd import Solver
    from paper_2304_00337_amd.native import BlochError
    runs = {}
    for lock in (0.0, 1.0):
        s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=10.0, precision=precision,
                   tol=1e-9, max_iter=300, lock_rel=lock)
        runs[lock] = (s.solve_path(ks, start=start), s.info()["locked_columns"])
    assert runs[0.0][1] == 0 and runs[1.0][1] > 0
    tol = 1e-9 if precision == "fp64" else 1e-6
    for lock, (r, _) in runs.items():
        assert r["converged"], lock
        for t, k in enumerate(ks):
            ref, _, _ = dense_eigs(fem.Discretization(n, n, 1.0, 1.0, eps, *k), nev)
            assert np.max(np.abs(r["evals"][t] - ref) / ref) < tol, (lock, t)
    assert np.sum(runs[1.0][0]["iterations"]) <= 1.1 * np.sum(runs[0.0][0]["iterations"]) + 2
    with pytest.raises(BlochError):
        Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, lock_rel=1.5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fewer_preconditioned_throwaway_vectors_keep_the_results(precision):
    """Only the first throw-away vector gets a preconditioned direction (throw_precond = 1),
    the others stay in the block and are refined by the Ritz step alone: the path's
    eigenvalues still match the dense solve at the stated tolerance, with at most a third
    more iterations, and the option is checked."""
    n = 32
    eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
    ks = synth.path_gxmg(3)[:5]
    nev, nthrow = 8, 4
    start = synth.start_block(2 * n * n, nev + nthrow, 6)
    from paper_2304_00337_amd import Solver
    from paper_2304_00337_amd.native import BlochError
    its = {}
    tol = 1e-9 if precision == "fp64" else 1e-6
    for tp in (0, 1):
        s = Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, mu=10.0, precision=precision,
                   tol=1e-9, max_iter=300, throw_precond=tp)
        r = s.solve_path(ks, start=start)
        assert r["converged"], tp
        for t, k in enumerate(ks):
            ref, _, _ = dense_eigs(fem.Discretization(n, n, 1.0, 1.0, eps, *k), nev)
            assert np.max(np.abs(r["evals"][t] - ref) / ref) < tol, (tp, t)
        its[tp] = int(np.sum(r["iterations"]))
        if tp:
            assert s.info()["locked_columns"] >= 3 * its[tp] - 3 * len(ks)
    assert its[1] <= 1.35 * its[0] + 2
    with pytest.raises(BlochError):
        Solver(n, n, 1.0, 1.0, eps, nev=nev, nthrow=nthrow, throw_precond=-1)


def test_mixed_equals_fp64_and_alone_equals_repeat():
    prob = synth.config_c1()
    s64 = _solver(prob, "fp64", levels=3, nthrow=4, max_iter=300)
    s32 = _solver(prob, "mixed", levels=3, nthrow=4, max_iter=300)
    E0 = synth.start_block(prob.n_edges, 12, 0)
    a = s64.solve_k(*prob.ks[0], start=E0)
    b = s32.solve_k(*prob.ks[0], start=E0)
    assert np.max(np.abs(a["evals"] - b["evals"]) / a["evals"]) < 1e-6
    c = s64.solve_k(*prob.ks[0], start=E0)
    assert np.max(np.abs(a["evals"] - c["evals"]) / a["evals"]) < 1e-12


def test_errors_are_reported():
    from paper_2304_00337_amd import Solver
    from paper_2304_00337_amd.native import BlochError
    n = 16
    s = Solver(n, n, 1.0, 1.0, np.ones(n * n), nev=4, nthrow=2, max_iter=1)
    with pytest.raises(BlochError):
        s.solve_k(0.3, 0.2)              # no start block and no history
    r = s.solve_k(0.3, 0.2, start=synth.start_block(2 * n * n, 6, 0), allow_noconv=True)
    assert not r["converged"] and r["iterations"] == 1
    with pytest.raises(BlochError):
        s.solve_k(float("nan"), 0.0, start=synth.start_block(2 * n * n, 6, 0))


def test_autotuned_launch_shapes_do_not_change_results():
    """The autotuner only picks launch shapes (threads per block, columns per thread, block
    order, output tiles): every candidate shape reproduces the default one bit for bit."""
    import os
    prob = synth.config_c1()
    E0 = synth.start_block(prob.n_edges, 12, 3)
    base = _solver(prob, "mixed", levels=3, nthrow=4, max_iter=300, autotune=0)
    assert base.info()["edge_smooth_shape"] == [256, 1, 0]
    ref = base.solve_k(*prob.ks[0], start=E0)
    tuned = _solver(prob, "mixed", levels=3, nthrow=4, max_iter=300, autotune=1)
    it = tuned.info()
    assert it["edge_smooth_shape"][0] in (64, 128, 256) and it["rr_tile"] in (48, 64)
    got = [tuned.solve_k(*prob.ks[0], start=E0)]
    try:
        for shape in ("64,1,0", "128,2,1", "256,2,0", "64,2,1"):
            for tile in ("48", "64"):
                os.environ["BL_SMOOTH_SHAPE"] = shape
                os.environ["BL_RR_TILE"] = tile
                s = _solver(prob, "mixed", levels=3, nthrow=4, max_iter=300, autotune=1)
                assert s.info()["edge_smooth_shape"] == [int(v) for v in shape.split(",")]
                assert s.info()["rr_tile"] == int(tile)
                got.append(s.solve_k(*prob.ks[0], start=E0))
    finally:
        os.environ.pop("BL_SMOOTH_SHAPE", None)
        os.environ.pop("BL_RR_TILE", None)
    for r in got:
        assert np.array_equal(r["evals"], ref["evals"]) and r["iterations"] == ref["iterations"]
