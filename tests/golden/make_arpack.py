"""Writes arpack_<workload>.json: the smallest non-zero eigenvalues of the 256 x 256 lattice
workload (eps = 12 discs of radius 0.3 on eps = 1, 16 pairs) at four points of the
Gamma-X-M-Gamma path with 10 intervals per leg (the first point after Gamma, X, M and the
last point before Gamma); with --z2, of the band-structure experiment's cell (eps = 11.56 in
the disc of radius 0.18, 16 pairs) at 256 x 256 on its kappa = 30 raster at the two points
next to Gamma, (i, j) = (14, 14) and (15, 14); with --c3, of the 1024 x 1024 random
two-phase workload (32 pairs) at its first point after Gamma and at X (the stored file also
holds M and the last point before Gamma, indices 40 and 59, added with --add); with --c4small, of
the six problems of synth.config_c4_small (n 64..128, nev 4..16); with --c3 --add i,j, the
listed path points of the 1024 x 1024 workload, merged into its existing file.  Source:
oracle.dense.gradient_free_eigs (ARPACK on the pencil restricted to the complement of the
null space by exact sparse projections; the kernel cluster of dimension nm would defeat the
plain shift-invert certificate).  Calls only oracle/ and the input generators.

Run from the repository root:  python tests/golden/make_arpack.py [--z2 | --c3 [--add i,j] | --c4small]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import fem  # noqa: E402
from oracle.extrapolation import raster_k  # noqa: E402
from oracle.dense import gradient_free_eigs  # noqa: E402


def run(prob, idx, count):
    pts = []
    for i in idx:
        k1, k2 = (float(v) for v in prob.ks[i])
        t0 = time.time()
        d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, k1, k2)
        lam, _ = gradient_free_eigs(d, count)
        lam = [float(x) for x in lam]
        pts.append({"index": int(i), "k": [k1, k2], "evals": lam, "seconds": round(time.time() - t0, 1)})
        print(f"point {i} k=({k1:.4f},{k2:.4f}) lam1={lam[0]:.10g} lam{count}={lam[-1]:.10g} "
              f"({time.time() - t0:.0f}s)", flush=True)
    return pts


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    if "--c4small" in sys.argv:
        pts = []
        for i, prob in enumerate(synth.config_c4_small()):
            k1, k2 = (float(v) for v in prob.ks[0])
            d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, k1, k2)
            lam, _ = gradient_free_eigs(d, prob.nev)
            pts.append({"index": i, "n": prob.n, "nev": prob.nev, "k": [k1, k2], "evals": [float(x) for x in lam]})
            print(f"problem {i} n={prob.n} nev={prob.nev} lam1={lam[0]:.10g}", flush=True)
        out = {"workload": "synth.config_c4_small: six single-k disc-lattice problems, n 64..128, nev 4..16",
               "source": "oracle.dense.gradient_free_eigs (ARPACK on the complement of the null space)",
               "points": pts}
        name = "arpack_c4small.json"
    elif "--z2" in sys.argv:
        n = 256
        prob = synth.Problem(n, n, 1.0, 1.0, synth.paper_z2_eps(n),
                             np.array([raster_k(30, 14, 14), raster_k(30, 15, 14)]), 16, 8, 5)
        pts = run(prob, [0, 1], 16)
        for pt, ij in zip(pts, [(14, 14), (15, 14)]):
            pt["ij"] = list(ij)
        out = {"workload": "256x256, a=b=1, eps=11.56 in the disc r=0.18 centred, kappa=30 raster "
                           "points (14,14) and (15,14)",
               "source": "oracle.dense.gradient_free_eigs (ARPACK on the complement of the null space)",
               "points": pts}
        name = "arpack_z2_256.json"
    elif "--c3" in sys.argv and "--add" in sys.argv:
        # further points of the 1024 x 1024 path, merged into the stored file under a lock
        # (several of these runs may go in parallel, one point each)
        import fcntl
        prob = synth.config_c3()
        idx = [int(v) for v in sys.argv[sys.argv.index("--add") + 1].split(",")]
        pts = run(prob, idx, 32)
        path = os.path.join(here, "arpack_c3_1024.json")
        with open(path + ".lock", "w") as lk:
            fcntl.flock(lk, fcntl.LOCK_EX)
            with open(path) as f:
                out = json.load(f)
            have = {p["index"]: p for p in out["points"]}
            for pt in pts:
                have[pt["index"]] = pt
            out["points"] = [have[i] for i in sorted(have)]
            with open(path, "w") as f:
                json.dump(out, f, indent=1)
        try:
            os.remove(path + ".lock")
        except FileNotFoundError:   # the other run removed it first
            pass
        print(f"merged points {idx} into {path}")
        return
    elif "--c3" in sys.argv:
        prob = synth.config_c3()
        out = {"workload": "1024x1024, a=b=1, smoothed random field {1, 11.4} (seed 2), 61 points "
                           "on Gamma-X-M-Gamma (20 per leg)",
               "source": "oracle.dense.gradient_free_eigs (ARPACK on the complement of the null space)",
               "points": run(prob, [1, 20], 32)}
        name = "arpack_c3_1024.json"
    else:
        prob = synth.config_c2()
        out = {"workload": "256x256, a=b=1, eps=12 disc lattice r=0.3, 31 points on "
                           "Gamma-X-M-Gamma (10 per leg)",
               "source": "oracle.dense.gradient_free_eigs (ARPACK on the complement of the null space)",
               "points": run(prob, [1, 10, 20, 29], 16)}
        name = "arpack_c2_256.json"
    with open(os.path.join(here, name), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
