"""Writes c1_dense.json: the smallest non-zero eigenvalues of the 32 x 32 workload
(eps = 8.9 in the centred disc of radius 0.2, and eps = 1, k = (pi/2, 0)) from the dense
generalized eigensolve of the oracle.  Calls only oracle/ and the input generators.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fem  # noqa: E402
from oracle.dense import dense_eigs  # noqa: E402


def main():
    out = {"workload": "32x32, a=b=1, eps=8.9 disc r=0.2 (cell centres) or eps=1, k=(pi/2,0)",
           "source": "oracle.dense.dense_eigs (scipy.linalg.eigh on the assembled pencil)"}
    for key, one in (("disc", False), ("eps1", True)):
        prob = synth.config_c1(eps_one=one)
        d = fem.Discretization(prob.n, prob.m, prob.a, prob.b, prob.eps, *prob.ks[0])
        lam, _, _ = dense_eigs(d, 16)
        out[key] = [float(x) for x in lam]
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_dense.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
