"""Run the autotuner for a list of engine shapes and write its choices as a table.

    python -m paper_2304_00337_amd.tune_table OUT [n:p:precision:slots ...]

Each shape is tuned on a fresh engine of that many slots (the table that ships with the
library is ignored while doing so) and written as one line of `OUT` in the format that
libbloch.so reads at start-up (tuning.txt next to the library):

    n m p precision  edge_threads edge_columns edge_xcd  nodal_threads nodal_columns nodal_xcd  rr_tile

Shapes the table lacks are tuned when an engine is created and kept for the process.
"""
import os
import sys

DEFAULT_SHAPES = ["256:24:1:4", "256:24:0:1", "256:24:1:1", "128:12:1:8", "64:6:1:8"]


def tune(shapes):
    os.environ["BL_TUNE_IGNORE_TABLE"] = "1"
    import numpy as np
    import synth
    from .api import Batch
    lines = []
    for spec in shapes:
        n, p, prec, slots = (int(v) for v in spec.split(":"))
        nev = max(1, (2 * p) // 3)
        eps = synth.eps_disc_lattice(n, n, 1.0, 1.0, 12.0, 0.3)
        probs = [dict(n=n, m=n, a=1.0, b=1.0, eps=eps, nev=nev, nthrow=p - nev, ks=np.array([[0.5, 0.25]]),
                      start=synth.start_block(2 * n * n, p, 7 + i)) for i in range(slots)]
        with Batch(max_slots=slots, precision=prec, max_iter=1, autotune=1) as b:
            b.run(probs)
            for inf in b.engines():
                e, nd = inf["edge_smooth_shape"], inf["nodal_smooth_shape"]
                lines.append(f"{inf['n']} {inf['m']} {inf['p']} {inf['precision']}  {e[0]} {e[1]} {e[2]}  "
                             f"{nd[0]} {nd[1]} {nd[2]}  {inf['rr_tile']}")
                print(f"# {spec}: {lines[-1]} (tuning {inf['autotune_ms']:.1f} ms)", flush=True)
    return lines


def main():
    if len(sys.argv) < 2:
        print(__doc__)
        sys.exit(2)
    out = sys.argv[1]
    lines = tune(sys.argv[2:] or DEFAULT_SHAPES)
    seen = set()
    with open(out, "w") as f:
        f.write("# n m p precision  edge_threads edge_columns edge_xcd  nodal_threads nodal_columns "
                "nodal_xcd  rr_tile\n")
        for ln in lines:
            key = tuple(ln.split()[:4])
            if key not in seen:
                seen.add(key)
                f.write(ln + "\n")


if __name__ == "__main__":
    main()
