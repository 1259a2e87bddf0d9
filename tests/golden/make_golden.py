"""Write tests/golden/rmat20_u12.json: the oracle's colourful count on the full-size R-MAT scale-20
configuration (edge factor 16, seed 1; 12-vertex Pruefer tree, seed 12; one PCG64 colouring, seed 777).

Calls only inputs/ (to build the inputs) and oracle/ (to compute the expected values). Takes tens
of minutes and tens of GB of host memory: run it by hand, e.g. `python tests/golden/make_golden.py`.
Stores the total X (long double, as a decimal string) and the per-vertex counts of 2000 vertices:
the 50 of highest degree and 1950 drawn uniformly (seed 5).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat20_u12.json")


def main():
    scale, ef, gseed, k, tseed, cseed, root = 20, 16, 1, 12, 12, 777, 11
    rp, cl = inputs.rmat_graph(scale, ef, gseed)
    T = inputs.pruefer_tree(k, tseed)
    col = inputs.colours(len(rp) - 1, k, cseed)
    t0 = time.time()
    X, pv = oracle.count(rp, cl, col, T, root=root, per_vertex=True, longdouble=True)
    secs = time.time() - t0
    deg = np.diff(rp)
    rng = np.random.default_rng(5)
    top = np.argsort(-deg, kind="stable")[:50]
    rest = rng.choice(len(deg), size=1950, replace=False)
    sample = np.unique(np.concatenate([top, rest]))
    out = {
        "citation": "Section 2.1, Eq. 1 and Algorithm 1 (the colourful count for one colouring); values computed "
                    "by oracle/ (long-double compensated accumulation)",
        "graph": {"kind": "rmat", "scale": scale, "edge_factor": ef, "seed": gseed, "nnz": int(len(cl))},
        "template": {"kind": "pruefer", "k": k, "seed": tseed, "root": root},
        "colouring": {"kind": "pcg64", "seed": cseed},
        "X": repr(float(X)),
        "X_longdouble": np.format_float_scientific(X, precision=25, unique=False),
        "vertices": [int(v) for v in sample],
        "vertex_counts": [repr(float(pv[v])) for v in sample],
        "oracle_seconds": round(secs, 1),
        "oracle_threads": oracle.threads(),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}: X={X!r} in {secs:.0f}s")


if __name__ == "__main__":
    main()
