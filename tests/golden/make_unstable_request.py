"""Writes unstable_request.json: the oracle's own run of request 138 of the
1000-request serving stream (seed 2; 430 x 1952 cells, m = 2, n = 3, 449
steps), which turns non-physical between steps 350 and 400: the counts of
non-finite cells and of cells with rho <= 0 or T <= 0 every 50 steps.  The
GPU test holds the float64 path to the same verdict and the server to
reporting the request failed.

Calls only the CPU oracle (oracle/).  The workload numbers come from
paper_1308_0653_amd.workloads, which holds no arithmetic of the method.
Run:  python tests/golden/make_unstable_request.py   (about 40 s on 8 cores)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1308_0653_amd import workloads as W  # noqa: E402

INDEX = 138


def main():
    w = W.serving_stream(count=1000, rate=30.0)[INDEX][1]
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    counts = {}
    for s in range(50, 451, 50):
        o.step(50)
        F = o.fields()
        nonfinite = ~np.isfinite(F).all(axis=0)
        nonphys = ~nonfinite & ((F[0] <= 0) | (F[3] <= 0))
        counts[s] = {"n_nonfinite": int(nonfinite.sum()), "n_nonphys": int(nonphys.sum())}
        print(s, counts[s], flush=True)
    out = {"index": INDEX, "nr": w.nr, "ntheta": w.ntheta, "nsteps": w.nsteps, "m": w.m, "n": w.n,
           "oracle_bad_cells": counts,
           "note": "written by tests/golden/make_unstable_request.py from the oracle alone"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "unstable_request.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
