"""Writes tgv128_oracle_series.json: the FP64 oracle's diagnostic series of the
precision workload, the compressible Taylor-Green vortex at 128^3 (Mach 1.25,
Re 1600, the recipe of paper_2609_16361_amd.inputs.tgv), 4000 steps with the
channels of Sec. 3.3 reduced every 50 steps: volume sums of the kinetic energy and
of the solenoidal and dilatational dissipation densities, divided by the cell count
(lattice units), at the steps t = 0, 50, ..., 3950.

Calls only the oracle and the seeded input generator.  About an hour on 8 cores:
    python tests/golden/make_tgv128_oracle_series.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2609_16361_amd import inputs  # noqa: E402

N_GRID, STEPS, EVERY, CHUNK = 128, 4000, 50, 200


def main(out=os.path.join(HERE, "tgv128_oracle_series.json")):
    case = inputs.tgv(n=N_GRID, steps=STEPS, diag_every=EVERY)
    f = oracle.init(case.params, case.Q0)
    rows = []
    t0 = time.time()
    for s in range(0, STEPS, CHUNK):
        f, d = oracle.run(case.params, f, CHUNK, EVERY)
        rows += [list(r) for r in d]
        print(f"step {s + CHUNK}/{STEPS}  {time.time() - t0:.0f} s", flush=True)
    rows = np.array(rows)
    assert rows.shape[0] == STEPS // EVERY and np.all(rows[:, 8] == 0)
    rec = {"workload": f"compressible Taylor-Green vortex {N_GRID}^3, Mach 1.25, Re 1600, {STEPS} steps",
           "source": "FP64 oracle (oracle/oracle.c), written by tests/golden/make_tgv128_oracle_series.py",
           "steps": list(range(0, STEPS, EVERY)),
           "cells": case.cells,
           "Ek": list(rows[:, 0] / case.cells),
           "eps_s": list(rows[:, 1] / case.cells),
           "eps_d": list(rows[:, 2] / case.cells),
           "omega": case.params["omega"][0], "r": case.meta["r"]}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
