"""Writes the stored oracle summaries in this folder (calls only oracle/ and
the seeded input generators).  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import crp_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def summary(fin, cnt):
    fin = O.sort_finished(fin)
    return {
        "counts": cnt,
        "nsteps_sum": int(fin["nsteps"].sum()),
        "first": {k: (v[:4].tolist()) for k, v in fin.items()},
        "E_mean": float(fin["E"].mean()),
        "x_abs_mean": float(np.abs(fin["x"]).mean()),
    }


def main():
    w = I.W_SMALL
    g = O.GridRef(w.make_grid(), w.spacing_m)
    t = O.TablesRef(w.make_tables())
    inj = w.make_injection()
    out = {"workload": w.name, "description": "1000 protons at 1e19 eV, 32^3 FP64 grid of "
           "100 kpc cells (band 2..16 cells, 1 nG, seed 1), rising loss table, 10 Mpc"}
    fin, _, cnt, _ = O.propagate(O.config_for(w), g, t, inj)
    out["fp64"] = summary(fin, cnt)
    g32 = O.GridRef(w.make_grid().astype(np.float32), w.spacing_m)
    fin, _, cnt, _ = O.propagate(O.config_for(w, precision=O.MIX), g32, t, inj)
    out["mix"] = summary(fin, cnt)
    with open(os.path.join(HERE, "small_workload_oracle.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
