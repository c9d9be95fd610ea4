"""Writes the stored oracle trajectories under tests/golden/ (calls only oracle/ and synth).

Run from the repository root:  python tests/golden/make_golden.py
The paper prints no worked-example values (its figures carry no data and it has no tables),
so the fixtures here are oracle outputs on seeded synthetic inputs; they pin the oracle against
accidental change. A change to them must name, in its commit message, the passage of the paper
(or the reading of it) that justifies the oracle change.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import sweep  # noqa: E402


def trajectory(desc, n_sweeps):
    aux = synth.initial_aux(desc)
    paths = synth.initial_paths(desc)
    tab = sweep.ChainTables(desc)
    logz0 = None
    for s in range(n_sweeps):
        aux, paths, lz = sweep.sweep(desc, aux, paths, s, tab)
        if logz0 is None:
            logz0 = lz
    return {"desc": desc.__dict__, "n_sweeps": n_sweeps, "logZ_sweep0": logz0.tolist(),
            "aux": aux.tolist(), "paths": paths.tolist()}


def main():
    out = {
        "small_gauss_4x4": trajectory(synth.config_small_fp64()[0], 10),
        "small_hirsch_4x4_blocks": trajectory(
            synth.ChainDesc(L=4, L_tau=12, n_up=8, n_dn=8, hs_kind=synth.HS_HIRSCH, block_len=5,
                            t=1.0, U=4.0, dtau=0.1, seed=3), 10),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_trajectories.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
