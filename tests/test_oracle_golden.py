"""The oracle reproduces its stored seeded trajectories (written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np

import synth
from oracle import sweep

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_trajectories.json")


def test_oracle_trajectories_unchanged():
    with open(GOLD) as f:
        gold = json.load(f)
    for name, rec in gold.items():
        desc = synth.ChainDesc(**rec["desc"])
        aux = synth.initial_aux(desc)
        paths = synth.initial_paths(desc)
        tab = sweep.ChainTables(desc)
        for s in range(rec["n_sweeps"]):
            aux, paths, lz = sweep.sweep(desc, aux, paths, s, tab)
            if s == 0:
                assert np.allclose(lz, rec["logZ_sweep0"], rtol=1e-13), name
        assert np.array_equal(paths, np.array(rec["paths"])), name
        assert np.allclose(aux, np.array(rec["aux"]), rtol=1e-12, atol=1e-13), name
