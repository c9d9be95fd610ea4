"""One sweep of the joint worldline / auxiliary-field chain (test infrastructure, FP64).

Composition (Sec. 3.5 and Appendix A.1, each move leaves the joint measure of eq. joint
invariant): first every worldline's blocks are redrawn by FFBS given the field at sweep start,
then the field is redrawn site by site from its exact conditional given the new worldlines.
Permutations stay the identity.
"""
from __future__ import annotations

import numpy as np

from . import ffbs, gibbs, hs, lattice


class ChainTables:
    """Dense transfer matrix of one chain (built once per (L, t, dtau))."""

    def __init__(self, desc):
        self.desc = desc
        self.Gmat = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)


def sweep(desc, aux: np.ndarray, paths: np.ndarray, s: int, tables: ChainTables | None = None,
          return_margin: bool = False):
    """Returns (new_aux [L_tau, N], new_paths [L_tau, Np] int32, logZ [Np], margins?)."""
    tables = tables or ChainTables(desc)
    W_up, W_dn = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)
    new_paths = paths.astype(np.int64).copy()
    logZ = np.zeros(desc.n_particles)
    marg = np.full(paths.shape, np.inf)
    for W, parts in ((W_up, np.arange(desc.n_up)),
                     (W_dn, np.arange(desc.n_up, desc.n_particles))):
        if len(parts) == 0:
            continue
        res = ffbs.ffbs_spin(tables.Gmat, W, paths, parts, desc.seed, s, desc.block_len,
                             return_margin)
        new_paths[:, parts] = res[0]
        logZ[parts] = res[1]
        if return_margin:
            marg[:, parts] = res[2]
    cu, cd = gibbs.occupancy(new_paths, desc.n_up, desc.N)
    new_aux = gibbs.gibbs_field(desc.hs_kind, desc.U, desc.dtau, cu, cd, desc.seed, s)
    out = (new_aux, new_paths.astype(np.int32), logZ)
    if return_margin:
        return out + (marg,)
    return out


def run(desc, aux: np.ndarray, paths: np.ndarray, first_sweep: int, n_sweeps: int):
    tables = ChainTables(desc)
    for s in range(first_sweep, first_sweep + n_sweeps):
        aux, paths, _ = sweep(desc, aux, paths, s, tables)
    return aux, paths
