"""Exact Gibbs draws of the auxiliary field given the worldlines (test infrastructure, FP64).

Sec. 3.5.3-3.5.5: given the fermion paths the field factorises over (site, slice).
  Hirsch:   P(s_rl = +1 | paths) = (1 + tanh(lambda m_rl)) / 2,  m = n_up - n_dn
            draw: s = +1 iff u < (1 + tanh(lambda m)) / 2, u a Philox uniform.
  Gaussian: sigma_rl | paths ~ N(a (n_rl - 1/2), 1),  n = n_up + n_dn      (eq. gaussCond)
            draw: sigma = a (n - 1/2) + z, z a Philox Box-Muller normal.
n_up, n_dn count the worldlines of each spin at site r on slice l.
"""
from __future__ import annotations

import numpy as np

from . import hs, philox


def occupancy(paths: np.ndarray, n_up: int, N: int):
    """(n_up[l, r], n_dn[l, r]) counts from worldlines paths[l, p] (up particles first)."""
    L_tau = paths.shape[0]
    cu = np.zeros((L_tau, N), dtype=np.int64)
    cd = np.zeros((L_tau, N), dtype=np.int64)
    for l in range(L_tau):
        cu[l] = np.bincount(paths[l, :n_up], minlength=N)
        cd[l] = np.bincount(paths[l, n_up:], minlength=N)
    return cu, cd


def hirsch_p_plus(lam: float, m: np.ndarray) -> np.ndarray:
    return (1.0 + np.tanh(lam * m)) / 2.0


def gibbs_field(hs_kind: int, U: float, dtau: float, n_up_cnt: np.ndarray,
                n_dn_cnt: np.ndarray, seed: int, sweep: int) -> np.ndarray:
    """New auxiliary field [L_tau, N] drawn from its exact conditional."""
    L_tau, N = n_up_cnt.shape
    sites = np.arange(N, dtype=np.uint64)[None, :]
    slices = np.arange(L_tau, dtype=np.uint64)[:, None]
    x0, x1, _, _ = philox.draw_words(seed, sites, slices, sweep, philox.TAG_GIBBS)
    if hs_kind == hs.HS_GAUSS:
        a = hs.gauss_coupling(U, dtau)
        n = (n_up_cnt + n_dn_cnt).astype(np.float64)
        return a * (n - 0.5) + philox.gaussian(x0, x1)
    lam = hs.hirsch_lambda(U, dtau)
    m = (n_up_cnt - n_dn_cnt).astype(np.float64)
    u = philox.uniform(x0)
    return np.where(u < hirsch_p_plus(lam, m), 1.0, -1.0)
