"""Stationarity of the oracle's sweep (Appendix A.1: each move leaves eq. joint invariant) on a
lattice small enough to enumerate the joint measure exactly."""
import itertools

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import hs, lattice, sweep


def exact_path_marginal(desc):
    """pi(up path, down path) with the field summed / integrated out exactly, P = identity.

    Ising: sum_s exp(lambda s m) = 2 cosh(lambda m) per (site, slice).
    Gaussian: int ds exp(-s^2/2 - a s/2 + a s n) ∝ exp(a^2 (n - 1/2)^2 / 2) per (site, slice).
    """
    L, L_tau, N = desc.L, desc.L_tau, desc.N
    Gm = lattice.transfer_matrix(L, desc.t, desc.dtau)
    lam = hs.hirsch_lambda(desc.U, desc.dtau)
    a = hs.gauss_coupling(desc.U, desc.dtau)
    states = list(itertools.product(range(N), repeat=L_tau))
    dn_states = states if desc.n_dn else [(-1,) * L_tau]
    prob = np.zeros((len(states), len(dn_states)))
    for iu, pu in enumerate(states):
        wu = np.prod([Gm[pu[(l + 1) % L_tau], pu[l]] for l in range(L_tau)])
        for idn, pd in enumerate(dn_states):
            if pd[0] < 0:
                wd = 1.0
            else:
                wd = np.prod([Gm[pd[(l + 1) % L_tau], pd[l]] for l in range(L_tau)])
            w = wu * wd
            for l in range(L_tau):
                for r in range(N):
                    nu, nd = int(pu[l] == r), int(pd[l] == r)
                    if desc.hs_kind == synth.HS_HIRSCH:
                        w *= np.cosh(lam * (nu - nd))
                    else:
                        w *= np.exp(0.5 * a * a * (nu + nd - 0.5) ** 2)
            prob[iu, idn] = w
    return states, prob / prob.sum()


def field_sign_conditional(desc, states):
    """P(aux[0, 0] > 0 | up path, down path): the exact field conditional at (slice 0, site 0)."""
    lam = hs.hirsch_lambda(desc.U, desc.dtau)
    a = hs.gauss_coupling(desc.U, desc.dtau)
    n_up = np.array([int(p[0] == 0) for p in states])
    nu = n_up[:, None]
    nd = n_up[None, :] if desc.n_dn else np.zeros((1, 1), dtype=int)
    if desc.hs_kind == synth.HS_HIRSCH:
        return (1 + np.tanh(lam * (nu - nd))) / 2
    return scipy.stats.norm.cdf(a * (nu + nd - 0.5))


def run_histogram(desc, n_sweeps, n_thin=2):
    """Visits of (up path, down path, [aux[0,0] > 0]) along the oracle's chain."""
    aux = synth.initial_aux(desc)
    paths = synth.initial_paths(desc)
    tab = sweep.ChainTables(desc)
    N, L_tau = desc.N, desc.L_tau
    counts = np.zeros((N ** L_tau, N ** L_tau if desc.n_dn else 1, 2))
    for s in range(n_sweeps):
        aux, paths, _ = sweep.sweep(desc, aux, paths, s, tab)
        if s >= 20 and s % n_thin == 0:
            cu = sum(int(paths[l, 0]) * N ** (L_tau - 1 - l) for l in range(L_tau))
            cd = sum(int(paths[l, 1]) * N ** (L_tau - 1 - l) for l in range(L_tau)) if desc.n_dn else 0
            counts[cu, cd, int(aux[0, 0] > 0)] += 1
    return counts


def exact_joint(desc):
    states, prob = exact_path_marginal(desc)
    p_pos = field_sign_conditional(desc, states)
    return np.stack([prob * (1 - p_pos), prob * p_pos], axis=-1)


# The chi-square test takes the visits as independent draws, so the samples are thinned beyond
# the chain's autocorrelation: the Gaussian-field chain needs every sixth sweep (at every second
# one its statistic runs near twice its degrees of freedom for any random stream).
@pytest.mark.parametrize("kind,L_tau,B,n_dn,n_sweeps,n_thin", [
    (synth.HS_HIRSCH, 2, 0, 1, 14000, 2),
    (synth.HS_GAUSS, 2, 0, 1, 28000, 6),
    (synth.HS_HIRSCH, 4, 2, 0, 12000, 2),
])
def test_sweep_leaves_joint_measure_invariant(kind, L_tau, B, n_dn, n_sweeps, n_thin):
    desc = synth.ChainDesc(L=2, L_tau=L_tau, n_up=1, n_dn=n_dn, hs_kind=kind, block_len=B,
                           t=1.0, U=4.0, dtau=0.3, seed=17)
    prob = exact_joint(desc)
    counts = run_histogram(desc, n_sweeps, n_thin)
    M = counts.sum()
    exp = prob.ravel() * M
    obs = counts.ravel()
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    chi2 = ((o - e) ** 2 / e).sum()
    assert scipy.stats.chi2.sf(chi2, len(e) - 1) > 1e-4, chi2
