"""Pins of the oracle's local link updates (Sec. 3.5.1, eq. Rlocal): the update must leave the
exact path law invariant and reach it from any start. The law is obtained by enumerating every
closed path of one worldline on a tiny lattice, independently of the update's own formula."""
import itertools

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import hs, lattice, local


def exact_ring_law(desc, aux, spin=0):
    """All closed paths (r_0, ..., r_{L_tau-1}) of one worldline and their probabilities under
    prod_l W_l(r_l) G(r_{l+1} - r_l) (eq. joint, one worldline, the ring closing on itself)."""
    N = desc.L * desc.L
    Gm = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)
    W = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)[spin]
    paths = np.array(list(itertools.product(range(N), repeat=desc.L_tau)), dtype=np.int64)
    w = np.ones(len(paths))
    for l in range(desc.L_tau):
        w *= W[l, paths[:, l]] * Gm[paths[:, (l + 1) % desc.L_tau], paths[:, l]]
    return paths, w / w.sum()


def code_of(paths, N):
    c = np.zeros(paths.shape[0], dtype=np.int64)
    for l in range(paths.shape[1]):
        c = c * N + paths[:, l]
    return c


def chi2_p(counts, prob):
    M = counts.sum()
    ex = prob * M
    keep = ex >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exv = np.append(ex[keep], ex[~keep].sum())
    chi2 = ((obs - exv) ** 2 / exv).sum()
    return scipy.stats.chi2.sf(chi2, len(exv) - 1)


CASES = [(2, 3, synth.HS_GAUSS, 0.5), (3, 2, synth.HS_HIRSCH, 0.4), (2, 4, synth.HS_HIRSCH, 0.3)]


@pytest.mark.parametrize("L,L_tau,kind,dtau", CASES)
def test_local_update_preserves_the_exact_path_law(L, L_tau, kind, dtau):
    """Worldlines drawn exactly from the path law stay distributed by it after one pass and
    after three passes (every worldline an independent chain on the same field)."""
    M = 40000
    desc = synth.ChainDesc(L=L, L_tau=L_tau, n_up=M, n_dn=0, hs_kind=kind, block_len=0,
                           t=1.0, U=4.0, dtau=dtau, seed=11)
    aux = synth.initial_aux(desc, rng_seed=3)
    paths, prob = exact_ring_law(desc, aux)
    pick = np.random.default_rng(5).choice(len(paths), size=M, p=prob)
    start = paths[pick].T.copy()                       # [L_tau, M]
    N = L * L
    for n_passes in (1, 3):
        out = local.local_update(desc, aux, start, sweep=4, n_passes=n_passes)
        counts = np.bincount(code_of(out.T, N), minlength=N ** L_tau)
        assert chi2_p(counts, prob) > 1e-4, n_passes


@pytest.mark.parametrize("L,L_tau,kind,dtau", CASES[:2])
def test_local_update_reaches_the_path_law_from_a_fixed_start(L, L_tau, kind, dtau):
    """From every worldline parked on site 0, repeated passes converge to the exact law."""
    M = 40000
    desc = synth.ChainDesc(L=L, L_tau=L_tau, n_up=M, n_dn=0, hs_kind=kind, block_len=0,
                           t=1.0, U=4.0, dtau=dtau, seed=12)
    aux = synth.initial_aux(desc, rng_seed=4)
    paths, prob = exact_ring_law(desc, aux)
    start = np.zeros((L_tau, M), dtype=np.int64)
    out = local.local_update(desc, aux, start, sweep=0, n_passes=60)
    counts = np.bincount(code_of(out.T, L * L), minlength=(L * L) ** L_tau)
    assert chi2_p(counts, prob) > 1e-4


def test_local_update_down_spin_uses_its_own_potential():
    """Ising field: a down worldline weighs W_dn = e^{-lambda s}; its stationary law is the
    down-spin ring law, which differs from the up-spin one."""
    M = 40000
    desc = synth.ChainDesc(L=2, L_tau=3, n_up=0, n_dn=M, hs_kind=synth.HS_HIRSCH, block_len=0,
                           t=1.0, U=6.0, dtau=0.5, seed=13)
    aux = synth.initial_aux(desc, rng_seed=6)
    paths, prob_dn = exact_ring_law(desc, aux, spin=1)
    _, prob_up = exact_ring_law(desc, aux, spin=0)
    assert np.abs(prob_dn - prob_up).max() > 0.02
    pick = np.random.default_rng(8).choice(len(paths), size=M, p=prob_dn)
    out = local.local_update(desc, aux, paths[pick].T.copy(), sweep=2, n_passes=2)
    counts = np.bincount(code_of(out.T, 4), minlength=4 ** 3)
    assert chi2_p(counts, prob_dn) > 1e-4


def test_proposal_is_a_nearest_neighbour_step():
    L = 5
    r = np.arange(L * L)
    for e, (dx, dy) in enumerate(((1, 0), (-1, 0), (0, 1), (0, -1))):
        nb = local.neighbour(r, np.full_like(r, e), L)
        assert np.array_equal(nb % L, (r % L + dx) % L)
        assert np.array_equal(nb // L, (r // L + dy) % L)
