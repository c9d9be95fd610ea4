"""Pins of the oracle's MALA field step. With one worldline the field's law given its anchor site
is exactly a finite Gaussian mixture: pick a closed path w through the anchor with probability
proportional to prod_l G(w_{l+1} - w_l), then sigma_rl ~ N(a (1[w_l = r] - 1/2), 1) independently
(the prior exp(-sigma^2/2 - a sigma/2) times exp(a sigma) at visited points). That law is
sampled exactly, independently of the MALA formula, and must stay invariant."""
import itertools

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import hs, lattice, mala


def exact_mixture(desc, anchor_site):
    N = desc.L * desc.L
    Gm = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)
    free = np.array(list(itertools.product(range(N), repeat=desc.L_tau - 1)), dtype=np.int64)
    paths = np.concatenate([np.full((len(free), 1), anchor_site), free], axis=1)
    w = np.ones(len(paths))
    for l in range(desc.L_tau):
        w *= Gm[paths[:, (l + 1) % desc.L_tau], paths[:, l]]
    return paths, w / w.sum()


def draw_exact(desc, paths, prob, rng, M):
    a = hs.gauss_coupling(desc.U, desc.dtau)
    N = desc.L * desc.L
    pick = rng.choice(len(paths), size=M, p=prob)
    mean = np.full((M, desc.L_tau, N), -0.5 * a)
    for l in range(desc.L_tau):
        mean[np.arange(M), l, paths[pick, l]] += a
    return mean + rng.standard_normal(mean.shape)


def mixture_cdf(desc, paths, prob, l, r, x):
    a = hs.gauss_coupling(desc.U, desc.dtau)
    visited = (paths[:, l] == r).astype(np.float64)
    mu = a * (visited - 0.5)
    return (prob[None, :] * scipy.stats.norm.cdf(x[:, None] - mu[None, :])).sum(axis=1)


DESC = synth.ChainDesc(L=2, L_tau=3, n_up=1, n_dn=0, hs_kind=synth.HS_GAUSS, block_len=0,
                       t=1.0, U=6.0, dtau=0.5, seed=19)


def run_chains(step_fn, M=1500, K=6, eps=0.8):
    desc = DESC
    anchor_site = 1
    paths, prob = exact_mixture(desc, anchor_site)
    rng = np.random.default_rng(23)
    fields = draw_exact(desc, paths, prob, rng, M)
    wl = np.full((desc.L_tau, 1), anchor_site, dtype=np.int64)
    acc = 0
    for i in range(M):
        s = fields[i]
        for k in range(K):
            s, ok, _ = step_fn(desc, s, wl, 0, eps, 1000 * i + k)
            acc += ok
        fields[i] = s
    return desc, paths, prob, fields, acc / (M * K)


def check_law(desc, paths, prob, fields):
    """KS of every coordinate against its exact mixture marginal, and the joint check that
    the anchor point carries mean a/2."""
    a = hs.gauss_coupling(desc.U, desc.dtau)
    worst = 1.0
    for l in range(desc.L_tau):
        for r in range(desc.L * desc.L):
            x = fields[:, l, r]
            p = scipy.stats.kstest(x, lambda v: mixture_cdf(desc, paths, prob, l, r, np.atleast_1d(v))).pvalue
            worst = min(worst, p)
    # Bonferroni over the 12 coordinates
    assert worst > 1e-4 / 12, worst
    anchor_mean = fields[:, 0, 1].mean()
    assert abs(anchor_mean - 0.5 * a) < 5.0 / np.sqrt(len(fields)), anchor_mean


def test_mala_preserves_the_exact_field_law():
    desc, paths, prob, fields, rate = run_chains(mala.mala_step)
    assert 0.2 < rate < 0.999, rate
    check_law(desc, paths, prob, fields)


def test_exact_mixture_sampler_matches_its_own_marginals():
    """The reference sampler itself: its draws pass the same KS checks (no MALA step)."""
    desc = DESC
    paths, prob = exact_mixture(desc, 1)
    fields = draw_exact(desc, paths, prob, np.random.default_rng(29), 1500)
    check_law(desc, paths, prob, fields)


def test_mala_rejects_the_ising_field():
    d = synth.ChainDesc(L=2, L_tau=3, n_up=1, n_dn=0, hs_kind=synth.HS_HIRSCH, block_len=0,
                        t=1.0, U=4.0, dtau=0.5, seed=3)
    with pytest.raises(ValueError):
        mala.mala_step(d, np.ones((3, 4)), np.zeros((3, 1), dtype=np.int64), 0, 0.5, 0)
