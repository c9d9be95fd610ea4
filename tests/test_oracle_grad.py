"""Pins of the oracle's log Z_path gradient: central finite differences, the marginal sum rule
and the U=0 closed form of d log Z / d t."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import grad, hs


def small_chain(L=4, L_tau=16, U=4.0, dtau=0.1, kind=synth.HS_GAUSS, seed=0, n=None):
    d = synth.half_filled(L, L_tau, kind, U, dtau, seed)
    if n is not None:
        d = dataclasses.replace(d, n_up=n[0], n_dn=n[1])
    return d


def test_aux_gradient_matches_central_differences():
    d = small_chain(L=3, L_tau=8, n=(2, 3))
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 4)
    _, g, _, _ = grad.logz_path_grad(d, aux, paths, 2)
    rng = np.random.default_rng(1)
    h = 1e-4
    for _ in range(16):
        l, r = rng.integers(0, d.L_tau), rng.integers(0, d.N)
        ap, am = aux.copy(), aux.copy()
        ap[l, r] += h
        am[l, r] -= h
        fd = (grad.logz_path(d, ap, paths, 2)[0] - grad.logz_path(d, am, paths, 2)[0]) / (2 * h)
        assert g[l, r] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    v = rng.standard_normal(aux.shape)
    fd = (grad.logz_path(d, aux + h * v, paths, 2)[0] - grad.logz_path(d, aux - h * v, paths, 2)[0]) / (2 * h)
    assert float((g * v).sum()) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("kind", [synth.HS_GAUSS, synth.HS_HIRSCH])
def test_t_gradient_matches_central_differences(kind):
    d = small_chain(L=4, L_tau=12, kind=kind, seed=3)
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 9)
    _, _, gt, _ = grad.logz_path_grad(d, aux, paths, 5)
    h = 1e-4
    fd = (grad.logz_path(d, aux, paths, 5, t=d.t + h)[0]
          - grad.logz_path(d, aux, paths, 5, t=d.t - h)[0]) / (2 * h)
    assert gt == pytest.approx(fd, rel=1e-7)


def test_marginal_sum_rule():
    # sum_r dlogZ/dlogW_l(r) = 1 per worldline and slice => sum_r grad[l, r] = a * N_p
    d = small_chain(L=4, L_tau=10, seed=2)
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 2)
    _, g, _, _ = grad.logz_path_grad(d, aux, paths, 0)
    a = hs.gauss_coupling(d.U, d.dtau)
    assert np.allclose(g.sum(axis=1), a * d.n_particles, rtol=1e-13)
    assert np.all(g >= 0)


@pytest.mark.parametrize("L,L_tau,dtau", [(4, 16, 0.1), (6, 8, 0.2)])
def test_u0_t_gradient_closed_form(L, L_tau, dtau):
    d = small_chain(L=L, L_tau=L_tau, U=0.0, dtau=dtau)
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 1)
    _, _, gt, per = grad.logz_path_grad(d, aux, paths, 3)
    beta = L_tau * dtau
    m = np.arange(L)
    c = np.cos(2 * np.pi * m / L)
    ck = (c[:, None] + c[None, :]).ravel()
    w = np.exp(2 * beta * ck)
    ref = (2 * beta * ck * w).sum() / w.sum()
    assert np.allclose(per, ref, rtol=1e-12)
    if (L, L_tau) == (4, 16):
        assert ref == pytest.approx(5.898678748201, abs=1e-10)


def enumerate_logz(desc, aux, paths, anchor, perm):
    """log Z_p by summing every path of the block: from p's anchor site over L_tau slices to the
    anchor site of perm[p], weight prod W_l(r_l) G(r_{l+1} - r_l) (brute force, tiny systems)."""
    import itertools
    from oracle import lattice
    Gm = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)
    W_up, W_dn = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)
    out = np.zeros(desc.n_particles)
    for p in range(desc.n_particles):
        W = W_up if p < desc.n_up else W_dn
        a, e = paths[anchor, p], paths[anchor, perm[p]]
        z = 0.0
        for mid in itertools.product(range(desc.N), repeat=desc.L_tau - 1):
            r = (a,) + mid + (e,)
            wgt = 1.0
            for j in range(desc.L_tau):
                wgt *= W[(anchor + j) % desc.L_tau, r[j]] * Gm[r[j + 1], r[j]]
            z += wgt
        out[p] = np.log(z)
    return out


def test_reconnected_logz_matches_enumeration():
    d = synth.ChainDesc(L=2, L_tau=4, n_up=3, n_dn=2, hs_kind=synth.HS_GAUSS, block_len=0, t=1.0,
                        U=4.0, dtau=0.3, seed=5)
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 7)
    perm = np.array([2, 0, 1, 4, 3])
    for anchor in (0, 2):
        _, per = grad.logz_path(d, aux, paths, anchor, perm=perm)
        assert np.allclose(per, enumerate_logz(d, aux, paths, anchor, perm), rtol=1e-12)
    # the identity permutation is the plain closed ring
    assert np.allclose(grad.logz_path(d, aux, paths, 1, perm=np.arange(5))[1],
                       grad.logz_path(d, aux, paths, 1)[1], rtol=0, atol=0)


def test_reconnected_gradients_match_central_differences():
    d = small_chain(L=3, L_tau=8, n=(3, 2))
    aux = synth.initial_aux(d)
    paths = synth.random_paths(d, 6)
    perm = np.array([1, 2, 0, 4, 3])
    _, g, gt, _ = grad.logz_path_grad(d, aux, paths, 3, perm=perm)
    rng = np.random.default_rng(4)
    h = 1e-4
    for _ in range(12):
        l, r = rng.integers(0, d.L_tau), rng.integers(0, d.N)
        ap, am = aux.copy(), aux.copy()
        ap[l, r] += h
        am[l, r] -= h
        fd = (grad.logz_path(d, ap, paths, 3, perm=perm)[0]
              - grad.logz_path(d, am, paths, 3, perm=perm)[0]) / (2 * h)
        assert g[l, r] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    fd = (grad.logz_path(d, aux, paths, 3, t=d.t + h, perm=perm)[0]
          - grad.logz_path(d, aux, paths, 3, t=d.t - h, perm=perm)[0]) / (2 * h)
    assert gt == pytest.approx(fd, rel=1e-7)
    # the smoothing marginals still sum to one per worldline and slice
    a = hs.gauss_coupling(d.U, d.dtau)
    assert np.allclose(g.sum(axis=1), a * d.n_particles, rtol=1e-13)
