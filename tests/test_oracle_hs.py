"""Pins of the field couplings and Gibbs conditionals (eq. hirsch, eq. gaussHS, eq. gaussCond)."""
import itertools

import numpy as np
import pytest
import scipy.integrate

from oracle import gibbs, hs, philox


@pytest.mark.parametrize("U,dtau", [(4.0, 0.0625), (4.0, 0.1), (2.0, 0.05), (6.0, 0.05), (0.0, 0.1)])
def test_hirsch_identity(U, dtau):
    lam = hs.hirsch_lambda(U, dtau)
    assert np.cosh(lam) == pytest.approx(np.exp(dtau * U / 2), rel=1e-15)
    ratios = []
    for nu, nd in itertools.product((0, 1), repeat=2):
        lhs = np.exp(-dtau * U * (nu - 0.5) * (nd - 0.5))
        rhs = 0.5 * sum(np.exp(lam * s * (nu - nd)) for s in (1, -1))
        ratios.append(rhs / lhs)
    # the decoupling holds up to an (n-independent) constant
    assert np.allclose(ratios, ratios[0], rtol=1e-14)


@pytest.mark.parametrize("U,dtau", [(4.0, 0.1), (4.0, 0.05), (1.0, 0.3)])
def test_gaussian_identity(U, dtau):
    a = hs.gauss_coupling(U, dtau)
    assert a * a == pytest.approx(abs(U) * dtau, rel=1e-15)
    ratios = []
    for nu, nd in itertools.product((0, 1), repeat=2):
        n = nu + nd
        val, _ = scipy.integrate.quad(
            lambda s: np.exp(-0.5 * s * s + a * s * (n - 0.5)) / np.sqrt(2 * np.pi), -40, 40,
            epsabs=0, epsrel=1e-13)
        ratios.append(val / np.exp(abs(U) * dtau * nu * nd))
    assert np.allclose(ratios, ratios[0], rtol=1e-11)
    # the constant is exp(+|U| dtau / 8) on the integral side
    assert ratios[0] == pytest.approx(np.exp(a * a / 8), rel=1e-11)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_gaussian_conditional_moments_from_joint(n):
    # conditional of sigma given n: prior exp(-s^2/2 - a s/2) times W^n = exp(a s n)
    a = hs.gauss_coupling(4.0, 0.1)
    dens = lambda s: np.exp(-0.5 * s * s - 0.5 * a * s + a * s * n)
    Z, _ = scipy.integrate.quad(dens, -40, 40, epsrel=1e-13)
    m1, _ = scipy.integrate.quad(lambda s: s * dens(s), -40, 40, epsrel=1e-13)
    m2, _ = scipy.integrate.quad(lambda s: s * s * dens(s), -40, 40, epsrel=1e-13)
    mean = m1 / Z
    assert mean == pytest.approx(a * (n - 0.5), abs=1e-12)
    assert m2 / Z - mean ** 2 == pytest.approx(1.0, abs=1e-11)


@pytest.mark.parametrize("m", [-3, -1, 0, 1, 2])
def test_hirsch_conditional_from_joint(m):
    lam = hs.hirsch_lambda(4.0, 0.1)
    # P(s) ∝ prior(1/2) * W_up^{n_up} W_dn^{n_dn} = exp(lam s (n_up - n_dn))
    w = {s: 0.5 * np.exp(lam * s * m) for s in (1, -1)}
    assert gibbs.hirsch_p_plus(lam, np.float64(m)) == pytest.approx(w[1] / (w[1] + w[-1]), rel=1e-14)


def test_gibbs_draws_follow_conditionals():
    L_tau, N = 64, 256
    rng = np.random.default_rng(5)
    cu = rng.integers(0, 3, size=(L_tau, N))
    cd = rng.integers(0, 3, size=(L_tau, N))
    lam = hs.hirsch_lambda(4.0, 0.0625)
    tot = {}
    for s in range(20):
        f = gibbs.gibbs_field(hs.HS_HIRSCH, 4.0, 0.0625, cu, cd, 11, s)
        for m in np.unique(cu - cd):
            sel = (cu - cd) == m
            k, n = tot.get(m, (0, 0))
            tot[m] = (k + int((f[sel] > 0).sum()), n + int(sel.sum()))
    for m, (k, n) in tot.items():
        p = float(gibbs.hirsch_p_plus(lam, np.float64(m)))
        z = (k - n * p) / np.sqrt(n * p * (1 - p))
        assert abs(z) < 4.5, (m, k, n, p)
    a = hs.gauss_coupling(4.0, 0.1)
    f = np.stack([gibbs.gibbs_field(hs.HS_GAUSS, 4.0, 0.1, cu, cd, 3, s) for s in range(8)])
    z = f - a * ((cu + cd) - 0.5)[None]
    assert abs(z.mean()) < 4.5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.5 * np.sqrt(2.0 / z.size)


def test_gibbs_uses_distinct_counters():
    cu = np.zeros((4, 9), dtype=np.int64)
    f0 = gibbs.gibbs_field(hs.HS_GAUSS, 4.0, 0.1, cu, cu, 1, 0)
    f1 = gibbs.gibbs_field(hs.HS_GAUSS, 4.0, 0.1, cu, cu, 1, 1)
    f2 = gibbs.gibbs_field(hs.HS_GAUSS, 4.0, 0.1, cu, cu, 2, 0)
    assert len(np.unique(np.concatenate([f0.ravel(), f1.ravel(), f2.ravel()]))) == 3 * 36
    x0, x1, _, _ = philox.draw_words(1, 0, 0, 0, philox.TAG_GIBBS)
    assert f0[0, 0] == pytest.approx(-0.5 * hs.gauss_coupling(4.0, 0.1) + philox.gaussian(x0, x1))
