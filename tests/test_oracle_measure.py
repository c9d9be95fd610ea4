"""Pins of the oracle's equal-time observables (Sec. 4: C(r), S(k), D, local moment): closed
forms on configurations whose answers are known, and the identities that tie S(k) to C(r)."""
import numpy as np
import pytest

from oracle import measure


def neel_paths(L, L_tau):
    """Up worldlines on (x+y)-even sites, down on odd ones, static in tau."""
    sites = np.arange(L * L)
    even = sites[(sites % L + sites // L) % 2 == 0]
    odd = sites[(sites % L + sites // L) % 2 == 1]
    return np.tile(np.concatenate([even, odd]), (L_tau, 1)), len(even)


@pytest.mark.parametrize("L", [2, 4, 6])
def test_neel_state_closed_forms(L):
    """S^z = +-1/2 staggered: S(Q) = N/4 at Q = (pi, pi) and 0 elsewhere, C(r) = (-1)^{x+y}/4,
    no double occupancy, local moment 3/4."""
    N = L * L
    paths, n_up = neel_paths(L, 5)
    Sk, Cr, D, S2 = measure.observables(L, n_up, paths)
    Q = (L // 2) + L * (L // 2)
    ref = np.zeros(N)
    ref[Q] = N / 4.0
    assert np.allclose(Sk, ref, atol=1e-12)
    r = np.arange(N)
    assert np.allclose(Cr, 0.25 * (-1.0) ** (r % L + r // L), atol=1e-15)
    assert D == 0.0 and S2 == pytest.approx(0.75)


def test_ferromagnet_and_doubly_occupied_closed_forms():
    """All up worldlines stacked on one site: S^z = n/2 there, so S(k) = n^2/(4N) for every k and
    C(r) = n^2/(4N) delta_{r,0}; with n up and n down worldlines on one site, S^z = 0 and
    D = n^2 / N."""
    L, n, L_tau = 4, 3, 4
    N = L * L
    paths = np.full((L_tau, n), 5)
    Sk, Cr, D, S2 = measure.observables(L, n, paths)
    assert np.allclose(Sk, n * n / (4.0 * N))
    ref = np.zeros(N)
    ref[0] = n * n / (4.0 * N)
    assert np.allclose(Cr, ref)
    assert D == 0.0 and S2 == pytest.approx(0.75 * n * n / N)
    paths = np.full((L_tau, 2 * n), 7)
    Sk, Cr, D, S2 = measure.observables(L, n, paths)
    assert np.allclose(Sk, 0.0) and np.allclose(Cr, 0.0)
    assert D == pytest.approx(n * n / N) and S2 == 0.0


@pytest.mark.parametrize("L,n_up,n_dn", [(3, 4, 5), (4, 8, 8), (6, 10, 7)])
def test_structure_factor_is_the_transform_of_the_correlation(L, n_up, n_dn):
    """Random configurations: S(k) = sum_r e^{i k.r} C(r) and (1/N) sum_k S(k) = C(0) =
    <(S^z)^2>, which ties the two independently written sums together."""
    N = L * L
    rng = np.random.default_rng(L + n_up)
    paths = rng.integers(0, N, size=(6, n_up + n_dn))
    Sk, Cr, D, S2 = measure.observables(L, n_up, paths)
    r = np.arange(N)
    kx, ky = r % L, r // L
    ph = 2.0 * np.pi * (np.outer(kx, r % L) + np.outer(ky, r // L)) / L
    assert np.allclose((np.exp(1j * ph) @ Cr).real, Sk, atol=1e-12)
    assert np.mean(Sk) == pytest.approx(Cr[0], abs=1e-14)
    assert S2 == pytest.approx(3.0 * Cr[0], rel=1e-14)
    assert np.all(Sk >= -1e-15)
