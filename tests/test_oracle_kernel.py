"""Pins of the oracle's hopping kernel (Sec. 3.3, eq. Tkk) against independent mathematics."""
import numpy as np
import pytest
import scipy.linalg
import scipy.special

from oracle import lattice

CASES = [(2, 1.0, 0.1), (3, 1.0, 0.1), (4, 1.0, 0.1), (6, 0.7, 0.3), (12, 1.0, 0.05),
         (16, 1.0, 0.0625), (32, 1.0, 0.05)]


def adjacency(L):
    """Nearest-neighbour adjacency of the periodic L x L lattice, every bond counted (so L=2
    doubles the periodic bond, the lattice on which eps_k = -2t(cos kx + cos ky) lives)."""
    N = L * L
    A = np.zeros((N, N))
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                A[((x + dx) % L) + L * ((y + dy) % L), i] += 1.0
    return A


@pytest.mark.parametrize("L,t,dtau", CASES)
def test_g_equals_fourier_definition(L, t, dtau):
    # the Fourier definition (1/L) sum_m ghat(m) cos(2 pi m d/L), accurate to rounding of its
    # largest term
    g = lattice.g_1d(L, t, dtau)
    ref = lattice.g_1d_fourier(L, t, dtau)
    assert np.max(np.abs(g - ref)) <= 2.2e-16 * L * ref.max()
    assert np.allclose(g[:3], ref[:3], rtol=1e-14)


def test_g_reference_values_L32():
    # I_d(0.1) for d = 0..4 (dtau = 0.05, t = 1): 1.002502, 5.006253e-2, 1.251042e-3, ...
    g = lattice.g_1d(32, 1.0, 0.05)
    ref = [1.0025015629340956, 5.0062526047092694e-2, 1.2510419921651e-3, 2.0846357422e-5,
           2.605469e-7]
    assert np.allclose(g[:5], ref, rtol=1e-6)


@pytest.mark.parametrize("L,t,dtau", CASES)
def test_transfer_matrix_is_expm_of_hopping(L, t, dtau):
    # exp(-dtau K) with K = -t A, the kinetic term of eq. hubbard
    ref = scipy.linalg.expm(t * dtau * adjacency(L))
    G = lattice.transfer_matrix(L, t, dtau)
    assert np.max(np.abs(G - ref)) < 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("L,t,dtau", CASES)
def test_normalisation_symmetry_positivity(L, t, dtau):
    G = lattice.kernel_2d(L, t, dtau)
    assert G.sum() == pytest.approx(np.exp(4 * t * dtau), rel=4e-16)
    x = np.arange(L)
    g = lattice.g_1d(L, t, dtau)
    assert np.allclose(g, g[(-x) % L], rtol=1e-15)
    assert np.all(g > 0)


@pytest.mark.parametrize("L", [3, 4, 8])
def test_semigroup(L):
    G1 = lattice.transfer_matrix(L, 1.0, 0.1)
    G2 = lattice.transfer_matrix(L, 1.0, 0.2)
    assert np.allclose(G1 @ G1, G2, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("L,t,dtau", [(3, 1.0, 0.1), (4, 0.8, 0.1), (8, 1.0, 0.05)])
def test_dt_derivative(L, t, dtau):
    # d/dt expm(t dtau A) = dtau A expm(t dtau A)
    A = adjacency(L)
    ref = dtau * A @ scipy.linalg.expm(t * dtau * A)
    dG = lattice.transfer_matrix_dt(L, t, dtau)
    assert np.max(np.abs(dG - ref)) < 1e-13 * np.max(np.abs(ref))


def test_ghat_is_fourier_transform_of_kernel():
    L = 6
    G = lattice.kernel_2d(L, 1.0, 0.2).reshape(L, L)
    Gh = np.fft.fft2(G).real.reshape(-1)
    assert np.allclose(Gh, lattice.ghat_2d(L, 1.0, 0.2), rtol=1e-14)
