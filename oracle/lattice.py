"""Lattice geometry and the hopping kernel (test infrastructure, FP64, no FFT).

Sec. 3.3 ("Derivation of the Momentum-Space Transfer Kernel"): K is diagonal in momentum with
dispersion eps_k = -2t sum_alpha cos k_alpha, so one kinetic step multiplies mode k by
Ghat(k) = exp(-dtau eps_k) = exp(2 t dtau (cos k_x + cos k_y)) (the product D(k)^2 of the
half steps used in eq. ffbsFwd). In real space that is the convolution kernel
G(d) = (1/N) sum_k Ghat(k) e^{i k.d}, which factorises as g(d_x) g(d_y) with
g(d) = (1/L) sum_m exp(2 t dtau cos(2 pi m / L)) cos(2 pi m d / L)
     = sum_{n = d (mod L)} I_n(2 t dtau)      (modified Bessel functions; all terms > 0 for t > 0).

Site index i = x + L*y on the periodic L x L lattice; r (-) r' is the componentwise difference
modulo L. Everything here is a closed-form sum or a dense matrix; no FFT.
"""
from __future__ import annotations

import numpy as np
import scipy.special


def coords(L: int):
    """x and y coordinate arrays of the N = L*L sites, in site-index order i = x + L*y."""
    i = np.arange(L * L)
    return i % L, i // L


def ghat_1d(L: int, t: float, dtau: float) -> np.ndarray:
    """One-dimensional factor exp(2 t dtau cos(2 pi m / L)), m = 0..L-1, of Ghat(k)."""
    m = np.arange(L)
    return np.exp(2.0 * t * dtau * np.cos(2.0 * np.pi * m / L))


def ghat_2d(L: int, t: float, dtau: float) -> np.ndarray:
    """Ghat(k) = exp(-dtau eps_k) on the L x L momentum grid, flattened as m_x + L*m_y."""
    h = ghat_1d(L, t, dtau)
    return np.outer(h, h).reshape(-1)


def _bessel_orders(L: int):
    n_max = 3 * L + 40
    return np.arange(-n_max, n_max + 1)


def g_1d(L: int, t: float, dtau: float) -> np.ndarray:
    """g(d), d = 0..L-1, as the positive closed form sum_{n = d (mod L)} I_n(2 t dtau).

    From exp(x cos th) = sum_n I_n(x) e^{i n th}: the Fourier definition
    (1/L) sum_m exp(2 t dtau cos(2 pi m/L)) cos(2 pi m d/L) collects the modified Bessel
    functions I_n(2 t dtau) with n = d (mod L). Unlike the cosine sum (accurate only to the
    rounding of its largest term) this keeps every entry, however small, to relative precision.
    """
    n = _bessel_orders(L)
    In = scipy.special.iv(n, 2.0 * t * dtau)
    return np.array([In[(n - d) % L == 0].sum() for d in range(L)])


def g_1d_fourier(L: int, t: float, dtau: float) -> np.ndarray:
    """g(d) by the direct cosine sum (1/L) sum_m ghat(m) cos(2 pi m d / L) (used as a check)."""
    m = np.arange(L)
    d = np.arange(L)
    phase = 2.0 * np.pi * (np.outer(d, m) % L) / L
    return (np.cos(phase) * ghat_1d(L, t, dtau)[None, :]).sum(axis=1) / L


def dg_dt_1d(L: int, t: float, dtau: float) -> np.ndarray:
    """d g(d) / d t = 2 dtau sum_{n = d (mod L)} I_n'(2 t dtau)."""
    n = _bessel_orders(L)
    dIn = scipy.special.ivp(n, 2.0 * t * dtau)
    return 2.0 * dtau * np.array([dIn[(n - d) % L == 0].sum() for d in range(L)])


def kernel_2d(L: int, t: float, dtau: float) -> np.ndarray:
    """G(d) = g(d_x) g(d_y), flattened as d_x + L*d_y."""
    g = g_1d(L, t, dtau)
    return np.outer(g, g).reshape(-1)


def _circulant_from(table2d: np.ndarray, L: int) -> np.ndarray:
    x, y = coords(L)
    dx = (x[:, None] - x[None, :]) % L
    dy = (y[:, None] - y[None, :]) % L
    return table2d[dx + L * dy]


def transfer_matrix(L: int, t: float, dtau: float) -> np.ndarray:
    """Dense N x N matrix Gmat[i, j] = G(r_i (-) r_j): the kinetic step as a circulant.

    (G * f)(r) = sum_r' G(r (-) r') f(r') = (Gmat @ f)[r].
    """
    return _circulant_from(kernel_2d(L, t, dtau), L)


def transfer_matrix_dt(L: int, t: float, dtau: float) -> np.ndarray:
    """Dense d Gmat / d t, from d/dt [g(d_x) g(d_y)] = g'(d_x) g(d_y) + g(d_x) g'(d_y)."""
    g = g_1d(L, t, dtau)
    dg = dg_dt_1d(L, t, dtau)
    table = (np.outer(dg, g) + np.outer(g, dg)).reshape(-1)
    return _circulant_from(table, L)


def site_diff(L: int, r_to: np.ndarray, r_from: np.ndarray) -> np.ndarray:
    """Flattened index of r_to (-) r_from."""
    dx = (r_to % L - r_from % L) % L
    dy = (r_to // L - r_from // L) % L
    return dx + L * dy
