"""Hubbard-Stratonovich fields: couplings, site potentials W and field priors (test infrastructure).

Hirsch (Ising) field, eq. hirsch (Sec. 3.2 and Sec. 3.5.4): cosh(lambda) = exp(dtau U / 2) and
the slice weight exp(lambda s (n_up - n_dn)); a spin-up worldline at site r on slice l picks up
W_up = exp(+lambda s_rl), a spin-down one W_dn = exp(-lambda s_rl). Field prior: 1/2 per value.

Gaussian field, eq. gaussHS (Sec. 3.5.5): coupling a = sqrt(|U| dtau) and the factor
exp(-sigma^2/2 + a sigma (n_up + n_dn - 1/2)); every worldline at (r, l) picks up
W = exp(a sigma_rl) whatever its spin, and the field carries the prior exp(-sigma^2/2 - a sigma/2).
The paper states this identity for U < 0; it is applied here literally with |U| (the reading
for the repulsive Gaussian configurations).
"""
from __future__ import annotations

import numpy as np

HS_GAUSS = 0
HS_HIRSCH = 1


def hirsch_lambda(U: float, dtau: float) -> float:
    """lambda = arccosh(exp(dtau U / 2))  (Appendix B.4.2)."""
    return float(np.arccosh(np.exp(dtau * U / 2.0)))


def gauss_coupling(U: float, dtau: float) -> float:
    """a = sqrt(|U| dtau)  (eq. gaussHS)."""
    return float(np.sqrt(abs(U) * dtau))


def log_weight_coeffs(hs_kind: int, U: float, dtau: float):
    """(c_up, c_dn) with log W_spin(r, l) = c_spin * aux(r, l)."""
    if hs_kind == HS_GAUSS:
        a = gauss_coupling(U, dtau)
        return a, a
    lam = hirsch_lambda(U, dtau)
    return lam, -lam


def potentials(aux: np.ndarray, hs_kind: int, U: float, dtau: float):
    """Site potentials (W_up, W_dn), each [L_tau, N]: W = exp(c_spin * aux)."""
    c_up, c_dn = log_weight_coeffs(hs_kind, U, dtau)
    return np.exp(c_up * aux), np.exp(c_dn * aux)
