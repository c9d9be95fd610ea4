"""Gradient-informed proposals for the Gaussian field (test infrastructure, FP64).

The field's law given the worldlines' sites at one anchor slice l0, with the worldlines' paths
summed out, is
    pi(sigma) ∝ prod_{r,l} exp(-sigma_rl^2 / 2 - a sigma_rl / 2) * Z_path(sigma),
the Gaussian HS prior of eq. gaussHS times Z_path = prod_p Z_p, the weight of all closed paths of
each worldline through its anchor site (log Z_path and its gradient as in `grad`). A
Metropolis-adjusted Langevin step (Roberts and Tweedie, 1996) targets it:
    g(sigma)  = d log pi / d sigma = -sigma - a/2 + d log Z_path / d sigma,
    sigma'    = sigma + h g(sigma) + eps xi,   h = eps^2 / 2,  xi_rl ~ N(0, 1),
    log alpha = log pi(sigma') - log pi(sigma)
                - |sigma - sigma' - h g(sigma')|^2 / (2 eps^2) + |sigma' - sigma - h g(sigma)|^2 / (2 eps^2),
and the whole field of the chain moves to sigma' iff u < exp(log alpha).
Random numbers: xi_rl from the Philox counter (site r, slice l, sweep, TAG_MALA) by Box-Muller,
u from counter (0, 0, sweep, TAG_MALA_ACCEPT), key (seed, 0). Only Gaussian-field chains have
this law; the Ising field keeps its Gibbs draw.
"""
from __future__ import annotations

import numpy as np

from . import grad, hs, philox

TAG_MALA = 3
TAG_MALA_ACCEPT = 4


def log_prior(desc, sigma: np.ndarray) -> float:
    a = hs.gauss_coupling(desc.U, desc.dtau)
    return float(np.sum(-0.5 * sigma * sigma - 0.5 * a * sigma))


def log_target(desc, sigma, paths, anchor, perm=None):
    """(log pi up to a constant, d log pi / d sigma); perm: reconnection (None = identity)."""
    a = hs.gauss_coupling(desc.U, desc.dtau)
    lz, g, _, _ = grad.logz_path_grad(desc, sigma, paths, anchor, perm=perm)
    return log_prior(desc, sigma) + lz, -sigma - 0.5 * a + g


def mala_step(desc, sigma: np.ndarray, paths: np.ndarray, anchor: int, eps: float, sweep: int,
              perm=None):
    """One MALA step of the chain's field. Returns (new field, accepted, log alpha). With a
    reconnection perm, Z_path is the weight of the paths joining each anchor site to that of the
    reconnected worldline (see `grad`)."""
    if desc.hs_kind != hs.HS_GAUSS:
        raise ValueError("MALA moves the Gaussian field only")
    L_tau, N = sigma.shape
    h = 0.5 * eps * eps
    lp0, g0 = log_target(desc, sigma, paths, anchor, perm)
    sites = np.arange(N, dtype=np.uint64)[None, :]
    slices = np.arange(L_tau, dtype=np.uint64)[:, None]
    x0, x1, _, _ = philox.draw_words(desc.seed, sites, slices, sweep, TAG_MALA)
    xi = philox.gaussian(x0, x1)
    prop = sigma + h * g0 + eps * xi
    lp1, g1 = log_target(desc, prop, paths, anchor, perm)
    fwd = np.sum((prop - sigma - h * g0) ** 2) / (2.0 * eps * eps)
    rev = np.sum((sigma - prop - h * g1) ** 2) / (2.0 * eps * eps)
    log_alpha = lp1 - lp0 - rev + fwd
    w0, _, _, _ = philox.draw_words(desc.seed, np.uint64(0), np.uint64(0), sweep, TAG_MALA_ACCEPT)
    u = float(philox.uniform(np.asarray(w0)))
    accepted = u < np.exp(min(log_alpha, 0.0))
    return (prop if accepted else sigma.copy()), bool(accepted), float(log_alpha)
