"""Local link updates of the worldlines (test infrastructure, FP64).

Sec. 3.5.1, eq. Rlocal: one worldline's position on one slice is changed while its positions on
the two adjacent slices stay fixed, and the change is accepted by Metropolis with the ratio of
the path weights. In the site basis taken for the whole sampler a worldline sitting at r_l on
slice l carries the potential W_l(r_l) and the two hops G(r_l - r_{l-1}) and G(r_{l+1} - r_l),
so moving r_l to r' is accepted with probability min(1, R),

    R = W_l(r') G(r' - r_{l-1}) G(r_{l+1} - r') / [ W_l(r_l) G(r_l - r_{l-1}) G(r_{l+1} - r_l) ].

Readings where the paper is silent:
  * proposal: r' = r_l + e with e one of the four lattice vectors (+x, -x, +y, -y), equally
    likely, periodic. The proposal is symmetric, so min(1, R) is the Metropolis acceptance;
  * order: a checkerboard in tau. One pass visits, for every worldline, first the odd interior
    slices l = 1, 3, ... <= L_tau-2, then the even interior slices l = 2, 4, ... <= L_tau-2, then
    slice 0, then slice L_tau-1. A move on slice l sees only slices l-1 and l+1, which belong to
    other phases, so the moves of one phase are independent of each other and the order inside
    a phase does not matter. The two end slices neighbour other worldlines when the worldlines
    reconnect at tau = beta (permutation perm: slice L_tau of p is slice 0 of perm[p]); they
    have phases of their own for the same reason. Without a permutation each worldline closes
    on itself;
  * random numbers: Philox counter (particle, slice, sweep, TAG_LOCAL + 256 * pass), key
    (seed, 0); the top two bits of word x1 select e (0: +x, 1: -x, 2: +y, 3: -y), word x0 gives
    the uniform u, and the move is taken iff u < R.
"""
from __future__ import annotations

import numpy as np

from . import hs, lattice, philox

TAG_LOCAL = 2


def neighbour(r: np.ndarray, e: np.ndarray, L: int) -> np.ndarray:
    """Site r + e on the periodic L x L lattice, site index x + L y; e in {0: +x, 1: -x, 2: +y,
    3: -y}."""
    x, y = r % L, r // L
    dx = np.where(e == 0, 1, np.where(e == 1, -1, 0))
    dy = np.where(e == 2, 1, np.where(e == 3, -1, 0))
    return (x + dx) % L + L * ((y + dy) % L)


def local_update(desc, aux: np.ndarray, paths: np.ndarray, sweep: int, n_passes: int,
                 return_margin: bool = False, perm: np.ndarray | None = None):
    """n_passes passes of local link updates over every worldline.

    aux [L_tau, N] field, paths [L_tau, n_particles] (up particles first), perm [n_particles]
    the reconnection at tau = beta (None: the identity). Returns the new paths and, if asked,
    the decision margins |u - R| of every proposal [n_passes, L_tau, particles] (a proposal
    whose margin is at round-off level is a near-tie).
    """
    L, L_tau, N = desc.L, desc.L_tau, desc.L * desc.L
    Gm = lattice.transfer_matrix(L, desc.t, desc.dtau)       # Gm[r', r] = G(r' - r)
    W_up, W_dn = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)
    W = np.stack([W_up, W_dn])                                # [spin, L_tau, N]
    P = desc.n_up + desc.n_dn
    parts = np.arange(P)
    spin = (parts >= desc.n_up).astype(np.int64)
    nxt = parts if perm is None else np.asarray(perm, dtype=np.int64)
    prv = np.empty(P, dtype=np.int64)
    prv[nxt] = parts                                          # slice -1 of p is slice L_tau-1 of prv[p]
    out = np.asarray(paths, dtype=np.int64).copy()
    margins = np.full((n_passes, L_tau, P), np.inf)

    def visit(l, ps, r_prev, r_next):
        x0, x1, _, _ = philox.draw_words(desc.seed, parts.astype(np.uint64), l, sweep,
                                         TAG_LOCAL + 256 * ps)
        e = (x1 >> np.uint64(62)).astype(np.int64)
        u = philox.uniform(x0)
        r = out[l].copy()
        r_new = neighbour(r, e, L)
        num = W[spin, l, r_new] * Gm[r_new, r_prev] * Gm[r_next, r_new]
        den = W[spin, l, r] * Gm[r, r_prev] * Gm[r_next, r]
        R = num / den
        margins[ps, l] = np.abs(u - R)
        out[l] = np.where(u < R, r_new, r)

    for ps in range(n_passes):
        for first in (1, 2):                       # odd, then even interior slices
            for l in range(first, L_tau - 1, 2):
                visit(l, ps, out[l - 1], out[l + 1])
        visit(0, ps, out[L_tau - 1, prv], out[1])
        visit(L_tau - 1, ps, out[L_tau - 2], out[0, nxt])
    if return_margin:
        return out, margins
    return out
