"""Permutation updates: reconnecting worldlines at tau = beta (test infrastructure, FP64).

Eq. joint sums over the permutations P_up, P_dn that reconnect the worldlines of each spin at
the time boundary, with the factor sgn(P_up) sgn(P_dn); Sec. 3.5.6 proposes pair swaps of the
reconnections. With slice L_tau of worldline p identified with slice 0 of worldline P(p), a
configuration weighs
    |pi| = prod_p prod_{l < L_tau} W_l(r^p_l) G(r^p_{l+1} - r^p_l),   r^p_{L_tau} = r^{P(p)}_0,
and the sign sgn(P) is carried alongside (observables are reweighted by it). Swapping the
reconnections of two same-spin worldlines p, q (P(p) <-> P(q)) changes only their two boundary
hops, so the Metropolis ratio on |pi| is
    R = G(r^{P(q)}_0 - r^p_{L-1}) G(r^{P(p)}_0 - r^q_{L-1}) / [G(r^{P(p)}_0 - r^p_{L-1}) G(r^{P(q)}_0 - r^q_{L-1})]
(L = L_tau), and every accepted swap flips sgn(P).

Readings where the paper is silent:
  * proposals: pass k pairs the worldlines of each spin as (p0 + o + 2i, p0 + o + 2i + 1),
    o = k mod 2, p0 the spin's first worldline; the pairs of a pass are disjoint, so their moves
    are independent, and adjacent transpositions generate every permutation;
  * random numbers: Philox counter (p, 0, sweep, TAG_PERM + 256 * pass) for the pair whose
    first worldline is p, key (seed, 0); the swap is taken iff u < R (u from word x0).
"""
from __future__ import annotations

import numpy as np

from . import lattice, philox

TAG_PERM = 5


def permutation_sign(perm: np.ndarray) -> int:
    """sgn of a permutation from its cycle decomposition: (-1)^(n - number of cycles)."""
    perm = np.asarray(perm, dtype=np.int64)
    seen = np.zeros(len(perm), dtype=bool)
    cycles = 0
    for i in range(len(perm)):
        if not seen[i]:
            cycles += 1
            j = i
            while not seen[j]:
                seen[j] = True
                j = perm[j]
    return 1 if (len(perm) - cycles) % 2 == 0 else -1


def perm_update(desc, paths: np.ndarray, perm: np.ndarray, sweep: int, n_passes: int,
                return_margin: bool = False):
    """n_passes passes of pair swaps. Returns (new perm, number of accepted swaps) and, if asked,
    the margins |u - R| of every proposal as a list per pass."""
    Gm = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)   # Gm[r', r] = G(r' - r)
    L_tau = desc.L_tau
    perm = np.asarray(perm, dtype=np.int64).copy()
    flips = 0
    margins = []
    for ps in range(n_passes):
        o = ps % 2
        m_pass = []
        for p0, n in ((0, desc.n_up), (desc.n_up, desc.n_dn)):
            p = np.arange(p0 + o, p0 + n - 1, 2, dtype=np.int64)
            if len(p) == 0:
                continue
            q = p + 1
            last_p = paths[L_tau - 1, p].astype(np.int64)
            last_q = paths[L_tau - 1, q].astype(np.int64)
            first_pp = paths[0, perm[p]].astype(np.int64)
            first_pq = paths[0, perm[q]].astype(np.int64)
            R = (Gm[first_pq, last_p] * Gm[first_pp, last_q]) / \
                (Gm[first_pp, last_p] * Gm[first_pq, last_q])
            x0, _, _, _ = philox.draw_words(desc.seed, p.astype(np.uint64), 0, sweep,
                                            TAG_PERM + 256 * ps)
            u = philox.uniform(x0)
            take = u < R
            m_pass.append(np.abs(u - R))
            a, b = perm[p[take]].copy(), perm[q[take]].copy()
            perm[p[take]], perm[q[take]] = b, a
            flips += int(take.sum())
        margins.append(np.concatenate(m_pass) if m_pass else np.zeros(0))
    if return_margin:
        return perm, flips, margins
    return perm, flips
