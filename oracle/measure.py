"""Equal-time observables of a worldline configuration (test infrastructure, FP64).

Sec. 4 measures, with S^z_j = (n_{j,up} - n_{j,dn}) / 2:
    C(r) = < S^z_0 S^z_r >,   S(k) = (1/N) sum_{i,j} e^{i k.(r_i - r_j)} < S^z_i S^z_j >,
the double occupancy D = < n_up n_dn > and the local moment < S_i^2 >. On a configuration the
expectation is estimated by the average over the L_tau slices (every slice of the periodic trace
is equivalent) and, for C, D and the local moment, over sites (translation invariance):
    C(r) = (1/(L_tau N)) sum_{l, j} S^z_{j+r,l} S^z_{j,l},
    S(k) = (1/L_tau) sum_l (1/N) | sum_j e^{i k.r_j} S^z_{j,l} |^2,   k = 2 pi (k_x, k_y) / L,
    D = (1/(L_tau N)) sum_{l, j} n_{j,up,l} n_{j,dn,l},
    <S^2> = (3/4) (1/(L_tau N)) sum_{l, j} (n_{j,up,l} - n_{j,dn,l})^2   (= 3 <(S^z)^2>).
Occupations are worldline counts per site and slice (with the permutation fixed to the identity
several same-spin worldlines may share a site, so n can exceed 1). Every sum here is written out
directly over sites; k and r are indexed like sites, k_x + L k_y and x + L y.
"""
from __future__ import annotations

import numpy as np

from . import gibbs


def observables(L: int, n_up: int, paths: np.ndarray):
    """(S(k) [N], C(r) [N], D, <S^2>) of worldlines paths[l, p] (up particles first)."""
    N = L * L
    L_tau = paths.shape[0]
    cu, cd = gibbs.occupancy(np.asarray(paths, dtype=np.int64), n_up, N)
    sz = 0.5 * (cu - cd).astype(np.float64)                      # [L_tau, N]
    x = np.arange(N) % L
    y = np.arange(N) // L
    # S(k): direct sum over sites for every k
    phase = 2.0 * np.pi * (np.outer(x, x) + np.outer(y, y)) / L   # [k, j] = k.r_j
    amp = sz @ np.exp(1j * phase).T                               # [L_tau, k]
    Sk = (np.abs(amp) ** 2).mean(axis=0) / N
    # C(r): direct sum over sites for every displacement r
    Cr = np.zeros(N)
    for r in range(N):
        shifted = ((x + x[r]) % L) + L * ((y + y[r]) % L)         # site j + r
        Cr[r] = (sz[:, shifted] * sz).mean()
    D = float((cu * cd).mean())
    S2 = float(0.75 * ((cu - cd) ** 2).mean())
    return Sk, Cr, D, S2
