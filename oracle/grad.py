"""log Z_path and its gradient by reverse mode (test infrastructure, FP64).

log Z_path(aux, t) = sum over worldlines p of log Z_p, where Z_p is the weight of all closed
paths of particle p that pass through its current site a_p at the anchor slice l0: the FFBS
forward filter of Sec. 3.5.2 run over one block of length L_tau anchored at (l0, a_p) and closed
on the same site. It is log p(anchor sites | field) up to a field-independent constant; the HS
prior is not included. The paper does not define this gradient; it is the adjoint of the
forward recursion:

  backward messages  beta_{L_tau-1}(r) = G(e (-) r),  e the site the block closes on (a),
                     beta_j = G * (W_{j+1} . beta_{j+1})            (G is symmetric)
  so that Z = sum_r f_j(r) beta_j(r) for every j, and
  d log Z / d log W_j(r) = f_j(r) beta_j(r) / Z      (the smoothing marginal of r_j)
  d log Z / d t = sum_j <u_{j+1}, (dG/dt) * f_j> / <u_{j+1}, G * f_j>,
                  u_{j+1} = W_{j+1} . beta_{j+1}  (u_{L_tau} = delta_e).
With log W_spin = c_spin * aux (c = a for the Gaussian field, +-lambda for the Ising one),
d log Z_path / d aux(l, r) = sum_p c_spin(p) P(r_l^(p) = r).
All messages are kept normalised; every ratio above is scale-free.

With reconnections at tau = beta (eq. joint's sum over permutations, slice L_tau of worldline p
being slice 0 of worldline perm[p]) the block of p anchored at (l0, a_p) runs through tau = beta
onto perm[p] and closes on the anchor site of perm[p]: Z_p is the weight of all paths from a_p
to a_{perm[p]} over L_tau slices (the same recursion with end site a_{perm[p]} in place of a_p),
and log Z_path is still the log-probability of the anchor sites given the field, up to a
field-independent constant.
"""
from __future__ import annotations

import numpy as np

from . import ffbs, hs, lattice


def _spins(desc, aux):
    W_up, W_dn = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)
    c_up, c_dn = hs.log_weight_coeffs(desc.hs_kind, desc.U, desc.dtau)
    out = []
    if desc.n_up:
        out.append((W_up, c_up, np.arange(desc.n_up)))
    if desc.n_dn:
        out.append((W_dn, c_dn, np.arange(desc.n_up, desc.n_particles)))
    return out


def _ends(desc, paths, anchor_slice, parts, perm):
    """Anchor sites of the worldlines each block closes on (itself, or its reconnection)."""
    nxt = parts if perm is None else np.asarray(perm, dtype=np.int64)[parts]
    return paths[anchor_slice, nxt].astype(np.int64)


def logz_path(desc, aux: np.ndarray, paths: np.ndarray, anchor_slice: int, t: float | None = None,
              perm: np.ndarray | None = None):
    """(total log Z_path, per-particle log Z_p [Np]); perm: reconnection (None = identity)."""
    t = desc.t if t is None else t
    Gmat = lattice.transfer_matrix(desc.L, t, desc.dtau)
    per = np.zeros(desc.n_particles)
    for W, _, parts in _spins(desc, aux):
        a = paths[anchor_slice, parts].astype(np.int64)
        e = _ends(desc, paths, anchor_slice, parts, perm)
        _, lz, _ = ffbs.forward_filter(Gmat, W, anchor_slice, desc.L_tau, a, e)
        per[parts] = lz
    return float(per.sum()), per


def logz_path_grad(desc, aux: np.ndarray, paths: np.ndarray, anchor_slice: int,
                   perm: np.ndarray | None = None):
    """Returns (log Z_path, grad_aux [L_tau, N], d log Z_path / d t, per-particle dt [Np])."""
    L_tau, N = desc.L_tau, desc.N
    Gmat = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)
    dGmat = lattice.transfer_matrix_dt(desc.L, desc.t, desc.dtau)
    grad = np.zeros((L_tau, N))
    dt_per = np.zeros(desc.n_particles)
    total = 0.0
    for W, coef, parts in _spins(desc, aux):
        P = len(parts)
        rows = np.arange(P)
        a = paths[anchor_slice, parts].astype(np.int64)
        e = _ends(desc, paths, anchor_slice, parts, perm)
        filt, lz, _ = ffbs.forward_filter(Gmat, W, anchor_slice, L_tau, a, e)
        total += float(lz.sum())
        u_next = np.zeros((P, N))
        u_next[rows, e] = 1.0                       # u_{L_tau} = delta_e
        dt = np.zeros(P)
        for j in range(L_tau - 1, -1, -1):
            f = filt[:, j, :]
            beta = u_next @ Gmat                    # beta_j(r) = sum_r' G(r' - r) u(r')
            beta /= beta.sum(axis=1, keepdims=True)
            Gf = f @ Gmat.T
            dGf = f @ dGmat.T
            dt += (u_next * dGf).sum(axis=1) / (u_next * Gf).sum(axis=1)
            fb = f * beta
            marg = fb / fb.sum(axis=1, keepdims=True)
            grad[(anchor_slice + j) % L_tau] += coef * marg.sum(axis=0)
            u_next = W[(anchor_slice + j) % L_tau][None, :] * beta
            u_next /= u_next.sum(axis=1, keepdims=True)
        dt_per[parts] = dt
    return total, grad, float(dt_per.sum()), dt_per
