"""Forward filtering, backward sampling of worldline blocks (test infrastructure, FP64).

Sec. 3.5.2 ("Forward-Filtering Backward-Sampling"), read in the site basis. For a block that
starts at slice l0 with the worldline at site a, has length n and ends at slice l0+n (mod L_tau)
at site e, with the endpoints held fixed:

  forward:   f_0 = W_l0(a) delta_a;   f_j = W_{l0+j} . (G * f_{j-1}),  j = 1 .. n-1
             Z = (G * f_{n-1})(e)      (the block's partition function given its endpoints)
  backward:  r_n = e;  for j = n-1 .. 1 draw r_j with P(r_j = r | r_{j+1}) ∝ f_j(r) G(r_{j+1} (-) r)

(the site-basis form of the paper's exact conditional P(k_l | k_{l+1})). The weight of the end
slice belongs to the next block. Convolutions are dense matrix products (Gmat @ f), no FFT.

Scaling: each f_j is divided by its sum c_j (c_0 = W_l0(a)), and
log Z = sum_j log c_j + log (G * f~_{n-1})(e). The paper does not fix a normaliser; the sum is
used here.

Inverse CDF: weights w(r) = max(f~_j(r), 0) G(r_{j+1} (-) r) in site order, C its running sum,
T = u * C_{N-1}; the draw is the smallest r with C_r > T (zero-weight sites are never chosen);
if rounding leaves no such r the last r with w(r) > 0 is taken.
"""
from __future__ import annotations

import numpy as np

from . import philox


def block_schedule(L_tau: int, block_len: int, sweep: int):
    """[(start, length)] of the FFBS blocks of a sweep.

    Block length B (0 means L_tau); the block starts are o_s + j*B (mod L_tau) with
    o_s = (s * floor(B/2)) mod L_tau, so each sweep moves the fixed endpoints by half a block
    (for B dividing L_tau and B even, o_s alternates between 0 and B/2); a last block shorter
    than B closes the ring. The paper only says the endpoints are held fixed; moving them is
    what lets every slice be redrawn.
    """
    B = L_tau if block_len == 0 else block_len
    o = ((sweep % L_tau) * (B // 2)) % L_tau
    nb = -(-L_tau // B)
    out = []
    for j in range(nb):
        length = B if j < nb - 1 else L_tau - (nb - 1) * B
        out.append(((o + j * B) % L_tau, length))
    return out


def forward_filter(Gmat: np.ndarray, W: np.ndarray, start: int, length: int,
                   anchors: np.ndarray, ends: np.ndarray):
    """Normalised forward messages of one block for a batch of worldlines of one spin.

    Gmat: [N, N] dense transfer matrix; W: [L_tau, N] site potentials of this spin;
    anchors, ends: [P] sites at slices start and start+length.
    Returns (filters [P, length, N] with filters[:, j] = f~_j, logZ [P], logc [P, length]).
    """
    L_tau, N = W.shape
    P = anchors.shape[0]
    rows = np.arange(P)
    filt = np.zeros((P, length, N))
    logc = np.zeros((P, length))
    filt[rows, 0, anchors] = 1.0
    logc[:, 0] = np.log(W[start, anchors])
    for j in range(1, length):
        h = (filt[:, j - 1, :] @ Gmat.T) * W[(start + j) % L_tau][None, :]
        c = h.sum(axis=1)
        filt[:, j, :] = h / c[:, None]
        logc[:, j] = np.log(c)
    z_end = (filt[:, length - 1, :] @ Gmat.T)[rows, ends]
    logZ = logc.sum(axis=1) + np.log(z_end)
    return filt, logZ, logc


def sample_index(w: np.ndarray, u: np.ndarray, return_margin: bool = False):
    """Row-wise inverse-CDF draw: w [P, N] non-negative weights, u [P] uniforms in [0,1)."""
    C = np.cumsum(w, axis=1)
    total = C[:, -1]
    T = u * total
    above = C > T[:, None]
    idx = np.argmax(above, axis=1)
    none = ~above.any(axis=1)
    if np.any(none):
        pos = w[none] > 0
        last = w.shape[1] - 1 - np.argmax(pos[:, ::-1], axis=1)
        idx[none] = last
    if not return_margin:
        return idx
    rows = np.arange(w.shape[0])
    hi = C[rows, idx] - T
    lo = T - np.where(idx > 0, C[rows, np.maximum(idx - 1, 0)], 0.0)
    return idx, np.minimum(hi, lo) / total


def backward_sample(Gmat: np.ndarray, filt: np.ndarray, anchors: np.ndarray,
                    ends: np.ndarray, u: np.ndarray, return_margin: bool = False):
    """Backward pass of one block. u: [P, length] uniforms, u[:, j] used for slice j (j >= 1).

    Returns positions [P, length+1] (column 0 = anchors, column length = ends) and, optionally,
    the relative CDF margin of every draw (distance of T to the nearest boundary / total).
    """
    P, length, N = filt.shape
    pos = np.zeros((P, length + 1), dtype=np.int64)
    pos[:, 0] = anchors
    pos[:, length] = ends
    margins = np.full((P, length), np.inf)
    for j in range(length - 1, 0, -1):
        w = np.maximum(filt[:, j, :], 0.0) * Gmat[pos[:, j + 1], :]
        if return_margin:
            pos[:, j], margins[:, j] = sample_index(w, u[:, j], True)
        else:
            pos[:, j] = sample_index(w, u[:, j])
    if return_margin:
        return pos, margins
    return pos


def ffbs_spin(Gmat, W, paths, particles, seed, sweep, block_len, return_margin=False,
              perm=None):
    """FFBS of every block of the given particles (one spin) for one sweep.

    paths: [L_tau, n_particles] current worldlines (endpoints are read from it).
    perm: optional [n_particles] permutation of the worldline connections at tau = beta (eq.
    joint; Sec. 3.5.6): slice L_tau of worldline p is slice 0 of worldline perm[p]. A block that
    runs past slice L_tau - 1 of its owner p continues on worldline perm[p]: its end site and
    its interior slices from L_tau on are read from / written to perm[p]'s column. With a
    permutation, `particles` must be all of the spin's worldlines (perm maps them onto
    themselves); None is the identity.
    Returns (new positions for these particles [L_tau, P], logZ summed over blocks [P],
    and margins [L_tau, P] if asked; margins at fixed endpoints are +inf).
    """
    L_tau = W.shape[0]
    particles = np.asarray(particles, dtype=np.int64)
    P = len(particles)
    out = paths[:, particles].astype(np.int64).copy()
    col = np.arange(P)                       # column of each particle's own slices
    if perm is None:
        nxt = col                            # column holding each worldline's slices >= L_tau
    else:
        where = {int(q): k for k, q in enumerate(particles)}
        nxt = np.array([where[int(perm[q])] for q in particles], dtype=np.int64)
    logZ = np.zeros(P)
    marg = np.full((L_tau, P), np.inf)
    for start, length in block_schedule(L_tau, block_len, sweep):
        anchors = paths[start, particles].astype(np.int64)
        end_col = nxt if start + length >= L_tau else col
        ends = paths[(start + length) % L_tau, particles[end_col]].astype(np.int64)
        filt, lz, _ = forward_filter(Gmat, W, start, length, anchors, ends)
        logZ += lz
        u = np.zeros((P, length))
        for j in range(1, length):
            u[:, j] = philox.path_uniforms(seed, np.asarray(particles, dtype=np.uint64),
                                           (start + j) % L_tau, sweep)
        res = backward_sample(Gmat, filt, anchors, ends, u, return_margin)
        pos, m = res if return_margin else (res, None)
        for j in range(1, length):
            c = nxt if start + j >= L_tau else col
            out[(start + j) % L_tau, c] = pos[:, j]
            if return_margin:
                marg[(start + j) % L_tau, c] = m[:, j]
    if return_margin:
        return out, logZ, marg
    return out, logZ
