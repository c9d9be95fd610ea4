"""Pins of the permutation sector (eq. joint with P != id; Sec. 3.5.6): on systems of two
worldlines small enough to enumerate every (paths, permutation) state, each move that sees the
permutation (pair swaps, FFBS with reconnected blocks, local updates) must leave |pi| invariant,
and at U = 0 the enumerated sign average must equal the free-fermion closed form."""
import itertools

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import ffbs, hs, lattice, local, perm as operm


def joint_states(desc, aux):
    """Every (paths [L_tau, 2], perm) state of two up worldlines, |pi| and sgn."""
    L_tau, N = desc.L_tau, desc.L * desc.L
    Gm = lattice.transfer_matrix(desc.L, desc.t, desc.dtau)
    W = hs.potentials(aux, desc.hs_kind, desc.U, desc.dtau)[0]
    conf = np.array(list(itertools.product(range(N), repeat=2 * L_tau)), dtype=np.int64)
    conf = conf.reshape(-1, L_tau, 2)                 # [state, slice, worldline]
    states, weights, signs = [], [], []
    for pm, sg in (((0, 1), 1), ((1, 0), -1)):
        w = np.ones(len(conf))
        for p in range(2):
            for l in range(L_tau):
                w *= W[l, conf[:, l, p]]
                nxt = conf[:, l + 1, p] if l + 1 < L_tau else conf[:, 0, pm[p]]
                w *= Gm[nxt, conf[:, l, p]]
        states.append(conf)
        weights.append(w)
        signs.append(np.full(len(conf), sg))
    perms = np.repeat(np.array([[0, 1], [1, 0]]), len(conf), axis=0)
    return np.concatenate(states), perms, np.concatenate(weights), np.concatenate(signs)


def code(paths, perms, N):
    """State index matching joint_states' order: perm block, then paths in row-major order."""
    L_tau = paths.shape[1]
    c = np.zeros(paths.shape[0], dtype=np.int64)
    for l in range(L_tau):
        for p in range(2):
            c = c * N + paths[:, l, p]
    return c + (perms[:, 0] == 1) * N ** (2 * L_tau)


def chi2_p(counts, prob):
    ex = prob * counts.sum()
    keep = ex >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exv = np.append(ex[keep], ex[~keep].sum())
    return scipy.stats.chi2.sf(((obs - exv) ** 2 / exv).sum(), len(exv) - 1)


def system(L_tau, U, kind=synth.HS_GAUSS, M=1, seed=3):
    """M independent two-worldline systems as one chain of 2M up worldlines: pairs (2i, 2i+1)."""
    return synth.ChainDesc(L=2, L_tau=L_tau, n_up=2 * M, n_dn=0, hs_kind=kind, block_len=0,
                           t=1.0, U=U, dtau=0.4, seed=seed)


def draw_exact(desc, aux, M, rng):
    st, pm, w, _ = joint_states(desc, aux)
    pick = rng.choice(len(w), size=M, p=w / w.sum())
    paths = np.empty((desc.L_tau, 2 * M), dtype=np.int64)
    perm = np.empty(2 * M, dtype=np.int64)
    paths[:, 0::2] = st[pick, :, 0].T
    paths[:, 1::2] = st[pick, :, 1].T
    perm[0::2] = 2 * np.arange(M) + pm[pick, 0]
    perm[1::2] = 2 * np.arange(M) + pm[pick, 1]
    return paths, perm, w / w.sum()


def to_states(paths, perm, M):
    p = np.stack([paths[:, 0::2].T, paths[:, 1::2].T], axis=2)      # [M, L_tau, 2]
    pm = np.stack([perm[0::2] - 2 * np.arange(M), perm[1::2] - 2 * np.arange(M)], axis=1)
    return p, pm


@pytest.mark.parametrize("L_tau,dtau", [(2, 0.4), (3, 0.3)])
def test_u0_sign_average_is_the_free_fermion_closed_form(L_tau, dtau):
    d = synth.ChainDesc(L=2, L_tau=L_tau, n_up=2, n_dn=0, hs_kind=synth.HS_GAUSS, block_len=0,
                        t=1.0, U=0.0, dtau=dtau, seed=1)
    _, _, w, sg = joint_states(d, np.zeros((L_tau, 4)))
    beta = L_tau * dtau
    c = np.cos(np.pi * np.arange(2))
    lam = np.exp(2 * beta * (c[:, None] + c[None, :]).ravel())
    ref = (lam.sum() ** 2 - (lam ** 2).sum()) / (lam.sum() ** 2 + (lam ** 2).sum())
    assert (sg * w).sum() / w.sum() == pytest.approx(ref, rel=1e-12)


def test_permutation_sign_by_cycles():
    assert operm.permutation_sign([0, 1, 2]) == 1
    assert operm.permutation_sign([1, 0, 2]) == -1
    assert operm.permutation_sign([1, 2, 0]) == 1
    assert operm.permutation_sign([3, 2, 1, 0]) == 1
    assert operm.permutation_sign([1, 2, 3, 0]) == -1


def test_pair_swaps_preserve_the_joint_law():
    M = 60000
    d = system(2, 4.0, M=M)
    aux = synth.initial_aux(d, rng_seed=9)
    paths, perm, prob = draw_exact(d, aux, M, np.random.default_rng(1))
    signs0 = [operm.permutation_sign(perm[2 * i:2 * i + 2] - 2 * i) for i in range(5)]
    new, flips = operm.perm_update(d, paths, perm, sweep=7, n_passes=1)
    assert 0 < flips < M
    st, pm = to_states(paths, new, M)
    counts = np.bincount(code(st, pm, 4), minlength=len(prob))
    assert chi2_p(counts, prob) > 1e-4
    # each accepted swap flips that system's sign
    for i in range(5):
        changed = not np.array_equal(new[2 * i:2 * i + 2], perm[2 * i:2 * i + 2])
        assert operm.permutation_sign(new[2 * i:2 * i + 2] - 2 * i) == signs0[i] * (-1 if changed else 1)


@pytest.mark.parametrize("block_len", [0, 2])
def test_ffbs_with_reconnected_blocks_preserves_the_joint_law(block_len):
    M = 60000
    d = synth.ChainDesc(L=2, L_tau=3, n_up=2 * M, n_dn=0, hs_kind=synth.HS_GAUSS,
                        block_len=block_len, t=1.0, U=4.0, dtau=0.4, seed=4)
    aux = synth.initial_aux(d, rng_seed=11)
    paths, perm, prob = draw_exact(d, aux, M, np.random.default_rng(2))
    Gm = lattice.transfer_matrix(d.L, d.t, d.dtau)
    W = hs.potentials(aux, d.hs_kind, d.U, d.dtau)[0]
    for s in (1, 2):   # block offsets 0 and floor(B/2): blocks that cross tau = beta
        out, _ = ffbs.ffbs_spin(Gm, W, paths, np.arange(2 * M), d.seed, s, d.block_len,
                                perm=perm)
        st, pm = to_states(out, perm, M)
        counts = np.bincount(code(st, pm, 4), minlength=len(prob))
        assert chi2_p(counts, prob) > 1e-4, s
        assert not np.array_equal(out, paths)


def test_local_updates_with_reconnections_preserve_the_joint_law():
    M = 60000
    d = system(3, 4.0, M=M, seed=5)
    aux = synth.initial_aux(d, rng_seed=12)
    paths, perm, prob = draw_exact(d, aux, M, np.random.default_rng(3))
    out = local.local_update(d, aux, paths, sweep=3, n_passes=2, perm=perm)
    st, pm = to_states(out, perm, M)
    counts = np.bincount(code(st, pm, 4), minlength=len(prob))
    assert chi2_p(counts, prob) > 1e-4


def free_fermion_energy(L, t, beta, n):
    """Canonical energy of n free fermions (one spin) on the periodic L x L lattice: levels
    eps_k = -2t(cos kx + cos ky), weights of the n-fermion states prod lambda_k over k-subsets."""
    ks = 2 * np.pi * np.arange(L) / L
    eps = (-2 * t * (np.cos(ks)[:, None] + np.cos(ks)[None, :])).ravel()
    num = den = 0.0
    for sub in itertools.combinations(range(len(eps)), n):
        e = eps[list(sub)].sum()
        w = np.exp(-beta * e)
        num += e * w
        den += w
    return num / den


@pytest.mark.parametrize("L_tau,dtau", [(3, 0.3), (4, 0.25)])
def test_u0_fermion_energy_from_reconnected_gradients(L_tau, dtau):
    """At U = 0 the sign-weighted average, over every (anchor sites, permutation) of two up
    worldlines weighted by prod_p Z_p, of the Rao-Blackwellised kinetic energy
    -(t/beta) sum_p d log Z_p / dt (Z_p closing on the anchor of perm[p]) is the canonical energy
    of two free fermions: the permutation sum antisymmetrises the propagator."""
    from oracle import grad as ograd
    d = synth.ChainDesc(L=2, L_tau=L_tau, n_up=2, n_dn=0, hs_kind=synth.HS_GAUSS, block_len=0,
                        t=1.0, U=0.0, dtau=dtau, seed=1)
    aux = np.zeros((L_tau, d.N))
    beta = L_tau * dtau
    num = den = 0.0
    for a in itertools.product(range(d.N), repeat=2):
        paths = np.tile(np.array(a), (L_tau, 1))
        for pm, sg in (((0, 1), 1), ((1, 0), -1)):
            lz, _, dt, _ = ograd.logz_path_grad(d, aux, paths, 0, perm=np.array(pm))
            w = sg * np.exp(lz)
            num += w * (-d.t / beta) * dt
            den += w
    assert num / den == pytest.approx(free_fermion_energy(2, d.t, beta, 2), rel=1e-11)
    # without the permutation sum the same average gives distinguishable particles' energy
    num_b = den_b = 0.0
    for a in itertools.product(range(d.N), repeat=2):
        paths = np.tile(np.array(a), (L_tau, 1))
        lz, _, dt, _ = ograd.logz_path_grad(d, aux, paths, 0)
        num_b += np.exp(lz) * (-d.t / beta) * dt
        den_b += np.exp(lz)
    assert abs(num_b / den_b - free_fermion_energy(2, d.t, beta, 2)) > 1e-3
