"""Pins of the oracle's FFBS (Sec. 3.5.2): brute-force path enumeration, U=0 closed forms,
FFT convolution, chi-square of sampled paths and the inverse-CDF rules."""
import itertools

import numpy as np
import pytest
import scipy.stats

from oracle import ffbs, lattice


def brute_force_law(Gmat, W, start, length, a, e):
    """All interior paths of one block with their unnormalised weights (eq. joint, one worldline)."""
    L_tau, N = W.shape
    paths = np.array(list(itertools.product(range(N), repeat=length - 1)), dtype=np.int64)
    if length == 1:
        paths = np.zeros((1, 0), dtype=np.int64)
    full = np.concatenate([np.full((len(paths), 1), a), paths, np.full((len(paths), 1), e)], axis=1)
    w = np.ones(len(paths))
    for j in range(length):
        w *= W[(start + j) % L_tau, full[:, j]] * Gmat[full[:, j + 1], full[:, j]]
    return paths, w


@pytest.mark.parametrize("L,length", [(2, 2), (2, 5), (2, 7), (3, 3), (3, 5)])
def test_forward_filter_partition_function_matches_enumeration(L, length):
    rng = np.random.default_rng(L * 10 + length)
    L_tau = 8
    N = L * L
    Gmat = lattice.transfer_matrix(L, 1.0, 0.3)
    W = np.exp(0.6 * rng.standard_normal((L_tau, N)))
    for start in (0, 5):
        for a, e in ((0, 0), (1, N - 1)):
            _, w = brute_force_law(Gmat, W, start, length, a, e)
            _, lz, _ = ffbs.forward_filter(Gmat, W, start, length, np.array([a]), np.array([e]))
            assert lz[0] == pytest.approx(np.log(w.sum()), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("L,length", [(2, 5), (3, 4)])
def test_backward_conditionals_equal_exact_path_law(L, length):
    rng = np.random.default_rng(7)
    L_tau, N = 6, L * L
    Gmat = lattice.transfer_matrix(L, 1.0, 0.4)
    W = np.exp(0.8 * rng.standard_normal((L_tau, N)))
    a, e, start = 1, 2, 3
    paths, w = brute_force_law(Gmat, W, start, length, a, e)
    exact = w / w.sum()
    filt, _, _ = ffbs.forward_filter(Gmat, W, start, length, np.array([a]), np.array([e]))
    # probability the backward recursion assigns to each interior path
    prob = np.ones(len(paths))
    nxt = np.full(len(paths), e)
    for j in range(length - 1, 0, -1):
        cur = paths[:, j - 1]
        wj = filt[0, j][None, :] * Gmat[nxt][:, :]
        prob *= wj[np.arange(len(paths)), cur] / wj.sum(axis=1)
        nxt = cur
    assert np.allclose(prob, exact, rtol=1e-12, atol=1e-15)


def test_backward_sampler_chi2_against_enumeration():
    L, length, L_tau = 2, 5, 5
    N = L * L
    rng = np.random.default_rng(3)
    Gmat = lattice.transfer_matrix(L, 1.0, 0.5)
    W = np.exp(0.7 * rng.standard_normal((L_tau, N)))
    a, e = 0, 3
    paths, w = brute_force_law(Gmat, W, 0, length, a, e)
    exact = w / w.sum()
    M = 60000
    filt, _, _ = ffbs.forward_filter(Gmat, W, 0, length, np.full(M, a), np.full(M, e))
    u = np.random.default_rng(11).random((M, length))
    pos = ffbs.backward_sample(Gmat, filt, np.full(M, a), np.full(M, e), u)
    code = np.zeros(M, dtype=np.int64)
    for j in range(1, length):
        code = code * N + pos[:, j]
    counts = np.bincount(code, minlength=N ** (length - 1))
    ref = np.zeros(N ** (length - 1))
    for p, pr in zip(paths, exact):
        c = 0
        for v in p:
            c = c * N + v
        ref[c] = pr
    exp = ref * M
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    chi2 = ((obs - ex) ** 2 / ex).sum()
    assert scipy.stats.chi2.sf(chi2, len(ex) - 1) > 1e-4


def closed_form_ring_logz(L, L_tau, dtau, t=1.0):
    # U = 0: W = 1, K commutes with itself, Z_p = G^{(L_tau)}(0) = (1/N) sum_k exp(-beta eps_k)
    m = np.arange(L)
    c = np.cos(2 * np.pi * m / L)
    eps = -2 * t * (c[:, None] + c[None, :])
    return np.log(np.exp(-L_tau * dtau * eps).sum() / (L * L))


@pytest.mark.parametrize("L,L_tau,dtau", [(4, 16, 0.1), (2, 4, 0.1), (3, 4, 0.1), (8, 20, 0.05),
                                          (6, 10, 0.1)])
def test_u0_ring_closed_form(L, L_tau, dtau):
    N = L * L
    Gmat = lattice.transfer_matrix(L, 1.0, dtau)
    W = np.ones((L_tau, N))
    anchors = np.arange(N)
    _, lz, _ = ffbs.forward_filter(Gmat, W, 3 % L_tau, L_tau, anchors, anchors)
    assert np.allclose(lz, closed_form_ring_logz(L, L_tau, dtau), rtol=1e-13)


def test_u0_ring_reference_value_small_config():
    # 4x4, L_tau=16, dtau=0.1 (beta = 1.6): (1/N) sum_k e^{-beta eps_k}
    assert closed_form_ring_logz(4, 16, 0.1) == pytest.approx(3.787224610410, abs=1e-11)


def test_u0_open_block_closed_form():
    L, B, dtau = 4, 8, 0.1
    N = L * L
    Gmat = lattice.transfer_matrix(L, 1.0, dtau)
    W = np.ones((B, N))
    m = np.arange(L)
    c = np.cos(2 * np.pi * m / L)
    x, y = lattice.coords(L)
    for e in range(N):
        # G^{(B)}(d) = (1/N) sum_k exp(-B dtau eps_k) cos(k.d)
        ph = np.cos(2 * np.pi * (np.outer(m, np.ones(L)) * x[e] + np.outer(np.ones(L), m) * y[e]) / L)
        ref = (np.exp(2 * B * dtau * (c[:, None] + c[None, :])) * ph).sum() / N
        _, lz, _ = ffbs.forward_filter(Gmat, W, 0, B, np.array([0]), np.array([e]))
        assert np.exp(lz[0]) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("L", [4, 6, 12, 32])
def test_fft_convolution_equals_direct(L):
    rng = np.random.default_rng(L)
    f = np.exp(3 * rng.standard_normal((5, L * L)))
    direct = f @ lattice.transfer_matrix(L, 1.0, 0.05).T
    Gh = lattice.ghat_2d(L, 1.0, 0.05).reshape(L, L)
    # numpy arrays are [y, x]; ghat_2d is symmetric in (mx, my)
    viafft = np.fft.ifft2(np.fft.fft2(f.reshape(5, L, L)) * Gh).real.reshape(5, -1)
    assert np.linalg.norm(viafft - direct) <= 1e-13 * np.linalg.norm(direct)


def test_block_schedule_covers_ring():
    for L_tau, B in ((16, 0), (16, 4), (10, 4), (7, 3), (160, 64), (5, 2)):
        for s in (0, 1, 2):
            blocks = ffbs.block_schedule(L_tau, B, s)
            seen = np.zeros(L_tau, dtype=int)
            for start, n in blocks:
                assert n >= 1
                for j in range(n):
                    seen[(start + j) % L_tau] += 1
            assert np.all(seen == 1)
            BB = L_tau if B == 0 else B
            assert blocks[0][0] == (s * (BB // 2)) % L_tau


@pytest.mark.parametrize("L_tau,B", [(16, 0), (16, 4), (10, 4), (7, 3), (160, 64), (5, 2),
                                     (9, 0), (1024, 64), (6, 5)])
def test_block_schedule_reaches_every_slice(L_tau, B):
    interior = np.zeros(L_tau, dtype=bool)
    for s in range(2 * L_tau):
        for start, n in ffbs.block_schedule(L_tau, B, s):
            for j in range(1, n):
                interior[(start + j) % L_tau] = True
    assert interior.all()


def test_sample_index_rules():
    w = np.array([[0.0, 1.0, 0.0, 2.0, 0.0]])
    assert ffbs.sample_index(w, np.array([0.0]))[0] == 1
    assert ffbs.sample_index(w, np.array([1.0 / 3.0 - 1e-12]))[0] == 1
    assert ffbs.sample_index(w, np.array([0.5]))[0] == 3
    # u -> 1 with T rounding onto the total: last positive weight
    assert ffbs.sample_index(w, np.array([1.0]))[0] == 3
    assert ffbs.sample_index(np.array([[0.0, 0.0, 1e-300]]), np.array([0.99]))[0] == 2


def test_filters_positive_and_normalised():
    L, L_tau = 4, 16
    rng = np.random.default_rng(0)
    Gmat = lattice.transfer_matrix(L, 1.0, 0.1)
    W = np.exp(0.63 * rng.standard_normal((L_tau, L * L)))
    filt, lz, logc = ffbs.forward_filter(Gmat, W, 0, L_tau, np.arange(8), np.arange(8))
    assert np.all(filt > 0) or np.all(filt[:, 1:] > 0)
    assert np.allclose(filt.sum(axis=2), 1.0, rtol=1e-14)
    assert np.all(np.isfinite(lz))
