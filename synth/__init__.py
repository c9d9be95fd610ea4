"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the benchmark.

This module holds only input recipes: chain descriptors for the lattice workloads, initial
auxiliary fields and initial worldlines drawn from numpy's seeded generator. It contains none
of the sampler's arithmetic (no kernels, potentials, filters or conditionals), so the CPU
oracle and the GPU library can both take its outputs as inputs without sharing method code.

Workload shapes follow the paper's experiments: half-filled periodic square lattices with
nearest-neighbour hopping t=1 (Sec. 4, "Physical Setup" and "Computational Performance").
No public dataset is involved; every input is synthetic.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

HS_GAUSS = 0
HS_HIRSCH = 1


@dataclasses.dataclass(frozen=True)
class ChainDesc:
    """One Markov chain: an L x L periodic lattice with L_tau imaginary-time slices.

    n_up / n_dn: number of spin-up / spin-down worldlines (particle index p < n_up is up).
    hs_kind: HS_GAUSS (continuous field) or HS_HIRSCH (Ising field, stored as +-1.0).
    block_len: FFBS block length, 0 means one block of length L_tau (the whole ring).
    """

    L: int
    L_tau: int
    n_up: int
    n_dn: int
    hs_kind: int
    block_len: int
    t: float
    U: float
    dtau: float
    seed: int

    @property
    def N(self) -> int:
        return self.L * self.L

    @property
    def n_particles(self) -> int:
        return self.n_up + self.n_dn


def half_filled(L: int, L_tau: int, hs_kind: int, U: float, dtau: float, seed: int,
                t: float = 1.0, block_len: int = 0) -> ChainDesc:
    n = (L * L) // 2
    return ChainDesc(L=L, L_tau=L_tau, n_up=n, n_dn=n, hs_kind=hs_kind, block_len=block_len,
                     t=t, U=U, dtau=dtau, seed=seed)


def initial_aux(desc: ChainDesc, rng_seed: int | None = None) -> np.ndarray:
    """Initial auxiliary field, shape [L_tau, N] float64, slice-major, site i = x + L*y.

    Gaussian kind: independent N(0,1) values. Hirsch kind: independent +-1 with p=1/2.
    """
    rng = np.random.default_rng(desc.seed if rng_seed is None else rng_seed)
    shape = (desc.L_tau, desc.N)
    if desc.hs_kind == HS_GAUSS:
        return rng.standard_normal(shape)
    return np.where(rng.random(shape) < 0.5, 1.0, -1.0)


def _site_order(L: int, first_parity: int) -> List[int]:
    even = [x + L * y for y in range(L) for x in range(L) if (x + y) % 2 == first_parity]
    odd = [x + L * y for y in range(L) for x in range(L) if (x + y) % 2 != first_parity]
    return even + odd


def initial_paths(desc: ChainDesc) -> np.ndarray:
    """Static initial worldlines, shape [L_tau, n_up + n_dn] int32.

    Up particles occupy the (x+y)-even sites in increasing site index, then the odd ones;
    down particles the (x+y)-odd sites first. Every slice holds the same positions.
    """
    N = desc.N
    up = _site_order(desc.L, 0)
    dn = _site_order(desc.L, 1)
    pos = [up[p % N] for p in range(desc.n_up)] + [dn[q % N] for q in range(desc.n_dn)]
    return np.tile(np.asarray(pos, dtype=np.int32), (desc.L_tau, 1))


def random_paths(desc: ChainDesc, rng_seed: int) -> np.ndarray:
    """Uniformly random worldlines [L_tau, n_particles] int32 (used for parity of single steps)."""
    rng = np.random.default_rng(rng_seed)
    return rng.integers(0, desc.N, size=(desc.L_tau, desc.n_particles), dtype=np.int32)


def random_walk_paths(desc: ChainDesc, rng_seed: int, hop: float = 0.3) -> np.ndarray:
    """Worldlines that look like sampled ones: a uniformly random site at slice 0, then at each
    slice a nearest-neighbour hop with probability `hop` (the wrap from the last slice back to
    slice 0 is not constrained).
    Shape [L_tau, n_particles] int32."""
    rng = np.random.default_rng(rng_seed)
    L = desc.L
    x = rng.integers(0, L, size=desc.n_particles)
    y = rng.integers(0, L, size=desc.n_particles)
    out = np.empty((desc.L_tau, desc.n_particles), dtype=np.int32)
    for l in range(desc.L_tau):
        out[l] = x + L * y
        move = rng.random(desc.n_particles) < hop
        d = rng.integers(0, 4, size=desc.n_particles)
        x = np.where(move & (d == 0), (x + 1) % L, np.where(move & (d == 1), (x - 1) % L, x))
        y = np.where(move & (d == 2), (y + 1) % L, np.where(move & (d == 3), (y - 1) % L, y))
    return out


# --- the workload configurations ---------------------------------------------------------

def config_small_fp64() -> List[ChainDesc]:
    """4x4, U=4, dtau=0.1, L_tau=16 (beta=1.6), 8+8 fermions, Gaussian field, seed 0."""
    return [half_filled(4, 16, HS_GAUSS, 4.0, 0.1, seed=0)]


def config_16x16_hirsch(n_chains: int = 64) -> List[ChainDesc]:
    """16x16, U=4, dtau=0.0625, L_tau=64 (beta=4), 128+128 fermions, Ising field, seeds 0.."""
    return [half_filled(16, 64, HS_HIRSCH, 4.0, 0.0625, seed=s) for s in range(n_chains)]


def config_32x32(U: float = 4.0, n_chains: int = 16) -> List[ChainDesc]:
    """32x32, dtau=0.05, L_tau=160 (beta=8), 512+512 fermions, Gaussian field, seeds 0.."""
    return [half_filled(32, 160, HS_GAUSS, U, 0.05, seed=s) for s in range(n_chains)]


def config_uneven(n_chains: int = 256, gen_seed: int = 2510) -> List[ChainDesc]:
    """Uneven batch: L from {8,12,16,24,32}, beta from {2,4,8}, dtau=0.05, U ~ U[2,6],
    half filling, Gaussian / Ising field 50/50. Chain c has seed c."""
    rng = np.random.default_rng(gen_seed)
    out = []
    for c in range(n_chains):
        L = int(rng.choice([8, 12, 16, 24, 32]))
        beta = float(rng.choice([2.0, 4.0, 8.0]))
        L_tau = int(round(beta / 0.05))
        U = float(rng.uniform(2.0, 6.0))
        kind = HS_GAUSS if rng.random() < 0.5 else HS_HIRSCH
        out.append(half_filled(L, L_tau, kind, U, 0.05, seed=c))
    return out


def config_paper_shape(L: int = 32, block_len: int = 64, n_chains: int = 4) -> List[ChainDesc]:
    """The paper's performance shape (Sec. 4): beta=32, dtau=1/32 (L_tau=1024), FFBS blocks of
    32 or 64 slices, L x L at half filling; U=4, Gaussian field (the paper gives no U here)."""
    return [half_filled(L, 1024, HS_GAUSS, 4.0, 1.0 / 32.0, seed=s, block_len=block_len)
            for s in range(n_chains)]


def config_gradient(n_chains: int = 8) -> List[ChainDesc]:
    """32x32, dtau=0.05, L_tau=128, U=4, Gaussian field, seeds 0.."""
    return [half_filled(32, 128, HS_GAUSS, 4.0, 0.05, seed=s) for s in range(n_chains)]


def pack(descs: Sequence[ChainDesc], per_chain: Sequence[np.ndarray]) -> np.ndarray:
    """Concatenate per-chain arrays (flattened) in chain order: the packed batch layout."""
    return np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in per_chain])
