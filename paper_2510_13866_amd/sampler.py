"""Torch-facing helpers over the C ABI: device buffers in the packed batch layout, a Sampler
object, and LogZPath, a torch.autograd.Function whose backward is the library's hand-written
adjoint (fh_logZ_grad). Torch provides device memory and streams only; every step of the
sweep and of the gradient runs in the HIP library.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from . import fhmc


class Sampler:
    """A plan over a batch of chains plus helpers to move per-chain arrays in and out."""

    def __init__(self, descs: Sequence, precision: int = fhmc.FH_FP64, flags: int = 0,
                 device: str = "cuda:0"):
        self.descs = list(descs)
        self.precision = precision
        self.device = torch.device(device)
        self.plan = fhmc.fh_init(self.descs, precision, flags)
        self.dtype = torch.float64 if precision == fhmc.FH_FP64 else torch.float32
        self.aux_elems, self.path_elems, self.n_particles = fhmc.fh_sizes(self.plan)
        self.layouts = [fhmc.fh_layout(self.plan, c) for c in range(len(self.descs))]
        self.t_values = [float(d.t) for d in self.descs]
        self._chain_index = None

    def close(self):
        if self.plan is not None:
            fhmc.fh_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers --------------------------------------------------------------------------
    def pack_aux(self, per_chain: Sequence[np.ndarray]) -> torch.Tensor:
        flat = np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in per_chain])
        return torch.from_numpy(flat).to(device=self.device, dtype=self.dtype)

    def pack_paths(self, per_chain: Sequence[np.ndarray]) -> torch.Tensor:
        flat = np.concatenate([np.asarray(a, dtype=np.int32).reshape(-1) for a in per_chain])
        return torch.from_numpy(flat).to(device=self.device)

    def unpack_aux(self, aux: torch.Tensor) -> List[np.ndarray]:
        host = aux.detach().to("cpu", torch.float64).numpy()
        return [host[l["aux_offset"]:l["aux_offset"] + l["aux_count"]].reshape(l["L_tau"], l["N"])
                for l in self.layouts]

    def unpack_paths(self, paths: torch.Tensor) -> List[np.ndarray]:
        host = paths.detach().cpu().numpy()
        return [host[l["path_offset"]:l["path_offset"] + l["path_count"]].reshape(
            l["L_tau"], l["n_particles"]) for l in self.layouts]

    def unpack_particles(self, vals: torch.Tensor) -> List[np.ndarray]:
        host = vals.detach().cpu().numpy()
        return [host[l["particle_offset"]:l["particle_offset"] + l["n_particles"]]
                for l in self.layouts]

    def chain_index(self) -> torch.Tensor:
        """Chain id of every element of the packed aux array (device, int64)."""
        if self._chain_index is None:
            idx = np.concatenate([np.full(l["aux_count"], c, dtype=np.int64)
                                  for c, l in enumerate(self.layouts)])
            self._chain_index = torch.from_numpy(idx).to(self.device)
        return self._chain_index

    # -- calls ----------------------------------------------------------------------------
    def forward_filter(self, aux, paths, sweep, stream=None) -> torch.Tensor:
        logZ = torch.empty(self.n_particles, dtype=torch.float64, device=self.device)
        fhmc.fh_forward_filter(self.plan, aux, paths, sweep, logZ, stream)
        return logZ

    def backward_sample(self, paths, sweep, stream=None):
        fhmc.fh_backward_sample(self.plan, paths, sweep, stream)

    def gibbs_aux(self, paths, aux, sweep, stream=None):
        fhmc.fh_gibbs_aux(self.plan, paths, aux, sweep, stream)

    def local_update(self, aux, paths, sweep, n_passes=1, stream=None):
        fhmc.fh_local_update(self.plan, aux, paths, sweep, n_passes, stream)

    def set_permutation(self, per_chain: Sequence[np.ndarray]):
        """Reconnections at tau = beta, one chain-local permutation per chain."""
        fhmc.fh_set_permutation(self.plan, np.concatenate([np.asarray(q).ravel()
                                                           for q in per_chain]))

    def permutation(self):
        """(per-chain permutations, per-chain signs)."""
        perm, sign = fhmc.fh_get_permutation(self.plan, self.n_particles, len(self.descs))
        perm = np.asarray(perm)
        return [perm[l["particle_offset"]:l["particle_offset"] + l["n_particles"]]
                for l in self.layouts], np.asarray(sign)

    def permutation_update(self, paths, sweep, n_passes=1, stream=None):
        fhmc.fh_permutation_update(self.plan, paths, sweep, n_passes, stream)

    def measure(self, paths, stream=None):
        """Per-chain (S(k) [N], C(r) [N], D, local moment) of the worldlines, as numpy arrays."""
        total = sum(lay["N"] for lay in self.layouts)
        Sk = torch.empty(total, dtype=torch.float64, device=self.device)
        Cr = torch.empty_like(Sk)
        D = torch.empty(len(self.descs), dtype=torch.float64, device=self.device)
        S2 = torch.empty_like(D)
        fhmc.fh_measure(self.plan, paths, Sk, Cr, D, S2, stream)
        Sk, Cr, D, S2 = (t.cpu().numpy() for t in (Sk, Cr, D, S2))
        out, o = [], 0
        for c, lay in enumerate(self.layouts):
            n = lay["N"]
            out.append((Sk[o:o + n], Cr[o:o + n], float(D[c]), float(S2[c])))
            o += n
        return out

    def sweep(self, aux, paths, first_sweep, n_sweeps, stream=None):
        fhmc.fh_sweep(self.plan, aux, paths, first_sweep, n_sweeps, stream)

    def set_hopping(self, t_values: Sequence[float]):
        fhmc.fh_set_hopping(self.plan, t_values)
        self.t_values = [float(v) for v in t_values]

    def logz_grad(self, aux, paths, anchor_slice, stream=None):
        n = len(self.descs)
        logZ = torch.empty(n, dtype=torch.float64, device=self.device)
        grad_aux = torch.empty_like(aux)
        grad_t = torch.empty(n, dtype=torch.float64, device=self.device)
        fhmc.fh_logZ_grad(self.plan, aux, paths, anchor_slice, logZ, grad_aux, grad_t, stream)
        return logZ, grad_aux, grad_t

    def mala_field(self, aux, paths, anchor_slice, eps, sweep, stream=None) -> np.ndarray:
        """One MALA move of every Gaussian field (fh_mala_field); per-chain 1 / 0 accepted,
        -1 for Ising-field chains."""
        acc = torch.empty(len(self.descs), dtype=torch.int32, device=self.device)
        fhmc.fh_mala_field(self.plan, aux, paths, anchor_slice, eps, sweep, acc, stream)
        return acc.cpu().numpy()

    def kinetic_energy(self, aux, paths, anchor_slice, stream=None) -> np.ndarray:
        """Rao-Blackwellised kinetic-energy estimate per chain (fh_kinetic_energy)."""
        out = torch.empty(len(self.descs), dtype=torch.float64, device=self.device)
        fhmc.fh_kinetic_energy(self.plan, aux, paths, anchor_slice, out, stream)
        return out.cpu().numpy()

    def filters(self, chain, particle) -> np.ndarray:
        rows = fhmc.fh_get_filters(self.plan, chain, particle)
        N = self.layouts[chain]["N"]
        dst = torch.empty(rows * N, dtype=self.dtype, device=self.device)
        fhmc.fh_get_filters(self.plan, chain, particle, dst)
        return dst.cpu().double().numpy().reshape(rows, N)

    def status(self):
        return fhmc.fh_get_status(self.plan)


class LogZPath(torch.autograd.Function):
    """logZ[c] = log Z_path of chain c (per-chain tensor) as a function of the packed field
    `aux` and the hopping amplitudes `t` ([n_chains] float64); the backward pass is the
    library's adjoint. Usage: LogZPath.apply(aux, t, sampler, paths, anchor_slice)."""

    @staticmethod
    def forward(ctx, aux, t, sampler: Sampler, paths, anchor_slice: int):
        tv = [float(v) for v in t.detach().cpu().tolist()]
        if tv != sampler.t_values:
            sampler.set_hopping(tv)
        logZ, grad_aux, grad_t = sampler.logz_grad(aux.detach(), paths, anchor_slice)
        ctx.save_for_backward(grad_aux, grad_t)
        ctx.chain_index = sampler.chain_index()
        ctx.t_device, ctx.t_dtype = t.device, t.dtype
        return logZ

    @staticmethod
    def backward(ctx, g):
        grad_aux, grad_t = ctx.saved_tensors
        scale = g.to(grad_aux.device)[ctx.chain_index].to(grad_aux.dtype)
        ga = grad_aux * scale
        gt = (grad_t * g.to(grad_t.device)).to(device=ctx.t_device, dtype=ctx.t_dtype)
        return ga, gt, None, None, None
