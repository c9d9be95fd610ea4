"""ctypes binding of the C ABI in include/fh.h (argument marshalling only).

Every sampling step runs in the HIP library libfhmc.so built next to this file; importing this
module raises ImportError when that library is missing, so there is no silent CPU path.
Array arguments are torch tensors on the GPU (their data pointers are passed through);
`stream` defaults to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_uint32, c_uint64, c_void_p

# PyTorch ships its own HIP and HSA runtimes under the same sonames as the system ROCm ones.
# Loading torch first makes libfhmc.so bind to those already-loaded runtimes, so the process has
# one HIP runtime and torch's device pointers and streams are valid in the library. Loaded the
# other way round, the process would hold two runtimes and torch would find no GPU.
import torch  # noqa: E402,F401  (load order only)

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfhmc.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError("libfhmc.so is not built (%s); run paper_2510_13866_amd.build.build() "
                      "or __graft_entry__.build() first" % _LIB_PATH)
lib = ctypes.CDLL(_LIB_PATH)

FH_OK = 0
FH_ERR_INVALID_ARG = -1
FH_ERR_UNSUPPORTED = -2
FH_ERR_OOM = -3
FH_ERR_HIP = -4
FH_ERR_NONFINITE = -5
FH_ERR_ZERO_WEIGHT = -6
FH_ERR_STATE = -7
FH_ERR_BAD_PATH = -8

FH_HS_GAUSS = 0
FH_HS_HIRSCH = 1

FH_FP64 = 0
FH_FP32 = 1
FH_FP32_MFMA3 = 2

FH_FLAG_NONE = 0
FH_FLAG_GRAPH = 1
FH_FLAG_AUTOTUNE = 2
FH_FLAG_FULL_ROW_DRAW = 4
FH_FLAG_FFT_CONV = 8
FH_FLAG_GRAD_CHECKPOINT = 16


class fh_chain_desc(ctypes.Structure):
    _fields_ = [("L", c_int32), ("L_tau", c_int32), ("n_up", c_int32), ("n_dn", c_int32),
                ("hs_kind", c_int32), ("block_len", c_int32), ("t", c_double), ("U", c_double),
                ("dtau", c_double), ("seed", c_uint64)]


class fh_chain_layout(ctypes.Structure):
    _fields_ = [("aux_offset", c_int64), ("aux_count", c_int64), ("path_offset", c_int64),
                ("path_count", c_int64), ("particle_offset", c_int64), ("L", c_int32),
                ("N", c_int32), ("L_tau", c_int32), ("n_particles", c_int32)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("fh_init", c_int32, POINTER(c_void_p), POINTER(fh_chain_desc), c_int32, c_int32, c_uint32)
_sig("fh_destroy", c_int32, c_void_p)
_sig("fh_layout", c_int32, c_void_p, c_int32, POINTER(fh_chain_layout))
_sig("fh_sizes", c_int32, c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64))
_sig("fh_forward_filter", c_int32, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p, c_void_p)
_sig("fh_backward_sample", c_int32, c_void_p, c_void_p, c_uint64, c_void_p)
_sig("fh_gibbs_aux", c_int32, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p)
_sig("fh_sweep", c_int32, c_void_p, c_void_p, c_void_p, c_uint64, c_int32, c_void_p)
_sig("fh_local_update", c_int32, c_void_p, c_void_p, c_void_p, c_uint64, c_int32, c_void_p)
_sig("fh_set_permutation", c_int32, c_void_p, POINTER(c_int32))
_sig("fh_get_permutation", c_int32, c_void_p, POINTER(c_int32), POINTER(c_int32))
_sig("fh_permutation_update", c_int32, c_void_p, c_void_p, c_uint64, c_int32, c_void_p)
_sig("fh_measure", c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p)
_sig("fh_measure_noalloc", c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
     c_void_p)
_sig("fh_mala_field", c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_uint64, c_void_p,
     c_void_p)
_sig("fh_logZ_grad", c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
     c_void_p, c_void_p)
_sig("fh_kinetic_energy", c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p)
_sig("fh_set_hopping", c_int32, c_void_p, POINTER(c_double))
_sig("fh_get_status", c_int32, c_void_p, POINTER(c_int32), POINTER(c_int32))
_sig("fh_get_filters", c_int32, c_void_p, c_int32, c_int32, c_void_p, c_int64, POINTER(c_int64),
     c_void_p)
_sig("fh_get_radix_plan", c_int32, c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32))
_sig("fh_strerror", ctypes.c_char_p, c_int32)
_sig("fh_debug_fft2d_host", c_int32, POINTER(c_double), c_int32, c_int32)
_sig("fh_debug_fft2d_host_plan", c_int32, POINTER(c_double), c_int32, POINTER(c_int32), c_int32,
     c_int32)
_sig("fh_debug_radix_orders", c_int32, c_int32, POINTER(c_int32), c_int32)
_sig("fh_debug_kernel_table", c_int32, c_int32, c_double, c_double, POINTER(c_double))
_sig("fh_debug_philox", c_int32, c_uint64, c_uint64, c_uint64, c_uint64, c_uint64, c_uint64,
     POINTER(c_uint64))
_sig("fh_debug_window_select", c_int32, POINTER(c_double), c_int32, POINTER(c_int32),
     POINTER(c_double))
_sig("fh_debug_window_draw", c_int32, c_int32, c_int32, POINTER(c_double), c_double,
     POINTER(c_double), c_int32, c_double, POINTER(c_int32), POINTER(c_int32))
_sig("fh_debug_inflate_window_bound", c_int32, c_void_p, c_double)
_sig("fh_debug_backward_kernels", c_int32, c_void_p, POINTER(c_int32), POINTER(c_int32))
_sig("fh_debug_forward_kernels", c_int32, c_void_p, POINTER(c_int32))
_sig("fh_debug_backward_adapt", c_int32, c_void_p, c_int32, POINTER(c_int32))
_sig("fh_debug_rescue_holds", c_int32, c_void_p, POINTER(c_int32))
_sig("fh_debug_rescue_causes", c_int32, c_void_p, POINTER(c_int32))
_sig("fh_debug_fill_filter_row", c_int32, c_void_p, c_int32, c_int32, c_int32, c_double)
_sig("fh_debug_representatives", c_int32, c_void_p, POINTER(c_int32), c_int64, POINTER(c_int64))
_sig("fh_debug_share_filters", c_int32, c_void_p, c_int32)
_sig("fh_debug_rescue", c_int32, c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int64),
     POINTER(c_int32), c_int32)
_sig("fh_debug_sweep_timing", c_int32, c_void_p, c_int32)
_sig("fh_debug_sweep_times", c_int32, c_void_p, POINTER(ctypes.c_float))


class FhError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, lib.fh_strerror(code).decode(), code))


def _check(code, where):
    if code != FH_OK:
        raise FhError(code, where)


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def make_descs(descs):
    arr = (fh_chain_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = fh_chain_desc(int(d.L), int(d.L_tau), int(d.n_up), int(d.n_dn), int(d.hs_kind),
                               int(d.block_len), float(d.t), float(d.U), float(d.dtau),
                               int(d.seed))
    return arr


# ---- C ABI, one Python function per entry point ------------------------------------------

def fh_init(descs, precision, flags=FH_FLAG_NONE):
    """descs: sequence of objects with the fh_chain_desc fields (e.g. synth.ChainDesc)."""
    plan = c_void_p()
    arr = make_descs(descs)
    _check(lib.fh_init(byref(plan), arr, len(descs), int(precision), int(flags)), "fh_init")
    return plan


def fh_destroy(plan):
    _check(lib.fh_destroy(plan), "fh_destroy")


def fh_layout(plan, chain):
    out = fh_chain_layout()
    _check(lib.fh_layout(plan, int(chain), byref(out)), "fh_layout")
    return {k: getattr(out, k) for k, _ in fh_chain_layout._fields_}


def fh_sizes(plan):
    a, p, n = c_int64(), c_int64(), c_int64()
    _check(lib.fh_sizes(plan, byref(a), byref(p), byref(n)), "fh_sizes")
    return a.value, p.value, n.value


def fh_forward_filter(plan, aux, paths, sweep, logZ=None, stream=None):
    _check(lib.fh_forward_filter(plan, _ptr(aux), _ptr(paths), int(sweep), _ptr(logZ),
                                 _stream(stream)), "fh_forward_filter")


def fh_backward_sample(plan, paths, sweep, stream=None):
    _check(lib.fh_backward_sample(plan, _ptr(paths), int(sweep), _stream(stream)),
           "fh_backward_sample")


def fh_gibbs_aux(plan, paths, aux, sweep, stream=None):
    _check(lib.fh_gibbs_aux(plan, _ptr(paths), _ptr(aux), int(sweep), _stream(stream)),
           "fh_gibbs_aux")


def fh_sweep(plan, aux, paths, first_sweep, n_sweeps, stream=None):
    _check(lib.fh_sweep(plan, _ptr(aux), _ptr(paths), int(first_sweep), int(n_sweeps),
                        _stream(stream)), "fh_sweep")


def fh_logZ_grad(plan, aux, paths, anchor_slice, logZ=None, grad_aux=None, grad_t=None,
                 stream=None):
    _check(lib.fh_logZ_grad(plan, _ptr(aux), _ptr(paths), int(anchor_slice), _ptr(logZ),
                            _ptr(grad_aux), _ptr(grad_t), _stream(stream)), "fh_logZ_grad")


def fh_kinetic_energy(plan, aux, paths, anchor_slice, energy, stream=None):
    _check(lib.fh_kinetic_energy(plan, _ptr(aux), _ptr(paths), int(anchor_slice), _ptr(energy),
                                 _stream(stream)), "fh_kinetic_energy")


def fh_set_hopping(plan, t_values):
    arr = (c_double * len(t_values))(*[float(v) for v in t_values])
    _check(lib.fh_set_hopping(plan, arr), "fh_set_hopping")


def fh_get_status(plan):
    code, chain = c_int32(), c_int32()
    _check(lib.fh_get_status(plan, byref(code), byref(chain)), "fh_get_status")
    return code.value, chain.value


def fh_get_filters(plan, chain, particle, dst=None, stream=None):
    """Returns the row count; copies the rows into dst (a flat device tensor) if given."""
    rows = c_int64()
    cap = 0 if dst is None else dst.numel()
    _check(lib.fh_get_filters(plan, int(chain), int(particle), _ptr(dst), cap, byref(rows),
                              _stream(stream)), "fh_get_filters")
    return rows.value


def fh_local_update(plan, aux, paths, sweep, n_passes, stream=None):
    _check(lib.fh_local_update(plan, _ptr(aux), _ptr(paths), int(sweep), int(n_passes),
                               _stream(stream)), "fh_local_update")


def fh_measure(plan, paths, Sk=None, Cr=None, D=None, S2=None, stream=None):
    _check(lib.fh_measure(plan, _ptr(paths), _ptr(Sk), _ptr(Cr), _ptr(D), _ptr(S2),
                          _stream(stream)), "fh_measure")


def fh_measure_noalloc(plan, paths, Sk=None, Cr=None, D=None, S2=None, stream=None):
    _check(lib.fh_measure_noalloc(plan, _ptr(paths), _ptr(Sk), _ptr(Cr), _ptr(D), _ptr(S2),
                                  _stream(stream)), "fh_measure_noalloc")


def fh_set_permutation(plan, perm):
    """perm: host sequence [particles] (chain-local indices, packed like logZ)."""
    arr = (c_int32 * len(perm))(*[int(v) for v in perm])
    _check(lib.fh_set_permutation(plan, arr), "fh_set_permutation")


def fh_get_permutation(plan, particles, n_chains):
    """(perm list [particles], sign list [n_chains])."""
    perm = (c_int32 * particles)()
    sign = (c_int32 * n_chains)()
    _check(lib.fh_get_permutation(plan, perm, sign), "fh_get_permutation")
    return list(perm), list(sign)


def fh_permutation_update(plan, paths, sweep, n_passes, stream=None):
    _check(lib.fh_permutation_update(plan, _ptr(paths), int(sweep), int(n_passes),
                                     _stream(stream)), "fh_permutation_update")


def fh_mala_field(plan, aux, paths, anchor_slice, eps, sweep, accepted=None, stream=None):
    _check(lib.fh_mala_field(plan, _ptr(aux), _ptr(paths), int(anchor_slice), float(eps),
                             int(sweep), _ptr(accepted), _stream(stream)), "fh_mala_field")


def fh_get_radix_plan(plan, chain):
    """The radix stage order of chain `chain`'s FFTs, as a tuple of radices."""
    rad = (c_int32 * 6)()
    n = c_int32()
    _check(lib.fh_get_radix_plan(plan, int(chain), rad, byref(n)), "fh_get_radix_plan")
    return tuple(rad[i] for i in range(n.value))


def fh_strerror(code):
    return lib.fh_strerror(int(code)).decode()


def fh_debug_rescue(plan, cap=0):
    """(queued blocks of the last forward pass incl. its backward, blocks redrawn in FP64 since
    the previous call, [(chain, particle, block)] of the first `cap` queued blocks, chains
    queued whole)."""
    import numpy as np
    last, whole, total = c_int32(), c_int32(), c_int64()
    buf = np.zeros((max(cap, 1), 3), dtype=np.int32)
    _check(lib.fh_debug_rescue(plan, byref(last), byref(whole), byref(total),
                               buf.ctypes.data_as(POINTER(c_int32)), cap), "fh_debug_rescue")
    n = min(cap, last.value)
    return last.value, total.value, [tuple(int(v) for v in buf[i]) for i in range(n)], whole.value


def fh_debug_rescue_causes(plan):
    """Blocks queued for the FP64 re-filter since fh_init, by floor: (step mass, end weight,
    backward draw, FP32 FFT forward)."""
    import numpy as np
    buf = np.zeros(4, dtype=np.int32)
    _check(lib.fh_debug_rescue_causes(plan, buf.ctypes.data_as(POINTER(c_int32))),
           "fh_debug_rescue_causes")
    return buf


def fh_debug_rescue_holds(plan, n_chains):
    """Per chain, the forward passes it stays on the FP64 re-filter (FP32 plans)."""
    import numpy as np
    buf = np.zeros(n_chains, dtype=np.int32)
    _check(lib.fh_debug_rescue_holds(plan, buf.ctypes.data_as(POINTER(c_int32))),
           "fh_debug_rescue_holds")
    return buf


def fh_debug_representatives(plan):
    """The representative map of the shared forward filters (numpy int32, empty when the plan
    shares none)."""
    import numpy as np
    n = c_int64()
    _check(lib.fh_debug_representatives(plan, None, 0, byref(n)), "fh_debug_representatives")
    buf = np.zeros(max(n.value, 1), dtype=np.int32)
    _check(lib.fh_debug_representatives(plan, buf.ctypes.data_as(POINTER(c_int32)), n.value,
                                        byref(n)), "fh_debug_representatives")
    return buf[:n.value]


def fh_debug_sweep_times(plan):
    """(forward, backward, FP64 re-filter, its phase A beside the first two) milliseconds of the
    last sweep (timing enabled)."""
    ms = (ctypes.c_float * 4)()
    _check(lib.fh_debug_sweep_times(plan, ms), "fh_debug_sweep_times")
    return ms[0], ms[1], ms[2], ms[3]
