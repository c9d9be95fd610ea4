"""CPU-side checks of the HIP library: it loads, exports every declared entry point, validates
descriptors before touching the device, and its host-side mirrors of the device arithmetic
(FFT stages, kernel table, Philox) agree with numpy / the oracle. No GPU compute is called."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fh.h", "fh_debug.h")]


@pytest.fixture(scope="module")
def fhmc():
    from paper_2510_13866_amd import fhmc as m
    return m


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(fh_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(fhmc):
    names = declared_functions()
    assert "fh_init" in names and "fh_sweep" in names and "fh_logZ_grad" in names
    for n in names:
        assert hasattr(fhmc.lib, n), n


def test_binding_leaves_one_hip_runtime_in_the_process():
    """PyTorch ships HIP and HSA runtimes under the system ROCm sonames. Importing the binding
    first (before torch) must still leave one runtime of each in the process, so that torch's
    device pointers and streams are valid in the library (checked in a fresh interpreter)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2510_13866_amd import fhmc\n"
            "import torch\n"
            "libs = set(l.split()[-1] for l in open('/proc/self/maps') if '/' in l)\n"
            "print(sum('libamdhip64' in l for l in libs), sum('libhsa-runtime64' in l for l in libs))\n"
            % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    n_hip, n_hsa = (int(v) for v in out.stdout.split()[-2:])
    assert n_hip == 1 and n_hsa == 1, out.stdout


def test_library_resolves_every_symbol_at_load(fhmc):
    """Loading with immediate binding fails on any symbol the library uses but does not define
    (a shared library links without them)."""
    lib = ctypes.CDLL(fhmc._LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)
    assert lib.fh_strerror is not None


def test_struct_sizes_match_header(fhmc):
    assert ctypes.sizeof(fhmc.fh_chain_desc) == 56
    assert ctypes.sizeof(fhmc.fh_chain_layout) == 56


@pytest.mark.parametrize("L", [2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 32, 36, 48, 64])
@pytest.mark.parametrize("inverse", [0, 1])
def test_host_fft_stages_match_numpy(fhmc, L, inverse):
    rng = np.random.default_rng(L)
    z = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))  # [y, x]
    buf = np.empty(2 * L * L)
    buf[0::2] = z.real.ravel()
    buf[1::2] = z.imag.ravel()
    rc = fhmc.lib.fh_debug_fft2d_host(buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), L,
                                      inverse)
    assert rc == 0
    got = (buf[0::2] + 1j * buf[1::2]).reshape(L, L)
    ref = np.fft.fft2(z) if not inverse else np.fft.ifft2(z) * L * L
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_host_fft_rejects_unsupported_lengths(fhmc):
    buf = np.zeros(2 * 25)
    p = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert fhmc.lib.fh_debug_fft2d_host(p, 5, 0) == fhmc.FH_ERR_UNSUPPORTED
    assert fhmc.lib.fh_debug_fft2d_host(p, 1, 0) == fhmc.FH_ERR_UNSUPPORTED


@pytest.mark.parametrize("L,t,dtau", [(2, 1.0, 0.1), (3, 1.0, 0.1), (4, 1.0, 0.1), (12, 1.0, 0.05),
                                      (32, 1.0, 0.05), (16, 0.7, 0.3)])
def test_kernel_table_matches_oracle(fhmc, L, t, dtau):
    from oracle import lattice
    out = np.zeros(L)
    assert fhmc.lib.fh_debug_kernel_table(L, t, dtau, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    ref = lattice.g_1d(L, t, dtau)
    assert np.allclose(out, ref, rtol=1e-13, atol=0)
    assert np.all(out > 0)


def test_philox_matches_oracle_and_numpy(fhmc):
    from oracle import philox
    rng = np.random.default_rng(9)
    out = (ctypes.c_uint64 * 4)()
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        k = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        assert fhmc.lib.fh_debug_philox(*c, *k, out) == 0
        ref = philox.philox4x64(*[np.uint64(v) for v in c], np.uint64(k[0]), np.uint64(k[1]))
        assert list(out) == [int(r) for r in ref]
        if c[0] >= 1:
            bg = np.random.Philox(key=np.array(k, dtype=np.uint64),
                                  counter=np.array([c[0] - 1] + c[1:], dtype=np.uint64))
            assert list(out) == [int(v) for v in bg.random_raw(4)]


def bad_descs():
    import synth
    good = synth.half_filled(4, 16, synth.HS_GAUSS, 4.0, 0.1, 0)
    import dataclasses
    r = dataclasses.replace
    return [r(good, L=1), r(good, L=5), r(good, L=128), r(good, L_tau=1), r(good, n_up=-1),
            r(good, n_up=0, n_dn=0), r(good, hs_kind=7), r(good, block_len=1),
            r(good, block_len=17), r(good, t=0.0), r(good, t=float("nan")), r(good, dtau=-0.1),
            r(good, U=float("inf")), r(good, hs_kind=synth.HS_HIRSCH, U=-1.0)]


def test_init_validates_before_touching_the_device(fhmc):
    for d in bad_descs():
        with pytest.raises(fhmc.FhError) as e:
            fhmc.fh_init([d], fhmc.FH_FP64)
        assert e.value.code in (fhmc.FH_ERR_INVALID_ARG, fhmc.FH_ERR_UNSUPPORTED), d
    import synth
    good = synth.half_filled(4, 16, synth.HS_GAUSS, 4.0, 0.1, 0)
    with pytest.raises(fhmc.FhError) as e:
        fhmc.fh_init([good], 9)
    assert e.value.code == fhmc.FH_ERR_INVALID_ARG
    with pytest.raises(fhmc.FhError) as e:
        fhmc.fh_init([good], fhmc.FH_FP64, flags=0x100)
    assert e.value.code == fhmc.FH_ERR_INVALID_ARG


def test_null_plan_calls_are_rejected(fhmc):
    assert fhmc.lib.fh_destroy(None) == fhmc.FH_ERR_INVALID_ARG
    assert fhmc.lib.fh_sweep(None, None, None, 0, 1, None) == fhmc.FH_ERR_INVALID_ARG
    assert fhmc.lib.fh_get_status(None, None, None) == fhmc.FH_ERR_INVALID_ARG
    assert fhmc.lib.fh_debug_rescue_causes(None, None) == fhmc.FH_ERR_INVALID_ARG
    assert fhmc.lib.fh_debug_forward_kernels(None, None) == fhmc.FH_ERR_INVALID_ARG
    assert fhmc.fh_strerror(fhmc.FH_ERR_STATE) == "call order violated"


def _radix_orders_brute(L):
    """Every sequence over {2, 3, 4} of length <= 6 with product L (independent enumeration)."""
    out = set()
    for n in range(1, 7):
        for seq in itertools.product((2, 3, 4), repeat=n):
            if int(np.prod(seq)) == L:
                out.add(seq)
    return out


def _smooth_lengths():
    res = []
    for L in range(2, 65):
        r = L
        for f in (2, 3):
            while r % f == 0:
                r //= f
        if r == 1:
            res.append(L)
    return res


@pytest.mark.parametrize("L", _smooth_lengths())
def test_radix_order_candidates_are_every_valid_order(fhmc, L):
    cap = 200
    out = np.zeros(cap * 7, dtype=np.int32)
    n = fhmc.lib.fh_debug_radix_orders(L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    got = [tuple(out[7 * k + 1:7 * k + 1 + out[7 * k]]) for k in range(n)]
    assert len(got) == len(set(got)), "duplicate candidates"
    assert set(got) == _radix_orders_brute(L)


def test_radix_order_candidates_reject_unsupported(fhmc):
    out = np.zeros(7, dtype=np.int32)
    p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    for L in (1, 5, 7, 10, 81, 96):
        assert fhmc.lib.fh_debug_radix_orders(L, p, 1) == 0


@pytest.mark.parametrize("L", [6, 8, 12, 16, 24, 32, 48, 64])
def test_every_radix_order_computes_the_dft(fhmc, L):
    """Each stage order the autotuner may choose, run through the kernels' stage code on the
    host, against numpy's FFT (forward and unscaled inverse)."""
    cap = 200
    out = np.zeros(cap * 7, dtype=np.int32)
    n = fhmc.lib.fh_debug_radix_orders(L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    rng = np.random.default_rng(L)
    x = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    ref_f = np.fft.fft2(x)
    ref_i = np.fft.ifft2(x) * L * L
    for k in range(n):
        ns = int(out[7 * k])
        rad = np.ascontiguousarray(out[7 * k + 1:7 * k + 1 + ns], dtype=np.int32)
        for inverse, ref in ((0, ref_f), (1, ref_i)):
            buf = np.empty(2 * L * L)
            buf[0::2], buf[1::2] = x.real.ravel(), x.imag.ravel()
            rc = fhmc.lib.fh_debug_fft2d_host_plan(
                buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), L,
                rad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ns, inverse)
            assert rc == 0
            y = (buf[0::2] + 1j * buf[1::2]).reshape(L, L)
            assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref)), (L, tuple(rad), inverse)


def test_fft_plan_rejects_invalid_orders(fhmc):
    buf = np.zeros(2 * 64)
    p = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for L, rad in ((8, [4, 4]), (8, [8]), (12, [4, 3, 1]), (8, [2, 2, 2, 1]), (6, [5, 1])):
        r = np.array(rad, dtype=np.int32)
        assert fhmc.lib.fh_debug_fft2d_host_plan(
            p, L, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(rad), 0) == fhmc.FH_ERR_INVALID_ARG
