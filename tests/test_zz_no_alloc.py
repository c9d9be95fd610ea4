"""fh_measure_noalloc (per-slice rows in the library's static device array) against fh_measure
(rows in a buffer the plan allocates) through the C ABI: identical outputs on two calls in a row,
the second on a smaller batch, and the size limit."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _outputs(S):
    total = sum(lay["N"] for lay in S.layouts)
    Sk = torch.full((total,), float("nan"), dtype=torch.float64, device=S.device)
    Cr = torch.full_like(Sk, float("nan"))
    D = torch.full((len(S.descs),), float("nan"), dtype=torch.float64, device=S.device)
    S2 = torch.full_like(D, float("nan"))
    return Sk, Cr, D, S2


def test_measure_noalloc_equals_measure(gpu):
    from paper_2510_13866_amd import fhmc
    from paper_2510_13866_amd.sampler import Sampler
    big = [synth.half_filled(16, 64, synth.HS_HIRSCH, 4.0, 0.0625, seed=s) for s in range(3)] + [
        synth.ChainDesc(L=12, L_tau=24, n_up=60, n_dn=70, hs_kind=synth.HS_GAUSS, block_len=0,
                        t=1.0, U=4.0, dtau=0.05, seed=9),
        synth.ChainDesc(L=6, L_tau=10, n_up=18, n_dn=5, hs_kind=synth.HS_GAUSS, block_len=4,
                        t=1.0, U=3.0, dtau=0.1, seed=7)]
    small = [synth.config_small_fp64()[0],
             synth.ChainDesc(L=3, L_tau=7, n_up=4, n_dn=3, hs_kind=synth.HS_HIRSCH, block_len=0,
                             t=1.0, U=4.0, dtau=0.1, seed=5)]
    stream = torch.cuda.current_stream()
    for k, descs in enumerate((big, small)):   # the second call on a smaller batch
        print("measure_noalloc call", k, [(d.L, d.L_tau, d.n_particles) for d in descs], flush=True)
        S = Sampler(descs, fhmc.FH_FP64)
        P = S.pack_paths([synth.random_walk_paths(d, 40 + 10 * k + i) for i, d in enumerate(descs)])
        ref, got = _outputs(S), _outputs(S)
        fhmc.fh_measure(S.plan, P, *ref, stream)
        fhmc.fh_measure_noalloc(S.plan, P, *got, stream)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b)
        assert S.status() == (0, -1)
        S.close()


def test_measure_noalloc_rejects_plans_beyond_its_array(gpu):
    from paper_2510_13866_amd import fhmc
    from paper_2510_13866_amd.sampler import Sampler
    # two chains of 32 x 32 sites and 2048 slices: 2 * 2^22 + 2 * 4096 doubles of rows, above 2^22
    descs = [synth.ChainDesc(L=32, L_tau=2048, n_up=1, n_dn=0, hs_kind=synth.HS_GAUSS, block_len=0,
                             t=1.0, U=4.0, dtau=0.05, seed=s) for s in range(2)]
    S = Sampler(descs, fhmc.FH_FP64)
    P = S.pack_paths([synth.initial_paths(d) for d in descs])
    Sk, Cr, D, S2 = _outputs(S)
    with pytest.raises(fhmc.FhError) as e:
        fhmc.fh_measure_noalloc(S.plan, P, Sk, Cr, D, S2)
    assert e.value.code == fhmc.FH_ERR_UNSUPPORTED
    fhmc.fh_measure(S.plan, P, Sk, Cr, D, S2)   # the allocating entry point still serves it
    torch.cuda.synchronize()
    assert np.all(np.isfinite(D.cpu().numpy()))
    assert S.status() == (0, -1)
    S.close()
