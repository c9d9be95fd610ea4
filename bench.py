#!/usr/bin/env python3
"""Throughput of the FFBS worldline sweep on one MI355X: site-slice updates/s.

Workload: 16 chains of a 32x32 periodic lattice, L_tau = 160 (beta = 8, dtau = 0.05), U = 4,
512 + 512 worldlines per chain, Gaussian HS field, 500 sweeps; synthetic seeded inputs already
resident in HBM. One step = one sweep of the chain as it runs (forward filter + backward sample
of every worldline, then the Gibbs draw of every field value, for all 16 chains), replayed from
a captured hipGraph, each sweep continuing from the state the previous one left. The warmup
sweeps start from the initial state (the first one captures the graph); the timed sweeps carry
the chain on, 500 sweeps in all by default. The chain clusters within a few sweeps (the
worldlines are distinguishable while the permutation is the identity), so the timed sweeps
include the transitional ones, whose out-of-range blocks the FP32 plan re-filters in FP64, and
then the settled state; `per_sweep_ms` gives both parts, and the same chain is also run at
U = 2 and U = 6.

Prints one JSON line. `roofline` is for the dominant kernel (the longer of the forward filter and
the backward sampler per sweep), timed with HIP events on the stream it runs on; `cpu_baseline` times the FP64 oracle on host cores on a
bounded sample (one chain, six sweeps) and scales it to the same unit. `err_vs_fp64_plain`
compares the FP32 plan's log Z and filters with the FP64 plain path's on the same GPU and the
same states (the initial one and a transitional one).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_mfma3": 2}
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFS = 2500.0   # dense bf16 matrix-core peak
FP64_PEAK_TFS = 78.6     # FP64 matrix-core peak
FP32_VECTOR_PEAK_TFS = 157.3
KERNEL_SOURCES = {"forward": {"fp32_mfma3": "fh_mfma.hip", "fp32": "fh_kernels.hip",
                              "fp64": "fh_mfma.hip"},
                  "backward": {"fp32_mfma3": "fh_kernels.hip", "fp32": "fh_kernels.hip",
                               "fp64": "fh_kernels.hip"}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=499)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32_mfma3", choices=sorted(PRECISIONS))
    ap.add_argument("--chains", type=int, default=16)
    ap.add_argument("--U", type=float, default=4.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-error", action="store_true", help="skip the filter error sample against the FP64 plain path")
    ap.add_argument("--no-other-u", action="store_true",
                    help="skip the same chain at U = 2 and U = 6")
    ap.add_argument("--full-row-draw", action="store_true",
                    help="backward draws scan whole filter rows (FH_FLAG_FULL_ROW_DRAW)")
    ap.add_argument("--autotune", action="store_true",
                    help="FFT plans (--precision fp32 or fp64 with L > 32): time every radix-2/3/4 "
                         "stage order per lattice size at plan creation (FH_FLAG_AUTOTUNE)")
    ap.add_argument("--grad-checkpoint", action="store_true",
                    help="grad / mala workloads: the adjoint keeps every ceil(sqrt(L_tau))-th "
                         "ring row and recomputes the rest (FH_FLAG_GRAD_CHECKPOINT)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--workload", default="32x32",
                    choices=["32x32", "uneven", "hirsch16", "grad", "small", "paper64", "paper32",
                             "local", "measure", "mala", "perm", "64x64"],
                    help="32x32: the headline workload; the others time the remaining "
                         "configurations (uneven batch, 16x16 Ising field, adjoint, 4x4 FP64) "
                         "and the paper's own shape (32x32, L_tau=1024, blocks of 64 or 32)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(name):
    import hashlib
    path = os.path.join(ROOT, "paper_2510_13866_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel, precision, kernel_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the same kernel and on the current kernel source; None otherwise."""
    src = KERNEL_SOURCES[kernel][precision]
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s_%s_32x32_Ltau160.md" % (kernel, precision))
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_json:"):
            rec = json.loads(line[len("traffic_json:"):])
            if rec.get("source_sha256") != source_sha(src):
                return None
            if not rec.get("kernel", "").startswith(kernel_name):
                return None
            return rec["fetch_bytes"] + rec["write_bytes"]
    return None


def run_chain(S, A, P, first, n, stream):
    """n consecutive sweeps (sweep indices first .. first + n - 1) continuing the chain in A, P,
    with a HIP event after each; returns (total ms, [ms of each sweep])."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    with torch.cuda.stream(stream):
        for i in range(n):
            S.sweep(A, P, first + i, 1, stream)
            ev[i + 1].record(stream)
    torch.cuda.synchronize()
    each = [ev[i].elapsed_time(ev[i + 1]) for i in range(n)]
    return ev[0].elapsed_time(ev[n]), each


def chain_summary(each, warmup):
    """Per-sweep figures of a timed chain: the first ten timed sweeps one by one, and the median
    of the second half (the settled state)."""
    import statistics
    half = each[len(each) // 2:] or each
    return {"first_timed_sweep_index": warmup,
            "first_10_ms": [round(x, 3) for x in each[:10]],
            "settled_median_ms": round(statistics.median(half), 4),
            "max_ms": round(max(each), 3)}


def copy_calibration(stream):
    """A plain device copy of 1 GiB, five times: its FETCH_SIZE / WRITE_SIZE counters give the
    factor that turns those counters into HBM bytes."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(5):
            b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def err_vs_fp64_plain(precision, descs, aux, paths, sweep, stream):
    """The FP32 plan against the FP64 plain path (an FP64 plan on the same GPU; its filters match
    the FP64 oracle to 1e-11 and its log Z to 1e-12 in the parity tests) on one state (aux as the
    FP32 plan holds it, paths) and sweep index: the relative log Z error of every worldline, and
    the normwise filter error of every stored row of 8 worldlines of chain 0, together with the
    number of blocks the FP32 plan re-filtered in FP64 on that state."""
    import numpy as np
    import torch
    from paper_2510_13866_amd import fhmc
    from paper_2510_13866_amd.sampler import Sampler
    out = {}
    S32 = Sampler(descs, precision)
    S64 = Sampler(descs, fhmc.FH_FP64)
    lz = []
    for S in (S32, S64):
        A, P = S.pack_aux(aux), S.pack_paths(paths)
        t = S.forward_filter(A, P, sweep, stream)
        torch.cuda.synchronize()   # the library wrote t on `stream`
        lz.append(t.cpu().numpy())
    rel = np.abs(lz[0] - lz[1]) / (1.0 + np.abs(lz[1]))
    errs = []
    for p in range(0, 1024, 128):
        ref = S64.filters(0, p)
        errs.extend(np.linalg.norm(S32.filters(0, p) - ref, axis=1) / np.linalg.norm(ref, axis=1))
    queued, _, _, whole = fhmc.fh_debug_rescue(S32.plan)
    for S in (S32, S64):
        code, _ = S.status()
        if code != 0:
            raise RuntimeError("device status in the error sample: " + fhmc.fh_strerror(code))
        S.close()
    out["logz_err"] = {"max": float(rel.max()), "median": float(np.median(rel)),
                       "worldlines": int(rel.size), "measure": "|dlogZ| / (1 + |logZ|)"}
    out["filter_err"] = {"max": float(np.max(errs)), "median": float(np.median(errs)),
                         "sample": "8 worldlines of chain 0, every stored row"}
    out["blocks_refiltered_fp64"] = int(queued)
    out["chains_refiltered_whole"] = int(whole)
    return out


def cpu_baseline(desc, aux, paths, n_sweeps=6):
    """The oracle as it stands, one chain, n_sweeps sweeps, on the host cores."""
    import numpy as np
    from oracle import sweep as osweep
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    tab = osweep.ChainTables(desc)
    t0 = time.perf_counter()
    for s in range(n_sweeps):
        aux, paths, _ = osweep.sweep(desc, aux, paths, s, tab)
    dt = time.perf_counter() - t0
    return {"value": n_sweeps * desc.N * desc.L_tau / dt, "unit": "site-slice updates/s",
            "cores": threads, "kind": "oracle",
            "sample": "1 chain x %d sweeps of 32x32, L_tau=160, 512+512 worldlines (%.1f s)"
                      % (n_sweeps, dt)}


def other_workload(args):
    """Secondary workloads: one JSON line each, same timing rules as the headline run."""
    import numpy as np
    import torch

    import synth
    from paper_2510_13866_amd import fhmc
    from paper_2510_13866_amd.sampler import Sampler

    prec_name = args.precision
    if args.workload == "uneven":
        descs = synth.config_uneven(256)
        label = "FFBS sweep, 256 uneven chains (L in {8,12,16,24,32}, L_tau in {40,80,160}, " \
                "dtau=0.05, U~U[2,6], half filling, Gaussian/Ising 50/50)"
    elif args.workload == "hirsch16":
        descs = synth.config_16x16_hirsch(64)
        label = "FFBS sweep, 64 chains x 16x16 lattice, L_tau=64, dtau=0.0625, U=4, 128+128 " \
                "worldlines, Ising field"
    elif args.workload in ("paper64", "paper32"):
        B = 64 if args.workload == "paper64" else 32
        descs = synth.config_paper_shape(32, B, 4)
        label = "FFBS sweep, 4 chains x 32x32 lattice, L_tau=1024 (beta=32, dtau=1/32), " \
                "FFBS blocks of %d slices, U=4, 512+512 worldlines, Gaussian field" % B
    elif args.workload == "64x64":
        descs = [synth.half_filled(64, 160, synth.HS_GAUSS, 4.0, 0.05, seed=s) for s in range(4)]
        label = "FFBS sweep, 4 chains x 64x64 lattice, L_tau=160, dtau=0.05, U=4, 2048+2048 " \
                "worldlines, Gaussian field"
    elif args.workload == "small":
        descs = synth.config_small_fp64()
        prec_name = "fp64"
        label = "FFBS sweep, 1 chain x 4x4 lattice, L_tau=16, dtau=0.1, U=4, 8+8 worldlines, " \
                "Gaussian field"
    elif args.workload == "mala":
        descs = synth.config_gradient(8)
        label = "MALA move of the Gaussian field (two log Z_path gradients + proposal + " \
                "accept), 8 chains x 32x32, L_tau=128, dtau=0.05, U=4, 512+512 worldlines"
    elif args.workload == "measure":
        descs = synth.config_32x32(4.0, 16)
        label = "equal-time observables S(k), C(r), D, local moment (Sec. 4), 16 chains x " \
                "32x32 lattice, L_tau=160, 512+512 worldlines"
    elif args.workload == "local":
        descs = synth.config_32x32(4.0, 16)
        label = "local link updates (Sec. 3.5.1), 16 chains x 32x32 lattice, L_tau=160, " \
                "512+512 worldlines, Gaussian field, 4 passes per step"
    elif args.workload == "perm":
        descs = synth.config_32x32(4.0, 16)
        label = "FFBS sweep with random reconnections at tau=beta plus 2 passes of pair swaps " \
                "(Sec. 3.5.6), 16 chains x 32x32 lattice, L_tau=160, 512+512 worldlines"
    else:
        descs = synth.config_gradient(8)
        label = "log Z_path and its gradient (field and t), 8 chains x 32x32, L_tau=128, " \
                "dtau=0.05, U=4, 512+512 worldlines, Gaussian field"
    prec = PRECISIONS[prec_name]
    aux = [synth.initial_aux(d) for d in descs]
    paths = [synth.initial_paths(d) for d in descs]
    stream = torch.cuda.Stream()
    sites = sum(d.N * d.L_tau for d in descs)
    log("bench: %s workload, %s, %d chains" % (args.workload, prec_name, len(descs)))
    flags = fhmc.FH_FLAG_GRAPH | (fhmc.FH_FLAG_AUTOTUNE if args.autotune else 0)
    if args.grad_checkpoint:
        flags |= fhmc.FH_FLAG_GRAD_CHECKPOINT
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    S = Sampler(descs, prec, flags)
    A, P = S.pack_aux(aux), S.pack_paths(paths)
    torch.cuda.synchronize()
    extra = {}
    if args.grad_checkpoint:
        extra["grad_checkpoint"] = True
    if args.autotune:  # the stage order chosen per lattice size
        chosen = {}
        for c, d in enumerate(descs):
            if d.L not in chosen:
                chosen[d.L] = list(fhmc.fh_get_radix_plan(S.plan, c))
        extra["radix_plans"] = {str(L): v for L, v in sorted(chosen.items())}
    if args.workload == "grad":
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            logZ = torch.empty(len(descs), dtype=torch.float64, device="cuda")
            gA = torch.empty_like(A)
            gT = torch.empty(len(descs), dtype=torch.float64, device="cuda")
            for _ in range(args.warmup):
                fhmc.fh_logZ_grad(S.plan, A, P, 0, logZ, gA, gT, stream)
            torch.cuda.synchronize()
            # device memory taken by the plan and the call's buffers (the library allocates
            # with hipMalloc; free memory before the plan and after the warm-up calls)
            extra["device_bytes_plan_and_buffers"] = free0 - torch.cuda.mem_get_info()[0]
            e0.record(stream)
            for i in range(args.steps):
                fhmc.fh_logZ_grad(S.plan, A, P, i % descs[0].L_tau, logZ, gA, gT, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        metric = "gradient evaluations/s (log Z_path, d/d field, d/d t) at 32x32 L_tau=128, 8 chains"
        value = args.steps / (ms / 1e3)
        unit = "evaluations/s"
        extra["site_slices_per_s"] = sites * args.steps / (ms / 1e3)
    elif args.workload == "mala":
        acc = torch.empty(len(descs), dtype=torch.int32, device="cuda")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            for i in range(max(1, args.warmup)):
                fhmc.fh_mala_field(S.plan, A, P, 0, 0.02, i, acc, stream)
            torch.cuda.synchronize()
            extra["device_bytes_plan_and_buffers"] = free0 - torch.cuda.mem_get_info()[0]
            e0.record(stream)
            for i in range(args.steps):
                fhmc.fh_mala_field(S.plan, A, P, i % descs[0].L_tau, 0.02, 100 + i, acc, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        metric = "MALA field moves/s (all 8 chains per move; 32x32, L_tau=128)"
        value = args.steps / (ms / 1e3)
        unit = "moves/s"
        extra["last_accepted"] = acc.cpu().tolist()
    elif args.workload == "measure":
        total = sum(d.N for d in descs)
        Sk = torch.empty(total, dtype=torch.float64, device="cuda")
        Cr = torch.empty_like(Sk)
        Dv = torch.empty(len(descs), dtype=torch.float64, device="cuda")
        S2 = torch.empty_like(Dv)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            for _ in range(max(1, args.warmup)):
                fhmc.fh_measure(S.plan, P, Sk, Cr, Dv, S2, stream)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                fhmc.fh_measure(S.plan, P, Sk, Cr, Dv, S2, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        metric = "measured slices/s (S(k), C(r), D, local moment; 32x32, 16 chains)"
        value = sum(d.L_tau for d in descs) * args.steps / (ms / 1e3)
        unit = "slices/s"
    elif args.workload == "local":
        passes = 4
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            for i in range(args.warmup):
                fhmc.fh_local_update(S.plan, A, P, i, passes, stream)
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(args.steps):
                fhmc.fh_local_update(S.plan, A, P, args.warmup + i, passes, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        proposals = sum(d.n_particles * d.L_tau for d in descs) * passes
        metric = "local link proposals/s (32x32, L_tau=160, 16 chains)"
        value = proposals * args.steps / (ms / 1e3)
        unit = "proposals/s"
    elif args.workload == "perm":
        rng = np.random.default_rng(2510)
        S.set_permutation([np.concatenate([rng.permutation(d.n_up),
                                           d.n_up + rng.permutation(d.n_dn)]) for d in descs])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):  # one chain run on from the initial state
            for i in range(args.warmup):
                S.sweep(A, P, i, 1, stream)
                fhmc.fh_permutation_update(S.plan, P, i, 2, stream)
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(args.steps):
                S.sweep(A, P, args.warmup + i, 1, stream)
                fhmc.fh_permutation_update(S.plan, P, args.warmup + i, 2, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        metric = "site-slice updates/s with reconnections and pair swaps (32x32, L_tau=160, " \
                 "16 chains)"
        value = sites * args.steps / (ms / 1e3)
        unit = "site-slice updates/s"
        _, signs = S.permutation()
        extra["sign_sum"] = int(np.sum(signs))
    else:  # one chain run on from the initial state: warmup sweeps, then the timed ones
        run_chain(S, A, P, 0, args.warmup, stream)
        fhmc.fh_debug_rescue(S.plan)
        ms, each = run_chain(S, A, P, args.warmup, args.steps, stream)
        metric = "site-slice updates/s (%s)" % args.workload
        value = sites * args.steps / (ms / 1e3)
        unit = "site-slice updates/s"
        extra["per_sweep_ms"] = chain_summary(each, args.warmup)
        extra["blocks_redrawn_fp64"] = int(fhmc.fh_debug_rescue(S.plan)[1])
    code, _ = S.status()
    if code != 0:
        raise RuntimeError("device status: " + fhmc.fh_strerror(code))
    S.close()
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec_name == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": label, "chains": len(descs), "precision": prec_name,
                      "site_slices_per_step": sites, "graph": True, "autotune": args.autotune}}
    out.update(extra)
    log("  %.3f ms/step, %.4g %s" % (ms / args.steps, value, unit))
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (chains are "
              "independent, so each GPU would run its own share of them). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "32x32":
        other_workload(args)
        return
    import numpy as np
    import torch

    import synth
    from paper_2510_13866_amd import fhmc
    from paper_2510_13866_amd.sampler import Sampler

    descs = synth.config_32x32(args.U, n_chains=args.chains)
    aux = [synth.initial_aux(d) for d in descs]
    paths = [synth.initial_paths(d) for d in descs]
    stream = torch.cuda.Stream()
    prec = PRECISIONS[args.precision]
    if args.calibrate_copy:
        copy_calibration(stream)
    sites = sum(d.N * d.L_tau for d in descs)

    log("bench: %s, %d chains 32x32 L_tau=160, warmup %d, steps %d (one chain run on)" %
        (args.precision, args.chains, args.warmup, args.steps))
    draw_flag = fhmc.FH_FLAG_FULL_ROW_DRAW if args.full_row_draw else 0

    def chain(U, precision, flags, warmup, steps):
        """The headline chain at coupling U: warmup sweeps from the initial state, then `steps`
        timed sweeps continuing it; the status is checked after the timed sweeps."""
        ds = synth.config_32x32(U, n_chains=args.chains)
        S = Sampler(ds, precision, fhmc.FH_FLAG_GRAPH | flags)
        A = S.pack_aux([synth.initial_aux(d) for d in ds])
        P = S.pack_paths([synth.initial_paths(d) for d in ds])
        run_chain(S, A, P, 0, warmup, stream)
        fhmc.fh_debug_rescue(S.plan)  # restart the count of FP64-redrawn blocks
        ms, each = run_chain(S, A, P, warmup, steps, stream)
        code, _ = S.status()
        if code != 0:
            raise RuntimeError("device status after the timed sweeps (U=%g): %s" %
                               (U, fhmc.fh_strerror(code)))
        _, redrawn, last, _ = fhmc.fh_debug_rescue(S.plan, cap=1 << 20)
        per_chain = [0] * len(ds)
        for (c, _, _) in last:
            per_chain[c] += 1
        log("  U=%g: blocks queued for FP64 in the last sweep, per chain: %s" % (U, per_chain))
        causes = fhmc.fh_debug_rescue_causes(S.plan)
        log("  U=%g: blocks queued since the start, by floor (step, end, draw, fft): %s" %
            (U, list(causes)))
        return S, A, P, ms, each, redrawn, causes

    S, A, P, ms, each, redrawn, causes = chain(args.U, prec, draw_flag, args.warmup, args.steps)
    ms_step = ms / args.steps
    value = sites * args.steps / (ms / 1e3)
    n_blocks = sum(d.n_particles for d in descs) * args.steps
    log("  %.3f ms/sweep, %.3e site-slice updates/s; blocks redrawn in FP64: %d of %d" %
        (ms_step, value, redrawn, n_blocks))
    extra = {"per_sweep_ms": chain_summary(each, args.warmup),
             "blocks_redrawn_fp64": {"count": int(redrawn), "of": int(n_blocks)},
             "fp64_queue_causes": {"step_floor": int(causes[0]), "end_weight": int(causes[1]),
                                   "draw_floor": int(causes[2]), "fft_forward": int(causes[3]),
                                   "counted": "blocks queued by the FP32 kernels since the "
                                              "plan was made, warmup included"}}
    log("  per sweep: %s" % extra["per_sweep_ms"])

    # The kernels of the timed sweeps, timed with HIP events the library records in each sweep
    # (fh_debug_sweep_timing) around the forward-filter kernels, the backward kernels and the
    # FP64 re-filter: the same chain is run again from the same input, eagerly (it is
    # deterministic, so it passes through the same states; checked below), reading the events
    # after every sweep, and the segments are averaged over the timed sweeps. Per sweep it also
    # counts the chains the FP32 kernels worked on: the forward kernels skip the chains held on
    # the FP64 re-filter at the start of the sweep, the backward kernels every chain re-filtered
    # whole in it.
    St = Sampler(descs, prec, fhmc.FH_FLAG_GRAPH | draw_flag)
    At, Pt = St.pack_aux(aux), St.pack_paths(paths)
    assert fhmc.lib.fh_debug_sweep_timing(St.plan, 1) == 0
    run_chain(St, At, Pt, 0, args.warmup, stream)
    seg = [0.0, 0.0, 0.0, 0.0]
    fwd_chains, fwd_reps, bwd_chains = [], [], []
    d0 = descs[0]                                                  # every chain has this shape
    own = np.repeat(np.arange(d0.n_particles), 1)                  # one block per worldline
    with torch.cuda.stream(stream):
        for i in range(args.steps):
            held = fhmc.fh_debug_rescue_holds(St.plan, len(descs))
            fhmc.fh_debug_rescue(St.plan)  # the queue counters restart for this sweep
            St.sweep(At, Pt, args.warmup + i, 1, stream)
            for k, v in enumerate(fhmc.fh_debug_sweep_times(St.plan)):
                seg[k] += v
            whole = fhmc.fh_debug_rescue(St.plan)[3]
            # worldlines whose forward recursion ran: the representatives of the shared forward
            # filters (every worldline on plans that share none), in the chains not held
            rep = fhmc.fh_debug_representatives(St.plan)
            shared = len(rep) > 0
            n_rep = 0
            for c in range(len(descs)):
                if held[c] == 0:
                    n_rep += (d0.n_particles if len(rep) == 0 else
                              int(np.sum(rep[c * d0.n_particles:(c + 1) * d0.n_particles] == own)))
            fwd_chains.append(int(np.sum(held == 0)))
            fwd_reps.append(n_rep)
            bwd_chains.append(len(descs) - whole)
    torch.cuda.synchronize()
    if not (torch.equal(At, A) and torch.equal(Pt, P)):
        raise RuntimeError("the timing replay did not reproduce the timed chain")
    St.close()
    fwd_ms, bwd_ms, rescue_ms, beside_ms = (v / args.steps for v in seg)
    extra["kernel_ms_per_sweep"] = {
        "forward": round(fwd_ms, 4), "backward": round(bwd_ms, 4),
        "fp64_refilter": round(rescue_ms, 4), "fp64_refilter_beside": round(beside_ms, 4),
        "timing": "HIP events inside every timed sweep, averaged; fp64_refilter_beside is the "
                  "held chains' re-filter on the plan's side stream, concurrent with forward "
                  "and backward"}
    log("  per sweep: forward %.3f ms, backward %.3f ms, FP64 re-filter %.3f ms "
        "(+ %.3f ms beside the FP32 passes)" % (fwd_ms, bwd_ms, rescue_ms, beside_ms))
    rsz = 8 if args.precision == "fp64" else 4
    rows = d0.n_particles * (d0.L_tau - 1)                         # per chain: one block each
    N = d0.N
    w_bytes = 2 * d0.L_tau * N * rsz                               # site potentials, both spins
    # backward: the full-row kernel reads every filter row; the windowed one reads the 7 x 7
    # window around the next slice's site (half-width 3 at dtau = 0.05), fallbacks aside
    read_per_row = N * rsz if args.full_row_draw else 49 * rsz
    # per launch, averaged over the timed sweeps: the chains each launch worked on, and the
    # worldlines whose recursion the forward ran (rows written: L_tau - 1 per worldline plus the
    # end tile of the shared filters)
    fwd_avg = sum(fwd_chains) / args.steps
    rep_avg = sum(fwd_reps) / args.steps
    bwd_avg = sum(bwd_chains) / args.steps
    rows_per_rep = (d0.L_tau - 1) + (1 if shared else 0)
    algo = {"forward": round(rep_avg * rows_per_rep * N * rsz + fwd_avg * w_bytes),
            "backward": round(bwd_avg * rows * (read_per_row + 4))}  # + the drawn site (int32)
    extra["fp32_kernel_chains_per_launch"] = {
        "forward": fwd_avg, "forward_worldlines": rep_avg, "backward": bwd_avg,
        "of": len(descs), "worldlines_per_chain": d0.n_particles,
        "last_3_sweeps": {"forward": fwd_chains[-3:], "forward_worldlines": fwd_reps[-3:],
                          "backward": bwd_chains[-3:]}}
    times = {"forward": fwd_ms, "backward": bwd_ms}
    fwd_kernel = {"fp32_mfma3": "k_forward_mfma2", "fp64": "k_forward_dmfma"}.get(args.precision,
                                                                                 "k_forward_fft")
    names = {"forward": "forward filter (%s)" % fwd_kernel,
             "backward": "backward sampler (%s)" % ("k_backward_l32" if args.full_row_draw
                                                    else "k_backward_win, full-row kernels")}
    knames = {"forward": fwd_kernel,
              "backward": "k_backward_l32" if args.full_row_draw else "k_backward_win"}
    roofs = {}
    for k in ("forward", "backward"):
        gbs = algo[k] / (times[k] / 1e3) / 1e9
        roofs[k] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(k, args.precision, knames[k]),
                    "kernel": names[k], "ms_per_launch": round(times[k], 4),
                    "algorithmic_bytes_per_launch": algo[k],
                    "timing": "average over the timed sweeps",
                    # a worldline's recursion (forward) or its draws (backward) are L_tau - 1
                    # dependent steps; once the chain has clustered, the forward runs one
                    # recursion per start site (the shared forward filters), so both launches
                    # are then bound by that chain of steps, not by HBM
                    "critical_path": {
                        "dependent_steps": d0.L_tau - 1,
                        "us_per_step": round(times[k] * 1e3 / (d0.L_tau - 1), 2)}}
        log("  %s %.3f ms/launch, %.0f GB/s algorithmic" % (names[k], times[k], gbs))
    if args.precision == "fp32_mfma3":
        # the same forward launch against the matrix cores: 24 bf16 MFMA 32x32x16 per
        # worldline-step (two circulant products, three-term splits, six products each); a
        # block of L_tau slices takes L_tau - 1 steps and one more product for its end weight
        flops = round(rep_avg * d0.L_tau * 24 * 32 * 32 * 16 * 2)
        tf = flops / (times["forward"] / 1e3) / 1e12
        roofs["forward"]["matrix_cores"] = {
            "achieved": round(tf, 1), "peak": BF16_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(tf / BF16_PEAK_TFS, 4), "flops_per_launch": flops, "dtype": "bf16"}
    elif args.precision == "fp64":
        # FP64 circulant: 64 v_mfma_f64_16x16x4_f64 per worldline-step
        flops = round(rep_avg * d0.L_tau * 64 * 16 * 16 * 4 * 2)
        tf = flops / (times["forward"] / 1e3) / 1e12
        roofs["forward"]["matrix_cores"] = {
            "achieved": round(tf, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(tf / FP64_PEAK_TFS, 4), "flops_per_launch": flops, "dtype": "f64"}
    else:
        # FFT convolution in FP32 on the vector ALUs: two worldlines share one complex signal,
        # so each worldline-step costs half of a forward and an inverse complex 2D FFT
        # (5 N log2 N flops each) plus ~6N for the spectral product, W and the normaliser
        import math
        flops = int(sum(d.n_particles * d.L_tau for d in descs) * (5 * N * math.log2(N) + 6 * N))
        tf = flops / (times["forward"] / 1e3) / 1e12
        roofs["forward"]["alu"] = {
            "achieved": round(tf, 2), "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(tf / FP32_VECTOR_PEAK_TFS, 4), "flops_per_launch": flops, "dtype": "f32"}
    dominant = "forward" if fwd_ms >= bwd_ms else "backward"
    roof = roofs[dominant]
    S.close()

    if not args.no_other_u:
        for U in (2.0, 4.0, 6.0):
            if U == args.U:
                continue
            So, _, _, msu, eachu, redu, causu = chain(U, prec, draw_flag, args.warmup, args.steps)
            So.close()
            extra["U=%g" % U] = {"ms_per_step": round(msu / args.steps, 4),
                                 "value": sites * args.steps / (msu / 1e3),
                                 "per_sweep_ms": chain_summary(eachu, args.warmup),
                                 "blocks_redrawn_fp64": int(redu),
                                 "fp64_queue_causes": [int(x) for x in causu]}
            log("  U=%g: %.3f ms/sweep" % (U, msu / args.steps))
    if not args.no_error and args.precision != "fp64":
        # the FP32 plan against the FP64 plain path on the initial state and on the state after
        # two sweeps of the FP32 chain (a transitional one)
        Sx = Sampler(descs, prec, fhmc.FH_FLAG_GRAPH)
        Ax, Px = Sx.pack_aux(aux), Sx.pack_paths(paths)
        errs = {"initial": err_vs_fp64_plain(prec, descs, Sx.unpack_aux(Ax), paths, 0, stream)}
        run_chain(Sx, Ax, Px, 0, 2, stream)
        errs["after_2_sweeps"] = err_vs_fp64_plain(prec, descs, Sx.unpack_aux(Ax),
                                                   Sx.unpack_paths(Px), 2, stream)
        Sx.close()
        extra["err_vs_fp64_plain"] = errs
        log("  error vs the FP64 plain path: %s" % errs)

    if not args.no_plain and args.precision != "fp64":
        S64, _, _, ms64, each64, _, _ = chain(args.U, fhmc.FH_FP64, 0, args.warmup, args.steps)
        S64.close()
        ms64 /= args.steps
        extra["fp64_plain"] = {"ms_per_step": round(ms64, 4),
                               "value": sites / (ms64 / 1e3),
                               "per_sweep_ms": chain_summary(each64, args.warmup),
                               "convolution": "FP64 circulant on the matrix cores"}
        extra["speedup_vs_fp64_plain"] = round(ms64 / ms_step, 3)
        log("  fp64 plain %.3f ms/sweep" % ms64)
        # the first sweep from the initial state with FFT convolutions in FP64: an FFT resolves a
        # filter only to ~eps of its largest value, which the end weights of the chain's next
        # sweeps fall below
        S64 = Sampler(descs, fhmc.FH_FP64, fhmc.FH_FLAG_FFT_CONV)
        Af, Pf = S64.pack_aux(aux), S64.pack_paths(paths)
        run_chain(S64, Af.clone(), Pf.clone(), 0, 1, stream)   # module load, untimed
        ms64f, _ = run_chain(S64, Af, Pf, 0, 1, stream)
        code, _ = S64.status()
        S64.close()
        if code != 0:
            raise RuntimeError("device status of the FP64 FFT sweep: " + fhmc.fh_strerror(code))
        extra["fp64_fft_plain"] = {"ms_per_step": round(ms64f, 4),
                                   "value": sites / (ms64f / 1e3),
                                   "sweeps": "the first sweep from the initial state"}
        log("  fp64 FFT plain %.3f ms/sweep" % ms64f)

    cpu = None
    if not args.no_cpu_baseline:
        log("  cpu baseline (oracle, 1 chain, 6 sweeps)...")
        cpu = cpu_baseline(descs[0], aux[0], paths[0])

    out = {
        "metric": "site-slice updates/s at 32x32 L_tau=160",
        "value": value,
        "unit": "site-slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "FFBS sweep, %d chains x 32x32 lattice, L_tau=160, dtau=0.05, "
                               "U=%g, 512+512 worldlines, Gaussian field, %d consecutive sweeps "
                               "from the initial state (%d untimed)" %
                               (args.chains, args.U, args.warmup + args.steps, args.warmup),
                   "chains": args.chains, "L": 32, "L_tau": 160, "precision": args.precision,
                   "graph": True,
                   "backward_draw": "full row" if args.full_row_draw else "window"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "roofline_other_kernel": roofs["backward" if dominant == "forward" else "forward"],
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
