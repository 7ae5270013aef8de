#!/usr/bin/env python3
"""Throughput of the NEDNER reconstruction operator on one MI355X.

One step = one forward execute of the whole operator (spread, lateral FFTs and
deconvolution, NER column FFT + gather + weight, inverse 3D FFT) on one
resident batch of synthetic sensor data. The default workload is the largest
single-GPU one: 65536 sensors drawn 4x denser near the aperture centre, 1024
samples, 30 balls and 5 bead-chain cylinders, output 256x256x512, in the
compensated FP32 precision. Prints ONE JSON line:

  value        non-uniform points per second, M * Nt / t_step, in Mpts/s
  roofline     the slowest kernel against its bound (HBM bytes or ALU flops),
               timed live with HIP events on the execute stream
  cpu_baseline the FP64 oracle timed on the host on the whole workload, and the
               rel-L2 of every GPU precision against its volume
  fp64_plain, fp32_plain, fp32   the same operator in the other precisions:
               time, speedup of the headline precision, rel-L2
  kaiser_bessel_w8   the Kaiser-Bessel window at 8 taps on the same data
  adjoint      the exact adjoint A* (volume -> data) on the same plan
  forward_model_q    the forward operator Q of the wave equation and Q*
  image_measures     App. B measures of the reconstruction
  least_squares      20 projected-gradient iterations through the autograd
               functions on the 192x192-sensor workload, device time
  cache_resident_c2  the 128x128-sensor workload (its 202 MB workspace fits
               in the 256 MB Infinity Cache), with its own oracle error
  two_dimensional    sensors on a line, 1024 x 256 grid
  batch_c4     64 reconstructions of uneven size in one persistent launch per
               stage: aggregate roofline, oracle baseline, max rel-L2
  paper_timings      the paper's own reconstruction times (hardware not stated)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NEDNER-NUFFT recon Mpts/s & %HBM roofline, FP32 vs FP64 plain at rel err 1e-5"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
ORACLE_WORKERS = 16

WORKLOADS = {
    "c3": "65536 sensors 4x denser near the centre, 1024 samples, 30 balls + 5 bead chains -> 256x256x512",
    "c2": "128x128 sensors jittered +/-0.45 pitch, 512 samples, 10 balls + 1% noise -> 128x128x256",
    "c5": "192x192 sensors jittered +/-0.4 pitch, 768 samples, 20 balls + 1% noise -> 192x192x384",
    "c1": "32x32 sensors jittered +/-0.4 pitch, 128 samples, one ball -> 32x32x64",
    "c6": "equi-steradian mask: ~1600 sensors on a 240x240 grid, h ~ r^3, 512 samples, 10 balls "
          "+ 1% noise -> 240x240x256",
    "c7": "128x128 sensors on the output grid nodes (equispaced, NER-only path), 512 samples, "
          "10 balls + 1% noise -> 128x128x256",
    "c8": "1024 sensors on a line (two-dimensional problem), 2048 samples, 10 balls + 1% noise "
          "-> 1024x1x256",
    "c4": "64 problems, M ~ U[1024,16384] jittered, Nt in {256,512,1024}, 1-10 balls, s x s x Nt/2, "
          "one persistent launch per stage",
}

# Reconstruction times the paper reports (Sec. 4, Table 1; Sec. 7). It names
# neither the hardware nor the precision of these runs.
PAPER_TIMINGS = [
    dict(workload="star target, Fabry-Perot scan", method="NER-NUFFT, K = 6", seconds=140.0,
         source="Sec. 4, Table 1", hardware="not stated"),
    dict(workload="star target", method="k-Wave FFT + linear interpolation", seconds=189.0,
         source="Sec. 4, Table 1", hardware="not stated"),
    dict(workload="USAF chart, 146x146 sensors", method="NER-NUFFT", seconds=298.0,
         source="Sec. 4, Table 1", hardware="not stated"),
    dict(workload="USAF chart", method="k-Wave FFT + linear interpolation", seconds=384.0,
         source="Sec. 4, Table 1", hardware="not stated"),
    dict(workload="yarn, 226x226 = 51076 sensors, 452x452 lateral output", method="NER-NUFFT",
         seconds=154.0, source="Sec. 7", hardware="not stated"),
    dict(workload="yarn, equi-steradian mask of 1625 sensors", method="NEDNER-NUFFT",
         seconds=134.0, source="Sec. 7", hardware="not stated"),
]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stage_model(p, info, prec, equi=False, w=12):
    """Algorithmic bytes and flops of each forward stage (one launch each).
    On the equispaced path the spreading is a placement: one product per sample."""
    rs = 8 if prec == "fp64" else 4
    cs = 2 * rs
    M, Nt, N1, N2, N3 = p.m, p.nt, p.n1, p.n2, p.n3
    n1, n2, ntt = info["n1_os"], info["n2_os"], info["nt_os"]
    K2, J1, W = N2 // 2 + 1, N1 + 1, w
    return {
        "spread": dict(bytes=rs * M * Nt + rs * n1 * n2 * Nt,
                       flops=M * Nt if equi else 2 * W * W * M * Nt),
        "lat_a": dict(bytes=rs * n1 * n2 * Nt + cs * n1 * K2 * Nt,
                      flops=int(2.5 * n1 * n2 * Nt * math.log2(n2))),
        "lat_b": dict(bytes=cs * n1 * K2 * Nt + cs * K2 * J1 * Nt,
                      flops=int(5 * n1 * K2 * Nt * math.log2(n1))),
        "column": dict(bytes=cs * K2 * J1 * Nt + cs * K2 * J1 * N3,
                       flops=int(K2 * J1 * (5 * ntt * math.log2(ntt) + (N3 + 1) * 4 * W
                                            + 5 * N3 * math.log2(N3)))),
        "pass_c": dict(bytes=cs * K2 * J1 * N3 + cs * K2 * N1 * N3,
                       flops=int(5 * K2 * N1 * N3 * math.log2(N1))),
        "pass_d": dict(bytes=cs * K2 * N1 * N3 + rs * N1 * N2 * N3,
                       flops=int(2.5 * N1 * N2 * N3 * math.log2(N2))),
    }


def adjoint_stage_model(p, info, prec, w=12):
    """Algorithmic bytes of the adjoint stages (the forward stages' transposes)."""
    fw = stage_model(p, info, prec, w=w)
    rs = 8 if prec == "fp64" else 4
    return {"adj_d": fw["pass_d"], "adj_c": fw["pass_c"], "column_adj": fw["column"],
            "adj_b": fw["lat_b"], "adj_a": fw["lat_a"],
            "gather": dict(bytes=rs * p.m * p.nt + rs * info["n1_os"] * info["n2_os"] * p.nt,
                           flops=2 * w * w * p.m * p.nt)}


def spread_peak(prec):
    """ALU peak of the spreading's multiply-adds: FP64 vector for FP64 sums,
    the chip's FP32 vector peak (packed issue) for FP32 sums."""
    return FP64_VECTOR_TFLOPS if prec in ("fp64", "fp32w") else FP32_VECTOR_TFLOPS


# FP32 multiply-adds issued one per lane (the kernels are built without packed
# FP32 instructions): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# kernel name prefix -> stage, and the source file that defines the kernel
STAGE_KERNELS = {
    "k_spread": ("spread", "k_spread_impl.hpp"), "k_lat_a": ("lat_a", "k_passes.hip"),
    "k_lat_b": ("lat_b", "k_passes.hip"), "k_column": ("column", "k_column_impl.hpp"),
    "k_pass_c": ("pass_c", "k_passes.hip"), "k_pass_d": ("pass_d", "k_passes.hip"),
}


def kernel_source_hash(stage):
    """Hash of the source that defines a stage's kernel and the shared transform code."""
    src = {v[0]: v[1] for v in STAGE_KERNELS.values()}[stage]
    h = hashlib.sha256()
    for f in (src, "fft_lds.hpp"):
        with open(os.path.join(ROOT, "paper_1501_02946_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# the launch-shape fields each stage's kernel depends on
STAGE_SHAPE = {
    "spread": ("rows_per_wave", "time_per_lane", "spread_depth"),
    "lat_a": ("pass_lines", "pass_threads", "pass_inplace"),
    "lat_b": ("pass_lines", "pass_threads", "pass_inplace"),
    "pass_c": ("pass_lines", "pass_threads", "pass_inplace"),
    "pass_d": ("pass_lines", "pass_threads", "pass_inplace"),
    "column": (),
}


def traffic_key(workload, prec, stage, tuning):
    shape = ",".join(f"{k}={tuning[k]}" for k in STAGE_SHAPE[stage])
    return f"{workload}:{prec}:{stage}" + (f":{shape}" if shape else "")


def measured_traffic(workload, prec, stage, tuning):
    """HBM bytes per launch from committed rocprofv3 counters, if still current:
    same kernel source and same launch shape of that kernel, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or stage not in STAGE_SHAPE:
        return None
    with open(path) as fh:
        d = json.load(fh)
    rec = d.get(traffic_key(workload, prec, stage, tuning))
    if not rec or rec.get("source_hash") != kernel_source_hash(stage):
        return None
    return rec.get("bytes")


def summarize_counters(root, workload, prec):
    """HBM traffic per stage from rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE) of this script, each scaled by what the same counter reads for
    a plain device copy of known size (the --copy-calibration run).

    Layout under root: copy_calibration.json and copy_<COUNTER>/ (the copy
    runs), and one folder per counted launch shape holding bench_line.json
    (the JSON line the FETCH_SIZE run printed, with its launch shape) and
    <COUNTER>/<workload>_counter_collection.csv."""
    from paper_1501_02946_amd.profiling import counter_means
    with open(os.path.join(root, "copy_calibration.json")) as fh:
        nbytes = json.load(fh)["copy_bytes"]
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = counter_means(os.path.join(root, f"copy_{c}", "copy_counter_collection.csv"))
        kib, _ = cal["__amd_rocclr_copyBuffer"][c]
        # the copy reads and writes copy_bytes each
        scale[c] = nbytes / (kib * 1024.0)
    out = {}
    for sub in sorted(os.listdir(root)):
        line = os.path.join(root, sub, "bench_line.json")
        if not os.path.exists(line):
            continue
        with open(line) as fh:
            tuning = json.loads(fh.read().strip().splitlines()[-1])["tuning"]
        fetch = counter_means(os.path.join(root, sub, "FETCH_SIZE", f"{workload}_counter_collection.csv"))
        write = counter_means(os.path.join(root, sub, "WRITE_SIZE", f"{workload}_counter_collection.csv"))
        for kname, (stage, _) in STAGE_KERNELS.items():
            if kname not in fetch or kname not in write:
                continue
            fk, n = fetch[kname]["FETCH_SIZE"]
            wk, _ = write[kname]["WRITE_SIZE"]
            b = fk * 1024 * scale["FETCH_SIZE"] + wk * 1024 * scale["WRITE_SIZE"]
            out[traffic_key(workload, prec, stage, tuning)] = dict(
                bytes=int(round(b)), fetch_kib=round(fk, 1), write_kib=round(wk, 1),
                fetch_scale=round(scale["FETCH_SIZE"], 4), write_scale=round(scale["WRITE_SIZE"], 4),
                dispatches=n, source_hash=kernel_source_hash(stage),
                shape={k: tuning[k] for k in STAGE_SHAPE[stage]})
    return out


def time_op(torch, plan, fn, steps, warmup, profile=False):
    """Mean time of fn() (one operator call on the plan's stream) over `steps`
    calls, HIP events around them on that stream; with profile, the plan's
    per-stage times (HIP events recorded by the library between its kernels)."""
    import ctypes
    import paper_1501_02946_amd as N
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if profile:
        N._check(N.lib().nedner_profile_begin(plan._plan, steps))
    stream = torch.cuda.current_stream(plan.device)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    stages = None
    if profile:
        arr = (ctypes.c_double * 16)()
        ns = ctypes.c_int(0)
        names = ctypes.c_char_p()
        N._check(N.lib().nedner_profile_end(plan._plan, arr, 16, ctypes.byref(ns), ctypes.byref(names)))
        stages = dict(zip(names.value.decode().split(","), [arr[i] for i in range(ns.value)]))
    return ms, stages


def roofline_of(stages, model, prec, equi=False):
    """The slowest stage against its bound: the spreading's multiply-adds
    against the ALU peak of its accumulation type, every other stage's
    algorithmic bytes against the HBM peak."""
    dom = max(stages, key=stages.get)
    tdom = stages[dom] / 1e3
    if dom in ("spread", "gather") and not equi:
        peak = spread_peak(prec)
        ach = model[dom]["flops"] / tdom / 1e12
        roof = dict(bound="alu", achieved=round(ach, 3), peak=peak, unit="TFLOP/s",
                    frac=round(ach / peak, 4))
        if peak == FP32_VECTOR_TFLOPS:
            # the published peak counts packed FP32 issue, which this build
            # does not use; the rate its unpacked multiply-adds can reach
            roof["peak_unpacked_fp32"] = round(FP32_UNPACKED_TFLOPS, 1)
            roof["frac_unpacked_fp32"] = round(ach / FP32_UNPACKED_TFLOPS, 4)
    else:
        ach = model[dom]["bytes"] / tdom / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4))
    roof["kernel"] = dom
    roof["ms"] = round(stages[dom], 5)
    roof["alg_bytes"] = model[dom]["bytes"]
    roof["alg_flops"] = model[dom]["flops"]
    return roof


def stage_report(stages, model):
    rep = {}
    for name, t in stages.items():
        m = model.get(name, {})
        gbs = m.get("bytes", 0) / (t / 1e3) / 1e9 if t > 0 else 0.0
        rep[name] = dict(ms=round(t, 5), alg_bytes=m.get("bytes"), alg_flops=m.get("flops"),
                         hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
    return rep


# ---------------------------------------------------------------- oracle side

def _limit_threads():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[k] = "1"


def _oracle_volume_task(args):
    """Worker: the oracle volume of one problem (one BLAS thread per worker)."""
    idx, xy, h, g, geo_kw = args
    import oracle as O
    geo = O.geometry(**geo_kw)
    t = time.perf_counter()
    v = O.forward(xy, h, g, geo)
    return idx, v, time.perf_counter() - t


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def oracle_full(p):
    """The FP64 oracle on the whole workload in this process: volume and time."""
    import oracle as O
    geo = O.geometry(**p.geometry_kwargs())
    t = time.perf_counter()
    F = O.spectrum(p.xy, p.h, p.g, geo)
    v = O.volume_from_spectrum(F)
    return v, time.perf_counter() - t


def rel_l2(a, ref):
    import numpy as np
    return float(np.linalg.norm(a.astype(np.float64) - ref) / max(float(np.linalg.norm(ref)), 1e-300))


def q_sample_error(p, vol, dq, nsens=48, ntimes=4, seed=3):
    """rel-L2 of Q's output at sampled (sensor, time) pairs against the oracle's
    sums at those times (each time on its own: Q at t_n needs only t_n)."""
    import dataclasses

    import numpy as np
    import oracle as O
    geo = O.geometry(**p.geometry_kwargs())
    rng = np.random.default_rng(seed)
    ms = rng.choice(p.m, nsens, replace=False)
    ns = np.sort(rng.choice(p.nt, ntimes, replace=False))
    v = vol.astype(np.float64)
    want = np.empty((nsens, ntimes))
    for i, n in enumerate(ns):
        want[:, i] = O.trace(v, p.xy[ms], dataclasses.replace(geo, nt=1, t0=geo.t0 + n * geo.dt))[:, 0]
    got = dq[np.ix_(ms, ns)].astype(np.float64)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


# ---------------------------------------------------------------- legs

def make_plan(N, p, precision, **kw):
    return N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0, a1=p.a1, a2=p.a2,
                  d1=p.d1, d2=p.d2, d3=p.d3, precision=precision, **kw)


def leg_precision(torch, N, p, prec, a, flags=(), tuning=None, **kw):
    """Time one precision on the workload (with the given launch shape, else
    the plan's default); returns (record, volume on the host)."""
    plan = make_plan(N, p, prec, flags=list(flags), **kw)
    if tuning:
        t = dict(tuning)
        if plan.tuning["gather_rows"] == 0:
            # FP64 plans and wide windows take the tile-staged gather only
            t["gather_rows"] = 0
        plan.set_tuning(t)
    g = torch.as_tensor(p.g, dtype=plan.dtype, device=plan.device).contiguous()
    out = torch.empty((p.n1, p.n2, p.n3), dtype=plan.dtype, device=plan.device)
    ms, _ = time_op(torch, plan, lambda: plan.forward(g, out=out), a.steps, a.warmup)
    _, st = time_op(torch, plan, lambda: plan.forward(g, out=out), a.steps, 1, profile=True)
    rec = dict(ms_per_step=round(ms, 5), value=round(p.m * p.nt / (ms / 1e3) / 1e6, 2),
               unit="Mpts/s", stages_ms={k: round(v, 5) for k, v in st.items()})
    vol = out.cpu().numpy()
    del plan, g, out
    return rec, vol


def leg_least_squares(torch, N, a):
    """20 projected-gradient iterations on the 192x192-sensor workload through the
    autograd functions (model A* and model Q), timed with HIP events on the
    stream the operators run on; the losses stay on the device until the end."""
    import synth
    p = synth.config("c5")
    plan = make_plan(N, p, a.precision)
    g = torch.as_tensor(p.g, dtype=plan.dtype, device=plan.device).contiguous()
    res = {"workload": f"c5: {WORKLOADS['c5']}"}
    iters = 20
    for model in ("adjoint", "q"):
        # the step is fixed from a power iteration before the timed region
        eta = 0.95 / max(N.power_norm(plan, iters=20, model=model), 1e-300)
        rhs = g if model == "adjoint" else plan.q(plan.forward(g))
        N.lsq(plan, rhs, iters=2, eta=eta, model=model)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(plan.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, losses = N.lsq(plan, rhs, iters=iters, eta=eta, model=model, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / iters
        losses = [float(v) for v in losses]
        res[model] = dict(ms_per_iteration=round(ms, 4), iterations=iters,
                          loss_ratio=float(losses[-1] / losses[0]) if losses[0] else None,
                          monotone=bool(all(b <= a_ * (1 + 1e-6) for a_, b in zip(losses, losses[1:]))))
    del plan, g
    return res


def leg_batch(torch, N, a, probs, pool):
    """The 64-problem batch: one execute_many per step; aggregate roofline;
    the oracle over every problem in worker processes (one per host thread)."""
    import ctypes

    import numpy as np
    kws = [dict(xy=p.xy, h=p.h, nt=p.nt, dt=p.dt, volume=(p.n1, p.n2, p.n3)) for p in probs]
    bp = N.BatchPlan(kws, precision=a.precision)
    tune = None if a.no_autotune else bp.autotune()
    dt = torch.float64 if a.precision == "fp64" else torch.float32
    gs = [torch.as_tensor(p.g, dtype=dt, device=bp.device) for p in probs]
    outs = [torch.empty((p.n1, p.n2, p.n3), dtype=dt, device=bp.device) for p in probs]
    for _ in range(a.warmup):
        bp(gs, outs)
    torch.cuda.synchronize()
    N._check(N.lib().nedner_profile_begin(bp._plan, a.steps))
    stream = torch.cuda.current_stream(bp.device)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(a.steps):
        bp(gs, outs)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / a.steps
    arr = (ctypes.c_double * 16)()
    ns = ctypes.c_int(0)
    names = ctypes.c_char_p()
    N._check(N.lib().nedner_profile_end(bp._plan, arr, 16, ctypes.byref(ns), ctypes.byref(names)))
    stages = dict(zip(names.value.decode().split(","), [arr[i] for i in range(ns.value)]))
    vols = [o.cpu().numpy() for o in outs]
    points = sum(p.m * p.nt for p in probs)
    # aggregate algorithmic bytes and flops of each stage over the problems
    agg = {}
    for p in probs:
        info = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, precision=a.precision)
        for k, v in stage_model(p, info, a.precision).items():
            s = agg.setdefault(k, dict(bytes=0, flops=0))
            s["bytes"] += v["bytes"]
            s["flops"] += v["flops"]
    roof = roofline_of(stages, agg, a.precision)
    total_bytes = sum(v["bytes"] for v in agg.values())
    rec = {"workload": f"c4: {WORKLOADS['c4']}", "problems": len(probs), "points": points,
           "ms_per_step": round(ms, 5), "value": round(points / (ms / 1e3) / 1e6, 2), "unit": "Mpts/s",
           "volumes_per_s": round(len(probs) * 1e3 / ms, 2),
           "spread_ps_per_sample": round(stages.get("spread", 0.0) * 1e9 / points, 3),
           "stages_ms": {k: round(v, 5) for k, v in stages.items()},
           "stage_hbm_frac": {k: round(agg[k]["bytes"] / (stages[k] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                              for k in stages if k in agg and stages[k] > 0},
           "whole_step_hbm_frac": round(total_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "autotune": tune, "roofline": roof}
    del bp, gs, outs
    if pool is not None:
        t = time.perf_counter()
        tasks = [(i, p.xy, p.h, p.g, p.geometry_kwargs()) for i, p in enumerate(probs)]
        # largest problems first, so that the last ones to finish are small
        tasks.sort(key=lambda tk: -(tk[3].size * tk[1].shape[0]))
        errs = [None] * len(probs)
        busy = 0.0
        for i, v, sec in pool.imap_unordered(_oracle_volume_task, tasks):
            errs[i] = rel_l2(vols[i], v)
            busy += sec
        wall = time.perf_counter() - t
        rec["max_rel_l2_vs_oracle"] = max(errs)
        rec["worst_problem"] = int(np.argmax(errs))
        rec["cpu_baseline"] = dict(
            value=round(points / wall / 1e6, 4), unit="Mpts/s", cores=ORACLE_WORKERS, kind="oracle",
            seconds=round(wall, 2), cpu_model=cpu_model(),
            sample=(f"all {len(probs)} problems, each on one worker process with one BLAS thread, "
                    f"{ORACLE_WORKERS} workers; {busy:.0f} worker-seconds"))
    return rec


def write_traffic(a):
    """Merge the measured per-stage HBM bytes into profiles/traffic.json and print
    them next to the algorithmic bytes, with the launch shape of each counted run."""
    import paper_1501_02946_amd as N
    import synth
    import torch  # noqa: F401  (the binding loads torch first)
    p = synth.config(a.workload)
    info = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, c=p.c, t0=p.t0,
                   precision=a.precision)
    rec = summarize_counters(a.summarize_counters, a.workload, a.precision)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = {}
    if os.path.exists(path):
        with open(path) as fh:
            d = json.load(fh)
    # entries of the same workload and precision are replaced as a whole
    d = {k: v for k, v in d.items() if not k.startswith(f"{a.workload}:{a.precision}:")}
    d.update(rec)
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
    model = stage_model(p, info, a.precision)
    print("| stage | launch shape | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | "
          "algorithmic bytes | ratio |")
    print("|---|---|---|---|---|---|---|")
    for k, r in sorted(rec.items()):
        st = k.split(":")[2]
        alg = model[st]["bytes"]
        shape = " ".join(f"{x}={y}" for x, y in r["shape"].items()) or "-"
        print(f"| {st} | {shape} | {r['fetch_kib']} | {r['write_kib']} | {r['bytes']} | {alg} | "
              f"{r['bytes'] / alg:.3f} |")
    r0 = next(iter(rec.values()))
    print(f"scale factors: FETCH_SIZE x{r0['fetch_scale']}, WRITE_SIZE x{r0['write_scale']}")
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32w", "fp32", "fp32_plain", "fp64"])
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the plan's default launch shape instead of the autotuner's")
    ap.add_argument("--shape", default="", metavar="K=V,...",
                    help="launch-shape fields to set instead of autotuning (e.g. rows_per_wave=64)")
    ap.add_argument("--quick", action="store_true",
                    help="headline and stage times only (no other legs, no oracle)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every oracle run")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the FP64-plain, FP32-plain and FP32 legs")
    ap.add_argument("--no-kb", action="store_true", help="skip the Kaiser-Bessel (8-tap) leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the exact adjoint leg")
    ap.add_argument("--no-q", action="store_true", help="skip the forward operator Q leg")
    ap.add_argument("--no-lsq", action="store_true", help="skip the least-squares leg")
    ap.add_argument("--no-c2", action="store_true", help="skip the cache-resident c2 leg")
    ap.add_argument("--no-2d", action="store_true", help="skip the two-dimensional leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="turn the rocprofv3 counter CSVs under DIR into profiles/traffic.json")
    a = ap.parse_args(argv)
    if a.summarize_counters:
        return write_traffic(a)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): this build has no multi-GPU "
              "path; how the operator would shard is a design note", file=sys.stderr)
        return 2
    if a.quick:
        a.no_cpu_baseline = a.no_precisions = a.no_kb = a.no_adjoint = a.no_q = True
        a.no_lsq = a.no_c2 = a.no_2d = a.no_batch = True
    if a.copy_calibration:
        import torch
        x = torch.ones(a.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "launches": 3}), flush=True)
        return 0

    pool = None
    if not a.no_cpu_baseline and not a.no_batch and a.workload != "c4":
        # oracle workers for the batch: fresh interpreters, started before this
        # process touches the GPU, one BLAS thread each
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(ORACLE_WORKERS, initializer=_limit_threads)

    import numpy as np
    import torch

    import paper_1501_02946_amd as N
    import synth

    if a.workload == "c4":
        rec = leg_batch(torch, N, a, synth.batch_c4(), None)
        res = {"metric": METRIC, "value": rec["value"], "unit": "Mpts/s", "n_gpus": 1, "steps": a.steps,
               "warmup": a.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32",
               "data": "synthetic", "config": {"workload": rec["workload"], "precision": a.precision},
               "roofline": rec["roofline"], "cpu_baseline": None, "batch": rec}
        print(json.dumps(res), flush=True)
        return 0

    p = synth.config(a.workload)
    equi = a.workload == "c7"
    flags = ["equispaced"] if equi else []
    plan = make_plan(N, p, a.precision, flags=flags)
    g = torch.as_tensor(p.g, dtype=plan.dtype, device=plan.device).contiguous()
    out = torch.empty((p.n1, p.n2, p.n3), dtype=plan.dtype, device=plan.device)
    if a.shape:
        t = dict(plan.tuning)
        for kv in a.shape.split(","):
            k, v = kv.split("=")
            if k not in t:
                raise SystemExit(f"unknown launch-shape field {k!r}")
            t[k] = int(v)
        plan.set_tuning(t)
    elif not a.no_autotune and not equi:
        # launch shape by timing candidates (sweep length, samples per lane,
        # FFT-pass shape) before the timed region; the legs below reuse it
        import tempfile
        plan.autotune(g, cache=os.path.join(tempfile.mkdtemp(prefix="nedner_bench_"), "tuning.json"))

    ms, _ = time_op(torch, plan, lambda: plan.forward(g, out=out), a.steps, a.warmup)
    _, stages = time_op(torch, plan, lambda: plan.forward(g, out=out), a.steps, 1, profile=True)
    vol = out.cpu().numpy()
    points = p.m * p.nt
    value = points / (ms / 1e3) / 1e6

    model = stage_model(p, plan.info, a.precision, equi)
    roof = roofline_of(stages, model, a.precision, equi)
    tuning = {k: v for k, v in plan.tuning.items() if not k.startswith("ms_")}
    roof["traffic"] = measured_traffic(a.workload, a.precision, roof["kernel"], tuning)
    whole_bytes = sum(v["bytes"] for v in model.values())

    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS[a.workload]}", "sensors": p.m,
                   "nt": p.nt, "volume": [p.n1, p.n2, p.n3], "precision": a.precision,
                   "window_taps": 12, "oversampling": 2},
        "volumes_per_s": round(1e3 / ms, 2),
        "whole_step_hbm_frac": round(whole_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "tuning": tuning,
        "roofline": roof,
        "stages": stage_report(stages, model),
    }
    vols = {}
    shape = {k: v for k, v in tuning.items()}
    if not a.no_precisions:
        for prec in ("fp64", "fp32_plain", "fp32c", "fp32w", "fp32"):
            if prec == a.precision:
                continue
            key = {"fp64": "fp64_plain", "fp32_plain": "fp32_plain", "fp32c": "fp32_compensated",
                   "fp32w": "fp32_wide_sums", "fp32": "fp32"}[prec]
            rec, vols[key] = leg_precision(torch, N, p, prec, a, flags, tuning=shape)
            rec[f"{a.precision}_speedup"] = round(rec["ms_per_step"] / ms, 3)
            res[key] = rec
    if not a.no_kb:
        # the paper's window choice: Kaiser-Bessel, 8 taps per axis instead of 12
        rec, vols["kaiser_bessel_w8"] = leg_precision(torch, N, p, a.precision, a, flags, tuning=shape, w=8,
                                                      window="kaiser_bessel")
        res["kaiser_bessel_w8"] = rec
    if not a.no_adjoint:
        # the exact adjoint (a transpose pass of every stage) on the reconstructed volume
        da = torch.empty((p.m, p.nt), dtype=plan.dtype, device=plan.device)
        msa, _ = time_op(torch, plan, lambda: plan.adjoint(out, out=da), a.steps, a.warmup)
        _, sta = time_op(torch, plan, lambda: plan.adjoint(out, out=da), a.steps, 1, profile=True)
        amodel = adjoint_stage_model(p, plan.info, a.precision)
        res["adjoint"] = dict(ms_per_step=round(msa, 5), value=round(points / (msa / 1e3) / 1e6, 2),
                              unit="Mpts/s", ratio_to_forward=round(msa / ms, 3),
                              stages=stage_report(sta, amodel))
        del da
    # image measures of App. B on the reconstruction (GPU kernels)
    phantom = torch.as_tensor(synth.phantom_volume(p), dtype=plan.dtype, device=plan.device)
    msm, _ = time_op(torch, plan, lambda: N.mip(out, 2), a.steps, a.warmup)
    ten = N.tenenbaum(N.mip(out, 2), normalized=True)
    res["image_measures"] = dict(corrcoef_vs_phantom=round(N.corrcoef(out, phantom), 6),
                                 tenenbaum_depth_mip_per_pixel=ten, mip_ms=round(msm, 5))
    del phantom
    qsample = None
    if not a.no_q:
        # the forward operator Q (initial pressure -> sensor traces) on the
        # reconstructed volume, and its adjoint on the data
        dq = torch.empty((p.m, p.nt), dtype=plan.dtype, device=plan.device)
        vq = torch.empty_like(out)
        msq, _ = time_op(torch, plan, lambda: plan.q(out, out=dq), a.steps, a.warmup)
        _, stq = time_op(torch, plan, lambda: plan.q(out, out=dq), a.steps, 1, profile=True)
        msqa, _ = time_op(torch, plan, lambda: plan.q_adjoint(g, out=vq), a.steps, a.warmup)
        _, stqa = time_op(torch, plan, lambda: plan.q_adjoint(g, out=vq), a.steps, 1, profile=True)
        res["forward_model_q"] = dict(
            ms_per_step=round(msq, 5), value=round(points / (msq / 1e3) / 1e6, 2), unit="Mpts/s",
            adjoint_ms_per_step=round(msqa, 5),
            stages_ms={k: round(v, 5) for k, v in stq.items()},
            adjoint_stages_ms={k: round(v, 5) for k, v in stqa.items()})
        qsample = dq.cpu().numpy()
        del dq, vq
    del plan, g, out
    torch.cuda.empty_cache()
    if not a.no_lsq:
        res["least_squares"] = leg_least_squares(torch, N, a)
    vol_c2 = p2 = None
    if not a.no_c2 and a.workload != "c2":
        p2 = synth.config("c2")
        rec, vol_c2 = leg_precision(torch, N, p2, a.precision, a)
        rec["workload"] = f"c2: {WORKLOADS['c2']}"
        rec["note"] = "cache-resident: the 202 MB workspace fits in the 256 MB Infinity Cache"
        res["cache_resident_c2"] = rec
    if not a.no_2d:
        p8 = synth.config("c8")
        rec, _ = leg_precision(torch, N, p8, a.precision, a)
        rec["workload"] = f"c8: {WORKLOADS['c8']}"
        res["two_dimensional"] = rec
    if not a.no_batch:
        res["batch_c4"] = leg_batch(torch, N, a, synth.batch_c4(), pool)
    torch.cuda.empty_cache()
    res["paper_timings"] = PAPER_TIMINGS
    if not a.no_cpu_baseline:
        vref, sec = oracle_full(p)
        threads = blas_threads()
        res["cpu_baseline"] = dict(
            value=round(points / sec / 1e6, 4), unit="Mpts/s", cores=threads, kind="oracle",
            seconds=round(sec, 2), cpu_model=cpu_model(),
            sample=(f"the whole workload ({p.m} sensors x {p.nt} samples -> {p.n1}x{p.n2}x{p.n3}): "
                    f"NED as BLAS GEMMs on {threads} threads, NER by Horner's rule (numpy, one "
                    "thread), numpy ifftn"))
        res["rel_l2_vs_oracle"] = rel_l2(vol, vref)
        for key, v in vols.items():
            res[key]["rel_l2_vs_oracle"] = rel_l2(v, vref)
        if qsample is not None:
            res["forward_model_q"]["sampled_rel_l2_vs_oracle"] = q_sample_error(p, vol, qsample)
        if vol_c2 is not None:
            vref2, _ = oracle_full(p2)
            res["cache_resident_c2"]["rel_l2_vs_oracle"] = rel_l2(vol_c2, vref2)
    else:
        res["cpu_baseline"] = None
    if pool is not None:
        pool.close()
        pool.join()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
