#!/usr/bin/env python3
"""Throughput of the NEDNER reconstruction operator on one MI355X.

One step = one forward execute of the whole operator (spread, lateral FFTs and
deconvolution, NER column FFT + gather + weight, inverse 3D FFT) on one
resident batch of synthetic sensor data. Prints ONE JSON line:

  value        non-uniform points per second, M * Nt / t_step, in Mpts/s
  roofline     the slowest kernel against its bound (HBM bytes or ALU flops),
               timed live with HIP events on the execute stream
  cpu_baseline the FP64 oracle timed on the host on the same workload
  fp64_plain   the same operator in FP64 on the GPU, and the FP32 speedup
  kaiser_bessel_w8  the same workload with the Kaiser-Bessel window at 8 taps
  adjoint      the exact adjoint A* (volume -> data) on the same plan, per stage
  image_measures    the App. B measures of the reconstruction: correlation with
               the rasterised phantom, Tenenbaum sharpness of the depth MIP
  least_squares     20 iterations of projected gradient descent through the
               autograd functions (model A* and model Q), per-iteration time
  two_dimensional   the two-dimensional problem (sensors on a line) at the grid
               of the paper's 2-D study, 1024 x 256
  forward_model_q   the forward operator Q of the wave equation (volume -> data)
               and its adjoint on the same plan, per-stage times, and sampled
               outputs of Q against the oracle

Inputs: 128x128 jittered sensors (+/-0.45 pitch), 512 samples, 10 random balls
and 1 % noise, output 128x128x256 (the FP32-vs-plain comparison workload).
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

WORKLOADS = {
    "c2": "128x128 sensors jittered +/-0.45 pitch, 512 samples, 10 balls + 1% noise -> 128x128x256",
    "c3": "65536 sensors 4x denser near the centre, 1024 samples, 30 balls + 5 bead chains -> 256x256x512",
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


def stage_model(p, info, prec, equi=False):
    """Algorithmic bytes and flops of each forward stage (one launch each).
    On the equispaced path the spreading is a placement: one product per sample."""
    rs = 8 if prec == "fp64" else 4
    cs = 2 * rs
    M, Nt, N1, N2, N3 = p.m, p.nt, p.n1, p.n2, p.n3
    n1, n2, ntt = info["n1_os"], info["n2_os"], info["nt_os"]
    K2, J1, W = N2 // 2 + 1, N1 + 1, 12
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


# kernel name prefix -> stage, and the source file that defines the kernel
STAGE_KERNELS = {
    "k_spread": ("spread", "k_spread.hip"), "k_lat_a": ("lat_a", "k_passes.hip"),
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


def measured_traffic(workload, prec, stage, tuning):
    """HBM bytes per launch from committed rocprofv3 counters, if still current:
    same kernel source and same launch shape, else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    rec = d.get(f"{workload}:{prec}:{stage}")
    if not rec or rec.get("source_hash") != kernel_source_hash(stage):
        return None
    if rec.get("tuning") != {k: tuning[k] for k in rec.get("tuning", {})}:
        return None
    return rec.get("bytes")


def _counter_means(path):
    """Mean counter value per kernel (KiB per dispatch) of a rocprofv3 counter CSV."""
    import csv
    acc = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").strip()
            name = name.split("::")[-1]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def summarize_counters(root, workload, prec, tuning):
    """HBM traffic per stage from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)
    of this script, each scaled by what the same counter reads for a plain
    device copy of known size (the --copy-calibration run)."""
    out, lines = {}, []
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = _counter_means(os.path.join(root, f"pmc_{c}", "copy_counter_collection.csv"))
        kib, _ = cal["__amd_rocclr_copyBuffer"]
        # the copy reads and writes copy_bytes each
        with open(os.path.join(root, "copy_calibration.json")) as fh:
            nbytes = json.load(fh)["copy_bytes"]
        scale[c] = nbytes / (kib * 1024.0)
    fetch = _counter_means(os.path.join(root, "pmc_FETCH_SIZE", f"{workload}_counter_collection.csv"))
    write = _counter_means(os.path.join(root, "pmc_WRITE_SIZE", f"{workload}_counter_collection.csv"))
    for kname, (stage, _) in STAGE_KERNELS.items():
        hit = [k for k in fetch if k == kname]
        if not hit or kname not in write:
            continue
        fk, n = fetch[kname]
        wk, _ = write[kname]
        b = fk * 1024 * scale["FETCH_SIZE"] + wk * 1024 * scale["WRITE_SIZE"]
        out[f"{workload}:{prec}:{stage}"] = dict(
            bytes=int(round(b)), fetch_kib=round(fk, 1), write_kib=round(wk, 1),
            fetch_scale=round(scale["FETCH_SIZE"], 4), write_scale=round(scale["WRITE_SIZE"], 4),
            dispatches=n, source_hash=kernel_source_hash(stage), tuning=tuning)
    return out


def time_steps(torch, plan, g, out, steps, warmup, profile=False):
    return time_op(torch, plan, lambda: plan.forward(g, out=out), steps, warmup, profile)


def time_op(torch, plan, fn, steps, warmup, profile=False):
    """Mean time of fn() (one operator call on the plan's stream) over `steps`
    calls, HIP events around them; with profile, the plan's stage times too."""
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


def cpu_baseline(p, leg_limit_s=60.0):
    """The FP64 oracle on the host: full forward operator on the same workload."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    geo = O.geometry(**p.geometry_kwargs())
    t = time.perf_counter()
    F = O.spectrum(p.xy, p.h, p.g, geo)
    v = O.volume_from_spectrum(F)
    dt = time.perf_counter() - t
    return v, dict(value=p.m * p.nt / dt / 1e6, unit="Mpts/s", cores=int(threads), kind="oracle",
                   seconds=round(dt, 3),
                   sample=(f"the full workload ({p.m} sensors x {p.nt} samples -> "
                           f"{p.n1}x{p.n2}x{p.n3}): NED as BLAS GEMMs on {threads} threads, "
                           "NER by Horner's rule (numpy, one thread), numpy ifftn"))


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


def bench_batch(a, torch, N, synth):
    """The 64-problem batch: one execute_many per step."""
    import ctypes
    probs = synth.batch_c4()
    kws = [dict(xy=p.xy, h=p.h, nt=p.nt, dt=p.dt, volume=(p.n1, p.n2, p.n3)) for p in probs]
    bp = N.BatchPlan(kws, precision=a.precision)
    tune = bp.autotune()
    dt = torch.float64 if a.precision == "fp64" else torch.float32
    gs = [torch.as_tensor(p.g, dtype=dt, device=bp.device) for p in probs]
    outs = [torch.empty((p.n1, p.n2, p.n3), dtype=dt, device=bp.device) for p in probs]
    for _ in range(a.warmup):
        bp(gs, outs)
    torch.cuda.synchronize()
    N._check(N.lib().nedner_profile_begin(bp._plan, a.steps))
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(a.steps):
        bp(gs, outs)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / a.steps
    arr = (ctypes.c_double * 16)()
    ns = ctypes.c_int(0)
    names = ctypes.c_char_p()
    N._check(N.lib().nedner_profile_end(bp._plan, arr, 16, ctypes.byref(ns), ctypes.byref(names)))
    stages = dict(zip(names.value.decode().split(","), [round(arr[i], 5) for i in range(ns.value)]))
    points = sum(p.m * p.nt for p in probs)
    return {"metric": METRIC, "value": round(points / (ms / 1e3) / 1e6, 2), "unit": "Mpts/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if a.precision == "fp64" else "f32", "data": "synthetic",
            "config": {"workload": f"c4: {WORKLOADS['c4']}", "problems": len(probs),
                       "points": points, "precision": a.precision},
            "volumes_per_s": round(len(probs) * 1e3 / ms, 2), "stages_ms": stages,
            "autotune": tune, "roofline": None, "cpu_baseline": None}


def write_traffic(a):
    """Merge the measured per-stage HBM bytes into profiles/traffic.json and print
    them next to the algorithmic bytes, with the launch shape of the counted run."""
    import paper_1501_02946_amd as N
    import synth
    import torch  # noqa: F401  (the binding loads torch first)
    p = synth.config(a.workload)
    info = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, c=p.c, t0=p.t0,
                   precision=a.precision)
    # the JSON line the FETCH_SIZE-counted bench run printed: its launch shape
    with open(os.path.join(a.summarize_counters, "bench_line.json")) as fh:
        tuning = json.loads(fh.read().strip().splitlines()[-1])["tuning"]
    rec = summarize_counters(a.summarize_counters, a.workload, a.precision, tuning)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    d = {}
    if os.path.exists(path):
        with open(path) as fh:
            d = json.load(fh)
    d.update(rec)
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
    model = stage_model(p, info, a.precision)
    print("| stage | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | algorithmic bytes | ratio |")
    print("|---|---|---|---|---|---|")
    for k, r in rec.items():
        st = k.split(":")[-1]
        alg = model[st]["bytes"]
        print(f"| {st} | {r['fetch_kib']} | {r['write_kib']} | {r['bytes']} | {alg} | "
              f"{r['bytes'] / alg:.3f} |")
    print(f"scale factors: FETCH_SIZE x{next(iter(rec.values()))['fetch_scale']}, "
          f"WRITE_SIZE x{next(iter(rec.values()))['write_scale']}")
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32c", choices=["fp32c", "fp32", "fp32_plain", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-kb", action="store_true",
                    help="skip the Kaiser-Bessel (8-tap) leg timed beside the headline")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the leg timing the exact adjoint")
    ap.add_argument("--no-lsq", action="store_true",
                    help="skip the leg timing the projected-gradient least squares")
    ap.add_argument("--no-2d", action="store_true",
                    help="skip the leg timing the two-dimensional problem")
    ap.add_argument("--no-q", action="store_true",
                    help="skip the leg timing the forward operator Q and its adjoint")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="turn the rocprofv3 counter CSVs under DIR into profiles/traffic.json")
    a = ap.parse_args(argv)
    if a.summarize_counters:
        return write_traffic(a)
    if a.copy_calibration:
        import torch
        x = torch.ones(a.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "launches": 3}), flush=True)
        return 0
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU split of the "
              "operator is a design note, not part of this build", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1501_02946_amd as N
    import synth

    if a.workload == "c4":
        print(json.dumps(bench_batch(a, torch, N, synth)), flush=True)
        return 0
    p = synth.config(a.workload)
    equi = a.workload == "c7"
    flags = ["equispaced"] if equi else []
    plan = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0,
                  precision=a.precision, flags=flags)
    g = torch.as_tensor(p.g, dtype=plan.dtype, device=plan.device).contiguous()
    out = torch.empty((p.n1, p.n2, p.n3), dtype=plan.dtype, device=plan.device)

    ms, _ = time_steps(torch, plan, g, out, a.steps, a.warmup)
    _, stages = time_steps(torch, plan, g, out, a.steps, 1, profile=True)
    vol = out.cpu().numpy()
    points = p.m * p.nt
    value = points / (ms / 1e3) / 1e6

    model = stage_model(p, plan.info, a.precision, equi)
    stage_rep = {}
    for name, t in stages.items():
        m = model.get(name, {})
        gbs = m.get("bytes", 0) / (t / 1e3) / 1e9 if t > 0 else 0.0
        stage_rep[name] = dict(ms=round(t, 5), alg_bytes=m.get("bytes"), alg_flops=m.get("flops"),
                               hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
    dom = max(stages, key=stages.get)
    tdom = stages[dom] / 1e3
    if dom == "spread" and not equi:
        # the spread is a W*W-tap multiply-add per (sensor, sample): ALU bound;
        # the compensated and FP64 paths accumulate with FP64 FMAs
        peak = FP64_VECTOR_TFLOPS if a.precision in ("fp32c", "fp64") else FP32_VECTOR_TFLOPS
        ach = model[dom]["flops"] / tdom / 1e12
        roof = dict(bound="alu", achieved=round(ach, 3), peak=peak, unit="TFLOP/s",
                    frac=round(ach / peak, 4))
    else:
        ach = model[dom]["bytes"] / tdom / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4))
    roof["kernel"] = dom
    roof["ms"] = round(stages[dom], 5)
    tuning = {k: v for k, v in plan.tuning.items() if not k.startswith("ms_")}
    roof["traffic"] = measured_traffic(a.workload, a.precision, dom, tuning)

    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS[a.workload]}", "sensors": p.m,
                   "nt": p.nt, "volume": [p.n1, p.n2, p.n3], "precision": a.precision,
                   "window_taps": 12, "oversampling": 2},
        "volumes_per_s": round(1e3 / ms, 2),
        "tuning": tuning,
        "roofline": roof,
        "stages": stage_rep,
    }
    if not a.no_fp64 and a.precision != "fp64":
        p64 = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0, precision="fp64",
                     flags=flags)
        g64 = torch.as_tensor(p.g, dtype=torch.float64, device=plan.device).contiguous()
        o64 = torch.empty((p.n1, p.n2, p.n3), dtype=torch.float64, device=plan.device)
        ms64, _ = time_steps(torch, p64, g64, o64, a.steps, a.warmup)
        res["fp64_plain"] = dict(ms_per_step=round(ms64, 5), value=round(points / (ms64 / 1e3) / 1e6, 2),
                                 fp32_speedup=round(ms64 / ms, 3))
        vol64 = o64.cpu().numpy()
        del p64
    else:
        vol64 = None
    volkb = None
    if not a.no_kb:
        # the paper's window choice: Kaiser-Bessel, 8 taps per axis instead of 12
        pkb = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0,
                     precision=a.precision, w=8, window="kaiser_bessel", flags=flags)
        okb = torch.empty((p.n1, p.n2, p.n3), dtype=plan.dtype, device=plan.device)
        mskb, _ = time_steps(torch, pkb, g, okb, a.steps, a.warmup)
        _, stkb = time_steps(torch, pkb, g, okb, a.steps, 1, profile=True)
        res["kaiser_bessel_w8"] = dict(ms_per_step=round(mskb, 5),
                                       value=round(points / (mskb / 1e3) / 1e6, 2),
                                       stages_ms={k: round(v, 5) for k, v in stkb.items()})
        volkb = okb.cpu().numpy()
        del pkb
    if not a.no_adjoint:
        # the exact adjoint (a transpose pass of every stage) on the reconstructed volume
        da = torch.empty((p.m, p.nt), dtype=plan.dtype, device=plan.device)
        msa, _ = time_op(torch, plan, lambda: plan.adjoint(out, out=da), a.steps, a.warmup)
        _, sta = time_op(torch, plan, lambda: plan.adjoint(out, out=da), a.steps, 1, profile=True)
        res["adjoint"] = dict(ms_per_step=round(msa, 5), value=round(points / (msa / 1e3) / 1e6, 2),
                              unit="Mpts/s", stages_ms={k: round(v, 5) for k, v in sta.items()})
        del da
    # image measures of App. B on the reconstruction (GPU kernels)
    phantom = torch.as_tensor(synth.phantom_volume(p), dtype=plan.dtype, device=plan.device)
    msm, _ = time_op(torch, plan, lambda: N.mip(out, 2), a.steps, a.warmup)
    res["image_measures"] = dict(corrcoef_vs_phantom=round(N.corrcoef(out, phantom), 6),
                                 tenenbaum_depth_mip=N.tenenbaum(N.mip(out, 2)),
                                 mip_ms=round(msm, 5))
    del phantom
    if not a.no_lsq:
        # the step is fixed from a power iteration before the timed region
        lsq_res = {}
        for model in ("adjoint", "q"):
            eta = 0.95 / max(N.power_norm(plan, iters=20, model=model), 1e-300)
            rhs = g if model == "adjoint" else plan.q(out)
            N.lsq(plan, rhs, iters=2, eta=eta, model=model)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, losses = N.lsq(plan, rhs, iters=20, eta=eta, model=model)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            lsq_res[model] = dict(ms_per_iteration=round(dt * 1e3 / 20, 4),
                                  loss_ratio=float(losses[-1] / losses[0]) if losses[0] else None)
        res["least_squares"] = lsq_res
    if a.workload == "c2" and not a.no_2d:
        p2 = synth.config("c8")
        plan2 = N.Plan(p2.xy, p2.nt, p2.dt, (p2.n1, p2.n2, p2.n3), c=p2.c, h=p2.h, d1=p2.d1,
                       d2=p2.d2, precision=a.precision)
        g2 = torch.as_tensor(p2.g, dtype=plan2.dtype, device=plan2.device).contiguous()
        o2 = torch.empty((p2.n1, p2.n2, p2.n3), dtype=plan2.dtype, device=plan2.device)
        ms2, _ = time_steps(torch, plan2, g2, o2, a.steps, a.warmup)
        _, st2 = time_steps(torch, plan2, g2, o2, a.steps, 1, profile=True)
        res["two_dimensional"] = dict(workload=f"c8: {WORKLOADS['c8']}", ms_per_step=round(ms2, 5),
                                      value=round(p2.m * p2.nt / (ms2 / 1e3) / 1e6, 2), unit="Mpts/s",
                                      stages_ms={k: round(v, 5) for k, v in st2.items()})
        del plan2, g2, o2
    qsample = None
    if not a.no_q:
        # the forward operator Q (initial pressure -> sensor traces) on the
        # reconstructed volume, and its adjoint on the data
        dq = torch.empty((p.m, p.nt), dtype=plan.dtype, device=plan.device)
        vq = torch.empty_like(out)
        msq, stq = time_op(torch, plan, lambda: plan.q(out, out=dq), a.steps, a.warmup)
        _, stq = time_op(torch, plan, lambda: plan.q(out, out=dq), a.steps, 1, profile=True)
        msqa, _ = time_op(torch, plan, lambda: plan.q_adjoint(g, out=vq), a.steps, a.warmup)
        _, stqa = time_op(torch, plan, lambda: plan.q_adjoint(g, out=vq), a.steps, 1, profile=True)
        res["forward_model_q"] = dict(
            ms_per_step=round(msq, 5), value=round(points / (msq / 1e3) / 1e6, 2), unit="Mpts/s",
            adjoint_ms_per_step=round(msqa, 5),
            stages_ms={k: round(v, 5) for k, v in stq.items()},
            adjoint_stages_ms={k: round(v, 5) for k, v in stqa.items()})
        qsample = dq.cpu().numpy()
    if not a.no_cpu_baseline:
        vref, cb = cpu_baseline(p)
        res["cpu_baseline"] = cb
        nrm = float(np.linalg.norm(vref))
        res["rel_l2_vs_oracle"] = float(np.linalg.norm(vol.astype(np.float64) - vref) / nrm)
        if vol64 is not None:
            res["fp64_plain"]["rel_l2_vs_oracle"] = float(np.linalg.norm(vol64 - vref) / nrm)
        if volkb is not None:
            res["kaiser_bessel_w8"]["rel_l2_vs_oracle"] = float(
                np.linalg.norm(volkb.astype(np.float64) - vref) / nrm)
        if qsample is not None:
            res["forward_model_q"]["sampled_rel_l2_vs_oracle"] = q_sample_error(p, vol, qsample)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
