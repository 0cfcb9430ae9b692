"""Benchmark: field updates (Nz x range steps) per second of the batched spectral
split-step Pade march on one MI355X.

Default workload (broadband): 256 frequencies uniformly in 50..300 Hz on the deep-ocean Munk
profile (H = 5000 m, c0 = 1500 m/s), Nz = round(16 H f / 1500) = 2667 .. 16000 (uneven),
[6/6] Pade, dr = 25 m, Neumann tol 1e-10 (cap 48), TL every 40 steps, one plan per
frequency, all marched together from device memory (ssp_march_batch_async, the launches
recorded in a HIP graph).  A bench "step" is one range step of the whole batch (every Pade
factor and every Neumann term of every solve); inputs are resident in HBM before the timed
region and the TL rows stay in device arrays.  Beside it: the deep Munk waveguide at
Nz = 4096 (512 solves, key "munk4096") and the continuous-batching server on a Poisson
request stream (key "serving", p50/p99 latency).

Other workloads (--workload): munk4096 (512 solves at Nz = 4096, 50 Hz), eddy16384 (Munk +
Gaussian eddy at 200 Hz, Nz = 16384, [8/8], Neumann <= 12, potential rebuilt on the device
every step), serving, homogeneous, modal8001.

Prints ONE JSON line (contract of the driver).  Beside the metric it reports the roofline of
the dominant kernel, the plain one-kernel-per-stage form and the fused kernel on a single
solve (same arithmetic, identical results), the stand-alone transforms and the FP64 oracle
on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

PEAK_FP32 = 157.3e12   # MI355X published FP32 vector peak (FLOP/s)
PEAK_HBM = 8.0e12      # MI355X HBM3E (B/s)

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE) of `bench.py [--steps 40 --warmup 40 | --workload munk4096 --steps 100 --warmup
# 10 | --workload eddy16384 --steps 50 --warmup 10] --roof-launches 2 --copy-calibration 1024
# --no-extras`, averaged over the two roofline launches, each counter scaled by its reading
# for a plain 1 GiB device copy in the same run (FETCH_SIZE reads 0.5x the bytes moved,
# WRITE_SIZE 1.0x).  Keyed by the workload's launch
# shape (workload, Nz or FFT length of the dominant group, solves, steps per launch) and a
# fingerprint of the kernel sources and layout table: any change to their code (comments
# aside) makes the figure stale, and it is then reported as null.
TRAFFIC = {
    ("broadband", 32768, 150, 40): {"fingerprint": "c910d553603787a2", "fetch": 5.5848e+11,
                                    "write": 2.3530e+11},
    ("munk4096", 4096, 512, 100): {"fingerprint": "c910d553603787a2", "fetch": 3.0074e+07,
                                   "write": 1.6567e+09},
    ("eddy16384", 16384, 256, 50): {"fingerprint": "c910d553603787a2", "fetch": 8.7358e+11,
                                    "write": 5.8745e+11},
}


def source_fingerprint(root=None):
    """Hash of the kernel sources and layout table with comments and blank lines removed, so
    that only code changes make a measured traffic figure stale."""
    import hashlib
    h = hashlib.sha256()
    for f in ("ssp_device.hip", "ssp_device.h", "ssp_tuned.h"):
        with open(os.path.join(root or ROOT, "paper_2511_03343_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        code = "\n".join(line.rstrip() for line in src.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, nz, batch, chunk, bc="dirichlet"):
    t = TRAFFIC.get((workload, nz, batch, chunk)) if bc == "dirichlet" else None
    if t is None or t["fingerprint"] != source_fingerprint():
        return None
    return t["fetch"] + t["write"]


def algorithmic_flops(nz, pade_order, terms, steps, outputs):
    """Algorithmic FP32 work of the range step: every Neumann term costs two DSTs
    (5 Nz log2 Nz each) plus 8 Nz pointwise; every Pade factor 16 Nz; every output one
    DST."""
    tr = 5.0 * nz * math.log2(nz)
    return terms * 2 * (tr + 8 * nz) + steps * pade_order * 16 * nz + outputs * tr


def _solve(workload, nz=None, nsteps=None, zs=None, index=None, bc="dirichlet"):
    """The Solve of one job of a workload (index: frequency index of the broadband set;
    bc: boundary condition of the device-batch workloads)."""
    if workload == "munk4096":
        s = W.munk_deep(nz=nz or 4096)
    elif workload == "homogeneous":
        s = W.homogeneous_waveguide()
    elif workload == "modal8001":
        s = W.first_experiment()
    elif workload == "eddy16384":
        s = W.munk_eddy(nz=nz or 16384)
    elif workload == "serving":
        s = W.serving_requests(duration=0.2)[index].solve
    else:
        s = W.broadband()[index]
    if nsteps is not None:
        s.nsteps = nsteps
    if zs is not None:
        s.zs = zs
    s.bc = bc
    return s


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_worker(args):
    """March one solve with the oracle: `skip` range steps untimed (the benchmark's warm-up),
    then timed chunks of range steps until `seconds` have passed (a step's cost changes along
    the range as the field spreads).  Returns (timed field updates, seconds, last step)."""
    workload, nz, seconds, zs, index, bc, layer, skip = args
    import scipy.fft  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)   # one thread per solve process: `cores` counts the processes
    from oracle import Plan
    s = _solve(workload, nz, None, zs, index, bc)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol,
              rotation=s.rotation, bc=s.bc)
    eta = None if layer is None else W.absorbing_layer(s.nz, s.depth, layer[0], layer[1], s.bc)
    chunk = 4
    psi, done, spent, timed = s.starter(), 0, 0.0, 0
    while done < s.nsteps and (done < skip or spent < seconds):
        k = min(chunk, s.nsteps - done, skip - done) if done < skip else min(chunk, s.nsteps - done)
        c = s.profile(done, k) if s.env == "munk+eddy" else s.profile()
        t = time.perf_counter()
        res = pl.march(psi, k, c, out_every=s.out_every, r0=done * s.dr, absorber=eta)
        if done >= skip:
            spent += time.perf_counter() - t
            timed += k
        psi, done = res.final, done + k
    return s.nz * timed, spent, done


def cpu_baseline(workload, nz, seconds_target=20.0, bc="dirichlet", layer=None, skip=0):
    """The FP64 oracle on the host cores: one solve per single-threaded process, each
    marching for a bounded time."""
    cores = max(1, min(16, os.cpu_count() or 1))
    if workload == "serving":
        jobs = [("serving", None, seconds_target, None, i, bc, None, skip) for i in range(cores)]
        what = f"the first {cores} requests of the stream"
    elif workload == "broadband":
        # every 16th frequency (uneven Nz)
        jobs = [(workload, None, seconds_target, None, i, bc, None, skip)
                for i in range(0, 256, 256 // cores)][:cores]
        what = f"{len(jobs)} of the 256 frequencies (every {256 // cores}th)"
    else:
        lo, hi = {"homogeneous": (20.0, 180.0), "modal8001": (100.0, 3900.0)}.get(workload, (50.0, 2000.0))
        zs = W.source_depths(cores, lo, hi)
        jobs = [(workload, nz, seconds_target, float(z), None, bc, layer, skip) for z in zs]
        what = f"{cores} solves of the Nz={nz} {workload} workload"
        if bc != "dirichlet":
            what += f" ({bc} boundaries)"
        if layer is not None:
            what += f" (absorbing layer {layer[0]:g} m, eta {layer[1]:g})"
        if workload == "modal8001":
            what += " (Gaussian starters: with every series cut at M = 2 a step costs the same for any starter)"
    log(f"cpu baseline: {what}, about {seconds_target:g} s each on {cores} processes")
    res = []
    with mp.get_context("spawn").Pool(cores) as pool:
        for r in pool.imap_unordered(_oracle_worker, jobs):
            res.append(r)
            log(f"cpu baseline: {len(res)}/{len(jobs)} solves done")
    total = sum(r[0] for r in res)
    spent = max(r[1] for r in res)
    lo_s, hi_s = min(r[2] for r in res), max(r[2] for r in res)
    # the processes run side by side: the host's rate is the sum of theirs
    rate = sum(r[0] / r[1] for r in res if r[1] > 0)
    return {"value": rate, "unit": "field updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}: {skip} warm-up range steps untimed (as on the GPU), then chunks of 4 "
                      f"steps for about {seconds_target:g} s each (up to step {lo_s} .. {hi_s}; "
                      f"{total:.3g} timed field updates; FP64, one single-threaded solve per process, "
                      f"{spent:.1f} s of the slowest process)"}


DEFAULTS = {  # batch, timed steps, warmup steps, steps per launch
    "munk4096": (512, 400, 20, 100),
    "homogeneous": (1024, 1000, 20, 200),
    "eddy16384": (256, 100, 10, 50),
    "broadband": (256, 400, 40, 40),
    "serving": (1024, 0, 0, 50),
    "modal8001": (512, 500, 20, 100),
}
DESCRIPTIONS = {
    "homogeneous": "homogeneous Dirichlet waveguide, H=200 m, c=1500 m/s, 100 Hz, Nz=256, rotated [4/4] "
                   "Pade (alpha=pi/16), dr=5 m, V=0 (no Neumann terms), TL every 10 steps",
    "munk4096": "deep Munk waveguide, Nz=4096, [6/6] Pade, dr=25 m, 50 Hz, Neumann tol 1e-10 "
                "(cap 48), TL every 4 steps",
    "eddy16384": "Munk + Gaussian eddy, Nz=16384, [8/8] Pade, dr=20 m, 200 Hz, Neumann tol 1e-10 "
                 "(cap 12), potential on device every step, TL every 5 steps",
    "broadband": "256 frequencies 50..300 Hz, Munk, Nz=2667..16000 (16 pts/wavelength), [6/6] Pade, "
                 "dr=25 m, Neumann tol 1e-10 (cap 48), TL every 40 steps to device arrays",
    "modal8001": "range-independent Munk waveguide of the paper's first experiment: H=4 km, 100 Hz, "
                 "Nz=8001, [4/4] Pade, dr=100 m, Neumann series cut at M=2, normal-mode starters "
                 "(one device eigendecomposition for all source depths), TL every 10 steps",
    "serving": "Poisson request stream: f ~ U[25, 400] Hz, Nz a power of two 512..16384 (>= 4 pts/"
               "wavelength), range U[10, 100] km, Munk or Munk + eddy, [6/6], dr = max(25 m, 5/k0), "
               "continuous batching, TL rows to host every tick",
}


def _describe(workload, nz):
    text = DESCRIPTIONS[workload]
    if nz is not None:
        text = re.sub(r"Nz=[0-9.]+(?:\.\.[0-9]+)?", f"Nz={nz}", text, count=1)
    return text


def make_plan(ssp, s):
    pl = ssp.ssp_plan_create_bc(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max,
                                s.tol, s.bc)
    if s.rotation:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ROTATION, s.rotation)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, s.out_every)
    if s.env == "munk+eddy":
        e = s.eddy or W.Eddy()
        ssp.ssp_set_profile_analytic(pl, eddy=(e.amp, e.r0, e.rr, e.z0, e.rz))
    else:
        ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
    return pl


def plain_vs_fused(ssp, s, nsteps):
    """The plain one-kernel-per-stage form and the fused kernel, each on one solve."""
    out = {}
    for engine, key in ((1, "plain_one_solve"), (0, "fused_one_solve")):
        p1 = make_plan(ssp, s)
        ssp.ssp_plan_set_option(p1, ssp.SSP_OPT_PLAIN, engine)
        ssp.ssp_march(p1, s.nz, s.starter(), 2, want_field=False, want_tl=False)
        t1 = time.perf_counter()
        ssp.ssp_march(p1, s.nz, None, nsteps, want_field=False, want_tl=True)
        dt = time.perf_counter() - t1
        ssp.ssp_plan_destroy(p1)
        out[key] = s.nz * nsteps / dt
    out["unit"] = "field updates/s"
    out["steps"] = nsteps
    out["nz"] = s.nz
    return out


def run_device_batch(args, ssp, torch, stream, dev):
    """One plan, a batch of B solves marched on the device (munk4096, eddy16384)."""
    s = _solve(args.workload, args.nz, bc=args.bc)
    B = args.batch
    pl = make_plan(ssp, s)
    if args.absorber is not None:
        ssp.ssp_set_absorber(pl, W.absorbing_layer(s.nz, s.depth, args.absorber[0], args.absorber[1], s.bc))
    ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GRAPH, 1 if args.graph else 0)
    layout, threads, P = ssp.ssp_plan_engine(pl)
    # direct transforms (no chirp-z): 1 periodic with P = Nz, 2 Dirichlet with P = 2 (Nz + 1)
    direct = 1 if (s.bc == "periodic" and P == s.nz) else (
        2 if (s.bc == "dirichlet" and P == 2 * (s.nz + 1)) else 0)

    zs = (W.source_depths(B, 20.0, 180.0) if args.workload == "homogeneous"
          else W.source_depths(B, 100.0, 3900.0) if args.workload == "modal8001"
          else W.source_depths(B, 50.0, 2000.0))
    starter_s = None
    if args.workload == "modal8001":
        t_st = time.perf_counter()
        psi, kappa = ssp.ssp_modal_starter(pl, s.profile()[0], zs)
        starter_s = time.perf_counter() - t_st
        log(f"modal starters: {B} sources, {len(kappa)} modes, {starter_s:.2f} s")
    else:
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z, s.bc) for z in zs])
    d_psi = torch.from_numpy(psi.astype(np.complex64)).to(dev)
    d_step = torch.zeros(B, dtype=torch.int64, device=dev)
    d_stats = torch.zeros((B, 48), dtype=torch.uint8, device=dev)
    nout_chunk = args.chunk // s.out_every + 1
    d_tl = torch.empty((B, nout_chunk, s.nz), dtype=torch.float32, device=dev)
    ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())

    # steps per launch: every timed and warm-up launch marches k steps, so that the
    # recorded graph is replayed in the timed region
    kstep = max(1, min(args.chunk, args.steps or args.chunk))

    def run(nsteps, with_tl=True, events=None):
        done = 0
        while done < nsteps:
            k = kstep
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            ssp.ssp_march_device(pl, B, d_psi.data_ptr(), d_step.data_ptr(), k,
                                 d_tl.data_ptr() if with_tl else 0, d_stats.data_ptr())
            if events is not None:
                e1.record(stream)
                events.append((e0, e1, k))
            done += k

    # warm-up, then the timed region: the whole workload (march + TL outputs)
    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_steps = -(-args.steps // kstep) * kstep if args.steps > 0 else 0
    updates = B * s.nz * timed_steps

    # roofline of the dominant kernel (the fused march): launches without outputs, timed
    # with events on the stream they run on; algorithmic work from the per-solve Neumann
    # term counts of each launch
    events, flops = [], []
    for _ in range(args.roof_launches):
        run(kstep, with_tl=False, events=events)
        torch.cuda.synchronize()
        st = _stats(d_stats)
        flops.append(sum(algorithmic_flops(s.nz, s.pade_order, t, kstep, 0)
                         for t in st["terms_list"]))
    launch_s = [a.elapsed_time(b) / 1e3 for a, b, _ in events]
    achieved = sum(flops) / sum(launch_s)
    stats = _stats(d_stats)
    ssp.ssp_plan_destroy(pl)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
            "traffic": measured_traffic(args.workload, s.nz, B, kstep, args.bc)
            if args.absorber is None else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": (f"k_march_direct<{P}, {layout}, {direct}>" if direct
                       else f"k_march<{P}, {layout}>") + f" ({threads} threads per workgroup)",
            "avg_launch_ms": 1e3 * sum(launch_s) / len(launch_s),
            "steps_per_launch": kstep,
            "neumann_terms_per_solve_step": stats["terms"] / B / kstep}
    config = {"batch_solves": B, "nz": s.nz, "range_steps_timed": timed_steps,
              "steps_per_launch": kstep, "hip_graph": bool(args.graph), "boundary": s.bc}
    if args.absorber is not None:
        config["absorber"] = {"thickness_m": args.absorber[0], "eta_max": args.absorber[1]}
    if starter_s is not None:
        config["modal_starters"] = {"sources": B, "modes": int(len(kappa)), "seconds": starter_s,
                                    "note": "FP64 eigendecomposition on the device, outside the timed region"}
    plain = None
    if args.plain_steps > 0 and not direct:
        plain = plain_vs_fused(ssp, s, args.plain_steps)
        plain["fused_batched_over_plain"] = (updates / wall) / plain["plain_one_solve"]
    return updates, wall, roof, config, sorted(set(stats["status"])), plain, s.nz


def run_broadband(args, ssp, torch, stream, dev):
    """The 256 plans of the broadband set (uneven Nz) marched together from device memory:
    ssp_march_batch_async, TL rows to device arrays, the launches recorded once in a HIP
    graph and replayed (one graph launch per call of `chunk` steps)."""
    solves = W.broadband()
    plans = [make_plan(ssp, s) for s in solves]
    nzs = [s.nz for s in solves]
    n = len(plans)
    for pl in plans:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, -2)   # layouts tuned on a mixed batch
    if args.layouts:
        chosen = {int(k): int(v) for k, v in (kv.split("=") for kv in args.layouts.split(","))}
        for pl in plans:
            P = ssp.ssp_plan_engine(pl)[2]
            if P in chosen:
                ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, chosen[P])
    ssp.ssp_plan_set_option(plans[0], ssp.SSP_OPT_GRAPH, 1 if args.graph else 0)
    for pl, s in zip(plans, solves):
        ssp.ssp_set_field(pl, s.starter(), s.nz)
    # steps per call: every timed call (and every warm-up call) marches k steps, so that the
    # recorded graph is replayed in the timed region
    k = max(1, min(args.chunk, args.steps or args.chunk))
    d_tl = [torch.empty((k // s.out_every + 1, s.nz), dtype=torch.float32, device=dev) for s in solves]
    tl_ptrs = [t.data_ptr() for t in d_tl]

    def call(sub, steps, ptrs):
        ssp.ssp_march_batch_async(sub, [steps] * len(sub), ptrs)

    warm_calls = -(-args.warmup // k) if args.warmup > 0 else 0
    for _ in range(warm_calls):
        call(plans, k, tl_ptrs)
    st, stats = ssp.ssp_batch_stats(plans)
    torch.cuda.synchronize()
    calls = -(-args.steps // k) if args.steps > 0 else 0
    t0 = time.perf_counter()
    for _ in range(calls):
        call(plans, k, tl_ptrs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed_steps = calls * k
    st, stats = ssp.ssp_batch_stats(plans)
    updates = sum(nzs) * timed_steps
    statuses = {x["status"] for x in stats}
    layouts = {}
    for pl in plans:
        v, t, P = ssp.ssp_plan_engine(pl)
        layouts[P] = v

    # roofline of the dominant kernel: the split-transform group (FFT length 32768, the
    # largest solves, whose launch sets the call's time) marched alone for roof_launches
    # calls of k steps without outputs, timed with events on the stream it runs on;
    # algorithmic work from the per-solve Neumann term counts of each call
    P_of = [ssp.ssp_plan_engine(pl)[2] for pl in plans]
    Pdom = max(P_of)
    sub = [pl for pl, P in zip(plans, P_of) if P == Pdom]
    sub_s = [s for s, P in zip(solves, P_of) if P == Pdom]
    events, flops = [], []
    for _ in range(args.roof_launches):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call(sub, k, None)
        e1.record(stream)
        _, sst = ssp.ssp_batch_stats(sub)
        events.append((e0, e1))
        flops.append(sum(algorithmic_flops(s.nz, s.pade_order, x["neumann_terms"], k, 0)
                         for s, x in zip(sub_s, sst)))
        statuses |= {x["status"] for x in sst}
    torch.cuda.synchronize()
    launch_s = [a.elapsed_time(b) / 1e3 for a, b in events]
    achieved = sum(flops) / sum(launch_s) if launch_s else 0.0
    terms_step = sum(x["neumann_terms"] for x in stats) / n / k
    v_dom, t_dom, _ = ssp.ssp_plan_engine(sub[0])
    for pl in plans:
        ssp.ssp_plan_destroy(pl)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
            "traffic": measured_traffic("broadband", Pdom, len(sub), k),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": f"k_march<{Pdom}, {v_dom}> ({t_dom} threads per workgroup): the {len(sub)} solves "
                      f"with FFT length {Pdom}, whose launch sets the call's time",
            "avg_launch_ms": 1e3 * sum(launch_s) / len(launch_s) if launch_s else None,
            "steps_per_launch": k,
            "neumann_terms_per_solve_step": sum(flops) and (
                sum(x["neumann_terms"] for x in sst) / len(sub) / k)}
    config = {"solves": n, "nz_min": min(nzs), "nz_max": max(nzs), "sum_nz": sum(nzs),
              "range_steps_timed": timed_steps, "warmup_steps_run": warm_calls * k, "steps_per_call": k,
              "hip_graph": bool(args.graph), "layouts_by_fft_length": layouts,
              "neumann_terms_per_solve_step": terms_step,
              "outputs": "TL every 40 steps to device arrays (no host copies in the timed region)"}
    plain = None
    if args.plain_steps > 0:
        plain = plain_vs_fused(ssp, solves[-1], args.plain_steps)
        plain["fused_batched_over_plain"] = (updates / wall) / plain["plain_one_solve"]
    return updates, wall, roof, config, sorted(statuses), plain, None


PEAK_FP16_MFMA = 2.5e15   # MI355X dense fp16/bf16 matrix peak (FLOP/s)


def transform_rooflines(ssp, torch, stream, dev, reps=20):
    """Stand-alone batched transforms, each timed with events on its stream:
    the FFT-path DST (HBM-bound: 16 B per point read + written), chirp-z at Nz = 4096 and
    direct at Nz = 4095, and
    the dense DST on the matrix cores at Nz = 2048 (three fp16 products of 2 Nz^2 flops per
    real column)."""
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    # achievable HBM bandwidth: a plain device copy of 1 GiB (read + write), the reference
    # beside the datasheet peak for the FFT-path fractions below
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        a.fill_(1.0)

    def copy_once():
        with torch.cuda.stream(stream):  # on the stream the events are recorded on
            b.copy_(a)
    tc = timed(copy_once)
    copy_gbs = 2.0 * a.numel() * 4 / tc
    del a, b
    out["hbm_copy"] = {"kernel": "torch copy_ (1 GiB)", "achieved": copy_gbs / 1e9, "peak": PEAK_HBM / 1e9,
                       "unit": "GB/s", "frac": copy_gbs / PEAK_HBM}
    # chirp-z at Nz = 4096; the direct sine transform (one FFT of length 2 (Nz + 1)) at 4095
    for key, nz, kernel in (("dst_fft", 4096, f"k_transform<{_fft_len(4096)}, 0>"),
                            ("dst_fft_direct", 4095, "k_transform<8192, 2>")):
        B = 4096
        pl = ssp.ssp_plan_create(nz, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10)
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        x = torch.randn((B, nz), dtype=torch.complex64, device=dev)
        y = torch.empty_like(x)
        t = timed(lambda: ssp.ssp_dst_device(pl, B, x.data_ptr(), y.data_ptr()))
        ssp.ssp_plan_destroy(pl)
        gbs = 16.0 * nz * B / t
        out[key] = {"kernel": kernel, "nz": nz, "vectors": B, "bound": "hbm", "achieved": gbs / 1e9,
                    "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": gbs / PEAK_HBM,
                    "frac_of_copy": gbs / copy_gbs, "ms_per_call": 1e3 * t}
    nz, B = 2048, 1024
    pl = ssp.ssp_plan_create(nz, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10)
    ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
    x = torch.randn((B, nz), dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    t = timed(lambda: ssp.ssp_dst_dense_device(pl, B, x.data_ptr(), y.data_ptr()))
    ssp.ssp_plan_destroy(pl)
    alg = 2.0 * nz * nz * 2 * B
    out["dst_dense"] = {"kernel": "k_dense_split + k_dense_gemm", "nz": nz, "vectors": B,
                        "bound": "mfma", "achieved": 3 * alg / t / 1e12,
                        "peak": PEAK_FP16_MFMA / 1e12, "unit": "TFLOP/s",
                        "frac": 3 * alg / t / PEAK_FP16_MFMA,
                        "algorithmic_tflops": alg / t / 1e12, "ms_per_call": 1e3 * t,
                        "dtype": "fp16x3 (FP32 accumulate)"}
    return out


def run_serving(args, ssp, torch, stream, dev):
    """Poisson request stream through the continuous-batching server (the whole stream, plan
    creation included, is the timed region)."""
    from paper_2511_03343_amd.serve import LibBackend, Server, from_solve, latency_summary
    stream_reqs = W.serving_requests(rate=args.rate, duration=args.duration)
    reqs = []
    for i, q in enumerate(stream_reqs):
        s = q.solve
        c = W.munk(W.depth_grid(s.nz, s.depth)) if s.env == "munk" else None
        reqs.append(from_solve(q.arrival, s, c_table=c, rid=i))
    srv = Server(LibBackend(stream.cuda_stream), max_active=args.batch, steps_per_tick=args.chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = srv.run(reqs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    updates = sum(r.nz * res[r.rid].steps_done for r in reqs)
    flops = sum(algorithmic_flops(r.nz, r.pade_order, res[r.rid].neumann_terms, res[r.rid].steps_done,
                                  res[r.rid].steps_done // r.out_every) for r in reqs)
    nzs = [r.nz for r in reqs]
    roof = {"bound": "alu", "achieved": flops / wall / 1e12, "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s", "frac": flops / wall / PEAK_FP32, "traffic": None,
            "kernel": "k_march family + per-length launches, whole stream",
            "neumann_terms_per_solve_step": sum(res[r.rid].neumann_terms for r in reqs) /
                                            max(1, sum(res[r.rid].steps_done for r in reqs))}
    config = {"requests": len(reqs), "arrival_rate_per_s": args.rate, "arrival_window_s": args.duration,
              "nz_min": min(nzs), "nz_max": max(nzs), "steps_per_tick": args.chunk,
              "max_active": args.batch, "ticks": srv.ticks, "peak_active": srv.peak_active,
              "host_plan_creation_s": srv.t_create, "march_calls_s": srv.t_march,
              "latency": latency_summary(res)}
    statuses = sorted({res[r.rid].status for r in reqs})
    return updates, wall, roof, config, statuses, None, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(DEFAULTS), default="broadband")
    ap.add_argument("--steps", type=int, default=None, help="timed range steps")
    ap.add_argument("--warmup", type=int, default=None, help="untimed range steps")
    ap.add_argument("--batch", type=int, default=None, help="solves marched together")
    ap.add_argument("--nz", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None, help="range steps per kernel launch")
    ap.add_argument("--roof-launches", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=8,
                    help="range steps of the plain-form comparison (0: skip)")
    ap.add_argument("--graph", type=int, default=1, help="replay recorded launches (HIP graph)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--duration", type=float, default=1.0, help="serving: arrival window (s)")
    ap.add_argument("--no-extras", action="store_true",
                    help="broadband: skip the deep Munk line and the serving stream")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB of a plain device copy run first (counter calibration)")
    ap.add_argument("--layouts", default=None, metavar="P=V[,P=V]",
                    help="broadband: engine layout per FFT length instead of the tuned one")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-transforms", action="store_true",
                    help="skip the stand-alone transform measurements")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--bc", choices=["dirichlet", "neumann", "periodic"], default="dirichlet",
                    help="boundary condition (Sec. 3.1) of the munk4096, eddy16384 and "
                         "homogeneous workloads")
    ap.add_argument("--absorber", default=None, metavar="THICKNESS,ETA",
                    help="complex absorbing layer at the bottom (Sec. 3.1): thickness in m and "
                         "the largest imaginary part of v, for the device-batch workloads")
    args = ap.parse_args()
    if (args.bc != "dirichlet" or args.absorber) and args.workload in ("broadband", "serving"):
        print("--bc and --absorber apply to the munk4096, eddy16384 and homogeneous workloads",
              file=sys.stderr)
        sys.exit(2)
    if args.absorber is not None:
        th, eta = (float(x) for x in args.absorber.split(","))
        args.absorber = (th, eta)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); every solve of the batch is "
              "independent, so several GPUs would each run their own batch", file=sys.stderr)
        sys.exit(2)
    b, st, wu, ch = DEFAULTS[args.workload]
    args.batch = args.batch or b
    args.steps = args.steps if args.steps is not None else st
    args.warmup = args.warmup if args.warmup is not None else wu
    args.chunk = args.chunk or ch

    import torch
    from paper_2511_03343_amd import ssp
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)           # default priority
    torch.cuda.set_stream(stream)

    if args.copy_calibration > 0:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # scale between those counters and bytes moved
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    runner = {"broadband": run_broadband, "serving": run_serving}.get(args.workload, run_device_batch)
    log(f"{args.workload}: batch {args.batch}, {args.warmup} warm-up + {args.steps} timed steps")
    updates, wall, roof, config, statuses, plain, nz = runner(args, ssp, torch, stream, dev)
    log(f"{args.workload}: {updates / wall:.4g} field updates/s")
    value = updates / wall
    # a step is one range step of the whole batch (serving: one tick)
    timed_steps = config.get("range_steps_timed") or config.get("ticks") or 1

    extras = {}
    if args.workload == "broadband" and not args.no_extras:
        # the deep Munk waveguide (Nz = 4096, 512 solves) and the Munk + eddy waveguide
        # (Nz = 16384, 256 solves) as device batches, and the continuous-batching server on
        # the Poisson stream
        ea = argparse.Namespace(**vars(args))
        ea.workload, ea.nz, ea.bc, ea.absorber = "munk4096", None, "dirichlet", None
        ea.batch, ea.steps, ea.warmup, ea.chunk, ea.plain_steps = 512, 100, 20, 100, 0
        ea.roof_launches = 1
        u2, w2, r2, c2, s2, _, _ = run_device_batch(ea, ssp, torch, stream, dev)
        extras["munk4096"] = {"workload": _describe("munk4096", None), "value": u2 / w2,
                              "unit": "field updates/s", "ms_per_step": 1e3 * w2 / c2["range_steps_timed"],
                              "status": s2, "roofline": r2, **c2}
        log(f"munk4096: {u2 / w2:.4g} field updates/s")
        # the range-dependent Munk + eddy waveguide at Nz = 16384 (potential on the device)
        eb = argparse.Namespace(**vars(args))
        eb.workload, eb.nz, eb.bc, eb.absorber = "eddy16384", None, "dirichlet", None
        eb.batch, eb.steps, eb.warmup, eb.chunk, eb.plain_steps = 256, 50, 10, 50, 0
        eb.roof_launches = 1
        u4, w4, r4, c4, s4, _, _ = run_device_batch(eb, ssp, torch, stream, dev)
        extras["eddy16384"] = {"workload": _describe("eddy16384", None), "value": u4 / w4,
                               "unit": "field updates/s", "ms_per_step": 1e3 * w4 / c4["range_steps_timed"],
                               "status": s4, "roofline": r4, **c4}
        log(f"eddy16384: {u4 / w4:.4g} field updates/s")
        sa = argparse.Namespace(**vars(args))
        sa.workload, sa.batch, sa.chunk = "serving", 1024, 50
        u3, w3, r3, c3, s3, _, _ = run_serving(sa, ssp, torch, stream, dev)
        lat = c3["latency"]
        extras["serving"] = {"workload": _describe("serving", None), "value": u3 / w3,
                             "unit": "field updates/s", "p50_s": lat.get("p50_s"), "p99_s": lat.get("p99_s"),
                             "requests": c3["requests"], "completed": lat.get("count"),
                             "arrival_rate_per_s": sa.rate, "arrival_window_s": sa.duration,
                             "clock": "virtual: each tick advances it by the tick's measured duration "
                                      "(admission, plan creation and the batched march), and it jumps to "
                                      "the next arrival when nothing is active; latency = finish - arrival",
                             "status": s3, **{k: v for k, v in c3.items() if k != "latency"}}
        log(f"serving: {u3 / w3:.4g} field updates/s, p50 {lat.get('p50_s')}, p99 {lat.get('p99_s')}")

    transforms = None if args.no_transforms else transform_rooflines(ssp, torch, stream, dev)
    if transforms is not None:
        log("stand-alone transforms measured")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.workload, nz, args.cpu_seconds, args.bc, args.absorber, args.warmup)

    out = {
        "metric": "field updates (Nz x range steps)/s at TL err<=0.1 dB",
        "value": value,
        "unit": "field updates/s",
        "n_gpus": 1,
        "steps": timed_steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / timed_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Munk profile and Gaussian starters)",
        "config": {"workload": _describe(args.workload, args.nz) + (
            f", {args.bc} boundaries (Sec. 3.1)" if args.bc != "dirichlet" else "") + (
            f", bottom absorbing layer {args.absorber[0]:g} m (eta up to {args.absorber[1]:g})"
            if args.absorber else ""), **config},
        "roofline": roof,
        "status": statuses,
        "plain_form": plain,
        "transforms": transforms,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


def _stats(d_stats):
    raw = d_stats.cpu().numpy()
    terms = raw[:, 16:24].copy().view(np.int64).ravel()
    status = raw[:, 40:44].copy().view(np.int32).ravel()
    return {"terms": int(terms.sum()), "terms_list": [int(t) for t in terms],
            "status": [int(x) for x in status]}


def _fft_len(nz):
    p = 128
    while p < 2 * nz - 1:
        p *= 2
    return p


if __name__ == "__main__":
    main()
