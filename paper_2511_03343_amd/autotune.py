"""Autotuner of the march: engine layouts per FFT length, the layouts of batches that mix
lengths, and the transform engine (FFT or dense) per (Nz, Pade order) class.

The march kernel of an FFT length P can run in up to three layouts (SSP_OPT_VARIANT):
different thread counts, i.e. different elements per thread and radix of the first and
last FFT passes, with different register / LDS residency (which of the series sum,
potential and multipliers stay in registers follows from the layout; layout 2 uses one LDS
buffer so that two workgroups share a compute unit).  For every length with more than one
layout this script marches a full device batch of a representative solve (deep Munk
waveguide at 50 Hz, [6/6], dr = 25 m) in each layout, times the launches with HIP events on
their stream, checks that the layouts agree to rounding, and writes the fastest into
csrc/ssp_tuned.h.  It does so for each transform kind, on a grid of that kind: chirp-z
(Dirichlet, Nz = P/2), direct Fourier (periodic, Nz = P) and direct sine (Dirichlet,
Nz = P/2 - 1).

--what mixed: the layouts of the lengths that share a batch of uneven Nz (SSP_OPT_VARIANT =
-2): the broadband set (256 frequencies, FFT lengths 8192, 16384 and 32768) plus 64 plans at
Nz = 2048 (length 4096) marched together by ssp_march_batch_async, every combination of the
layouts of 4096, 8192 and 16384 timed on the whole call (the split length has one layout).

--what engine: for Nz = 256, 512, 1024, 2048 and Pade orders 4, 6, 8 a device batch of 128
solves marched with the FFT engine and with the dense engine (SSP_ENGINE_AUTO then takes the
faster; orders above 8 take the order-8 choice).

Each part rewrites its own table of csrc/ssp_tuned.h and keeps the others.  Rebuild the
library afterwards.

    python -m paper_2511_03343_amd.autotune [--what layouts|mixed|engine|all] [--write [--out PATH]]

The synthetic inputs come from workloads/ (seeded); nothing here computes the method.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(HERE, "csrc", "ssp_tuned.h")
LENGTHS = [128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768]


def _engine_threads(P: int, v: int) -> int:
    """Thread counts of the layouts (the same rule as the kernels)."""
    PE = P // 2 if P > 16384 else P
    t0 = 64 if PE <= 512 else (128 if PE == 1024 else (256 if PE <= 4096 else 1024))
    if P > 16384:  # the split engine has one layout
        return t0
    t1 = {1024: 64, 2048: 128, 4096: 512, 8192: 512}.get(PE, t0)
    t2 = {4096: 128, 8192: 256, 16384: 512}.get(PE, t0)
    return (t0, t1, t2)[v]


# transform kinds: (name, boundary condition, grid length for FFT length P)
KINDS = [("chirp", "dirichlet", lambda P: P // 2), ("fourier", "periodic", lambda P: P),
         ("sine", "dirichlet", lambda P: P // 2 - 1)]


def time_layout(ssp, torch, P: int, variant: int, batch: int, steps: int, reps: int, kind=KINDS[0]):
    sys.path.insert(0, ROOT)
    import dataclasses
    import workloads as W
    nz = kind[2](P)
    s = dataclasses.replace(W.munk_deep(nz=nz), bc=kind[1])
    stream = torch.cuda.Stream()
    pl = ssp.ssp_plan_create_bc(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol, s.bc)
    try:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, variant)
        ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
        zs = W.source_depths(batch, 50.0, 2000.0)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z, s.bc) for z in zs])
        with torch.cuda.stream(stream):
            d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
            d_step = torch.zeros(batch, dtype=torch.int64, device="cuda")
        stream.synchronize()
        ssp.ssp_to_sine(pl, batch, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, batch, d_psi.data_ptr(), d_step.data_ptr(), 2)  # warm-up
        stream.synchronize()
        best = math.inf
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ssp.ssp_march_device(pl, batch, d_psi.data_ptr(), d_step.data_ptr(), steps)
            e1.record(stream)
            stream.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        out = d_psi.cpu().numpy()
    finally:
        ssp.ssp_plan_destroy(pl)
    return best, out


def read_tables(path: str = HEADER) -> dict:
    """The current tables of the header (kTunedVariant, kTunedDirect, kTunedMixed,
    kTunedEngine) as nested lists."""
    import re
    txt = open(path).read()
    out = {}
    for name in ("kTunedVariant", "kTunedDirect", "kTunedMixed", "kTunedEngine"):
        m = re.search(name + r"\[[^=]*=\s*(\{.*?\});", txt, flags=re.S)
        if m:
            out[name] = json.loads(m.group(1).replace("{", "[").replace("}", "]"))
    out.setdefault("kTunedVariant", [0] * 9)
    out.setdefault("kTunedDirect", [[0] * 9, [0] * 9])
    out.setdefault("kTunedMixed", list(out["kTunedVariant"]))
    out.setdefault("kTunedEngine", [[0] * 4 for _ in range(4)])
    return out


def write_header(tables: dict, path: str = HEADER) -> None:
    def arr(v):
        return "{" + ", ".join(arr(x) if isinstance(x, list) else str(int(x)) for x in v) + "}"
    with open(path, "w") as f:
        f.write("// ssp_tuned.h - engine layout of the fused march kernel per FFT length, chosen by\n"
                "// paper_2511_03343_amd/autotune.py (written by that script; do not edit by hand).\n"
                "#pragma once\n\n"
                "namespace ssp {\n"
                "// kTunedVariant[log2(P) - 7] for P = 128 ... 32768\n"
                f"constexpr int kTunedVariant[9] = {arr(tables['kTunedVariant'])};\n"
                "// kTunedDirect[kind - 1][log2(P) - 7]: direct Fourier (periodic Nz = P), direct sine\n"
                "// (Dirichlet Nz = P/2 - 1)\n"
                f"constexpr int kTunedDirect[2][9] = {arr(tables['kTunedDirect'])};\n"
                "// kTunedMixed[log2(P) - 7]: chirp-z layouts for batches that mix FFT lengths\n"
                "// (SSP_OPT_VARIANT = -2), measured on a mixed-length batch\n"
                f"constexpr int kTunedMixed[9] = {arr(tables['kTunedMixed'])};\n"
                "// kTunedEngine[Nz class][p class]: 1 = dense engine, 0 = FFT engine, for SSP_ENGINE_AUTO;\n"
                "// Nz classes <= 256, <= 512, <= 1024, <= 2048; p classes <= 4, 5-6, 7-8, >= 9\n"
                f"constexpr int kTunedEngine[4][4] = {arr(tables['kTunedEngine'])};\n"
                "\n"
                "inline int tuned_engine(int nz, int p) {\n"
                "    const int nc = nz <= 256 ? 0 : nz <= 512 ? 1 : nz <= 1024 ? 2 : 3;\n"
                "    const int pc = p <= 4 ? 0 : p <= 6 ? 1 : p <= 8 ? 2 : 3;\n"
                "    return nz <= 2048 ? kTunedEngine[nc][pc] : 0;\n"
                "}\n"
                "}  // namespace ssp\n")


def tune_layouts(ssp, torch, args, tables):
    choice = {}
    for kind in KINDS:
        for P in LENGTHS:
            if kind[0] != "chirp" and (P > 16384 or kind[2](P) < 2):
                continue  # direct transforms exist up to FFT length 16384
            layouts = [v for v in range(3) if v == 0 or _engine_threads(P, v) != _engine_threads(P, 0)]
            if len(layouts) == 1:
                choice[(kind[0], P)] = 0
                continue
            # enough solves for several workgroups per compute unit at every layout
            batch = 512 if P >= 8192 else 1024
            times, fields = [], []
            for v in layouts:
                t, f = time_layout(ssp, torch, P, v, batch, args.steps, args.reps, kind)
                times.append(t)
                fields.append(f)
            diffs = [float(np.linalg.norm(f - fields[0]) / np.linalg.norm(fields[0])) for f in fields]
            assert max(diffs) < 1e-5, f"layouts of {kind[0]} P={P} disagree beyond rounding ({max(diffs):.2e})"
            choice[(kind[0], P)] = layouts[int(np.argmin(times))]
            row = {"part": "layouts", "kind": kind[0], "P": P, "nz": kind[2](P), "batch": batch,
                   "steps": args.steps, "layouts": layouts, "threads": [_engine_threads(P, v) for v in layouts],
                   "ms": [round(1e3 * t, 3) for t in times], "chosen": choice[(kind[0], P)],
                   "layout_difference_relL2": max(diffs)}
            print(json.dumps(row), flush=True)
    tables["kTunedVariant"] = [choice.get(("chirp", P), 0) for P in LENGTHS]
    tables["kTunedDirect"] = [[choice.get((k, P), 0) for P in LENGTHS] for k in ("fourier", "sine")]


def _mixed_solves():
    sys.path.insert(0, ROOT)
    import workloads as W
    solves = W.broadband()
    for i in range(64):  # FFT length 4096: Nz = 2048 at 40 .. 120 Hz
        s = W.munk_deep(nz=2048)
        s.freq = 40.0 + 80.0 * i / 63
        s.out_every = 40
        solves.append(s)
    return solves


def tune_mixed(ssp, torch, args, tables):
    import itertools
    solves = _mixed_solves()
    stream = torch.cuda.Stream()
    plans = []
    try:
        for s in solves:
            pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
            ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
            ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
            plans.append(pl)
        P_of = [ssp.ssp_plan_engine(pl)[2] for pl in plans]
        cands = {P: [v for v in range(3) if v == 0 or _engine_threads(P, v) != _engine_threads(P, 0)]
                 for P in (4096, 8192, 16384)}
        best, best_t, rows = None, math.inf, []
        for combo in itertools.product(*(cands[P] for P in (4096, 8192, 16384))):
            lay = dict(zip((4096, 8192, 16384), combo))
            for pl, P in zip(plans, P_of):
                ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, lay.get(P, 0))
            t_best = math.inf
            for _ in range(args.reps):
                for pl, s in zip(plans, solves):
                    ssp.ssp_set_field(pl, s.starter(), s.nz)
                ssp.ssp_march_batch_async(plans, [args.mixed_steps] * len(plans), None)   # warm-up
                ssp.ssp_batch_stats(plans)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ssp.ssp_march_batch_async(plans, [args.mixed_steps] * len(plans), None)
                e1.record(stream)
                ssp.ssp_batch_stats(plans)
                t_best = min(t_best, e0.elapsed_time(e1) / 1e3)
            row = {"part": "mixed", "layouts": {str(k): v for k, v in lay.items()}, "plans": len(plans),
                   "steps": args.mixed_steps, "ms": round(1e3 * t_best, 3)}
            rows.append(row)
            print(json.dumps(row), flush=True)
            if t_best < best_t:
                best, best_t = lay, t_best
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    mixed = list(tables["kTunedVariant"])
    for P, v in best.items():
        mixed[LENGTHS.index(P)] = v
    tables["kTunedMixed"] = mixed
    print(json.dumps({"part": "mixed", "chosen": {str(k): v for k, v in best.items()}}), flush=True)


def time_engine(ssp, torch, nz, p, engine, batch, steps):
    sys.path.insert(0, ROOT)
    import time
    import workloads as W
    s = W.munk_deep(nz=nz)
    s.pade_order = p
    stream = torch.cuda.Stream()
    pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    try:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, engine)
        ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
        zs = W.source_depths(batch, 50.0, 2000.0)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z) for z in zs])
        with torch.cuda.stream(stream):
            d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
            d_step = torch.zeros(batch, dtype=torch.int64, device="cuda")
        stream.synchronize()
        ssp.ssp_to_sine(pl, batch, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, batch, d_psi.data_ptr(), d_step.data_ptr(), 1)  # warm-up
        stream.synchronize()
        # wall time: the dense engine's loop is driven from the host
        t0 = time.perf_counter()
        ssp.ssp_march_device(pl, batch, d_psi.data_ptr(), d_step.data_ptr(), steps)
        stream.synchronize()
        t = time.perf_counter() - t0
        out = d_psi.cpu().numpy()
    finally:
        ssp.ssp_plan_destroy(pl)
    return t, out


def tune_engine(ssp, torch, args, tables):
    eng = [[0] * 4 for _ in range(4)]
    for nc, nz in enumerate((256, 512, 1024, 2048)):
        for pc, p in enumerate((4, 6, 8)):
            tf, ff = time_engine(ssp, torch, nz, p, ssp.SSP_ENGINE_FFT, 128, args.engine_steps)
            td, fd = time_engine(ssp, torch, nz, p, ssp.SSP_ENGINE_DENSE, 128, args.engine_steps)
            diff = float(np.linalg.norm(fd - ff) / np.linalg.norm(ff))
            assert diff < 1e-4, f"engines disagree at Nz={nz}, p={p} ({diff:.2e})"
            eng[nc][pc] = 1 if td < tf else 0
            print(json.dumps({"part": "engine", "nz": nz, "p": p, "batch": 128, "steps": args.engine_steps,
                              "fft_ms": round(1e3 * tf, 3), "dense_ms": round(1e3 * td, 3),
                              "engine_difference_relL2": diff, "chosen": "dense" if eng[nc][pc] else "fft"}),
                  flush=True)
        eng[nc][3] = eng[nc][2]
    tables["kTunedEngine"] = eng


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", choices=["layouts", "mixed", "engine", "all"], default="all")
    ap.add_argument("--write", action="store_true", help="write csrc/ssp_tuned.h")
    ap.add_argument("--out", default=HEADER, help="where --write puts the header (default: csrc/ssp_tuned.h)")
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--mixed-steps", type=int, default=40,
                    help="range steps per call of the mixed batch (the broadband benchmark's call length)")
    ap.add_argument("--engine-steps", type=int, default=4)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    import torch
    sys.path.insert(0, ROOT)
    from paper_2511_03343_amd import ssp
    assert torch.cuda.is_available(), "the autotuner times kernels on the GPU"
    tables = read_tables(HEADER)
    if args.what in ("layouts", "all"):
        tune_layouts(ssp, torch, args, tables)
    if args.what in ("mixed", "all"):
        tune_mixed(ssp, torch, args, tables)
    if args.what in ("engine", "all"):
        tune_engine(ssp, torch, args, tables)
    print(json.dumps({"tables": tables}), flush=True)
    if args.write:
        write_header(tables, args.out)
        print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
