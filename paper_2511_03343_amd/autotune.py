"""Autotuner for the engine layout of the fused march kernel, per FFT length.

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
Nz = P/2 - 1).  Rebuild the library afterwards.

    python -m paper_2511_03343_amd.autotune [--write [--out PATH]]

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


def write_header(choice: dict, path: str = HEADER) -> None:
    def row(kind):
        return ", ".join(str(choice.get((kind, P), 0)) for P in LENGTHS)
    with open(path, "w") as f:
        f.write("// ssp_tuned.h - engine layout of the fused march kernel per FFT length, chosen by\n"
                "// paper_2511_03343_amd/autotune.py (written by that script; do not edit by hand).\n"
                "#pragma once\n\n"
                "namespace ssp {\n"
                "// kTunedVariant[log2(P) - 7] for P = 128 ... 32768\n"
                f"constexpr int kTunedVariant[9] = {{{row('chirp')}}};\n"
                "// kTunedDirect[kind - 1][log2(P) - 7]: direct Fourier (periodic Nz = P), direct sine\n"
                "// (Dirichlet Nz = P/2 - 1)\n"
                f"constexpr int kTunedDirect[2][9] = {{{{{row('fourier')}}}, {{{row('sine')}}}}};\n"
                "}  // namespace ssp\n")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="write csrc/ssp_tuned.h")
    ap.add_argument("--out", default=HEADER, help="where --write puts the header (default: csrc/ssp_tuned.h)")
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    import torch
    sys.path.insert(0, ROOT)
    from paper_2511_03343_amd import ssp
    assert torch.cuda.is_available(), "the autotuner times kernels on the GPU"
    choice, report = {}, []
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
            row = {"kind": kind[0], "P": P, "nz": kind[2](P), "batch": batch, "steps": args.steps,
                   "layouts": layouts, "threads": [_engine_threads(P, v) for v in layouts],
                   "ms": [round(1e3 * t, 3) for t in times], "chosen": choice[(kind[0], P)],
                   "layout_difference_relL2": max(diffs)}
            report.append(row)
            print(json.dumps(row), flush=True)
    if args.write:
        write_header(choice, args.out)
        print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
