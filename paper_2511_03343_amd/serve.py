"""Continuous-batching server for range-march requests on one GPU.

Requests arrive over time, each a complete solve description (grid, frequency, range step,
Pade order, Neumann cap and tolerance, number of range steps, starter, environment, output
interval).  The server works in ticks:

  1. Admission: arrived requests, in arrival order, get a plan of their own (device tables,
     resident field, output staging) while the HBM budget and the slot limit allow.
  2. March: every active request advances in ONE batched library call
     (ssp_march_batch_steps: a single launch for the FFT lengths that share the 1024-thread
     kernel, one per other length, the groups concurrent), so requests of different grids,
     frequencies and environments run side by side and their fields stay resident in HBM
     between ticks.  The costliest request per range step advances steps_per_tick steps;
     every other request advances as many steps as fit in the same time by the cost model
     (FFT length P log P times its Neumann terms per step, measured in its previous tick),
     so small requests are not held back by large ones.
  3. Drain: the transmission-loss rows of the tick are appended to each request's result;
     finished requests release their plan and record their latency.

Each request's arithmetic does not depend on what runs beside it or on where ticks cut its
march (a resumed march is bitwise identical), so its result equals the result of running it
alone.  PyTorch is used only to query free device memory.

The backend is the HIP library through its C ABI; tests substitute a host-only stand-in to
check the scheduling logic without a GPU.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class ServeRequest:
    """One range-march request.  `profile` is 'munk' (range-independent Munk profile) or
    'munk+eddy' (Munk plus a Gaussian eddy evaluated on the device every step)."""
    arrival: float                 # seconds from the start of the stream
    nz: int
    depth: float
    freq: float
    c0: float
    dr: float
    pade_order: int
    neumann_max: int
    tol: float
    nsteps: int
    out_every: int
    starter: np.ndarray            # complex128 [nz]
    profile: str = "munk"
    munk: tuple = (1500.0, 0.00737, 1300.0)
    eddy: Optional[tuple] = None   # (amp, r0, rr, z0, rz) for 'munk+eddy'
    c_table: Optional[np.ndarray] = None  # [nz] sound speed for a tabulated profile
    rid: int = -1


def from_solve(arrival: float, s, c_table: Optional[np.ndarray] = None, rid: int = -1) -> ServeRequest:
    """A request from a solve description with the attributes of workloads.Solve (the starter
    from s.starter(); the eddy, if any, from s.eddy).  c_table: sound speed on the grid for a
    tabulated range-independent profile, else the analytic profile of s.env is used."""
    e = getattr(s, "eddy", None)
    return ServeRequest(arrival=arrival, nz=s.nz, depth=s.depth, freq=s.freq, c0=s.c0, dr=s.dr,
                        pade_order=s.pade_order, neumann_max=s.neumann_max, tol=s.tol,
                        nsteps=s.nsteps, out_every=s.out_every, starter=s.starter(), profile=s.env,
                        eddy=(e.amp, e.r0, e.rr, e.z0, e.rz) if (e is not None and s.env == "munk+eddy") else None,
                        c_table=c_table, rid=rid)


@dataclass
class ServeResult:
    rid: int
    tl: List[np.ndarray] = field(default_factory=list)   # TL rows in range order
    steps_done: int = 0
    neumann_terms: int = 0
    not_converged: int = 0
    fields: List[np.ndarray] = field(default_factory=list)  # field rows (run(march_fields=True))
    status: int = 0
    admitted: float = math.nan
    finished: float = math.nan
    latency: float = math.nan

    def tl_array(self) -> np.ndarray:
        return np.concatenate(self.tl, axis=0) if self.tl else np.zeros((0, 0), np.float32)


def fft_length(nz: int) -> int:
    P = 128
    while P < 2 * nz - 1:
        P *= 2
    return P


def step_cost(nz: int, terms_per_step: float) -> float:
    """Relative cost of one range step: every Neumann term is two transforms of length P."""
    P = fft_length(nz)
    return P * math.log2(P) * max(terms_per_step, 1.0)


def plan_device_bytes(nz: int, pade_order: int, out_rows: int) -> int:
    """Device memory of one plan: chirp spectra and twiddles, pointwise and Pade tables,
    potential, field and per-solve scratch, and output staging for out_rows rows."""
    P = fft_length(nz)
    PE = P // 2 if P > 16384 else P
    tables = (8 * P + 16 * (64 + P // 64) if P > 16384 else 2 * 8 * P) + 12 * (PE // 8 + 1) + 3 * 8 * nz + 3 * 16 * pade_order * nz + 16 * pade_order
    if P > 16384:
        tables += 16 * (P // 2)
    state = 4 * nz + 8 * nz + 5 * 8 * (P // 2) + 8 + 48 + 512   # work stride P/2 (>= nz)
    staging = 12 * nz * max(out_rows, 1)
    return tables + state + staging


class LibBackend:
    """The HIP library: one plan per admitted request.  Plans take the engine layouts the
    autotuner measured on a mixed-length batch (SSP_OPT_VARIANT = -2) and the engine chosen
    for their (Nz, Pade order) class (SSP_OPT_ENGINE = SSP_ENGINE_AUTO); both are fixed per
    plan, so a request's arithmetic does not depend on what it is batched with."""

    def __init__(self, stream_ptr: Optional[int] = None, variant: int = -2, engine: Optional[int] = None):
        from . import ssp
        self.ssp = ssp
        self.stream = stream_ptr
        self.variant = variant
        self.engine = ssp.SSP_ENGINE_AUTO if engine is None else engine

    def create(self, r: ServeRequest):
        s = self.ssp
        pl = s.ssp_plan_create(r.nz, r.depth, r.freq, r.c0, r.dr, r.pade_order, r.neumann_max, r.tol)
        try:
            if self.stream is not None:
                s.ssp_plan_set_stream(pl, self.stream)
            s.ssp_plan_set_option(pl, s.SSP_OPT_OUT_EVERY, r.out_every)
            s.ssp_plan_set_option(pl, s.SSP_OPT_VARIANT, self.variant)
            dense_ok = r.nz <= s.ssp_max_dense_nz()
            s.ssp_plan_set_option(pl, s.SSP_OPT_ENGINE, self.engine if (self.engine != s.SSP_ENGINE_DENSE or dense_ok)
                                  else s.SSP_ENGINE_FFT)
            if r.c_table is not None:
                s.ssp_set_profile(pl, 0, -1, r.c_table)
            else:
                s.ssp_set_profile_analytic(pl, munk=r.munk,
                                           eddy=r.eddy if r.profile == "munk+eddy" else None)
            s.ssp_set_field(pl, r.starter, r.nz)
        except Exception:
            s.ssp_plan_destroy(pl)
            raise
        return pl

    def march(self, handles: Sequence, nzs: Sequence[int], steps: Sequence[int]):
        st, _, tl, stats = self.ssp.ssp_march_batch_steps(list(handles), list(nzs), list(steps),
                                                          want_field=False, want_tl=True)
        return tl, stats

    def march_fields(self, handles: Sequence, nzs: Sequence[int], steps: Sequence[int]):
        """march() that also returns each plan's field rows (for checks against the oracle)."""
        st, fl, tl, stats = self.ssp.ssp_march_batch_steps(list(handles), list(nzs), list(steps),
                                                           want_field=True, want_tl=True)
        return fl, tl, stats

    def destroy(self, handle) -> None:
        self.ssp.ssp_plan_destroy(handle)

    def error_status(self, exc: Exception) -> Optional[int]:
        """The library status of an exception raised by create(), or None if it is not one."""
        return getattr(exc, "status", None) if isinstance(exc, self.ssp.SspError) else None

    @staticmethod
    def free_bytes() -> int:
        import torch
        free, _ = torch.cuda.mem_get_info()
        return int(free)


class Server:
    """Continuous batching over a request stream (see the module docstring).

    hbm_budget: bytes the active plans may hold (default: half the free device memory when
    the server starts); max_active: slot limit; steps_per_tick: range steps per tick."""

    def __init__(self, backend=None, hbm_budget: Optional[int] = None, max_active: int = 1024,
                 steps_per_tick: int = 50, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend if backend is not None else LibBackend()
        if hbm_budget is None:
            hbm_budget = self.backend.free_bytes() // 2
        if steps_per_tick < 1 or max_active < 1 or hbm_budget <= 0:
            raise ValueError("steps_per_tick, max_active and hbm_budget must be positive")
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.k = int(steps_per_tick)
        self.clock = clock
        self.ticks = 0
        self.peak_active = 0
        self.peak_bytes = 0
        self.t_create = 0.0   # host time creating plans
        self.t_march = 0.0    # time in the batched march calls
        self.failed = 0       # requests that ended with an error status

    def tick_steps_cap(self, r: ServeRequest) -> int:
        """The most range steps one tick gives request r; its output staging is budgeted for
        that many (see _cost), and run() never gives more."""
        return min(r.nsteps, self.k * max(1, int(step_cost(16384, 1.0) / step_cost(r.nz, 1.0))) * 4)

    def _cost(self, r: ServeRequest) -> int:
        rows = self.tick_steps_cap(r) // max(r.out_every, 1) + 1
        return plan_device_bytes(r.nz, r.pade_order, rows)

    def run(self, requests: Sequence[ServeRequest], realtime: bool = False,
            march_fields: bool = False) -> Dict[int, ServeResult]:
        """Serve the stream.  realtime: requests become visible at their arrival time on the
        wall clock (the server idles until then); otherwise the server keeps a virtual clock
        that advances by the measured duration of each tick (admission and march) and jumps
        to the next arrival when nothing is active, so latencies are those of an arrival
        process replayed against the device's own pace.  A request whose plan cannot be
        created (e.g. unstable coefficients) or whose march fails (e.g. a diverged series)
        ends with that status; the others continue.  march_fields: keep every request's
        field rows too (ServeResult.fields), for checks.  Returns the results by request id."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for i, r in enumerate(reqs):
            if r.rid < 0:
                r.rid = i
            if self._cost(r) > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs more device memory than the budget")
        pending: Deque[ServeRequest] = deque(reqs)
        queue: Deque[ServeRequest] = deque()
        active: List[dict] = []
        results: Dict[int, ServeResult] = {r.rid: ServeResult(r.rid) for r in reqs}
        used = 0
        t_wall0 = self.clock()
        vclock = 0.0

        def now() -> float:
            return self.clock() - t_wall0 if realtime else vclock

        try:
            while pending or queue or active:
                t = now()
                while pending and pending[0].arrival <= t:
                    queue.append(pending.popleft())
                if not queue and not active:
                    nxt = pending[0].arrival
                    if realtime:
                        time.sleep(max(0.0, nxt - now()))
                    else:
                        vclock = nxt
                    continue
                tick0 = self.clock()
                # admission in arrival order (no overtaking)
                tc = self.clock()
                while queue and len(active) < self.max_active and used + self._cost(queue[0]) <= self.hbm_budget:
                    r = queue.popleft()
                    cost = self._cost(r)
                    results[r.rid].admitted = t
                    try:
                        h = self.backend.create(r)
                    except Exception as exc:  # this request fails, the stream goes on
                        code = self.backend.error_status(exc) if hasattr(self.backend, "error_status") else None
                        if code is None:
                            raise
                        results[r.rid].status = int(code)
                        results[r.rid].finished = t
                        self.failed += 1
                        continue
                    used += cost
                    active.append({"req": r, "h": h, "left": r.nsteps, "cost": cost, "tps": 40.0,
                                   "cap": self.tick_steps_cap(r)})
                self.t_create += self.clock() - tc
                self.peak_active = max(self.peak_active, len(active))
                self.peak_bytes = max(self.peak_bytes, used)
                if active:
                    costs = [step_cost(a["req"].nz, a["tps"]) for a in active]
                    cmax = max(costs)
                    steps = [max(1, min(a["left"], a["cap"], int(round(self.k * cmax / c))))
                             for a, c in zip(active, costs)]
                    tm = self.clock()
                    handles, nzs = [a["h"] for a in active], [a["req"].nz for a in active]
                    if march_fields:
                        fl, tl, stats = self.backend.march_fields(handles, nzs, steps)
                    else:
                        fl = [None] * len(active)
                        tl, stats = self.backend.march(handles, nzs, steps)
                    self.t_march += self.clock() - tm
                    self.ticks += 1
                    for a, rows, frows, st, k in zip(active, tl, fl, stats, steps):
                        res = results[a["req"].rid]
                        if rows is not None and len(rows):
                            res.tl.append(np.array(rows, copy=True))
                        if frows is not None and len(frows):
                            res.fields.append(np.array(frows, copy=True))
                        res.steps_done += int(st["steps_done"])
                        res.neumann_terms += int(st["neumann_terms"])
                        res.not_converged += int(st["not_converged"])
                        if st["steps_done"] > 0:
                            a["tps"] = st["neumann_terms"] / st["steps_done"]
                        if st["status"] < 0 or (st["status"] > 0 and res.status == 0):
                            res.status = int(st["status"])
                        a["left"] = 0 if st["status"] < 0 else a["left"] - k
                if not realtime:
                    vclock += self.clock() - tick0
                t_end = now()
                keep = []
                for a in active:
                    if a["left"] > 0:
                        keep.append(a)
                        continue
                    self.backend.destroy(a["h"])
                    used -= a["cost"]
                    res = results[a["req"].rid]
                    res.finished = t_end
                    if res.status >= 0:
                        res.latency = t_end - a["req"].arrival
                    else:
                        self.failed += 1
                active = keep
        finally:
            for a in active:  # an exception left requests on the device: release their plans
                self.backend.destroy(a["h"])
        return results


def latency_summary(results: Dict[int, ServeResult]) -> dict:
    """p50 / p99 / max / mean latency (s) of the requests that completed (status >= 0)."""
    lat = np.array([r.latency for r in results.values() if np.isfinite(r.latency)])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "max_s": float(lat.max()),
            "mean_s": float(lat.mean())}
