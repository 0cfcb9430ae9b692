"""Continuous-batching server: scheduling logic on the host (a stand-in backend that only
counts steps, fails requests on purpose and records what each tick asks for), and on the
GPU every request of a Poisson mix equal, bitwise, to the same request run alone, and served
requests against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from paper_2511_03343_amd.serve import (Server, ServeRequest, from_solve, latency_summary,
                                         plan_device_bytes)


def to_request(arrival, s, rid=-1):
    c = W.munk(W.depth_grid(s.nz, s.depth)) if s.env == "munk" else None
    return from_solve(arrival, s, c_table=c, rid=rid)


class PlanError(Exception):
    def __init__(self, status):
        super().__init__(f"status {status}")
        self.status = status


class CountingBackend:
    """Host stand-in: plans are step counters; a tick returns one TL row per output step.
    fail_create: request ids whose plan creation fails (status -5, unstable coefficients);
    diverge: request id -> step at which its march reports a diverged series (status -4)."""

    def __init__(self, fail_create=(), diverge=None):
        self.live = {}
        self.max_live = 0
        self.created = []
        self.next = 0
        self.fail_create = set(fail_create)
        self.diverge = dict(diverge or {})
        self.max_steps = {}   # request id -> most steps one tick gave it

    def create(self, r):
        if r.rid in self.fail_create:
            raise PlanError(-5)
        h = self.next
        self.next += 1
        self.live[h] = {"n": 0, "every": r.out_every, "nz": r.nz, "rid": r.rid}
        self.created.append(r.rid)
        self.max_live = max(self.max_live, len(self.live))
        return h

    def march(self, handles, nzs, steps):
        tl, stats = [], []
        for h, nz, k in zip(handles, nzs, steps):
            st = self.live[h]
            self.max_steps[st["rid"]] = max(self.max_steps.get(st["rid"], 0), k)
            n0 = st["n"]
            stop = self.diverge.get(st["rid"])
            status, done = 0, k
            if stop is not None and n0 < stop <= n0 + k:
                status, done = -4, stop - 1 - n0   # the step `stop` diverged: the field stays before it
            rows = [n for n in range(n0 + 1, n0 + done + 1) if n % st["every"] == 0]
            st["n"] += done
            tl.append(np.array([[st["rid"] * 1000 + n] * 2 for n in rows], dtype=np.float32).reshape(-1, 2))
            stats.append({"steps_done": done, "neumann_terms": 3 * done, "not_converged": 0, "status": status})
        return tl, stats

    def destroy(self, h):
        del self.live[h]

    @staticmethod
    def error_status(exc):
        return getattr(exc, "status", None) if isinstance(exc, PlanError) else None

    @staticmethod
    def free_bytes():
        return 1 << 40


def fake_stream(n, seed=5):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += rng.exponential(0.01)
        nz = int(rng.choice([512, 1024, 4096, 16384]))
        out.append(ServeRequest(arrival=t, nz=nz, depth=5000.0, freq=50.0, c0=1500.0, dr=25.0,
                                pade_order=6, neumann_max=48, tol=1e-10,
                                nsteps=int(rng.integers(1, 400)), out_every=int(rng.integers(1, 30)),
                                starter=np.zeros(nz, complex)))
    return out


def test_scheduler_completes_every_request_with_all_outputs():
    reqs = fake_stream(200)
    ticks = iter(np.arange(0, 1e6, 0.003))
    srv = Server(CountingBackend(), hbm_budget=1 << 40, max_active=64, steps_per_tick=50,
                 clock=lambda: float(next(ticks)))
    res = srv.run(reqs)
    assert len(res) == len(reqs)
    for r in reqs:
        out = res[r.rid]
        assert out.steps_done == r.nsteps
        rows = out.tl_array()
        expect = [n for n in range(1, r.nsteps + 1) if n % r.out_every == 0]
        assert rows.shape[0] == len(expect)
        if expect:
            assert np.array_equal(rows[:, 0], r.rid * 1000 + np.array(expect, dtype=np.float32))
        assert out.latency >= 0 and out.admitted >= r.arrival - 1e-12
    assert srv.backend.max_live <= 64
    assert srv.backend.created == sorted(srv.backend.created)   # admission in arrival order
    s = latency_summary(res)
    assert s["count"] == len(reqs) and s["p99_s"] >= s["p50_s"]


def test_scheduler_respects_the_memory_budget():
    reqs = fake_stream(60, seed=9)
    big = max(plan_device_bytes(r.nz, r.pade_order, 50 // r.out_every + 1) for r in reqs)
    budget = 3 * big
    ticks = iter(np.arange(0, 1e6, 0.001))
    srv = Server(CountingBackend(), hbm_budget=budget, max_active=1000, steps_per_tick=50,
                 clock=lambda: float(next(ticks)))
    res = srv.run(reqs)
    assert all(res[r.rid].steps_done == r.nsteps for r in reqs)
    assert srv.peak_bytes <= budget
    assert srv.backend.max_live <= 3 * big // min(plan_device_bytes(512, 6, 2), big) + 1


def test_failed_requests_do_not_stop_the_stream():
    # one request's plan cannot be created, another's march diverges half way: both end with
    # their status, every plan is released, and every other request completes with all of
    # its outputs
    reqs = fake_stream(40, seed=11)
    for i, r in enumerate(reqs):
        r.rid = i
    reqs[7].nsteps = max(reqs[7].nsteps, 60)
    backend = CountingBackend(fail_create=[3], diverge={7: 30})
    ticks = iter(np.arange(0, 1e6, 0.002))
    srv = Server(backend, hbm_budget=1 << 40, max_active=16, steps_per_tick=20,
                 clock=lambda: float(next(ticks)))
    res = srv.run(reqs)
    assert res[3].status == -5 and res[3].steps_done == 0 and not np.isfinite(res[3].latency)
    assert res[7].status == -4 and res[7].steps_done == 29 and not np.isfinite(res[7].latency)
    assert srv.failed == 2 and not backend.live
    for r in reqs:
        if r.rid in (3, 7):
            continue
        out = res[r.rid]
        expect = [n for n in range(1, r.nsteps + 1) if n % r.out_every == 0]
        assert out.status == 0 and out.steps_done == r.nsteps and out.tl_array().shape[0] == len(expect)
    assert latency_summary(res)["count"] == len(reqs) - 2


def test_tick_never_exceeds_the_budgeted_output_rows():
    # the output staging of a request is budgeted for tick_steps_cap steps; the scheduler
    # never gives a request more steps in one tick, whatever its measured cost
    reqs = fake_stream(80, seed=13)
    backend = CountingBackend()
    ticks = iter(np.arange(0, 1e6, 0.002))
    srv = Server(backend, hbm_budget=1 << 40, max_active=32, steps_per_tick=25,
                 clock=lambda: float(next(ticks)))
    srv.run(reqs)
    for r in reqs:
        assert backend.max_steps[r.rid] <= srv.tick_steps_cap(r)


class RaisingBackend(CountingBackend):
    def march(self, handles, nzs, steps):
        raise RuntimeError("device lost")


def test_an_exception_releases_every_active_plan():
    backend = RaisingBackend()
    srv = Server(backend, hbm_budget=1 << 40, max_active=8, steps_per_tick=10)
    with pytest.raises(RuntimeError):
        srv.run(fake_stream(12, seed=3))
    assert backend.created and not backend.live


def test_scheduler_rejects_a_request_above_the_budget():
    reqs = fake_stream(3)
    srv = Server(CountingBackend(), hbm_budget=1000, steps_per_tick=10)
    with pytest.raises(ValueError):
        srv.run(reqs)


def small_mix():
    """A seeded Poisson mix with the serving distribution's structure at test size:
    Nz 512..2048, short ranges, Munk and Munk + eddy."""
    rng = np.random.default_rng(W.SEED + 7)
    t, out = 0.0, []
    for i in range(10):
        t += rng.exponential(0.005)
        f = float(rng.uniform(25.0, 120.0))
        nz = int(rng.choice([512, 1024, 2048]))
        k0 = 2 * np.pi * f / 1500.0
        dr = max(25.0, 5.0 / k0)
        env = "munk" if rng.random() < 0.5 else "munk+eddy"
        nsteps = int(rng.integers(20, 140))
        s = W.Solve(nz=nz, depth=5000.0, freq=f, c0=1500.0, dr=dr, pade_order=6, neumann_max=48,
                    tol=1e-10, nsteps=nsteps, zs=float(rng.uniform(50.0, 2000.0)), env=env,
                    out_every=max(1, nsteps // 10),
                    eddy=W.Eddy(r0=1500.0, rr=800.0) if env == "munk+eddy" else None)
        out.append(to_request(t, s, rid=i))
    return out


@pytest.mark.gpu
def test_mix_equals_alone_bitwise(ssp, gpu):
    from paper_2511_03343_amd.serve import LibBackend
    mix = Server(LibBackend(), steps_per_tick=16)
    res_mix = mix.run(small_mix())
    assert mix.peak_active > 1
    for r in small_mix():
        r.arrival = 0.0
        alone = Server(LibBackend(), steps_per_tick=1000).run([r])[r.rid]
        got = res_mix[r.rid]
        assert got.status == alone.status and got.status >= 0
        assert got.steps_done == alone.steps_done == r.nsteps
        assert got.neumann_terms == alone.neumann_terms
        a, b = got.tl_array(), alone.tl_array()
        assert a.shape == b.shape == (r.nsteps // r.out_every, r.nz)
        assert np.array_equal(a, b)
    print(f"[serving mix] ticks={mix.ticks} peak_active={mix.peak_active} "
          f"{latency_summary(res_mix)}", flush=True)


def _oracle_for_request(r):
    """The FP64 oracle's march of a served request (its starter, environment, range step and
    output interval)."""
    from oracle import Plan as OraclePlan
    pl = OraclePlan(r.nz, r.depth, r.freq, r.c0, r.dr, r.pade_order, r.neumann_max, r.tol)
    if r.c_table is not None:
        c = np.asarray(r.c_table)[None, :]
    elif r.profile == "munk+eddy":
        c = W.profile_steps("munk+eddy", r.nz, r.depth, r.dr, 0, r.nsteps, W.Eddy(*r.eddy))
    else:
        c = W.munk(W.depth_grid(r.nz, r.depth))[None, :]
    return pl.march(r.starter, r.nsteps, c, out_every=r.out_every)


@pytest.mark.gpu
def test_served_requests_vs_oracle(ssp, gpu):
    # a Poisson mix with unequal step counts served in ticks on the mixed-batch layouts,
    # with a Munk + eddy request at FFT length 8192 (Nz = 4096, its eddy on the device) and
    # a Munk request at 16384 (Nz = 8192) among the small ones; served field and TL rows of
    # every output step against the FP64 oracle
    from paper_2511_03343_amd.serve import LibBackend
    mix = small_mix()
    big = []
    for rid, (nz, f, env, n) in enumerate([(4096, 60.0, "munk+eddy", 48), (8192, 110.0, "munk", 20)]):
        s = W.Solve(nz=nz, depth=5000.0, freq=f, c0=1500.0, dr=25.0, pade_order=6, neumann_max=48,
                    tol=1e-10, nsteps=n, zs=900.0 + 300.0 * rid, env=env, out_every=n // 4,
                    eddy=W.Eddy(r0=600.0, rr=400.0) if env == "munk+eddy" else None)
        big.append(to_request(0.002 * (rid + 1), s, rid=100 + rid))
    reqs = mix + big
    srv = Server(LibBackend(), steps_per_tick=12)
    res = srv.run(reqs, march_fields=True)
    assert srv.peak_active > 1
    check = [r for r in reqs if r.rid in (0, 3, 6, 9, 100, 101)]
    for r in check:
        got = res[r.rid]
        ref = _oracle_for_request(r)
        assert got.status >= 0 and got.steps_done == r.nsteps == ref.steps_done
        fld = np.concatenate(got.fields, axis=0).astype(np.complex128)
        tl = got.tl_array().astype(np.float64)
        assert fld.shape == ref.field.shape and tl.shape == ref.tl.shape
        err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
        mask = ref.tl < 120.0
        dtl = np.abs(tl - ref.tl)[mask]
        print(f"[served vs oracle] rid={r.rid} nz={r.nz} f={r.freq:.1f} env={r.profile} steps={r.nsteps} "
              f"relL2={err.max():.3e} dTL={dtl.max():.3e}", flush=True)
        assert err.max() <= 1e-4 and dtl.max() <= 0.1
