"""Continuous-batching server: scheduling logic on the host (a stand-in backend that only
counts steps), and on the GPU every request of a Poisson mix equal, bitwise, to the same
request run alone."""
import numpy as np
import pytest

import workloads as W
from paper_2511_03343_amd.serve import (Server, ServeRequest, from_solve, latency_summary,
                                         plan_device_bytes)


def to_request(arrival, s, rid=-1):
    c = W.munk(W.depth_grid(s.nz, s.depth)) if s.env == "munk" else None
    return from_solve(arrival, s, c_table=c, rid=rid)


class CountingBackend:
    """Host stand-in: plans are step counters; a tick returns one TL row per output step."""

    def __init__(self):
        self.live = {}
        self.max_live = 0
        self.created = []
        self.next = 0

    def create(self, r):
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
            n0 = st["n"]
            rows = [n for n in range(n0 + 1, n0 + k + 1) if n % st["every"] == 0]
            st["n"] += k
            tl.append(np.array([[st["rid"] * 1000 + n] * 2 for n in rows], dtype=np.float32).reshape(-1, 2))
            stats.append({"steps_done": k, "neumann_terms": 3 * k, "not_converged": 0, "status": 0})
        return tl, stats

    def destroy(self, h):
        del self.live[h]

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
