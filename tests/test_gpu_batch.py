"""GPU tests of the device-resident uneven batch (ssp_march_batch_async + ssp_batch_stats),
its HIP-graph replay, the plan options of the boundary, the contraction estimate and the
per-solve profile-range check of ssp_march_device.

Equivalences are exact (the same kernels run on the same data), parity against the FP64
oracle uses the bar of the other GPU tests.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Plan as OraclePlan

from test_gpu_parity import make_plan, oracle_march, _report

pytestmark = pytest.mark.gpu


def _uneven_solves():
    # FFT lengths 8192 (chirp-z), 16384 and 32768 (split) and a direct sine grid (Nz = 1023)
    out = []
    for nz, f in [(3000, 56.25), (6000, 112.5), (12000, 225.0), (1023, 40.0)]:
        s = W.munk_deep(nsteps=6, nz=nz)
        s.freq, s.out_every = f, 3
        out.append(s)
    return out


def test_async_batch_equals_host_batch_and_graph_replays(ssp, gpu):
    torch = gpu
    solves = _uneven_solves()
    k = 6
    nz = [s.nz for s in solves]
    host = [make_plan(ssp, s) for s in solves]
    dev = [make_plan(ssp, s) for s in solves]
    stream = torch.cuda.Stream()
    try:
        for a, b, s in zip(host, dev, solves):
            ssp.ssp_set_field(a, s.starter(), s.nz)
            ssp.ssp_set_field(b, s.starter(), s.nz)
            ssp.ssp_plan_set_stream(b, stream.cuda_stream)
            ssp.ssp_plan_set_option(b, ssp.SSP_OPT_VARIANT, -1)
        ssp.ssp_plan_set_option(dev[0], ssp.SSP_OPT_GRAPH, 1)
        d_tl = [torch.full((k // s.out_every + 1, s.nz), -1.0, dtype=torch.float32, device="cuda") for s in solves]
        ptrs = [t.data_ptr() for t in d_tl]
        for call in range(3):  # the first records the graph, the others replay it
            st, _, tl_h, stats_h = ssp.ssp_march_batch(host, nz, k, want_field=False)
            ssp.ssp_march_batch_async(dev, [k] * len(dev), ptrs)
            st2, stats_d = ssp.ssp_batch_stats(dev)
            assert st2 == st
            for s, th, td, a, b in zip(solves, tl_h, d_tl, stats_h, stats_d):
                rows = th.shape[0]
                got = td.cpu().numpy()[:rows]
                _report(f"async call {call} nz={s.nz}", rows=rows, terms=b["neumann_terms"])
                assert a == b
                assert np.array_equal(th, got)
            for a, b, s in zip(host, dev, solves):
                assert np.array_equal(ssp.ssp_get_field(a, s.nz), ssp.ssp_get_field(b, s.nz))
            assert ssp.ssp_count_outputs(dev[0], k) == ssp.ssp_count_outputs(host[0], k)
    finally:
        for pl in host + dev:
            ssp.ssp_plan_destroy(pl)


def test_batch_members_with_zero_steps(ssp, gpu):
    # a member given zero steps marches nothing (no rows, statistics of zero steps, its state
    # unchanged) while the other members of the same launches march as they would alone
    solves = _uneven_solves()
    steps = [0, 6, 0, 4]
    nz = [s.nz for s in solves]
    plans = [make_plan(ssp, s) for s in solves]
    alone = [make_plan(ssp, s) for s in solves]
    try:
        for a, b, s in zip(plans, alone, solves):
            ssp.ssp_set_field(a, s.starter(), s.nz)
            ssp.ssp_set_field(b, s.starter(), s.nz)
        before = [ssp.ssp_get_field(a, s.nz) for a, s in zip(plans, solves)]
        st, fl, tl, stats = ssp.ssp_march_batch_steps(plans, nz, steps)
        assert st >= 0  # (a factor's series may stop at the term cap: a warning)
        for a, b, s, k, f, t, x, f0 in zip(plans, alone, solves, steps, fl, tl, stats, before):
            _report(f"zero-step batch nz={s.nz}", steps=k, rows=f.shape[0], terms=x["neumann_terms"])
            if k == 0:
                assert f.shape[0] == 0 and t.shape[0] == 0
                assert x["steps_done"] == 0 and x["neumann_terms"] == 0
                assert np.array_equal(ssp.ssp_get_field(a, s.nz), f0)
            else:
                st1, f1, t1, x1 = ssp.ssp_march(b, s.nz, None, k)
                assert st1 == x["status"] and x["steps_done"] == k and x == x1
                assert f.shape[0] > 0 and np.array_equal(f, f1) and np.array_equal(t, t1)
    finally:
        for pl in plans + alone:
            ssp.ssp_plan_destroy(pl)


def test_async_batch_uneven_steps_vs_oracle(ssp, gpu):
    # a step count per plan, against the oracle
    torch = gpu
    solves = _uneven_solves()
    steps = [6, 3, 4, 5]
    plans = [make_plan(ssp, s) for s in solves]
    try:
        for pl, s in zip(plans, solves):
            ssp.ssp_set_field(pl, s.starter(), s.nz)
        d_tl = [torch.zeros((k // s.out_every + 1, s.nz), dtype=torch.float32, device="cuda")
                for k, s in zip(steps, solves)]
        ssp.ssp_march_batch_async(plans, steps, [t.data_ptr() for t in d_tl])
        st, stats = ssp.ssp_batch_stats(plans)
        finals = [ssp.ssp_get_field(pl, s.nz) for pl, s in zip(plans, solves)]
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for s, k, f, x in zip(solves, steps, finals, stats):
        ref = oracle_march(s, nsteps=k)
        assert x["steps_done"] == k == ref.steps_done
        err = np.linalg.norm(f - ref.final) / np.linalg.norm(ref.final)
        _report(f"async uneven nz={s.nz}", steps=k, relL2=f"{err:.3e}")
        assert err <= 1e-4


def test_form_and_gain_limit_options(ssp, gpu):
    s = W.homogeneous_waveguide()
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_FORM, ssp.SSP_FORM_PRODUCT)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_FORM, ssp.SSP_FORM_SUM)
        assert e.value.status == ssp.SSP_E_UNIMPL
        # the rotated [4/4] approximant exceeds 1 by ~4.5e-8: rejected under a 1e-9 limit,
        # accepted under the default one
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GAIN_LIMIT, 1e-9)
        assert e.value.status == ssp.SSP_E_UNSTABLE
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GAIN_LIMIT, 1e-6)
    finally:
        ssp.ssp_plan_destroy(pl)
    # the standard approximant (unitary on the real axis) passes a 1e-9 limit, and a
    # rotation that fails the limit is refused and the plan keeps its coefficients
    s = W.munk_deep(nsteps=2, nz=300)
    s.out_every = 1
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GAIN_LIMIT, 1e-9)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ROTATION, np.pi / 16)
        assert e.value.status == ssp.SSP_E_UNSTABLE
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), 2)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert np.linalg.norm(fld[-1] - ref.field[-1]) / np.linalg.norm(ref.field[-1]) < 1e-4


def _dense_operator_radius(s, j):
    # brute force: the spectral radius of b_j L_j^{-1} V as a dense matrix in the sine
    # basis (tiny grid), from the oracle's own Pade coefficients and eigenvalues
    from oracle import dst_matrix
    o = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    S = dst_matrix(s.nz)
    v = o.potential(s.profile()[0])
    b = o.b[j]
    K = b * np.diag(1.0 / (1.0 + b * o.x)) @ S @ np.diag(v) @ S
    return float(np.max(np.abs(np.linalg.eigvals(K))))


def test_contraction_estimate_vs_dense_eigenvalues(ssp, gpu):
    s = W.munk_deep(nsteps=1, nz=96)
    pl = make_plan(ssp, s)
    try:
        bound, est = ssp.ssp_plan_contraction(pl, s.pade_order, iterations=400)
        info = ssp.ssp_plan_info(pl, s.pade_order)
    finally:
        ssp.ssp_plan_destroy(pl)
    o = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    for j in range(s.pade_order):
        # the library's factor j is the oracle's factor with the same b_j
        jo = int(np.argmin(np.abs(o.b - info["b"][j])))
        rho = _dense_operator_radius(s, jo)
        _report("contraction", j=j, estimate=f"{est[j]:.6f}", dense=f"{rho:.6f}", bound=f"{bound[j]:.3e}")
        assert bound[j] >= rho * (1 - 1e-9)
        assert abs(est[j] - rho) <= 0.02 * rho + 1e-6


def test_contraction_check_refuses_divergent_plan(ssp, gpu):
    # sigma = 1 with [6/6] (on a grid that resolves the factors' poles): the Neumann
    # operators have spectral radius above 1, so a march with the check on returns
    # SSP_E_DIVERGED before any step; the deep Munk settings pass
    s = W.munk_deep(nsteps=4, nz=511, neumann_max=16)
    s.dr = 1.0 / s.k0
    pl = make_plan(ssp, s)
    try:
        _, est = ssp.ssp_plan_contraction(pl, s.pade_order, iterations=60)
        assert est.max() > 1.0
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_CONTRACTION_CHECK, 1)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_DIVERGED and "contraction" in str(e.value)
    finally:
        ssp.ssp_plan_destroy(pl)
    s = W.munk_deep(nsteps=2, nz=511)
    pl = make_plan(ssp, s)
    try:
        _, est = ssp.ssp_plan_contraction(pl, s.pade_order, iterations=60)
        assert est.max() < 1.0
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_CONTRACTION_CHECK, 1)
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert st == 0 and stats["steps_done"] == 2
    finally:
        ssp.ssp_plan_destroy(pl)


def test_device_march_profile_rows_checked_per_solve(ssp, gpu):
    # a tabulated profile of 5 rows: a solve whose counter runs past it stops with
    # SSP_E_INVAL in its statistics; the plan's own step counter is not touched
    torch = gpu
    s = W.munk_deep(nsteps=5, nz=500)
    s.env, s.eddy = "munk+eddy", W.Eddy()
    pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    try:
        ssp.ssp_set_profile(pl, 0, 5, s.profile(0, 5))
        stream = torch.cuda.Stream()
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        B = 2
        psi = np.stack([s.starter(), s.starter()]).astype(np.complex64)
        d_psi = torch.from_numpy(psi).cuda()
        steps = torch.tensor([0, 3], dtype=torch.int64, device="cuda")
        d_stats = torch.zeros((B, 48), dtype=torch.uint8, device="cuda")
        ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), 4, 0, d_stats.data_ptr())
        stream.synchronize()
        raw = d_stats.cpu().numpy()
        done = raw[:, 0:8].copy().view(np.int64).ravel()
        status = raw[:, 40:44].copy().view(np.int32).ravel()
        assert steps.cpu().tolist() == [4, 5]
        assert done.tolist() == [4, 2] and status.tolist() == [0, ssp.SSP_E_INVAL]
        assert ssp.ssp_count_outputs(pl, 10) == 10  # the plan's own counter is still 0
    finally:
        ssp.ssp_plan_destroy(pl)
