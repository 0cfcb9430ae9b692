"""GPU parity of the dense engine (SSP_ENGINE_DENSE): every DST-I of the Neumann series as the
dense product S X on the matrix cores over the batch (Sec. 3.1: S is the orthonormal DST-I
matrix, symmetric and its own inverse).

Bar as for the FFT engine: relative L2 field error <= 1e-4 at every output range against
the FP64 oracle and |dTL| <= 0.1 dB where TL < 120 dB; statuses and step counts exact; a
solve gives the same result alone and batched with others (bitwise).
"""
import numpy as np
import pytest

import workloads as W
from oracle import DIVERGED, NOT_CONVERGED, OK

from test_gpu_parity import compare, make_plan, oracle_march, _report

pytestmark = pytest.mark.gpu


def dense_plan(ssp, s, profile="table"):
    pl = make_plan(ssp, s, profile)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, ssp.SSP_ENGINE_DENSE)
    return pl


@pytest.mark.parametrize("nz,nsteps", [(512, 60), (1024, 40), (2048, 24), (1000, 30), (255, 40)])
def test_dense_march_vs_oracle(ssp, gpu, nz, nsteps):
    s = W.munk_deep(nsteps=nsteps, nz=nz)
    s.out_every = nsteps // 4
    pl = dense_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == OK == ref.status and stats["steps_done"] == s.nsteps
    _report(f"dense nz={nz}", terms=stats["neumann_terms"], oracle_terms=int(ref.iterations.sum()))
    # term counts: FP32 and FP64 series stop at the same term except near the tolerance
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.02 * ref.iterations.sum() + 6
    compare(f"dense nz={nz}", fld, tl, ref)


def test_dense_long_march_vs_oracle(ssp, gpu):
    # drift of the fixed fp16 high/low representation of S over a longer range (Nz = 512)
    s = W.munk_deep(nsteps=400, nz=512)
    s.out_every = 100
    pl = dense_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    compare("dense 400 steps", fld, tl, oracle_march(s))


def test_dense_eddy_analytic_vs_oracle(ssp, gpu):
    # range-dependent potential evaluated on the device each step
    s = W.munk_eddy(nsteps=30, nz=1023, neumann_max=48)
    s.freq, s.pade_order, s.dr = 60.0, 6, 25.0
    s.out_every = 10
    pl = dense_plan(ssp, s, profile="analytic")
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    compare("dense eddy", fld, tl, oracle_march(s))


def test_dense_equals_fft_engine_to_rounding(ssp, gpu):
    s = W.munk_deep(nsteps=20, nz=700)
    s.out_every = 20
    out = []
    for engine in (ssp.SSP_ENGINE_FFT, ssp.SSP_ENGINE_DENSE):
        pl = make_plan(ssp, s)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, engine)
        try:
            out.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)[1])
        finally:
            ssp.ssp_plan_destroy(pl)
    err = np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[0])
    _report("dense vs fft", relL2=f"{err:.3e}")
    assert err < 2e-5


def test_dense_batch_uneven_steps_equals_alone_bitwise(ssp, gpu):
    # solves of different grids, frequencies and step counts in one batched call (the dense
    # groups by grid size, an FFT-engine plan beside them): each gives what it gives alone
    cases = [(512, 50.0, 12), (512, 80.0, 7), (1024, 50.0, 10), (2048, 100.0, 5), (3000, 56.0, 6)]
    solves = []
    for nz, f, n in cases:
        s = W.munk_deep(nsteps=n, nz=nz)
        s.freq, s.out_every = f, 3
        solves.append(s)

    def make(s):
        pl = make_plan(ssp, s)
        if s.nz <= ssp.ssp_max_dense_nz():
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, ssp.SSP_ENGINE_DENSE)
        return pl

    alone = []
    for s in solves:
        pl = make(s)
        try:
            alone.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)[1:])
        finally:
            ssp.ssp_plan_destroy(pl)
    plans = [make(s) for s in solves]
    try:
        for pl, s in zip(plans, solves):
            ssp.ssp_set_field(pl, s.starter(), s.nz)
        st, fl, tl, stats = ssp.ssp_march_batch_steps(plans, [s.nz for s in solves], [s.nsteps for s in solves])
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for (f1, t1, s1), f2, t2, s2, s in zip(alone, fl, tl, stats, solves):
        assert s2["steps_done"] == s.nsteps and s1["neumann_terms"] == s2["neumann_terms"]
        assert np.array_equal(f1, f2) and np.array_equal(t1, t2)


def test_dense_device_batch_vs_oracle(ssp, gpu):
    # ssp_march_device with the dense engine: 64 solves of one plan, sampled against the oracle
    torch = gpu
    s = W.munk_deep(nsteps=16, nz=1024)
    s.out_every = 8
    B = 64
    zs = W.source_depths(B, 50.0, 2000.0)
    pl = dense_plan(ssp, s)
    try:
        stream = torch.cuda.Stream()
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z) for z in zs])
        d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
        steps = torch.zeros(B, dtype=torch.int64, device="cuda")
        d_tl = torch.zeros((B, s.nsteps // s.out_every + 1, s.nz), dtype=torch.float32, device="cuda")
        d_stats = torch.zeros((B, 48), dtype=torch.uint8, device="cuda")
        out = torch.empty_like(d_psi)
        ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), s.nsteps, d_tl.data_ptr(),
                             d_stats.data_ptr())
        ssp.ssp_from_sine(pl, B, d_psi.data_ptr(), steps.data_ptr(), out.data_ptr())
        stream.synchronize()
        fld = out.cpu().numpy().astype(np.complex128)
        tl = d_tl.cpu().numpy()
        raw = d_stats.cpu().numpy()
        assert steps.cpu().tolist() == [s.nsteps] * B
    finally:
        ssp.ssp_plan_destroy(pl)
    status = raw[:, 40:44].copy().view(np.int32).ravel()
    assert set(status.tolist()) == {0}
    for b in (0, 31, 63):
        s1 = W.Solve(**{**s.__dict__, "zs": float(zs[b])})
        ref = oracle_march(s1)
        err = np.linalg.norm(fld[b] - ref.final) / np.linalg.norm(ref.final)
        mask = ref.tl < 120.0
        dtl = np.abs(tl[b, :ref.tl.shape[0]].astype(np.float64) - ref.tl)[mask]
        _report(f"dense device b={b}", relL2=f"{err:.3e}", max_dTL=f"{dtl.max():.3e}")
        assert err <= 1e-4 and dtl.max() <= 0.1


def test_dense_divergence_and_not_converged(ssp, gpu):
    # sigma = 1, [6/6] on a grid fine enough to resolve the factors' poles: the series
    # diverges (oracle and library, field left at step 0)
    s = W.munk_deep(nsteps=4, nz=511, neumann_max=16)
    s.dr = 1.0 / s.k0
    pl = dense_plan(ssp, s)
    try:
        ssp.ssp_set_field(pl, s.starter(), s.nz)
        st, _, _, stats = ssp.ssp_march_batch([pl], [s.nz], s.nsteps, want_field=False, want_tl=False)
        assert st == ssp.SSP_E_DIVERGED and stats[0]["status"] == ssp.SSP_E_DIVERGED
        assert stats[0]["steps_done"] == 0
        back = ssp.ssp_get_field(pl, s.nz)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == DIVERGED and ref.steps_done == 0
    assert np.linalg.norm(back - s.starter()) / np.linalg.norm(s.starter()) < 2e-6
    # a cap of 3 terms: series far from the tolerance are reported not converged
    s = W.munk_deep(nsteps=3, nz=511, neumann_max=3)
    s.out_every = 1
    pl = dense_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == NOT_CONVERGED and st == ssp.SSP_W_NOT_CONVERGED
    assert int((ref.residuals > 10 * s.tol).sum()) <= stats["not_converged"] <= int((ref.residuals > 0.1 * s.tol).sum())
    compare("dense not converged", fld, tl, ref)


def test_dense_engine_option_limits(ssp, gpu):
    pl = ssp.ssp_plan_create(4096, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10)
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, ssp.SSP_ENGINE_DENSE)
        assert e.value.status == ssp.SSP_E_UNIMPL
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, ssp.SSP_ENGINE_AUTO)
    finally:
        ssp.ssp_plan_destroy(pl)
    pl = ssp.ssp_plan_create_bc(512, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10, "neumann")
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ENGINE, ssp.SSP_ENGINE_DENSE)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)
