"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Bar (floating point): relative L2 field error <= 1e-4 at every output range and
|TL_gpu - TL_oracle| <= 0.1 dB wherever TL_oracle < 120 dB.  Transforms alone: <= 2e-6.
Statuses, step counts and bitwise batch/resume equivalence are compared exactly.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import DIVERGED, NOT_CONVERGED, OK, Plan as OraclePlan, dst as odst

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
DTL = 0.1


def _report(tag, **kv):
    print(f"[{tag}] " + " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def make_plan(ssp, s, profile="table"):
    pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    if s.rotation:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_ROTATION, s.rotation)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, s.out_every)
    if s.env == "munk+eddy":
        if profile == "analytic":
            e = s.eddy or W.Eddy()
            ssp.ssp_set_profile_analytic(pl, eddy=(e.amp, e.r0, e.rr, e.z0, e.rz))
        else:
            ssp.ssp_set_profile(pl, 0, s.nsteps, s.profile())
    elif s.env == "munk":
        if profile == "analytic":
            ssp.ssp_set_profile_analytic(pl)
        else:
            ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
    return pl


def oracle_march(s, nsteps=None, out_every=None, psi0=None):
    pl = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol,
                    rotation=s.rotation)
    return pl.march(s.starter() if psi0 is None else psi0, nsteps or s.nsteps, s.profile(),
                    out_every=out_every or s.out_every)


def compare(tag, fld, tl, ref, rel=REL_L2, dtl=DTL):
    assert fld.shape == ref.field.shape
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dt = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report(tag, max_relL2=f"{err.max():.3e}", final_relL2=f"{err[-1]:.3e}",
            max_dTL=f"{dt.max() if dt.size else 0:.3e}")
    assert err.max() <= rel
    assert dt.size == 0 or dt.max() <= dtl


# ------------------------------------------------------------------------------- transform
# up to 8192: one FFT per transform; above: the split transform (two half-length cores)
@pytest.mark.parametrize("nz", [2, 3, 5, 16, 63, 64, 100, 255, 256, 257, 1000, 2047, 4096, 5000, 8192,
                                8193, 12345, 16384])
def test_dst_parity(ssp, gpu, nz):
    torch = gpu
    B = 3
    pl = ssp.ssp_plan_create(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)
    try:
        x = np.stack([W.random_field(nz, 100 + b) for b in range(B)])
        d_in = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_out = torch.empty_like(d_in)
        ssp.ssp_dst_device(pl, B, d_in.data_ptr(), d_out.data_ptr())
        torch.cuda.synchronize()
        got = d_out.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = np.stack([odst(v) for v in x])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    _report("dst", nz=nz, relL2=f"{err.max():.2e}")
    assert err.max() < 2e-6


# dense product on the matrix cores: fp16 high/low parts of S and of each scaled column
# (three partial products, FP32 accumulation) leave ~2^-22 of the result plus the FP32
# accumulation over Nz terms; the bar is the one of the FFT transform
@pytest.mark.parametrize("nz,B", [(2, 1), (3, 5), (100, 3), (127, 64), (128, 2), (129, 65), (1000, 7),
                                  (2047, 3), (2048, 100)])
def test_dense_dst_parity(ssp, gpu, nz, B):
    torch = gpu
    pl = ssp.ssp_plan_create(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)
    try:
        x = np.stack([W.random_field(nz, 300 + b) for b in range(B)])
        # columns of very different magnitude, and a zero vector
        x[0] *= 1e-30
        if B > 2:
            x[1] *= 1e30
            x[2] = 0.0
        d_in = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_out = torch.empty_like(d_in)
        ssp.ssp_dst_dense_device(pl, B, d_in.data_ptr(), d_out.data_ptr())
        ssp.ssp_dst_dense_device(pl, B, d_in.data_ptr(), d_in.data_ptr())  # in place
        torch.cuda.synchronize()
        got = d_out.cpu().numpy().astype(np.complex128)
        got_inplace = d_in.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    x32 = x.astype(np.complex64).astype(np.complex128)
    ref = np.stack([odst(v) for v in x32])
    nrm = np.linalg.norm(ref, axis=1)
    live = nrm > 0
    err = np.linalg.norm(got - ref, axis=1)[live] / nrm[live]
    _report("dense dst", nz=nz, B=B, relL2=f"{err.max():.2e}")
    assert err.max() < 2e-6
    assert np.all(got[~live] == 0)
    assert np.array_equal(got, got_inplace)


def test_dense_dst_rejects_large_grid(ssp, gpu):
    nz = ssp.ssp_max_dense_nz() + 1
    pl = ssp.ssp_plan_create(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_dst_dense_device(pl, 1, 1, 1)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)


def test_sine_roundtrip_and_carrier(ssp, gpu):
    torch = gpu
    s = W.munk_deep(nz=1000)
    pl = make_plan(ssp, s)
    try:
        B = 2
        x = np.stack([s.starter(), W.random_field(s.nz, 7)])
        d_x = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_s = torch.empty_like(d_x)
        d_y = torch.empty_like(d_x)
        steps = torch.tensor([0, 7], dtype=torch.int64, device="cuda")
        ssp.ssp_to_sine(pl, B, d_x.data_ptr(), d_s.data_ptr())
        ssp.ssp_from_sine(pl, B, d_s.data_ptr(), steps.data_ptr(), d_y.data_ptr())
        torch.cuda.synchronize()
        y = d_y.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    car = np.exp(1j * s.k0 * s.dr * np.array([0, 7]))[:, None]
    err = np.linalg.norm(y - car * x, axis=1) / np.linalg.norm(x, axis=1)
    assert err.max() < 2e-6


# ------------------------------------------------------------------------------- marches
def test_homogeneous_waveguide(ssp, gpu):
    # H = 200 m, c = 1500 m/s, 100 Hz, Nz = 256, rotated [4/4], dr = 5 m, 1000 steps, V = 0
    s = W.homogeneous_waveguide()
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == OK and stats["steps_done"] == s.nsteps
    compare("homogeneous", fld, tl, ref)


# 8192: the largest grid with one FFT per transform; 8193: the smallest with split transforms
@pytest.mark.parametrize("nz,nsteps", [(2, 50), (3, 50), (127, 200), (511, 400), (1000, 100), (8192, 10),
                                      (8193, 10), (9000, 12)])
def test_munk_small(ssp, gpu, nz, nsteps):
    s = W.munk_deep(nsteps=nsteps, nz=nz)
    # on the coarsest grids the source Gaussian falls between grid points: use a seeded
    # random starter there
    psi0 = s.starter() if nz >= 16 else W.random_field(nz, 21)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, psi0, s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s, psi0=psi0)
    assert st == ref.status and stats["steps_done"] == ref.steps_done
    compare(f"munk nz={nz}", fld, tl, ref)
    # the same Neumann iteration counts as the oracle, up to a few near-threshold cases
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.01 * ref.iterations.sum() + 2


def test_empty_inputs_and_zero_steps(ssp, gpu):
    # zero vectors or zero plans are refused before any device work; a march of zero steps
    # returns no rows and leaves the state as it was: the march that follows it equals a
    # march from the freshly installed starter, bitwise
    torch = gpu
    s = W.munk_deep(nsteps=12, nz=1000)
    pl = make_plan(ssp, s)
    try:
        d = torch.zeros((1, s.nz), dtype=torch.complex64, device="cuda")
        for call in (lambda: ssp.ssp_dst_device(pl, 0, d.data_ptr(), d.data_ptr()),
                     lambda: ssp.ssp_march_batch([], [], 4)):
            with pytest.raises(ssp.SspError) as e:
                call()
            assert e.value.status == ssp.SSP_E_INVAL
        st0, f0, t0, stats0 = ssp.ssp_march(pl, s.nz, s.starter(), 0)
        assert st0 == OK and f0.shape == (0, s.nz) and t0.shape == (0, s.nz)
        assert stats0["steps_done"] == 0 and stats0["neumann_terms"] == 0
        st1, f1, t1, _ = ssp.ssp_march(pl, s.nz, None, s.nsteps)
        st2, f2, t2, _ = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    assert st1 == OK and st2 == OK and f1.shape[0] > 0
    assert np.array_equal(f1, f2) and np.array_equal(t1, t2)


def test_munk_full_size_start(ssp, gpu):
    # deep Munk waveguide at its full size (Nz = 4096) for the first 24 steps
    s = W.munk_deep(nsteps=24)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == OK
    compare("munk full start", fld, tl, ref)


def test_munk_full_size_norm_is_conserved(ssp, gpu):
    # lossless medium, standard Pade, converged series: ||u|| is constant (any size)
    s = W.munk_deep(nsteps=400)
    s.out_every = 100
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    n0 = np.linalg.norm(s.starter())
    ratios = np.linalg.norm(fld, axis=1) / n0
    _report("norm", ratios=np.array2string(ratios, precision=8))
    assert st == OK and np.max(np.abs(ratios - 1)) < 2e-5


@pytest.mark.parametrize("profile", ["table", "analytic"])
def test_eddy_range_dependent(ssp, gpu, profile):
    s = W.munk_eddy(nsteps=150, nz=1023, neumann_max=24)
    s.dr = 250.0 / 3.0   # crosses the eddy core (r0 = 50 km) in a short run
    s.nsteps = 120
    s.out_every = 10
    s.eddy = W.Eddy(r0=5000.0, rr=2500.0)
    pl = make_plan(ssp, s, profile=profile)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"eddy {profile}", fld, tl, ref)


@pytest.mark.parametrize("nz,nsteps", [(2046, 24), (4096, 20), (6000, 16)])
@pytest.mark.parametrize("profile", ["table", "analytic"])
def test_eddy_in_two_workgroup_layouts(ssp, gpu, nz, nsteps, profile):
    # FFT lengths 4096 ... 16384 run layout 2 (the potential held in registers and reloaded
    # every step of a range-dependent environment); the eddy (r0 = 1.5 km) is crossed
    s = W.munk_eddy(nsteps=nsteps, nz=nz, neumann_max=24)
    s.dr = 250.0 / 3.0
    s.out_every = 4
    s.eddy = W.Eddy(r0=1500.0, rr=1000.0)
    pl = make_plan(ssp, s, profile=profile)
    try:
        assert ssp.ssp_plan_engine(pl)[0] == 2
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    # (series that end within rounding of the tolerance may stop a term apart in FP32 and
    # FP64 arithmetic: the term counts are reported, the fields compared)
    _report(f"eddy layout 2 terms nz={nz}", gpu=stats["neumann_terms"], oracle=int(ref.iterations.sum()))
    compare(f"eddy layout 2 {profile} nz={nz}", fld, tl, ref)


@pytest.mark.parametrize("profile,variant", [("table", 0), ("analytic", 0), ("analytic", 2)])
def test_eddy_full_size_start(ssp, gpu, profile, variant):
    # Munk + eddy at its full size (200 Hz, Nz = 16384, [8/8], Neumann <= 12, dr = 20 m):
    # the first 10 steps, split transforms throughout, in both layouts of the split engine
    s = W.munk_eddy(nsteps=10)
    pl = make_plan(ssp, s, profile=profile)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, variant)
        assert ssp.ssp_plan_engine(pl)[0] == variant
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    _report(f"eddy full start {profile} layout {variant}", status=st, oracle_status=ref.status,
            terms=stats["neumann_terms"], oracle_terms=int(ref.iterations.sum()),
            not_converged=stats["not_converged"])
    assert st in (OK, NOT_CONVERGED) and ref.status in (OK, NOT_CONVERGED)
    assert stats["steps_done"] == ref.steps_done == s.nsteps
    compare(f"eddy full start {profile} layout {variant}", fld, tl, ref)


# ------------------------------------------------------------------------------- statuses
def test_divergence_reported_and_field_kept(ssp, gpu):
    s = W.munk_deep(nsteps=5, nz=511)
    s.dr = 1.0 / s.k0
    s.neumann_max = 16
    pl = make_plan(ssp, s)
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_DIVERGED
        back = ssp.ssp_get_field(pl, s.nz)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == DIVERGED and ref.steps_done == 0
    assert np.linalg.norm(back - s.starter()) / np.linalg.norm(s.starter()) < 2e-6


@pytest.mark.parametrize("p", [1, 2, 12])
def test_pade_order_extremes_vs_oracle(ssp, gpu, p):
    # the smallest approximant ([1/1]) and the largest order a plan accepts ([12/12]), on a
    # 200 Hz Munk channel (H = 1000 m, Nz = 1000, dr = 20 m) where every factor's series
    # converges
    s = W.munk_deep(nsteps=40, nz=1000)
    s.pade_order, s.freq, s.dr, s.depth, s.zs = p, 200.0, 20.0, 1000.0, 200.0
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == OK and st == OK and stats["steps_done"] == s.nsteps
    compare(f"pade [{p}/{p}]", fld, tl, ref)
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.01 * ref.iterations.sum() + 2


def test_high_order_divergence_matches_oracle(ssp, gpu):
    # on the 50 Hz Munk channel at Nz = 1000 the series of a [12/12] factor diverges in the
    # first step: the device reports it there and keeps the starter, as the oracle stops
    s = W.munk_deep(nsteps=5, nz=1000)
    s.pade_order = 12
    pl = make_plan(ssp, s)
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_DIVERGED
        back = ssp.ssp_get_field(pl, s.nz)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == DIVERGED and ref.steps_done == 0
    assert np.linalg.norm(back - s.starter()) / np.linalg.norm(s.starter()) < 2e-6


@pytest.mark.parametrize("nz", [500, 4096])
def test_divergence_after_unwritten_steps(ssp, gpu, nz):
    # the field is written back after every step (the recovery point): a step that diverges
    # after good steps (here step 5, where a slow layer enters the tabulated profile) leaves
    # the state after the last good step, bitwise equal to a march that stops there, and the
    # oracle stops at the same step
    s = W.munk_deep(nsteps=8, nz=nz)
    z = (np.arange(nz) + 1) * s.depth / (nz + 1)
    c = np.repeat(s.profile()[0][None, :], 8, axis=0)
    c[4:, (z > 1000.0) & (z < 1500.0)] = 1000.0

    def run(nsteps):
        pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
        try:
            ssp.ssp_set_profile(pl, 0, 8, c)
            ssp.ssp_set_field(pl, s.starter(), s.nz)
            st, _, _, stats = ssp.ssp_march_batch([pl], [s.nz], nsteps, want_field=False, want_tl=False)
            return st, stats[0], ssp.ssp_get_field(pl, s.nz)
        finally:
            ssp.ssp_plan_destroy(pl)

    st, stats, back = run(8)
    st4, stats4, good = run(4)
    _report(f"diverged after unwritten steps nz={nz}", status=st, steps=stats["steps_done"])
    assert st == ssp.SSP_E_DIVERGED and stats["status"] == ssp.SSP_E_DIVERGED and stats["steps_done"] == 4
    assert st4 == OK and stats4["steps_done"] == 4
    assert np.array_equal(back, good)
    o = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    ref = o.march(s.starter(), 8, c, out_every=0)
    assert ref.status == DIVERGED and ref.steps_done == 4
    assert np.linalg.norm(back - ref.final) / np.linalg.norm(ref.final) <= 1e-4


def test_not_converged_reported(ssp, gpu):
    s = W.munk_deep(nsteps=3, nz=511, neumann_max=3)
    s.out_every = 1
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert ref.status == NOT_CONVERGED and st == ssp.SSP_W_NOT_CONVERGED
    # series whose final residual is far from tol must be classified alike; ones within a
    # factor 10 of tol may differ between FP32 and FP64 arithmetic
    clear_nc = int((ref.residuals > 10 * s.tol).sum())
    maybe_nc = int((ref.residuals > 0.1 * s.tol).sum())
    assert clear_nc <= stats["not_converged"] <= maybe_nc
    compare("not converged", fld, tl, ref)


# ------------------------------------------------------------------------------- equivalences
def test_resume_is_bitwise(ssp, gpu):
    s = W.munk_deep(nsteps=40, nz=700)
    s.out_every = 20
    a = make_plan(ssp, s)
    b = make_plan(ssp, s)
    try:
        _, f_all, _, _ = ssp.ssp_march(a, s.nz, s.starter(), 40)
        _, f1, _, _ = ssp.ssp_march(b, s.nz, s.starter(), 20)
        _, f2, _, _ = ssp.ssp_march(b, s.nz, None, 20)
    finally:
        ssp.ssp_plan_destroy(a)
        ssp.ssp_plan_destroy(b)
    assert np.array_equal(f_all, np.concatenate([f1, f2]))


def test_resume_in_ragged_chunks_is_bitwise(ssp, gpu):
    # outputs fall on the multiples of out_every after the start: chunks of 3, 4 and 13 steps
    # with out_every = 5 give 0, 1 and 3 rows, together those of one 20-step march
    s = W.munk_deep(nsteps=20, nz=700)
    s.out_every = 5
    a = make_plan(ssp, s)
    b = make_plan(ssp, s)
    try:
        _, f_all, t_all, _ = ssp.ssp_march(a, s.nz, s.starter(), 20)
        parts = [ssp.ssp_march(b, s.nz, s.starter() if i == 0 else None, k) for i, k in enumerate((3, 4, 13))]
    finally:
        ssp.ssp_plan_destroy(a)
        ssp.ssp_plan_destroy(b)
    assert [p[1].shape[0] for p in parts] == [0, 1, 3] and f_all.shape[0] == 4
    assert [p[3]["step_index"] for p in parts] == [3, 7, 20]
    assert np.array_equal(f_all, np.concatenate([p[1] for p in parts]))
    assert np.array_equal(t_all, np.concatenate([p[2] for p in parts]))


def test_batch_equals_alone_bitwise(ssp, gpu):
    sizes = [(300, 500.0), (777, 1500.0), (2000, 1000.0), (511, 100.0)]
    solves = [W.munk_deep(nsteps=16, nz=nz, zs=zs) for nz, zs in sizes]
    for s in solves:
        s.out_every = 8
    alone = []
    for s in solves:
        pl = make_plan(ssp, s)
        try:
            alone.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)[1])
        finally:
            ssp.ssp_plan_destroy(pl)
    plans = [make_plan(ssp, s) for s in solves]
    try:
        for pl, s in zip(plans, solves):
            ssp.ssp_set_field(pl, s.starter(), s.nz)
        st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], 16)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for a, b in zip(alone, fl):
        assert np.array_equal(a, b)


def test_uneven_lengths_one_batch_equal_alone_bitwise(ssp, gpu):
    # FFT lengths 8192, 16384 and 32768 (broadband frequencies) in one batched call (their
    # launch groups run concurrently; the graph-recorded form of the same batch is checked
    # in test_gpu_batch.py); each solve must give exactly what it gives alone
    solves = []
    for nz, f in [(3000, 56.25), (6000, 112.5), (12000, 225.0), (16000, 300.0)]:
        s = W.munk_deep(nsteps=6, nz=nz)
        s.freq = f
        s.out_every = 3
        solves.append(s)
    alone = []
    for s in solves:
        pl = make_plan(ssp, s)
        try:
            alone.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps))
        finally:
            ssp.ssp_plan_destroy(pl)
    plans = [make_plan(ssp, s) for s in solves]
    try:
        for pl, s in zip(plans, solves):
            ssp.ssp_set_field(pl, s.starter(), s.nz)
        st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], 6)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for (st1, f1, t1, s1), f2, t2, s2 in zip(alone, fl, tl, stats):
        assert s1 == s2
        assert np.array_equal(f1, f2) and np.array_equal(t1, t2)


def test_device_batch_matches_host_march(ssp, gpu):
    torch = gpu
    B = 5
    base = W.munk_deep(nsteps=12, nz=1500)
    zs = W.source_depths(B, 200.0, 2000.0, seed=4)
    pl = make_plan(ssp, base)
    try:
        psi = np.stack([W.gaussian_starter(base.nz, base.depth, base.freq, base.c0, z) for z in zs])
        d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
        steps = torch.zeros(B, dtype=torch.int64, device="cuda")
        ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), base.nsteps)
        out = torch.empty_like(d_psi)
        ssp.ssp_from_sine(pl, B, d_psi.data_ptr(), steps.data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert steps.cpu().tolist() == [base.nsteps] * B
        host = []
        for z in zs:
            ssp.ssp_set_field(pl, W.gaussian_starter(base.nz, base.depth, base.freq, base.c0, z), base.nz)
            ssp.ssp_march(pl, base.nz, None, base.nsteps, want_field=False, want_tl=False)
            host.append(ssp.ssp_get_field(pl, base.nz))
    finally:
        ssp.ssp_plan_destroy(pl)
    assert np.array_equal(got.astype(np.complex128), np.stack(host))


@pytest.mark.parametrize("nz,env", [(510, "munk"), (300, "munk+eddy"), (9000, "munk")])
def test_plain_form_equals_fused_bitwise(ssp, gpu, nz, env):
    # the one-kernel-per-stage form runs the same arithmetic in the same order
    s = W.munk_deep(nsteps=8, nz=nz) if env == "munk" else W.munk_eddy(nsteps=8, nz=nz, neumann_max=24)
    s.out_every = 4
    out = []
    for engine in (0, 1):
        pl = make_plan(ssp, s, profile="analytic" if env != "munk" else "table")
        try:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_PLAIN, engine)
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, 0)  # the plain kernels' layout
            out.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps))
        finally:
            ssp.ssp_plan_destroy(pl)
    (st0, f0, t0, s0), (st1, f1, t1, s1) = out
    assert st0 == st1 and s0 == s1
    assert np.array_equal(f0, f1) and np.array_equal(t0, t1)


# every engine layout of the lengths that have several (FFT lengths 1024 ... 32768; a layout
# a length does not have falls back to layout 0; Nz = 12000 runs the split transform, whose
# layout 2 is the 512-thread engine of the 16384-point halves)
@pytest.mark.parametrize("nz", [510, 1000, 2046, 4096, 6000, 12000])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_engine_layouts_vs_oracle(ssp, gpu, nz, variant):
    s = W.munk_deep(nsteps=16, nz=nz)
    s.out_every = 4
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, variant)
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status == OK
    compare(f"layout {variant} nz={nz}", fld, tl, ref)


def test_layout_option_and_engine_query(ssp, gpu):
    # the layout a plan reports: the tuned default, an explicit choice, or layout 0 where the
    # length has no such layout; invalid values are rejected and leave the plan unchanged
    pl = ssp.ssp_plan_create(4096, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10)
    try:
        v0, t0, p0 = ssp.ssp_plan_engine(pl)
        assert p0 == 8192 and v0 in (0, 1, 2)
        seen = {}
        for v in (0, 1, 2):
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, v)
            seen[v] = ssp.ssp_plan_engine(pl)
        assert seen[0][1] == 1024 and seen[1][1] == 512 and seen[2][1] == 256
        for bad in (3, -3, 0.5):
            with pytest.raises(ssp.SspError) as e:
                ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, bad)
            assert e.value.status == ssp.SSP_E_INVAL
        assert ssp.ssp_plan_engine(pl) == seen[2]
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, -1)
        assert ssp.ssp_plan_engine(pl) == (v0, t0, p0)
    finally:
        ssp.ssp_plan_destroy(pl)
    pl = ssp.ssp_plan_create(12000, 5000.0, 225.0, 1500.0, 25.0, 6, 48, 1e-10)  # split: 0 and 2
    try:
        got = {}
        for v in (0, 1, 2):
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, v)
            got[v] = ssp.ssp_plan_engine(pl)
        assert got[0] == (0, 1024, 32768) and got[1] == got[0] and got[2] == (2, 512, 32768)
    finally:
        ssp.ssp_plan_destroy(pl)
    pl = ssp.ssp_plan_create(300, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)  # FFT length 1024
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, 2)  # no layout 2 at this length
        assert ssp.ssp_plan_engine(pl)[0] == 0
    finally:
        ssp.ssp_plan_destroy(pl)


def test_plain_form_reports_divergence(ssp, gpu):
    s = W.munk_deep(nsteps=3, nz=510)
    s.dr = 1.0 / s.k0
    s.neumann_max = 16
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_PLAIN, 1)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_DIVERGED
        back = ssp.ssp_get_field(pl, s.nz)
    finally:
        ssp.ssp_plan_destroy(pl)
    assert np.linalg.norm(back - s.starter()) / np.linalg.norm(s.starter()) < 2e-6


def test_graph_replays_match_plain_launches(ssp, gpu):
    # device batch advanced in chunks: recorded-graph replays vs ordinary launches, with
    # eager work and synchronisations between the replays; every replay is compared
    torch = gpu
    B, chunk, nchunks = 3, 6, 3
    base = W.munk_deep(nsteps=chunk, nz=900)
    zs = [300.0, 900.0, 1700.0]
    results = []
    for graph in (0, 1):
        stream = torch.cuda.Stream()
        pl = make_plan(ssp, base)
        try:
            ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GRAPH, graph)
            psi = np.stack([W.gaussian_starter(base.nz, base.depth, base.freq, base.c0, z) for z in zs])
            with torch.cuda.stream(stream):
                d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
                steps = torch.zeros(B, dtype=torch.int64, device="cuda")
                tl = torch.zeros((B, chunk // base.out_every + 1, base.nz), dtype=torch.float32, device="cuda")
            stream.synchronize()
            ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
            snaps = []
            for c in range(nchunks):
                ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), chunk, tl.data_ptr())
                stream.synchronize()
                junk = torch.randn(1000, device="cuda").sum().item()  # eager work in between
                snaps.append((d_psi.cpu().numpy().copy(), tl.cpu().numpy().copy(), steps.cpu().tolist()))
                assert np.isfinite(junk)
        finally:
            ssp.ssp_plan_destroy(pl)
        results.append(snaps)
    for (a_psi, a_tl, a_st), (b_psi, b_tl, b_st) in zip(*results):
        assert a_st == b_st
        assert np.array_equal(a_psi, b_psi) and np.array_equal(a_tl, b_tl)
    assert results[0][-1][2] == [chunk * nchunks] * B


def _device_batch_vs_oracle(ssp, torch, s, B, nsteps, samples, profile):
    """The benchmark's launch configuration: B solves of one plan on a dedicated stream,
    graph-recorded launches, TL rows on the device; sampled solves against the oracle."""
    stream = torch.cuda.Stream()
    pl = make_plan(ssp, s, profile=profile)
    zs = W.source_depths(B, 50.0, 2000.0)
    try:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GRAPH, 1)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z) for z in zs])
        with torch.cuda.stream(stream):
            d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
            steps = torch.zeros(B, dtype=torch.int64, device="cuda")
            nout = nsteps // s.out_every + 1
            d_tl = torch.zeros((B, nout, s.nz), dtype=torch.float32, device="cuda")
            out = torch.empty_like(d_psi)
        stream.synchronize()
        ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), nsteps, d_tl.data_ptr())
        ssp.ssp_from_sine(pl, B, d_psi.data_ptr(), steps.data_ptr(), out.data_ptr())
        stream.synchronize()
        tl = d_tl.cpu().numpy()
        fld = out.cpu().numpy().astype(np.complex128)
        assert steps.cpu().tolist() == [nsteps] * B
    finally:
        ssp.ssp_plan_destroy(pl)
    for b in samples:
        s1 = W.Solve(**{**s.__dict__, "zs": float(zs[b]), "nsteps": nsteps})
        ref = oracle_march(s1)
        rows = ref.tl.shape[0]
        mask = ref.tl < 120.0
        dtl = np.abs(tl[b, :rows].astype(np.float64) - ref.tl)[mask]
        err = np.linalg.norm(fld[b] - ref.final) / np.linalg.norm(ref.final)
        _report(f"bench config b={b}", nz=s.nz, relL2=f"{err:.3e}", max_dTL=f"{dtl.max():.3e}")
        assert err <= REL_L2 and dtl.max() <= DTL


def test_munk_bench_launch_configuration_sampled(ssp, gpu):
    # 512 solves of the deep Munk waveguide at Nz = 4096, as bench.py times them
    s = W.munk_deep()
    _device_batch_vs_oracle(ssp, gpu, s, 512, 24, [0, 255, 511], "table")


def test_eddy_bench_launch_configuration_sampled(ssp, gpu):
    # 256 Munk + eddy solves at Nz = 16384 (split transforms), potential on the device
    s = W.munk_eddy()
    _device_batch_vs_oracle(ssp, gpu, s, 256, 10, [0, 255], "analytic")


def test_broadband_one_launch_sampled(ssp, gpu):
    # frequencies of the broadband set with lengths 8192, 16384 and 32768 in one batched call
    solves = [W.broadband()[i] for i in (0, 100, 255)]
    nsteps = 8
    plans = [make_plan(ssp, s) for s in solves]
    try:
        for pl, s in zip(plans, solves):
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, 4)
            ssp.ssp_set_field(pl, s.starter(), s.nz)
        st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], nsteps)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for s, f, t in zip(solves, fl, tl):
        s.out_every = 4
        compare(f"broadband f={s.freq:.1f} nz={s.nz}", f, t, oracle_march(s, nsteps=nsteps))


def test_munk_full_size_full_range_vs_stored_oracle(ssp, gpu):
    # the benchmark workload at its full size and range (Nz = 4096, 4000 steps, 100 km)
    # against the oracle's field every 10 km (tests/golden/make_golden.py munk4096)
    import os
    from oracle import transmission_loss
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "munk4096_zs1000.npz"))
    s = W.munk_deep()
    s.out_every = int(g["out_every"])
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), int(g["nsteps"]))
    finally:
        ssp.ssp_plan_destroy(pl)
    assert st == int(g["status"]) == OK

    class Ref:
        field = g["field"]
        tl = transmission_loss(g["field"], g["ranges"])
    compare("munk full range", fld, tl, Ref)


def test_eddy_full_size_long_range_vs_stored_oracle(ssp, gpu):
    # Munk + eddy at its full size (Nz = 16384, [8/8], split transforms, potential on the
    # device) for 3000 steps (60 km, through the eddy core), against the stored FP64 oracle
    import os
    from oracle import transmission_loss
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "eddy16384_zs1000.npz"))
    s = W.munk_eddy(nsteps=int(g["nsteps"]))
    s.out_every = int(g["out_every"])
    pl = make_plan(ssp, s, profile="analytic")
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    _report("eddy long range", status=st, oracle_status=int(g["status"]),
            terms=stats["neumann_terms"], oracle_terms=int(np.sum(g["iterations"])),
            not_converged=stats["not_converged"], oracle_not_converged=int(g["not_converged"]))
    assert st in (OK, NOT_CONVERGED) and int(g["status"]) in (OK, NOT_CONVERGED)
    assert stats["steps_done"] == s.nsteps

    class Ref:
        field = g["field"]
        tl = transmission_loss(g["field"], g["ranges"])
    compare("eddy long range", fld, tl, Ref)


@pytest.mark.timeout(900)
def test_eddy_full_size_full_range_vs_stored_oracle(ssp, gpu):
    # Munk + eddy over its whole range: Nz = 16384 (split transforms), [8/8], Neumann <= 12,
    # 10^4 steps (200 km), potential on the device, against the stored FP64 oracle every
    # 20 km (tests/golden/make_golden.py eddy16384_full)
    import os
    from oracle import transmission_loss
    path = os.path.join(os.path.dirname(__file__), "golden", "eddy16384_full_zs1000.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle field missing: python tests/golden/make_golden.py eddy16384_full")
    g = np.load(path)
    s = W.munk_eddy(nsteps=int(g["nsteps"]))
    s.out_every = int(g["out_every"])
    pl = make_plan(ssp, s, profile="analytic")
    fields, tls, stats_all = [], [], []
    try:
        ssp.ssp_set_field(pl, s.starter(), s.nz)
        chunk = 1000
        for n0 in range(0, s.nsteps, chunk):
            st, fld, tl, stats = ssp.ssp_march(pl, s.nz, None, chunk)
            assert st in (OK, NOT_CONVERGED) and stats["steps_done"] == chunk
            fields.append(fld)
            tls.append(tl)
            stats_all.append(stats)
            print(f"[eddy full range] step {n0 + chunk}: terms {stats['neumann_terms']}", flush=True)
    finally:
        ssp.ssp_plan_destroy(pl)
    fld = np.concatenate(fields)
    terms = sum(x["neumann_terms"] for x in stats_all)
    nc = sum(x["not_converged"] for x in stats_all)
    _report("eddy full range", oracle_status=int(g["status"]), terms=terms,
            oracle_terms=int(np.sum(g["iterations"])), not_converged=nc,
            oracle_not_converged=int(g["not_converged"]))
    ref_field = g["field"].astype(np.complex128)

    class Ref:
        field = ref_field
        tl = transmission_loss(ref_field, g["ranges"])
    err = np.linalg.norm(fld - Ref.field, axis=1) / np.linalg.norm(Ref.field, axis=1)
    for r, e in zip(g["ranges"], err):
        print(f"[eddy full range] r = {r / 1000:.0f} km relL2 {e:.3e}", flush=True)
    compare("eddy full range", fld, np.concatenate(tls), Ref)


BROADBAND_GOLDEN = (0, 20, 28, 64, 106, 107, 180, 255)


@pytest.mark.timeout(900)
def test_broadband_full_batch_full_range_vs_stored_oracle(ssp, gpu):
    # all 256 frequencies of the broadband set in one batch (FFT lengths 8192, 16384 and
    # 32768, the mixed-batch layouts) over the full 2000 steps (50 km); the sampled
    # frequencies against the stored FP64 oracle at 25 and 50 km
    # (tests/golden/make_golden.py broadband): the per-frequency error table
    import os
    from oracle import transmission_loss
    solves = W.broadband()
    paths = {i: os.path.join(os.path.dirname(__file__), "golden", f"broadband_f{i:03d}.npz") for i in BROADBAND_GOLDEN}
    missing = [i for i, q in paths.items() if not os.path.exists(q)]
    if missing:
        pytest.skip(f"stored oracle fields missing: python tests/golden/make_golden.py broadband {missing}")
    gold = {i: np.load(q) for i, q in paths.items()}
    plans = []
    try:
        for i, s in enumerate(solves):
            s.out_every = 1000
            pl = make_plan(ssp, s)
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, -2)
            ssp.ssp_set_field(pl, s.starter(), s.nz)
            plans.append(pl)
        rows = {i: [] for i in gold}
        terms = {i: 0 for i in gold}
        chunk = 200
        for n0 in range(0, 2000, chunk):
            st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], chunk)
            assert st in (OK, NOT_CONVERGED)
            for i in gold:
                if fl[i].shape[0]:
                    rows[i].append(fl[i])
                terms[i] += stats[i]["neumann_terms"]
            assert all(x["steps_done"] == chunk for x in stats)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    worst = 0.0
    for i, g in gold.items():
        s = solves[i]
        fld = np.concatenate(rows[i])
        ref = g["field"].astype(np.complex128)
        assert fld.shape == ref.shape
        err = np.linalg.norm(fld - ref, axis=1) / np.linalg.norm(ref, axis=1)
        tl_ref = transmission_loss(ref, g["ranges"])
        tl_got = transmission_loss(fld, g["ranges"])
        mask = tl_ref < 120.0
        dtl = np.abs(tl_got - tl_ref)[mask]
        print(f"[broadband per frequency] f = {s.freq:7.3f} Hz  Nz = {s.nz:5d}  relL2(25 km) = {err[0]:.2e}  "
              f"relL2(50 km) = {err[1]:.2e}  max dTL = {dtl.max():.3f} dB  terms {terms[i]} "
              f"(oracle {int(np.sum(g['iterations']))})", flush=True)
        worst = max(worst, err.max())
        assert err.max() <= REL_L2 and dtl.max() <= DTL
    _report("broadband full range", worst_relL2=f"{worst:.3e}")
