"""GPU parity of the complex absorbing potential (Sec. 3.1; v -> v + i eta in a bottom layer)
against the oracle.  Bar as for the other marches: relative L2 field error <= 1e-4 at every
output range, |TL_gpu - TL_oracle| <= 0.1 dB where TL_oracle < 120 dB; plain-form and
removal equivalences bitwise.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Plan as OraclePlan

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
DTL = 0.1
LAYER = (1000.0, 0.05)   # bottom 1000 m of the 5000 m waveguide, eta rising to 0.05


def _report(tag, **kv):
    print(f"[{tag}] " + " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def eta_of(s):
    return W.absorbing_layer(s.nz, s.depth, LAYER[0], LAYER[1], s.bc)


def make_plan(ssp, s, profile="table", absorber=True):
    pl = ssp.ssp_plan_create_bc(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max,
                                s.tol, s.bc)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, s.out_every)
    if s.env == "munk+eddy":
        if profile == "analytic":
            e = s.eddy or W.Eddy()
            ssp.ssp_set_profile_analytic(pl, eddy=(e.amp, e.r0, e.rr, e.z0, e.rz))
        else:
            ssp.ssp_set_profile(pl, 0, s.nsteps, s.profile())
    else:
        ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
    if absorber:
        ssp.ssp_set_absorber(pl, eta_of(s))
    return pl


def oracle_march(s):
    pl = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol, bc=s.bc)
    return pl.march(s.starter(), s.nsteps, s.profile(), out_every=s.out_every, absorber=eta_of(s))


def compare(tag, fld, tl, ref):
    assert fld.shape == ref.field.shape
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dt = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report(tag, max_relL2=f"{err.max():.3e}", final_relL2=f"{err[-1]:.3e}",
            max_dTL=f"{dt.max() if dt.size else 0:.3e}")
    assert err.max() <= REL_L2
    assert dt.size == 0 or dt.max() <= DTL


@pytest.mark.parametrize("bc,nz,nsteps", [("dirichlet", 1000, 100), ("dirichlet", 4096, 24),
                                          ("dirichlet", 9000, 12), ("neumann", 1000, 100),
                                          ("periodic", 1000, 100)])
def test_munk_with_absorber_vs_oracle(ssp, gpu, bc, nz, nsteps):
    s = dataclasses.replace(W.munk_deep(nsteps=nsteps, nz=nz), bc=bc)
    s.out_every = max(1, nsteps // 4)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status and stats["steps_done"] == ref.steps_done
    compare(f"absorber {bc} nz={nz}", fld, tl, ref)
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.01 * ref.iterations.sum() + 2


@pytest.mark.parametrize("profile", ["table", "analytic"])
def test_eddy_with_absorber_vs_oracle(ssp, gpu, profile):
    s = W.munk_eddy(nsteps=40, nz=1000, neumann_max=24)
    s.out_every = 10
    pl = make_plan(ssp, s, profile=profile)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"absorber eddy {profile}", fld, tl, ref)


def test_plain_form_equals_fused_bitwise_with_absorber(ssp, gpu):
    s = W.munk_deep(nsteps=8, nz=510)
    s.out_every = 4
    out = []
    for engine in (0, 1):
        pl = make_plan(ssp, s)
        try:
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_PLAIN, engine)
            ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, 0)
            out.append(ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps))
        finally:
            ssp.ssp_plan_destroy(pl)
    (st0, f0, t0, s0), (st1, f1, t1, s1) = out
    assert st0 == st1 and s0 == s1
    assert np.array_equal(f0, f1) and np.array_equal(t0, t1)


def test_removing_the_absorber_restores_the_lossless_march_bitwise(ssp, gpu):
    s = W.munk_deep(nsteps=10, nz=700)
    s.out_every = 5
    a = make_plan(ssp, s, absorber=False)
    b = make_plan(ssp, s, absorber=True)
    try:
        ssp.ssp_set_absorber(b, None)
        ra = ssp.ssp_march(a, s.nz, s.starter(), s.nsteps)
        rb = ssp.ssp_march(b, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(a)
        ssp.ssp_plan_destroy(b)
    assert np.array_equal(ra[1], rb[1]) and np.array_equal(ra[2], rb[2])


def test_absorber_rejects_non_finite(ssp, gpu):
    s = W.munk_deep(nsteps=1, nz=64)
    pl = make_plan(ssp, s, absorber=False)
    try:
        eta = np.zeros(s.nz)
        eta[3] = np.nan
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_set_absorber(pl, eta)
        assert e.value.status == ssp.SSP_E_INVAL
    finally:
        ssp.ssp_plan_destroy(pl)


def test_munk_bench_launch_configuration_with_absorber_sampled(ssp, gpu):
    # 512 solves at Nz = 4096 with the bottom layer, as `bench.py --absorber` times them
    torch = gpu
    s = W.munk_deep()
    B, nsteps = 512, 24
    stream = torch.cuda.Stream()
    pl = make_plan(ssp, s)
    zs = W.source_depths(B, 50.0, 2000.0)
    try:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GRAPH, 1)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z) for z in zs])
        with torch.cuda.stream(stream):
            d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
            steps = torch.zeros(B, dtype=torch.int64, device="cuda")
            d_tl = torch.zeros((B, nsteps // s.out_every + 1, s.nz), dtype=torch.float32, device="cuda")
            out = torch.empty_like(d_psi)
        stream.synchronize()
        ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
        ssp.ssp_march_device(pl, B, d_psi.data_ptr(), steps.data_ptr(), nsteps, d_tl.data_ptr())
        ssp.ssp_from_sine(pl, B, d_psi.data_ptr(), steps.data_ptr(), out.data_ptr())
        stream.synchronize()
        tl = d_tl.cpu().numpy()
        fld = out.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    for b in (0, 511):
        s1 = dataclasses.replace(s, zs=float(zs[b]), nsteps=nsteps)
        ref = oracle_march(s1)
        mask = ref.tl < 120.0
        dtl = np.abs(tl[b, :ref.tl.shape[0]].astype(np.float64) - ref.tl)[mask]
        err = np.linalg.norm(fld[b] - ref.final) / np.linalg.norm(ref.final)
        _report(f"absorber bench config b={b}", relL2=f"{err:.3e}", max_dTL=f"{dtl.max():.3e}")
        assert err <= REL_L2 and dtl.max() <= DTL
