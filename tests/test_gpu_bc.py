"""GPU parity of the Neumann and periodic boundary conditions (Sec. 3.1) against the oracle.

The HIP library runs every boundary condition through the same kernels; only the plan's
tables (chirp windows, modulations, eigenvalues) and grid differ.  Bar as for the
Dirichlet march: relative L2 field error <= 1e-4 at every output range and
|TL_gpu - TL_oracle| <= 0.1 dB wherever TL_oracle < 120 dB; transforms <= 2e-6; batch,
resume and plain-form equivalences bitwise.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import OK, Plan as OraclePlan
from oracle.bases import forward as oforward

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
DTL = 0.1
BCS = ["neumann", "periodic"]


def _report(tag, **kv):
    print(f"[{tag}] " + " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def make_plan(ssp, s, profile="table"):
    pl = ssp.ssp_plan_create_bc(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max,
                                s.tol, s.bc)
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


def oracle_march(s, psi0=None):
    pl = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol,
                    rotation=s.rotation, bc=s.bc)
    return pl.march(s.starter() if psi0 is None else psi0, s.nsteps, s.profile(),
                    out_every=s.out_every)


def compare(tag, fld, tl, ref):
    assert fld.shape == ref.field.shape
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dt = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report(tag, max_relL2=f"{err.max():.3e}", final_relL2=f"{err[-1]:.3e}",
            max_dTL=f"{dt.max() if dt.size else 0:.3e}")
    assert err.max() <= REL_L2
    assert dt.size == 0 or dt.max() <= DTL


def with_bc(s, bc):
    return dataclasses.replace(s, bc=bc)


# ------------------------------------------------------------------------------- transforms
# up to 8192 points one FFT per transform, above it the split transform
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nz", [2, 3, 64, 255, 1000, 4096, 8193, 16384])
def test_forward_transform_parity(ssp, gpu, bc, nz):
    torch = gpu
    B = 3
    pl = ssp.ssp_plan_create_bc(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10, bc)
    try:
        x = np.stack([W.random_field(nz, 300 + b) for b in range(B)])
        d_in = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_out = torch.empty_like(d_in)
        ssp.ssp_dst_device(pl, B, d_in.data_ptr(), d_out.data_ptr())
        torch.cuda.synchronize()
        got = d_out.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = np.stack([oforward(bc, v) for v in x])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    _report(f"transform {bc} nz={nz}", max_relL2=f"{err.max():.3e}")
    assert err.max() <= 2e-6


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nz", [100, 9000])
def test_coefficient_roundtrip_and_carrier(ssp, gpu, bc, nz):
    torch = gpu
    s = with_bc(W.munk_deep(nz=nz), bc)
    pl = make_plan(ssp, s)
    try:
        x = np.stack([s.starter(), W.random_field(s.nz, 7)])
        d_x = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_s = torch.empty_like(d_x)
        d_y = torch.empty_like(d_x)
        steps = torch.tensor([0, 7], dtype=torch.int64, device="cuda")
        ssp.ssp_to_sine(pl, 2, d_x.data_ptr(), d_s.data_ptr())
        ssp.ssp_from_sine(pl, 2, d_s.data_ptr(), steps.data_ptr(), d_y.data_ptr())
        torch.cuda.synchronize()
        y = d_y.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    car = np.exp(1j * s.k0 * s.dr * np.array([0, 7]))[:, None]
    err = np.linalg.norm(y - car * x, axis=1) / np.linalg.norm(x, axis=1)
    assert err.max() < 2e-6


def test_dense_transform_rejects_other_boundaries(ssp, gpu):
    pl = ssp.ssp_plan_create_bc(256, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10, "neumann")
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_dst_dense_device(pl, 1, 1, 1)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)


# ------------------------------------------------------------------------------- marches
@pytest.mark.parametrize("bc", BCS)
def test_homogeneous_waveguide(ssp, gpu, bc):
    # H = 200 m, c = c0, 100 Hz, Nz = 256, rotated [4/4], dr = 5 m, 1000 steps, V = 0
    s = with_bc(W.homogeneous_waveguide(), bc)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == OK and stats["steps_done"] == s.nsteps
    compare(f"homogeneous {bc}", fld, tl, ref)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nz,nsteps", [(3, 40), (127, 200), (1000, 100), (4096, 24), (6000, 12), (9000, 12)])
def test_munk_vs_oracle(ssp, gpu, bc, nz, nsteps):
    s = with_bc(W.munk_deep(nsteps=nsteps, nz=nz), bc)
    psi0 = s.starter() if nz >= 16 else W.random_field(nz, 21)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, psi0, s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s, psi0=psi0)
    assert st == ref.status and stats["steps_done"] == ref.steps_done
    compare(f"munk {bc} nz={nz}", fld, tl, ref)
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.01 * ref.iterations.sum() + 2


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("profile", ["table", "analytic"])
def test_eddy_range_dependent(ssp, gpu, bc, profile):
    # the analytic environment is evaluated on the device at the bc's grid points
    s = with_bc(W.munk_eddy(nsteps=40, nz=1000, neumann_max=24), bc)
    s.out_every = 10
    pl = make_plan(ssp, s, profile=profile)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"eddy {bc} {profile}", fld, tl, ref)


@pytest.mark.parametrize("bc", BCS)
def test_plain_form_equals_fused_bitwise(ssp, gpu, bc):
    s = with_bc(W.munk_deep(nsteps=8, nz=511), bc)
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


def test_mixed_boundaries_batch_equals_alone_bitwise(ssp, gpu):
    # plans of the three boundary conditions (and FFT lengths) marched in one batch call
    cases = [("dirichlet", 700), ("neumann", 700), ("periodic", 700), ("neumann", 3000),
             ("periodic", 2048)]
    solves = []
    for bc, nz in cases:
        s = with_bc(W.munk_deep(nsteps=12, nz=nz), bc)
        s.out_every = 6
        solves.append(s)
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
        st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], 12)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for a, b in zip(alone, fl):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("bc", BCS)
def test_munk_bench_launch_configuration_sampled(ssp, gpu, bc):
    # 512 solves at Nz = 4096 as `bench.py --bc` times them: one plan on a dedicated
    # stream, graph-recorded launches, TL rows on the device; sampled solves vs the oracle
    torch = gpu
    s = with_bc(W.munk_deep(), bc)
    B, nsteps = 512, 24
    stream = torch.cuda.Stream()
    pl = make_plan(ssp, s)
    zs = W.source_depths(B, 50.0, 2000.0)
    try:
        ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_GRAPH, 1)
        psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z, bc) for z in zs])
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
        assert steps.cpu().tolist() == [nsteps] * B
    finally:
        ssp.ssp_plan_destroy(pl)
    for b in (0, 511):
        s1 = dataclasses.replace(s, zs=float(zs[b]), nsteps=nsteps)
        ref = oracle_march(s1)
        mask = ref.tl < 120.0
        dtl = np.abs(tl[b, :ref.tl.shape[0]].astype(np.float64) - ref.tl)[mask]
        err = np.linalg.norm(fld[b] - ref.final) / np.linalg.norm(ref.final)
        _report(f"bench config {bc} b={b}", relL2=f"{err:.3e}", max_dTL=f"{dtl.max():.3e}")
        assert err <= REL_L2 and dtl.max() <= DTL


@pytest.mark.parametrize("bc", BCS)
def test_munk_long_range(ssp, gpu, bc):
    # 400 steps (10 km) at Nz = 1000: error growth over range stays within the bar
    s = with_bc(W.munk_deep(nsteps=400, nz=1000), bc)
    s.out_every = 100
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"munk long {bc}", fld, tl, ref)


@pytest.mark.parametrize("nz,nsteps", [(128, 100), (512, 100), (2048, 50), (8192, 12), (16384, 6)])
def test_periodic_direct_fft_lengths_vs_oracle(ssp, gpu, nz, nsteps):
    # periodic grids whose length is a power of two run direct FFTs of length Nz
    s = with_bc(W.munk_deep(nsteps=nsteps, nz=nz), "periodic")
    s.out_every = max(1, nsteps // 3)
    pl = make_plan(ssp, s)
    try:
        layout, threads, P = ssp.ssp_plan_engine(pl)
        assert P == nz
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"periodic direct nz={nz}", fld, tl, ref)


@pytest.mark.parametrize("nz", [1024, 2048, 4096, 8192])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_periodic_direct_layouts_vs_oracle(ssp, gpu, nz, variant):
    # every engine layout of the direct Fourier march (a layout the length does not have
    # falls back to layout 0)
    s = with_bc(W.munk_deep(nsteps=12, nz=nz), "periodic")
    s.out_every = 4
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, variant)
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    compare(f"periodic direct layout {variant} nz={nz}", fld, tl, ref)


def test_periodic_direct_rejects_the_plain_form(ssp, gpu):
    s = with_bc(W.munk_deep(nsteps=2, nz=1024), "periodic")
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_PLAIN, 1)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)
    # a periodic grid of another length keeps the chirp-z transform of length >= 2 Nz - 1
    pl = ssp.ssp_plan_create_bc(1000, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10, "periodic")
    try:
        assert ssp.ssp_plan_engine(pl)[2] == 2048
    finally:
        ssp.ssp_plan_destroy(pl)
