"""GPU parity of the direct sine transform (Dirichlet grids with Nz + 1 a power of two).

Such grids run each DST-I (Sec. 2.1) as one FFT of length 2(Nz + 1) over the odd extension
of the data instead of the two chirp-z FFTs of the general length.  Bars as for the chirp-z
path: transforms relative L2 <= 2e-6 against the oracle's DST; marches relative L2 <= 1e-4
at every output range and |dTL| <= 0.1 dB where TL < 120 dB; batch equivalence bitwise.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import Plan as OraclePlan
from oracle.bases import forward as oforward

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
DTL = 0.1
DIRECT = [63, 127, 1023, 4095, 8191]


def _report(tag, **kv):
    print(f"[{tag}] " + " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def make_plan(ssp, s):
    pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, s.out_every)
    ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
    return pl


def oracle_march(s):
    pl = OraclePlan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    return pl.march(s.starter(), s.nsteps, s.profile(), out_every=s.out_every)


@pytest.mark.parametrize("nz", DIRECT + [16383])
def test_engine_length(ssp, gpu, nz):
    # direct up to FFT length 16384; Nz = 16383 falls back to the chirp-z split transform
    pl = ssp.ssp_plan_create(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)
    try:
        layout, threads, P = ssp.ssp_plan_engine(pl)
    finally:
        ssp.ssp_plan_destroy(pl)
    assert P == (2 * (nz + 1) if nz < 16383 else 32768)


@pytest.mark.parametrize("nz", DIRECT)
def test_forward_transform_parity(ssp, gpu, nz):
    torch = gpu
    B = 3
    pl = ssp.ssp_plan_create(nz, 1000.0, 50.0, 1500.0, 10.0, 2, 0, 1e-10)
    try:
        x = np.stack([W.random_field(nz, 500 + b) for b in range(B)])
        d_in = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_out = torch.empty_like(d_in)
        ssp.ssp_dst_device(pl, B, d_in.data_ptr(), d_out.data_ptr())
        torch.cuda.synchronize()
        got = d_out.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = np.stack([oforward("dirichlet", v) for v in x])
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    _report(f"direct sine transform nz={nz}", max_relL2=f"{err.max():.3e}")
    assert err.max() <= 2e-6


@pytest.mark.parametrize("nz", DIRECT)
def test_coefficient_roundtrip_and_carrier(ssp, gpu, nz):
    torch = gpu
    s = W.munk_deep(nz=nz)
    pl = make_plan(ssp, s)
    try:
        x = np.stack([s.starter(), W.random_field(s.nz, 9)])
        d_x = torch.from_numpy(x.astype(np.complex64)).cuda()
        d_s = torch.empty_like(d_x)
        d_y = torch.empty_like(d_x)
        steps = torch.tensor([0, 5], dtype=torch.int64, device="cuda")
        ssp.ssp_to_sine(pl, 2, d_x.data_ptr(), d_s.data_ptr())
        ssp.ssp_from_sine(pl, 2, d_s.data_ptr(), steps.data_ptr(), d_y.data_ptr())
        torch.cuda.synchronize()
        y = d_y.cpu().numpy().astype(np.complex128)
    finally:
        ssp.ssp_plan_destroy(pl)
    car = np.exp(1j * s.k0 * s.dr * np.array([0, 5]))[:, None]
    err = np.linalg.norm(y - car * x, axis=1) / np.linalg.norm(x, axis=1)
    assert err.max() < 2e-6


@pytest.mark.parametrize("nz,nsteps", [(63, 200), (1023, 100), (4095, 24), (8191, 12)])
def test_munk_vs_oracle(ssp, gpu, nz, nsteps):
    s = W.munk_deep(nsteps=nsteps, nz=nz)
    s.out_every = max(1, nsteps // 4)
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status and stats["steps_done"] == ref.steps_done
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dtl = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report(f"direct sine munk nz={nz}", max_relL2=f"{err.max():.3e}", max_dTL=f"{dtl.max():.3e}")
    assert err.max() <= REL_L2 and dtl.max() <= DTL
    assert abs(stats["neumann_terms"] - int(ref.iterations.sum())) <= 0.01 * ref.iterations.sum() + 2


def test_plain_form_rejected(ssp, gpu):
    s = W.munk_deep(nsteps=2, nz=1023)
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_PLAIN, 1)
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)


def test_mixed_batch_equals_alone_bitwise(ssp, gpu):
    # direct and chirp-z plans of neighbouring lengths in one batch call
    sizes = [4095, 4096, 1023, 1000, 8191]
    solves = []
    for nz in sizes:
        s = W.munk_deep(nsteps=8, nz=nz)
        s.out_every = 4
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
        st, fl, tl, stats = ssp.ssp_march_batch(plans, [s.nz for s in solves], 8)
    finally:
        for pl in plans:
            ssp.ssp_plan_destroy(pl)
    for a, b in zip(alone, fl):
        assert np.array_equal(a, b)


def test_bench_launch_configuration_sampled(ssp, gpu):
    # 512 solves at Nz = 4095 as `bench.py --nz 4095` times them: one plan on a dedicated
    # stream, graph-recorded launches, TL rows on the device; sampled solves vs the oracle
    torch = gpu
    s = W.munk_deep(nz=4095)
    B, nsteps = 512, 24
    stream = torch.cuda.Stream()
    pl = make_plan(ssp, s)
    zs = W.source_depths(B, 50.0, 2000.0)
    try:
        assert ssp.ssp_plan_engine(pl)[2] == 8192
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
        assert steps.cpu().tolist() == [nsteps] * B
    finally:
        ssp.ssp_plan_destroy(pl)
    for b in (0, 257, 511):
        s1 = dataclasses.replace(s, zs=float(zs[b]), nsteps=nsteps)
        ref = oracle_march(s1)
        mask = ref.tl < 120.0
        dtl = np.abs(tl[b, :ref.tl.shape[0]].astype(np.float64) - ref.tl)[mask]
        err = np.linalg.norm(fld[b] - ref.final) / np.linalg.norm(ref.final)
        _report(f"direct sine bench config b={b}", relL2=f"{err:.3e}", max_dTL=f"{dtl.max():.3e}")
        assert err <= REL_L2 and dtl.max() <= DTL


def test_munk_long_range(ssp, gpu):
    # 600 steps (15 km) at Nz = 4095: error growth over range stays within the bar
    s = W.munk_deep(nsteps=600, nz=4095)
    s.out_every = 150
    pl = make_plan(ssp, s)
    try:
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dtl = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report("direct sine munk long", relL2=" ".join(f"{e:.2e}" for e in err), max_dTL=f"{dtl.max():.3e}")
    assert err.max() <= REL_L2 and dtl.max() <= DTL


@pytest.mark.parametrize("nz", [1023, 2047, 4095, 8191])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_layouts_vs_oracle(ssp, gpu, nz, variant):
    # every engine layout of the direct sine march (a layout the length does not have falls
    # back to layout 0)
    s = W.munk_deep(nsteps=12, nz=nz)
    s.out_every = 4
    pl = make_plan(ssp, s)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_VARIANT, variant)
        st, fld, tl, stats = ssp.ssp_march(pl, s.nz, s.starter(), s.nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    ref = oracle_march(s)
    assert st == ref.status
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    assert err.max() <= REL_L2
