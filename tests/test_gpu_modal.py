"""GPU parity of the normal-mode starter (Sec. 3.2) against the oracle, and the paper's first
experiment set-up (range-independent Munk waveguide, H = 4 km, zs = 1100 m, 100 Hz, [4/4],
dr = 100 m) started from it.

The starter is FP64 on both sides (dense eigenproblem of the same operator): bar 1e-8
relative L2 for the starter and 1e-12 for the mode wavenumbers.  Marches from it: the march
bar (relL2 <= 1e-4, dTL <= 0.1 dB where TL < 120 dB).
"""
import math

import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

import workloads as W
from oracle import Plan as OraclePlan
from oracle.modal import depth_modes, modal_starter

pytestmark = pytest.mark.gpu


def _report(tag, **kv):
    print(f"[{tag}] " + " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def _gpu_starter(ssp, nz, H, f, c0, c, zs, max_modes=0, bc="dirichlet"):
    pl = ssp.ssp_plan_create_bc(nz, H, f, c0, 25.0, 4, 8, 1e-10, bc)
    try:
        return ssp.ssp_modal_starter(pl, c, zs, max_modes)
    finally:
        ssp.ssp_plan_destroy(pl)


@pytest.mark.parametrize("nz,H,f,zs", [(255, 5000.0, 12.0, 1000.0), (1000, 5000.0, 50.0, 1000.0),
                                       (2001, 4000.0, 100.0, 1100.0), (2048, 4000.0, 100.0, 3999.0)])
def test_modal_starter_vs_oracle(ssp, gpu, nz, H, f, zs):
    c0 = 1500.0
    c = W.munk(W.depth_grid(nz, H))
    got, kap = _gpu_starter(ssp, nz, H, f, c0, c, zs)
    ref = modal_starter(nz, H, f, c0, c, zs)
    rk, _, _ = depth_modes(nz, H, f, c0, c)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    kerr = np.max(np.abs(kap - rk) / rk)
    _report(f"modal nz={nz}", modes=len(kap), relL2=f"{err:.3e}", kappa_rel=f"{kerr:.3e}")
    assert len(kap) == len(rk)
    assert err < 1e-8 and kerr < 1e-12
    assert np.all(got.imag == 0.0)


def test_modal_starter_mode_cap(ssp, gpu):
    nz, H, f, c0, zs = 500, 4000.0, 30.0, 1500.0, 1100.0
    c = W.munk(W.depth_grid(nz, H))
    got, kap = _gpu_starter(ssp, nz, H, f, c0, c, zs, max_modes=7)
    ref = modal_starter(nz, H, f, c0, c, zs, max_modes=7)
    assert len(kap) == 7
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-8


def test_modal_starter_rejects_bad_input(ssp, gpu):
    nz, H = 64, 1000.0
    c = np.full(nz, 1500.0)
    pl = ssp.ssp_plan_create_bc(nz, H, 50.0, 1500.0, 10.0, 4, 8, 1e-10, "neumann")
    try:
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_modal_starter(pl, c, 100.0)
        assert e.value.status == ssp.SSP_E_UNIMPL
    finally:
        ssp.ssp_plan_destroy(pl)
    pl = ssp.ssp_plan_create(nz, H, 50.0, 1500.0, 10.0, 4, 8, 1e-10)
    try:
        for zs in (0.0, H, -5.0):
            with pytest.raises(ssp.SspError) as e:
                ssp.ssp_modal_starter(pl, c, zs)
            assert e.value.status == ssp.SSP_E_INVAL
        bad = c.copy()
        bad[3] = -1.0
        with pytest.raises(ssp.SspError):
            ssp.ssp_modal_starter(pl, bad, 100.0)
    finally:
        ssp.ssp_plan_destroy(pl)


def _fd_kappa2(H, f, n, count):
    h = H / (n + 1)
    z = h * np.arange(1, n + 1)
    k2 = (2 * math.pi * f / W.munk(z)) ** 2
    w = eigh_tridiagonal(-2.0 / h ** 2 + k2, np.full(n - 1, 1.0 / h ** 2), eigvals_only=True,
                         select="i", select_range=(n - count, n - 1))
    return np.sort(w)[::-1]


def test_first_experiment_full_grid_mode_wavenumbers(ssp, gpu):
    # the paper's grid, 8001 points (dz = 0.5 m): the lowest modes' kappa^2 against
    # Richardson-extrapolated finite differences of the Sturm-Liouville problem
    H, f, c0, nz, zs = 4000.0, 100.0, 1500.0, 8001, 1100.0
    c = W.munk(W.depth_grid(nz, H))
    got, kap = _gpu_starter(ssp, nz, H, f, c0, c, zs)
    count = 6
    a, b = _fd_kappa2(H, f, 40000, count), _fd_kappa2(H, f, 80001, count)
    ext = (4 * b - a) / 3
    rel = np.abs(kap[:count] ** 2 - ext) / ext
    _report("E1 modes", modes=len(kap), kappa2_rel=f"{rel.max():.3e}", norm=f"{np.linalg.norm(got):.4e}")
    assert rel.max() < 1e-9
    assert np.all(np.isfinite(got)) and np.linalg.norm(got) > 0


def test_first_experiment_march_from_the_modal_starter(ssp, gpu):
    # the first experiment's set-up at a coarser grid (Nz = 2001): the GPU starter and march
    # against the oracle's starter and march; the paper's M = 2 (two Neumann terms per
    # factor, so series stop at the cap and report not converged)
    H, f, c0, nz, zs, dr, nsteps = 4000.0, 100.0, 1500.0, 2001, 1100.0, 100.0, 20
    c = W.munk(W.depth_grid(nz, H))
    pl = ssp.ssp_plan_create(nz, H, f, c0, dr, 4, 2, 1e-10)
    try:
        ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, 5)
        ssp.ssp_set_profile(pl, 0, -1, c)
        psi0, kap = ssp.ssp_modal_starter(pl, c, zs)
        st, fld, tl, stats = ssp.ssp_march(pl, nz, psi0, nsteps)
    finally:
        ssp.ssp_plan_destroy(pl)
    opl = OraclePlan(nz, H, f, c0, dr, 4, 2, 1e-10)
    ref = opl.march(modal_starter(nz, H, f, c0, c, zs), nsteps, c[None, :], out_every=5)
    assert st == ref.status
    err = np.linalg.norm(fld - ref.field, axis=1) / np.linalg.norm(ref.field, axis=1)
    mask = ref.tl < 120.0
    dtl = np.abs(tl.astype(np.float64) - ref.tl)[mask]
    _report("E1 march", status=st, relL2=f"{err.max():.3e}", max_dTL=f"{dtl.max():.3e}",
            not_converged=stats["not_converged"])
    assert err.max() <= 1e-4 and dtl.max() <= 0.1


def test_modal_starters_for_several_sources(ssp, gpu):
    # one eigendecomposition, several source depths (one of them on a grid point)
    nz, H, f, c0 = 800, 4000.0, 60.0, 1500.0
    z = W.depth_grid(nz, H)
    c = W.munk(z)
    zs = np.array([250.0, 1100.0, z[401], 3700.0])
    pl = ssp.ssp_plan_create(nz, H, f, c0, 25.0, 4, 8, 1e-10)
    try:
        got, kap = ssp.ssp_modal_starter(pl, c, zs)
    finally:
        ssp.ssp_plan_destroy(pl)
    assert got.shape == (len(zs), nz)
    for q, zq in enumerate(zs):
        ref = modal_starter(nz, H, f, c0, c, zq)
        err = np.linalg.norm(got[q] - ref) / np.linalg.norm(ref)
        _report(f"modal source {zq:.1f}", relL2=f"{err:.3e}")
        assert err < 1e-8
