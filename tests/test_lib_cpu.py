"""Host-side checks of the C-ABI library that need no GPU: exported symbols, the host
Pade construction against the oracle, and argument validation."""
import ctypes
import math

import numpy as np
import pytest

from oracle.pade import pade


def test_library_exports_every_header_function(ssp):
    names = ssp.header_functions()
    assert len(names) >= 18
    L = ctypes.CDLL(ssp.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("sigma,p,alpha", [
    (2.094395102393196, 4, 0.0), (2.094395102393196, 4, math.pi / 16),
    (5.235987755982989, 6, 0.0), (16.755160819145562, 8, 0.0), (31.4, 6, 0.0), (0.5, 1, 0.0),
    (41.8879, 4, 0.0)])
def test_host_pade_matches_oracle(ssp, sigma, p, alpha):
    got = ssp.ssp_pade_coefficients(sigma, p, alpha)
    ref = pade(sigma, p, alpha)
    scale = np.max(np.abs(ref.b))
    assert np.max(np.abs(got["b"] - ref.b)) < 1e-12 * scale
    assert np.max(np.abs(got["g"] - ref.a / ref.b)) < 1e-11
    assert abs(got["C"] - ref.C) < 1e-12
    dscale = np.max(np.abs(ref.d)) + 1
    assert np.max(np.abs(got["d"] - ref.d)) < 1e-11 * dscale
    assert abs(got["d0"] - ref.d0) < 1e-11 * dscale


def test_host_pade_rejects_bad_order(ssp):
    for p in (0, 13):
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_pade_coefficients(1.0, p)
        assert e.value.status == ssp.SSP_E_INVAL


@pytest.mark.parametrize("args,status", [
    ((1, 100.0, 50.0, 1500.0, 5.0, 4, 8, 1e-10), -1),
    ((64, -1.0, 50.0, 1500.0, 5.0, 4, 8, 1e-10), -1),
    ((64, 100.0, 0.0, 1500.0, 5.0, 4, 8, 1e-10), -1),
    ((64, 100.0, 50.0, float("nan"), 5.0, 4, 8, 1e-10), -1),
    ((64, 100.0, 50.0, 1500.0, 0.0, 4, 8, 1e-10), -1),
    ((64, 100.0, 50.0, 1500.0, 5.0, 0, 8, 1e-10), -1),
    ((64, 100.0, 50.0, 1500.0, 5.0, 13, 8, 1e-10), -1),
    ((64, 100.0, 50.0, 1500.0, 5.0, 4, -1, 1e-10), -1),
    ((64, 100.0, 50.0, 1500.0, 5.0, 4, 8, 0.0), -1),
    ((10 ** 6, 100.0, 50.0, 1500.0, 5.0, 4, 8, 1e-10), -7),
    ((16385, 5000.0, 50.0, 1500.0, 25.0, 6, 48, 1e-10), -7),   # one above the largest grid
])
def test_plan_create_validates_before_touching_the_device(ssp, args, status):
    with pytest.raises(ssp.SspError) as e:
        ssp.ssp_plan_create(*args)
    assert e.value.status == status


def test_status_strings(ssp):
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert ssp.ssp_status_string(s)
    assert ssp.ssp_max_nz() >= 8192
