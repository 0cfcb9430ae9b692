"""Pins of the oracle's normal-mode starter (Sec. 3.2).

Independent references: the closed-form modes of a homogeneous Dirichlet waveguide, a
second-order finite-difference solution of the Sturm-Liouville problem of the Munk
waveguide (Richardson-extrapolated, no spectral basis), the reciprocity of the point-source
field, and the exact one-way propagator of the same operator.
"""
import math

import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

import workloads as W
from oracle.modal import depth_modes, modal_field, modal_starter
from oracle.reference import dense_operator_from_c, dense_step


def test_homogeneous_starter_closed_form():
    nz, H, f, c0, zs = 255, 200.0, 100.0, 1500.0, 63.0
    k0 = 2 * math.pi * f / c0
    z = W.depth_grid(nz, H)
    got = modal_starter(nz, H, f, c0, np.full(nz, c0), zs)
    m = np.arange(1, nz + 1)
    mu = (m * math.pi / H) ** 2
    prop = mu < k0 ** 2
    kap = np.sqrt(k0 ** 2 - mu[prop])
    ref = math.sqrt(2 * math.pi) * ((2 / H) * np.sin(np.outer(z, m[prop]) * math.pi / H)
                                    @ (np.sin(m[prop] * math.pi * zs / H) / np.sqrt(kap)))
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))
    assert np.max(np.abs(got.imag)) == 0.0


def _fd_kappa2(H, f, c_of_z, n, count):
    # d_z^2 by second-order differences on n interior points, Dirichlet ends; the largest
    # eigenvalues of d_z^2 + k^2 are kappa^2 of the lowest modes
    h = H / (n + 1)
    z = h * np.arange(1, n + 1)
    k2 = (2 * math.pi * f / c_of_z(z)) ** 2
    d = -2.0 / h ** 2 + k2
    e = np.full(n - 1, 1.0 / h ** 2)
    w = eigh_tridiagonal(d, e, eigvals_only=True, select="i", select_range=(n - count, n - 1))
    return np.sort(w)[::-1]


def test_munk_mode_wavenumbers_match_finite_differences():
    # Munk waveguide of the paper's first experiment (H = 4 km) at 25 Hz: the lowest modes'
    # kappa^2 from the spectral eigenproblem against Richardson-extrapolated second-order
    # finite differences (an independent discretisation)
    H, f, c0, nz = 4000.0, 25.0, 1500.0, 1023
    kap, Y, A = depth_modes(nz, H, f, c0, W.munk(W.depth_grid(nz, H)))
    count = 6
    a = _fd_kappa2(H, f, W.munk, 20000, count)
    b = _fd_kappa2(H, f, W.munk, 40001, count)
    ext = (4 * b - a) / 3
    rel = np.abs(kap[:count] ** 2 - ext) / ext
    assert rel.max() < 1e-10, rel


def test_mode_values_between_grid_points_match_the_grid():
    # the basis expansion used for Psi_m(zs) reproduces the eigenvector at grid points
    nz, H, f, c0 = 300, 3000.0, 30.0, 1500.0
    z = W.depth_grid(nz, H)
    c = W.munk(z)
    for k in (17, 150, 299):
        u_grid = modal_starter(nz, H, f, c0, c, z[k])
        kap, Y, A = depth_modes(nz, H, f, c0, c)
        dz = H / (nz + 1)
        w = math.sqrt(2 * math.pi) * (Y[k] / math.sqrt(dz)) / (math.sqrt(dz) * np.sqrt(kap))
        assert np.max(np.abs(u_grid - Y @ w)) < 1e-10 * np.max(np.abs(u_grid))


def test_point_source_reciprocity():
    # source at z_j observed at z_k equals source at z_k observed at z_j
    nz, H, f, c0 = 200, 2000.0, 40.0, 1500.0
    z = W.depth_grid(nz, H)
    c = W.munk(z * 2.0)
    j, k = 31, 140
    a = modal_starter(nz, H, f, c0, c, z[j])[k]
    b = modal_starter(nz, H, f, c0, c, z[k])[j]
    assert abs(a - b) < 1e-12 * max(abs(a), 1e-30)


def test_modal_field_is_the_exact_one_way_propagation_of_the_starter():
    # u(r) = exp(i r k0 sqrt(1 + X)) u(0) for the same operator X (the starter holds only
    # propagating modes, so the evanescent part of the exact propagator plays no role)
    nz, H, f, c0, zs, r = 127, 1000.0, 20.0, 1500.0, 400.0, 750.0
    z = W.depth_grid(nz, H)
    c = W.munk(z * 4.0)
    k0 = 2 * math.pi * f / c0
    u = modal_field(nz, H, f, c0, c, zs, [0.0, r])
    X = dense_operator_from_c(nz, H, f, c0, c)
    ref = dense_step(X, u[0], lambda lam: np.exp(1j * k0 * r * np.sqrt(1 + lam + 0j)))
    assert np.linalg.norm(u[1] - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.parametrize("cap", [1, 5])
def test_max_modes_keeps_the_lowest_modes(cap):
    nz, H, f, c0 = 200, 2000.0, 40.0, 1500.0
    z = W.depth_grid(nz, H)
    c = W.munk(z * 2.0)
    kap_all, _, _ = depth_modes(nz, H, f, c0, c)
    kap, Y, _ = depth_modes(nz, H, f, c0, c, max_modes=cap)
    assert len(kap) == cap and np.array_equal(kap, kap_all[:cap])
    assert np.all(np.diff(kap_all) < 0)
