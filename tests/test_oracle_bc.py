"""Pins of the oracle under the Neumann and periodic boundary conditions of Sec. 3.1.

Independent references: the transform definitions written out, the sampled
eigenfunctions of d_z^2 (cos(l pi z/H), e^{2 pi i l z/H}) with their closed-form second
derivatives, the exact modal sum of a homogeneous waveguide (eigenfunction system solved
directly, no transform), dense operators on tiny grids, and the symmetries each boundary
condition implies (a constant mode under Neumann boundaries, translation under periodic
ones, reflection about mid-depth).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OK, Plan
from oracle.bases import (dct1, forward, forward_matrix, grid, inverse, orthonormal_matrix,
                          wavenumbers, weights)
from oracle.pade import pade
from oracle.reference import dense_operator_bc, dense_rational, dense_term, modal_field_bc

BCS = ["neumann", "periodic"]


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nz", [2, 3, 8, 37, 256])
def test_transform_matches_definition_and_inverts(bc, nz):
    x = W.random_field(nz, 5)
    T = forward_matrix(bc, nz)
    assert np.max(np.abs(forward(bc, x) - T @ x)) < 1e-12 * math.sqrt(nz)
    assert np.max(np.abs(inverse(bc, forward(bc, x)) - x)) < 1e-13 * math.sqrt(nz)
    # the written-out orthonormal matrix is unitary, and Parseval holds for the weighted
    # grid values
    Q = orthonormal_matrix(bc, nz)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(nz))) < 1e-12
    assert abs(np.linalg.norm(forward(bc, x)) - np.linalg.norm(weights(bc, nz) * x)) < 1e-12 * np.linalg.norm(x)


def test_dct1_is_symmetric_involution():
    nz = 33
    C = orthonormal_matrix("neumann", nz)
    assert np.max(np.abs(C - C.T)) == 0.0
    x = W.random_field(nz, 8)
    assert np.max(np.abs(dct1(dct1(x)) - x)) < 1e-13


def test_cosine_mode_is_a_basis_vector():
    # the forward Neumann transform maps the sampled mode cos(l pi z/H) on the Neumann grid
    # to sqrt((Nz-1)/2)/e_l times the l-th unit vector
    nz, H = 65, 1000.0
    z = W.depth_grid(nz, H, "neumann")
    assert z[0] == 0.0 and abs(z[-1] - H) < 1e-9
    for ell in (0, 1, 9, 64):
        y = forward("neumann", np.cos(ell * math.pi * z / H))
        e = np.zeros(nz)
        amp = math.sqrt((nz - 1) / 2) * (math.sqrt(2.0) if ell in (0, nz - 1) else 1.0)
        e[ell] = amp
        assert np.max(np.abs(y - e)) < 1e-11


def test_fourier_mode_is_a_basis_vector():
    nz, H = 64, 300.0
    z = W.depth_grid(nz, H, "periodic")
    for ell in (0, 1, 5, 32, -7):
        y = forward("periodic", np.exp(2j * math.pi * ell * z / H))
        e = np.zeros(nz, dtype=complex)
        e[ell % nz] = math.sqrt(nz)
        assert np.max(np.abs(y - e)) < 1e-11


@pytest.mark.parametrize("bc", BCS)
def test_spectral_second_derivative_of_band_limited_functions(bc):
    # d_z^2 = T^{-1} diag(-kappa^2) T equals the analytic second derivative of functions
    # built from the boundary condition's eigenfunctions
    nz, H = 96, 750.0
    z = W.depth_grid(nz, H, bc)
    if bc == "neumann":
        a, b = 3 * math.pi / H, 11 * math.pi / H
        f = np.cos(a * z) + 0.5 * np.cos(b * z)
        f2 = -a * a * np.cos(a * z) - 0.5 * b * b * np.cos(b * z)
    else:
        a, b = 2 * math.pi * 3 / H, 2 * math.pi * 17 / H
        f = np.exp(1j * a * z) + 0.5 * np.sin(b * z)
        f2 = -a * a * np.exp(1j * a * z) - 0.5 * b * b * np.sin(b * z)
    kap = wavenumbers(bc, nz, H)
    d2 = inverse(bc, -kap ** 2 * forward(bc, f))
    assert np.max(np.abs(d2 - f2)) < 1e-10 * np.max(np.abs(f2))


def test_oracle_grid_is_the_workload_grid():
    for bc in ("dirichlet",) + tuple(BCS):
        assert np.array_equal(grid(bc, 40, 123.0), W.depth_grid(40, 123.0, bc))


# ---------------------------------------------------------------- range march
def _homog(bc, nz=128, rotation=0.0):
    s = W.Solve(nz=nz, depth=200.0, freq=100.0, c0=1500.0, dr=5.0, pade_order=4,
                neumann_max=0, tol=1e-10, nsteps=60, zs=60.0, env="iso", rotation=rotation,
                out_every=30, bc=bc)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol,
              rotation=rotation, bc=bc)
    return s, pl


@pytest.mark.parametrize("bc", BCS)
def test_homogeneous_march_vs_modal_sum(bc):
    # exact modal sum of the waveguide; agreement is limited by the Pade approximant, so
    # compare the modes that propagate within 45 degrees
    s, pl = _homog(bc, rotation=math.pi / 16)
    psi0 = s.starter()
    res = pl.march(psi0, s.nsteps, s.profile(), out_every=s.out_every)
    assert res.status == OK and res.steps_done == s.nsteps
    ex = modal_field_bc(bc, psi0, W.depth_grid(s.nz, s.depth, bc), s.depth, pl.k0,
                        res.ranges[[0, -1]])
    T = forward_matrix(bc, s.nz)
    keep = wavenumbers(bc, s.nz, s.depth) <= pl.k0 * math.sin(math.radians(45))
    keep &= wavenumbers(bc, s.nz, s.depth) >= -pl.k0 * math.sin(math.radians(45))
    for got, ref in ((res.field[0], ex[0]), (res.field[-1], ex[1])):
        a, b = T @ got, T @ ref
        err = np.linalg.norm((a - b)[keep]) / np.linalg.norm(b[keep])
        assert err < 3e-4, err


@pytest.mark.parametrize("bc", BCS)
def test_single_mode_gains_the_pade_factor(bc):
    # with v = 0 a sampled eigenfunction stays one, multiplied per step by
    # e^{i sigma} R(x_m), x_m = -(kappa_m/k0)^2 from the mode's own wavenumber
    s, pl = _homog(bc, nz=64)
    z = W.depth_grid(s.nz, s.depth, bc)
    if bc == "neumann":
        kap = 5 * math.pi / s.depth
        u0 = np.cos(kap * z).astype(complex)
    else:
        kap = 2 * math.pi * 4 / s.depth
        u0 = np.exp(1j * kap * z)
    R = pade(pl.sigma, s.pade_order).R(-(kap / pl.k0) ** 2)
    res = pl.march(u0, 3, s.profile(), out_every=1)
    for n in range(3):
        assert np.max(np.abs(res.field[n] - (np.exp(1j * pl.sigma) * R) ** (n + 1) * u0)) < 1e-12


def test_neumann_constant_mode_is_carried_unchanged():
    # the l = 0 cosine mode has x = 0 and R(0) = 1: a constant field only gains the carrier
    s, pl = _homog("neumann", nz=50)
    u0 = np.full(s.nz, 0.7 - 0.2j)
    res = pl.march(u0, 5, s.profile(), out_every=5)
    assert np.max(np.abs(res.field[0] - np.exp(5j * pl.sigma) * u0)) < 1e-12


def test_periodic_march_commutes_with_translation():
    # periodic boundaries: shifting the starter and the environment by k grid points
    # shifts the solution by k points
    nz, H = 64, 400.0
    z = W.depth_grid(nz, H, "periodic")
    c = 1500.0 + 12.0 * np.cos(2 * math.pi * z / H) + 5.0 * np.sin(6 * math.pi * z / H)
    pl = Plan(nz, H, 60.0, 1500.0, 10.0, 4, 40, 1e-12, bc="periodic")
    u0 = W.random_field(nz, 21) * np.exp(-((z - 150.0) / 40.0) ** 2)
    a = pl.march(u0, 4, c[None, :], out_every=4)
    b = pl.march(np.roll(u0, 7), 4, np.roll(c, 7)[None, :], out_every=4)
    assert a.status == OK and b.status == OK
    assert np.max(np.abs(np.roll(a.field[0], 7) - b.field[0])) < 1e-11


def test_neumann_march_preserves_mirror_symmetry():
    # Neumann grid and basis are symmetric about mid-depth: a mirrored starter in a
    # mirrored environment gives the mirrored field (catches grid or endpoint-weight slips)
    nz, H = 81, 600.0
    z = W.depth_grid(nz, H, "neumann")
    c = 1500.0 + 20.0 * np.exp(-((z - 200.0) / 90.0) ** 2)
    pl = Plan(nz, H, 40.0, 1500.0, 10.0, 4, 40, 1e-12, bc="neumann")
    u0 = W.random_field(nz, 4) * np.exp(-((z - 250.0) / 60.0) ** 2)
    a = pl.march(u0, 3, c[None, :], out_every=3)
    b = pl.march(u0[::-1], 3, c[::-1][None, :], out_every=3)
    assert np.max(np.abs(a.field[0][::-1] - b.field[0])) < 1e-11


@pytest.mark.parametrize("bc", BCS)
def test_neumann_series_solves_the_dense_factor(bc):
    # per Pade factor: the series with a tight tolerance equals the dense LU solve of
    # (1 + b_j X) w = u, X built from the sampled eigenfunctions (no transform)
    nz, H, f, c0 = 24, 300.0, 30.0, 1500.0
    z = W.depth_grid(nz, H, bc)
    c = 1500.0 + 15.0 * np.exp(-((z - 120.0) / 50.0) ** 2)
    pl = Plan(nz, H, f, c0, 10.0, 4, 200, 1e-15, bc=bc)
    X = dense_operator_bc(bc, z, H, f, c0, c)
    u = W.random_field(nz, 2)
    v = pl.potential(c)
    for bj in pl.b:
        w, iters, res, st = pl.term_solve(u, bj, v)
        assert st == OK
        ref = dense_term(X, u, bj)
        assert np.linalg.norm(w - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("bc", BCS)
def test_step_equals_rational_function_of_dense_operator(bc):
    nz, H, f, c0 = 20, 250.0, 35.0, 1500.0
    z = W.depth_grid(nz, H, bc)
    c = 1500.0 - 10.0 * np.exp(-((z - 100.0) / 40.0) ** 2)
    pl = Plan(nz, H, f, c0, 8.0, 4, 200, 1e-15, bc=bc)
    X = dense_operator_bc(bc, z, H, f, c0, c)
    u = W.random_field(nz, 3)
    got, _, _, st = pl.step(u, pl.potential(c))
    ref = np.exp(1j * pl.sigma) * dense_rational(X, u, pl.pade.C, pl.pade.a, pl.pade.b)
    assert st == OK
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11
