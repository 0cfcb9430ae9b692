"""Pins of the oracle's complex absorbing potential (Sec. 3.1: an imaginary part added to the
wavenumber in a layer, v -> v + i eta).

Independent references: the closed form of a single mode under a uniform eta (the series
then sums exactly to (1 + b_j (x_m + i eta))^{-1}), dense solves of the vertical operator
with a complex diagonal, the decay of the field norm, and a truncated waveguide whose
absorbing layer must reproduce the field of a three times deeper waveguide that has no
layer.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OK, Plan
from oracle.bases import weights
from oracle.pade import pade
from oracle.reference import dense_operator_from_c, dense_rational, dense_term


def test_uniform_absorber_single_mode_closed_form():
    # c = c0 and eta constant: X = D + i eta, so the sine mode m gains e^{i sigma}
    # R(x_m + i eta) per step with x_m = -(m pi/(H k0))^2
    nz, H, f, c0, dr, eta = 63, 200.0, 100.0, 1500.0, 5.0, 0.01
    pl = Plan(nz, H, f, c0, dr, 4, 200, 1e-15)
    z = W.depth_grid(nz, H)
    m = 6
    u0 = np.sin(m * math.pi * z / H).astype(complex)
    xm = -(m * math.pi / (H * pl.k0)) ** 2
    R = pade(pl.sigma, 4).R(xm + 1j * eta)
    res = pl.march(u0, 3, np.full((1, nz), c0), out_every=1, absorber=np.full(nz, eta))
    assert res.status == OK
    for n in range(3):
        ref = (np.exp(1j * pl.sigma) * R) ** (n + 1) * u0
        assert np.max(np.abs(res.field[n] - ref)) < 1e-12
    assert abs(np.exp(1j * pl.sigma) * R) < 1.0   # the mode is damped


def test_absorber_series_and_step_vs_dense_operator():
    nz, H, f, c0 = 24, 300.0, 30.0, 1500.0
    z = W.depth_grid(nz, H)
    c = 1500.0 + 15.0 * np.exp(-((z - 120.0) / 50.0) ** 2)
    eta = W.absorbing_layer(nz, H, 100.0, 0.05)
    pl = Plan(nz, H, f, c0, 10.0, 4, 200, 1e-15)
    X = dense_operator_from_c(nz, H, f, c0, c) + 1j * np.diag(eta)
    u = W.random_field(nz, 2)
    v = pl.potential(c) + 1j * eta
    for bj in pl.b:
        w, iters, res, st = pl.term_solve(u, bj, v)
        assert st == OK
        ref = dense_term(X, u, bj)
        assert np.linalg.norm(w - ref) / np.linalg.norm(ref) < 1e-12
    got, _, _, st = pl.step(u, v)
    ref = np.exp(1j * pl.sigma) * dense_rational(X, u, pl.pade.C, pl.pade.a, pl.pade.b)
    assert st == OK and np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11


def _beam(H, nz, layer, nsteps=400, f=100.0, c0=1500.0, dr=5.0, tilt=15.0, bc="dirichlet"):
    # a Gaussian beam (30 m wide at 200 m) aimed at the bottom, homogeneous water
    k0 = 2 * math.pi * f / c0
    z = W.depth_grid(nz, H, bc)
    psi = np.exp(-((z - 200.0) / 30.0) ** 2) * np.exp(1j * k0 * math.sin(math.radians(tilt)) * z)
    eta = None if layer is None else W.absorbing_layer(nz, H, layer[0], layer[1], bc)
    pl = Plan(nz, H, f, c0, dr, 4, 80, 1e-10, bc=bc)
    return z, pl.march(psi, nsteps, np.full((1, nz), c0), out_every=nsteps // 4, absorber=eta)


def test_absorbing_layer_emulates_a_deeper_waveguide():
    # 600 m waveguide with a 300 m layer vs an 1800 m waveguide without one (same grid
    # points, dz = 600/256 m): above 350 m the two agree while the deep waveguide's bottom
    # echo is still far away; without the layer the 600 m bottom echo dominates
    z, deep = _beam(1800.0, 767, None)
    zt, cap = _beam(600.0, 255, (300.0, 0.05))
    _, hard = _beam(600.0, 255, None)
    keep = zt < 350.0
    assert np.array_equal(zt, z[:255])
    assert cap.status == OK
    for i in range(4):
        ref = deep.field[i][:255][keep]
        e_cap = np.linalg.norm(cap.field[i][keep] - ref) / np.linalg.norm(ref)
        assert e_cap < 0.05, (i, e_cap)
    e_hard = np.linalg.norm(hard.field[-1][keep] - deep.field[-1][:255][keep]) / np.linalg.norm(deep.field[-1][:255][keep])
    assert e_hard > 1.0


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_absorber_norm_is_non_increasing(bc):
    # eta >= 0 only removes energy: the norm (the coefficient-space one, with the endpoint
    # weights of the cosine basis) never grows and falls once the beam enters the layer;
    # without the layer the standard approximant keeps it (lossless medium)
    nz, H = 255, 600.0
    e = weights(bc, nz)
    _, cap = _beam(H, nz, (300.0, 0.05), nsteps=400, bc=bc)
    _, hard = _beam(H, nz, None, nsteps=400, bc=bc)
    norms = [np.linalg.norm(e * cap.field[i]) for i in range(4)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(norms, norms[1:]))
    assert norms[-1] < 0.5 * norms[0]
    h = [np.linalg.norm(e * hard.field[i]) for i in range(4)]
    assert max(h) - min(h) < 1e-9 * h[0]
