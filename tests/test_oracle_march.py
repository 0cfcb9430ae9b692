"""Pins of the oracle's transform and range march.

References used here are independent of the march: the DST-I definition, the exact
normal-mode sum of a homogeneous Dirichlet waveguide, a dense eigendecomposition of the
vertical operator on tiny grids, norm conservation of a unitary step, and the paper's
M = 0 special case.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import DIVERGED, NOT_CONVERGED, OK, Plan, dst, dst_direct, dst_matrix
from oracle.reference import (dense_operator_from_c, dense_step, dense_term,
                              normal_mode_field, propagation_angle)
from oracle.sssp import transmission_loss

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- transform (Sec. 3.1)
@pytest.mark.parametrize("nz", [2, 3, 16, 37, 256, 511])
def test_dst_matches_definition_and_is_involution(nz):
    x = W.random_field(nz, 11)
    assert np.max(np.abs(dst(x) - dst_direct(x))) < 1e-12 * math.sqrt(nz)
    assert np.max(np.abs(dst(dst(x)) - x)) < 1e-13 * math.sqrt(nz)


def test_dst_diagonalises_second_derivative():
    # S maps the sampled mode sin(l pi z/H) to sqrt((Nz+1)/2) e_l
    nz, H = 63, 1000.0
    z = W.depth_grid(nz, H)
    for ell in (1, 7, 63):
        y = dst(np.sin(ell * math.pi * z / H))
        e = np.zeros(nz)
        e[ell - 1] = math.sqrt((nz + 1) / 2)
        assert np.max(np.abs(y - e)) < 1e-12


# ---------------------------------------------------------------- paper constants
def test_munk_profile_against_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_settings.json")))["munk"]
    z = np.array([0.0, 1300.0, 4000.0])
    eta = 2 * (z - g["z_axis_m"]) / g["eta_scale_m"]
    c = g["c_axis_m_s"] * (1 + g["epsilon"] * (eta + np.exp(-eta) - 1))
    assert np.allclose(W.munk(z), c, rtol=0, atol=1e-9)
    assert W.munk(np.array([1300.0]))[0] == 1500.0          # sound-channel axis
    zz = np.linspace(0, 5000, 5001)
    assert zz[np.argmin(W.munk(zz))] == 1300.0


def test_transmission_loss_definition():
    r = np.array([1.0, 100.0])
    u = np.array([[1.0 + 0j], [10.0 + 0j]])
    tl = transmission_loss(u, r)
    assert abs(tl[0, 0]) < 1e-15 and abs(tl[1, 0]) < 1e-12


# ---------------------------------------------------------------- homogeneous waveguide
def _homog_plan(rotation, nsteps=1000):
    s = W.homogeneous_waveguide(nsteps=nsteps)
    return s, Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol,
                   rotation=rotation)


@pytest.mark.parametrize("rotation", [0.0, math.pi / 16])
def test_homogeneous_march_vs_normal_modes(rotation):
    # exact modal sum of the Dirichlet waveguide; agreement is limited by the Pade
    # approximant, so compare the modes that propagate within 45 degrees
    s, pl = _homog_plan(rotation)
    psi0 = s.starter()
    res = pl.march(psi0, s.nsteps, s.profile(), out_every=s.out_every)
    assert res.status == OK and res.steps_done == s.nsteps
    ex = normal_mode_field(psi0, s.depth, pl.k0, res.ranges[[0, -1]])
    keep = propagation_angle(s.nz, s.depth, pl.k0) <= 45.0
    for got, ref in ((res.field[0], ex[0]), (res.field[-1], ex[1])):
        a, b = dst_direct(got), dst_direct(ref)
        err = np.linalg.norm((a - b)[keep]) / np.linalg.norm(b[keep])
        assert err < 3e-4


def test_homogeneous_march_is_diagonal_power():
    # with V = 0 every step multiplies sine coefficient l by G_l = e^{i sigma} R(x_l)
    s, pl = _homog_plan(math.pi / 16, nsteps=200)
    psi0 = s.starter()
    res = pl.march(psi0, s.nsteps, s.profile(), out_every=50)
    G = np.exp(1j * pl.sigma) * pl.pade.R_product(pl.x)
    S = dst_matrix(s.nz)
    for k, n in enumerate((50, 100, 150, 200)):
        ref = S @ (G ** n * (S @ psi0))
        assert np.linalg.norm(res.field[k] - ref) / np.linalg.norm(ref) < 1e-12


def test_standard_pade_conserves_norm_homogeneous():
    s, pl = _homog_plan(0.0, nsteps=300)
    psi0 = s.starter()
    res = pl.march(psi0, s.nsteps, s.profile(), out_every=0)
    assert abs(np.linalg.norm(res.final) / np.linalg.norm(psi0) - 1) < 1e-12


# ---------------------------------------------------------------- Neumann series (Sec. 3)
def _tiny(nz=24, form="product", p=6, tol=1e-14, nmax=200, freq=50.0, dr=25.0, depth=300.0):
    c0 = 1500.0
    pl = Plan(nz, depth, freq, c0, dr, p, nmax, tol, form=form)
    z = W.depth_grid(nz, depth)
    c = 1500.0 + 12.0 * np.sin(z / 70.0)              # smooth, |v| ~ 1.6e-2
    v = pl.potential(c)
    return pl, c, v


@pytest.mark.parametrize("j", range(6))
def test_neumann_term_equals_dense_solve(j):
    pl, c, v = _tiny()
    u = W.random_field(pl.nz, 5)
    w, m, res, st = pl.term_solve(u, pl.b[j], v)
    X = dense_operator_from_c(pl.nz, pl.depth, pl.freq, pl.c0, c)
    ref = dense_term(X, u, pl.b[j])
    assert st == OK and m >= 1
    assert np.linalg.norm(w - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("form", ["product", "sum"])
def test_step_equals_rational_function_of_dense_operator(form):
    pl, c, v = _tiny(form=form)
    u = W.random_field(pl.nz, 6)
    out, iters, res, st = pl.step(u, v)
    X = dense_operator_from_c(pl.nz, pl.depth, pl.freq, pl.c0, c)
    ref = np.exp(1j * pl.sigma) * dense_step(X, u, lambda lam: pl.pade.R(lam))
    assert st == OK
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-11


def test_step_close_to_exact_propagator_for_propagating_part():
    # the exact step exp(i sigma sqrt(1+X)) from the same dense operator; the Pade error is
    # small for the eigenvalues near 0 (propagating, small angle)
    pl, c, v = _tiny(nz=40, p=8, depth=500.0)
    X = dense_operator_from_c(pl.nz, pl.depth, pl.freq, pl.c0, c)
    lam, Q = np.linalg.eigh(X)
    keep = lam > -0.5
    u = Q[:, keep] @ W.random_field(int(keep.sum()), 8)
    out, *_ = pl.step(u, v)
    ref = dense_step(X, u, lambda l: np.exp(1j * pl.sigma * np.sqrt(1 + l + 0j)))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-8


def test_sum_and_product_forms_agree_when_converged():
    s = W.munk_deep(nsteps=20, nz=255)
    u0 = s.starter()
    c = s.profile()
    outs = []
    for form in ("product", "sum"):
        pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, 64, 1e-13, form=form)
        outs.append(pl.march(u0, s.nsteps, c, out_every=0).final)
    assert np.linalg.norm(outs[0] - outs[1]) / np.linalg.norm(outs[1]) < 1e-9


def test_lossless_norm_conservation_munk():
    # real v, standard Pade: X is real symmetric and R(X) unitary, so a converged series
    # keeps the 2-norm
    s = W.munk_deep(nsteps=60, nz=255)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, 80, 1e-13)
    res = pl.march(s.starter(), s.nsteps, s.profile(), out_every=0)
    assert res.status == OK
    assert abs(np.linalg.norm(res.final) / np.linalg.norm(s.starter()) - 1) < 1e-9


def test_m0_is_isovelocity_case():
    # Sec. 4.1, Fig. 1a: M = 0 is equivalent to the isovelocity case
    s = W.munk_deep(nsteps=10, nz=127)
    pl0 = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, 0, s.tol)
    a = pl0.march(s.starter(), s.nsteps, s.profile(), out_every=0)
    iso = np.full((1, s.nz), s.c0)
    plv = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, 8, s.tol)
    b = plv.march(s.starter(), s.nsteps, iso, out_every=0)
    assert np.max(np.abs(a.final - b.final)) < 1e-13
    assert np.all(b.iterations == 1)         # v = 0: the first correction is zero


def test_divergence_detected():
    # sigma = k0 dr = 1 with p = 6 on the Munk profile: for the factor whose pole
    # 1 + b_j x = 0 lies inside the grid's eigenvalue range the series' terms grow
    s = W.munk_deep(nsteps=5, nz=511)
    dr = 1.0 / (2 * math.pi * s.freq / s.c0)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, dr, 6, 16, 1e-10)
    res = pl.march(s.starter(), 5, s.profile(), out_every=1)
    assert res.status == DIVERGED and res.steps_done == 0


def test_not_converged_reported():
    s = W.munk_deep(nsteps=3, nz=255, neumann_max=3)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, 3, 1e-10)
    res = pl.march(s.starter(), 3, s.profile(), out_every=1)
    assert res.status == NOT_CONVERGED and res.steps_done == 3
