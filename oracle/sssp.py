"""FP64 spectral split-step Pade range march (the oracle of the HIP library).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see oracle/__init__.py).

Follows the paper's method in its own order and notation:
  * Sec. 2: u(r + dr) ~ e^{i k0 dr} R(X) u(r), X = (delta k^2 + d_z^2)/k0^2, with the
    Pade approximant R in sum form d0 + sum_j d_j/(1 + b_j X) (w_j solves
    (1 + b_j X) w_j = u).
  * Sec. 3, eq. (1dHelmholtz): with b~_j = b_j/k0^2 the operator splits into the
    isovelocity part L_j = 1 + b~_j d_z^2 and the perturbation b~_j delta k^2(z).
  * Sec. 3, inverse of the isovelocity operator: L_j is diagonal in the transform basis;
    for Dirichlet boundaries (Sec. 3.1) the basis is the sine basis, where d_z^2 has the
    eigenvalues -(l pi/H)^2, so L_j^{-1} = S diag(1/(1 + b_j x_l)) S with
    x_l = -(l pi / (H k0))^2 and S the orthonormal DST-I.  Neumann and periodic
    boundaries (Sec. 3.1) swap in the cosine and Fourier bases of oracle.bases, with their
    grids and eigenvalues; everything else is unchanged.
  * Sec. 3, eq. (neumannseries): w_j = sum_{m=0..M} (-b~_j L_j^{-1} delta k^2)^m L_j^{-1} u,
    evaluated term by term, each term from the previous one.
  * Algorithm 1: for every range step, every Pade term's w_j from the series, then
    u_n = e^{i dr k0} (d0 u_{n-1} + sum_j d_j w_j).

Readings where the paper is silent (each also listed in the design notes):
  * Neumann stopping: the series for a term stops at the first m >= 1 with
    ||term_m|| <= tol ||w^{(m)}|| (2-norms over depth, in coefficient space: the
    trapezoidal norm of oracle.bases.weights for the cosine basis) or at m = neumann_max; with
    neumann_max = 0 only the m = 0 term is taken (the isovelocity case of Sec. 4.1).
  * Divergence: a series that reaches neumann_max without meeting tol and whose last
    term is not smaller than its first, or any non-finite value, stops the march.
  * Product form (numerically preferable in FP32, same approximant): R = C prod_j
    (1 + a_j X)/(1 + b_j X) and each factor equals g_j + (1 - g_j)(1 + b_j X)^{-1},
    g_j = a_j / b_j, applied in the fixed factor order of oracle.pade.
  * The carrier e^{i k0 dr} is applied every step (Algorithm 1), so outputs include it.
  * Transmission loss TL = -20 log10(|u| / sqrt(r)) in dB re 1 m (the field u carries
    no cylindrical spreading factor, Sec. 2).
  * Output steps are n = out_every, 2 out_every, ... up to nsteps.
  * Complex absorbing potential (Sec. 3.1 names it as a simple absorbing boundary): an
    imaginary part i eta(z) added to v, i.e. to delta k^2 / k0^2, fixed in range, its
    depth profile an input; eta > 0 damps (the one-way propagator
    exp(i sigma sqrt(1 + X)) then has modulus below one).  The series, its stopping rule
    and the step are unchanged, now in complex v.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import bases
from .pade import PadeCoeffs, pade

OK = 0
NOT_CONVERGED = 1
DIVERGED = -4


@dataclass
class MarchResult:
    field: np.ndarray            # complex128 [nout][Nz] (carrier included)
    tl: np.ndarray               # float64   [nout][Nz]
    ranges: np.ndarray           # float64   [nout]
    final: np.ndarray            # complex128 [Nz], field after the last good step
    status: int
    steps_done: int
    iterations: np.ndarray       # int [steps_done][p]: Neumann terms beyond m = 0
    residuals: np.ndarray        # float64 [steps_done][p]: final ||term||/||w||


class Plan:
    """Grid, Pade coefficients and eigenvalues for one (Nz, H, f, c0, dr, p) problem."""

    def __init__(self, nz: int, depth: float, freq: float, c0: float, dr: float,
                 pade_order: int, neumann_max: int, tol: float, rotation: float = 0.0,
                 form: str = "product", bc: str = "dirichlet"):
        if nz < 2 or depth <= 0 or freq <= 0 or c0 <= 0 or dr <= 0:
            raise ValueError("invalid plan parameters")
        if form not in ("product", "sum"):
            raise ValueError("form must be 'product' or 'sum'")
        self.bc = bases.check_bc(bc)
        self.nz, self.depth, self.freq, self.c0, self.dr = nz, depth, freq, c0, dr
        self.neumann_max, self.tol, self.form = int(neumann_max), float(tol), form
        self.k0 = 2.0 * math.pi * freq / c0
        self.sigma = self.k0 * dr
        self.z = bases.grid(bc, nz, depth)
        # eigenvalues of d_z^2/k0^2 in the basis of the boundary condition
        self.x = -(bases.wavenumbers(bc, nz, depth) / self.k0) ** 2
        # weights of the coefficient-space norm (all 1 except the Neumann boundary points)
        self.wnorm = bases.weights(bc, nz)
        self.pade: PadeCoeffs = pade(self.sigma, pade_order, rotation)
        self.b = self.pade.b
        self.g = self.pade.a / self.pade.b

    # --- pieces of the method ------------------------------------------------------------
    def potential(self, c: np.ndarray) -> np.ndarray:
        """v = delta k^2 / k0^2 = (c0/c)^2 - 1 (Sec. 2, X = (delta k^2 + d_z^2)/k0^2)."""
        return (self.c0 / np.asarray(c, dtype=np.float64)) ** 2 - 1.0

    def norm(self, u: np.ndarray) -> float:
        """2-norm over depth in coefficient space (Parseval): ||u|| for the sine and Fourier
        bases, the trapezoidal ||e u|| for the cosine basis."""
        return float(np.linalg.norm(self.wnorm * u))

    def l_inverse(self, u: np.ndarray, bj: complex) -> np.ndarray:
        """L_j^{-1} u = T^{-1} diag(1/(1 + b_j x)) T u (Sec. 3, isovelocity inverse; T the
        transform of the boundary condition, the DST-I for Dirichlet)."""
        return bases.inverse(self.bc, bases.forward(self.bc, u) / (1.0 + bj * self.x))

    def term_solve(self, u: np.ndarray, bj: complex, v: np.ndarray):
        """w = (1 + b_j X)^{-1} u by the Neumann series (eq. neumannseries).
        Returns (w, terms beyond m=0, final residual, status)."""
        term = self.l_inverse(u, bj)
        w = term.copy()
        first = self.norm(term)
        m, res = 0, 0.0
        for m in range(1, self.neumann_max + 1):
            term = -bj * self.l_inverse(v * term, bj)
            w = w + term
            tn, wn = self.norm(term), self.norm(w)
            res = tn / wn if wn > 0 else 0.0
            if not (np.isfinite(tn) and np.isfinite(wn)):
                return w, m, float("inf"), DIVERGED
            if tn <= self.tol * wn:
                return w, m, res, OK
        if self.neumann_max == 0:
            return w, 0, 0.0, OK
        if self.norm(term) >= first:
            return w, m, res, DIVERGED
        return w, m, res, NOT_CONVERGED

    def step(self, u: np.ndarray, v: np.ndarray):
        """One range step u_{n-1} -> u_n (Algorithm 1).  Returns (u_n, iters, res, status)."""
        p = len(self.b)
        iters = np.zeros(p, dtype=np.int64)
        res = np.zeros(p)
        status = OK
        if self.form == "sum":
            acc = self.pade.d0 * u
            for j in range(p):
                w, iters[j], res[j], st = self.term_solve(u, self.b[j], v)
                acc = acc + self.pade.d[j] * w
                status = _worse(status, st)
            out = acc
        else:
            out = u
            for j in range(p):
                w, iters[j], res[j], st = self.term_solve(out, self.b[j], v)
                out = self.g[j] * out + (1.0 - self.g[j]) * w
                status = _worse(status, st)
            out = self.pade.C * out
        out = np.exp(1j * self.sigma) * out
        if not np.all(np.isfinite(out)):
            status = DIVERGED
        return out, iters, res, status

    # --- the range march -----------------------------------------------------------------
    def march(self, psi0: np.ndarray, nsteps: int, c_steps: np.ndarray,
              out_every: int = 1, r0: float = 0.0,
              absorber: Optional[np.ndarray] = None) -> MarchResult:
        """March psi0 through nsteps range steps.  c_steps is [nsteps][Nz] (one sound-speed
        sample per step) or [1][Nz] (range independent).  absorber: imaginary part eta(z) of
        a complex absorbing potential (Sec. 3.1), v -> v + i eta, eta >= 0 absorbs."""
        u = np.asarray(psi0, dtype=np.complex128).copy()
        c_steps = np.atleast_2d(np.asarray(c_steps, dtype=np.float64))
        fields, ranges = [], []
        iters, resid = [], []
        status, done = OK, 0
        eta = None if absorber is None else np.asarray(absorber, dtype=np.float64)

        def pot(c):
            v = self.potential(c)
            return v if eta is None else v + 1j * eta

        v_fixed = pot(c_steps[0]) if c_steps.shape[0] == 1 else None
        for n in range(1, nsteps + 1):
            v = v_fixed if v_fixed is not None else pot(c_steps[n - 1])
            un, it, rs, st = self.step(u, v)
            if st == DIVERGED:
                status = DIVERGED
                break
            status = _worse(status, st)
            u = un
            done = n
            iters.append(it)
            resid.append(rs)
            if out_every > 0 and n % out_every == 0:
                fields.append(u.copy())
                ranges.append(r0 + n * self.dr)
        F = np.array(fields, dtype=np.complex128).reshape(-1, self.nz)
        R = np.array(ranges, dtype=np.float64)
        return MarchResult(field=F, tl=transmission_loss(F, R), ranges=R, final=u,
                           status=status, steps_done=done,
                           iterations=np.array(iters, dtype=np.int64).reshape(-1, len(self.b)),
                           residuals=np.array(resid).reshape(-1, len(self.b)))


def transmission_loss(field: np.ndarray, ranges: np.ndarray) -> np.ndarray:
    """TL = -20 log10(|u| / sqrt(r)) (dB re 1 m)."""
    field = np.atleast_2d(field)
    r = np.asarray(ranges, dtype=np.float64).reshape(-1, 1)
    with np.errstate(divide="ignore"):
        return -20.0 * np.log10(np.abs(field) / np.sqrt(r))


def _worse(a: int, b: int) -> int:
    if DIVERGED in (a, b):
        return DIVERGED
    return max(a, b)
