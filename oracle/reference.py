"""Closed-form and brute-force references that pin the oracle itself.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see oracle/__init__.py).  Nothing here
is used by the march; these are independent routes to quantities the march must reproduce.

  * normal_mode_field: exact one-way propagation in a homogeneous Dirichlet waveguide
    (Sec. 2 propagator exp(i r sqrt(d_z^2 + k^2)); modes sin(l pi z/H) with horizontal
    wavenumbers kappa_l = sqrt(k0^2 - (l pi/H)^2), Im kappa >= 0).  The starter is
    expanded with the definition-level DST matrix, not the library transform.
  * dense_operator / dense_step: the vertical operator X = k0^-2 (d_z^2 + k^2 - k0^2)
    built as a dense matrix S diag(x) S + diag(v) (S from its definition) and the
    propagator applied through a symmetric eigendecomposition (numpy.linalg.eigh), for
    tiny grids.  The rational step e^{i sigma} R(X) then needs no series, and the exact
    step exp(i sigma sqrt(1 + X)) is available for the same matrix.
  * modal_field_bc / dense_operator_bc: the same two references for the Neumann and
    periodic boundaries of Sec. 3.1.  The modal sum expands the starter by solving the
    linear system of the sampled eigenfunctions cos(l pi z/H) or e^{2 pi i l z/H} (no
    transform, no normalisation weights); the dense operator is d_z^2 = Phi diag(-mu)
    Phi^{-1} from the same sampled eigenfunctions (again no transform).
"""
from __future__ import annotations

import math

import numpy as np

from .dst import dst_matrix


def normal_mode_field(psi0: np.ndarray, depth: float, k0: float, ranges) -> np.ndarray:
    """Exact modal sum u(r, z_n) = sum_l c_l e^{i kappa_l r} S_{n l}, [len(ranges)][Nz]."""
    nz = len(psi0)
    S = dst_matrix(nz)
    coef = S @ np.asarray(psi0, dtype=np.complex128)
    mu = (np.arange(1, nz + 1) * math.pi / depth) ** 2
    kappa = np.sqrt((k0 ** 2 - mu).astype(np.complex128))
    kappa = np.where(kappa.imag < 0, -kappa, kappa)
    out = []
    for r in np.atleast_1d(ranges):
        out.append(S @ (coef * np.exp(1j * kappa * r)))
    return np.array(out)


def propagation_angle(nz: int, depth: float, k0: float) -> np.ndarray:
    """Grazing angle (deg) of each sine mode; NaN for evanescent modes."""
    kz = np.arange(1, nz + 1) * math.pi / depth
    s = kz / k0
    with np.errstate(invalid="ignore"):
        return np.where(s <= 1.0, np.degrees(np.arcsin(np.minimum(s, 1.0))), np.nan)


def dense_operator(nz: int, depth: float, k0: float, v: np.ndarray) -> np.ndarray:
    """X = S diag(x) S + diag(v) with x_l = -(l pi/(H k0))^2 (real symmetric)."""
    S = dst_matrix(nz)
    x = -(np.arange(1, nz + 1) * math.pi / (depth * k0)) ** 2
    return S @ np.diag(x) @ S + np.diag(np.asarray(v, dtype=np.float64))


def dense_step(X: np.ndarray, u: np.ndarray, func) -> np.ndarray:
    """func(X) u through X = Q diag(lam) Q^H (X real symmetric or Hermitian)."""
    lam, Q = np.linalg.eigh(X)
    return Q @ (func(lam) * (Q.conj().T @ u))


def dense_term(X: np.ndarray, u: np.ndarray, bj: complex) -> np.ndarray:
    """(1 + b_j X)^{-1} u by a dense LU solve."""
    return np.linalg.solve(np.eye(X.shape[0]) + bj * X, u)


def dense_operator_from_c(nz: int, depth: float, freq: float, c0: float,
                          c: np.ndarray) -> np.ndarray:
    """X = k0^-2 (d_z^2 + k^2 - k0^2) from its definition (Sec. 2) with k = 2 pi f / c(z),
    k0 = 2 pi f / c0, and d_z^2 = S diag(-(l pi/H)^2) S on the sine basis."""
    S = dst_matrix(nz)
    k0 = 2 * math.pi * freq / c0
    k = 2 * math.pi * freq / np.asarray(c, dtype=np.float64)
    d2 = S @ np.diag(-(np.arange(1, nz + 1) * math.pi / depth) ** 2) @ S
    return (d2 + np.diag(k ** 2 - k0 ** 2)) / k0 ** 2


def eigenfunctions(bc: str, z: np.ndarray, depth: float):
    """Sampled eigenfunctions of d_z^2 under boundary condition bc, as columns, and the
    squared vertical wavenumbers mu_l (d_z^2 phi_l = -mu_l phi_l)."""
    nz = len(z)
    if bc == "dirichlet":
        ell = np.arange(1, nz + 1)
        return np.sin(np.outer(z, ell) * math.pi / depth), (ell * math.pi / depth) ** 2
    if bc == "neumann":
        ell = np.arange(nz)
        return np.cos(np.outer(z, ell) * math.pi / depth), (ell * math.pi / depth) ** 2
    if bc == "periodic":
        ell = np.arange(nz) - (nz - 1) // 2          # -(Nz-1)/2 .. Nz/2
        return np.exp(2j * math.pi * np.outer(z, ell) / depth), (2 * math.pi * ell / depth) ** 2
    raise ValueError(bc)


def modal_field_bc(bc: str, psi0: np.ndarray, z: np.ndarray, depth: float, k0: float,
                   ranges) -> np.ndarray:
    """Exact one-way modal sum of a homogeneous waveguide with boundary condition bc:
    u(r, z_n) = sum_l c_l e^{i kappa_l r} phi_l(z_n), kappa_l = sqrt(k0^2 - mu_l)
    (Im kappa >= 0), the c_l from phi(z_n) c = psi0."""
    Phi, mu = eigenfunctions(bc, np.asarray(z, dtype=np.float64), depth)
    coef = np.linalg.solve(Phi.astype(np.complex128), np.asarray(psi0, dtype=np.complex128))
    kappa = np.sqrt((k0 ** 2 - mu).astype(np.complex128))
    kappa = np.where(kappa.imag < 0, -kappa, kappa)
    return np.array([Phi @ (coef * np.exp(1j * kappa * r)) for r in np.atleast_1d(ranges)])


def dense_operator_bc(bc: str, z: np.ndarray, depth: float, freq: float, c0: float,
                      c: np.ndarray) -> np.ndarray:
    """X = k0^-2 (d_z^2 + k^2 - k0^2) with d_z^2 = Phi diag(-mu) Phi^{-1}, Phi the sampled
    eigenfunctions of bc on the grid z (a dense, in general non-symmetric matrix)."""
    Phi, mu = eigenfunctions(bc, np.asarray(z, dtype=np.float64), depth)
    Phi = Phi.astype(np.complex128)
    d2 = Phi @ np.diag(-mu) @ np.linalg.inv(Phi)
    if bc != "periodic":
        d2 = d2.real
    k0 = 2 * math.pi * freq / c0
    k = 2 * math.pi * freq / np.asarray(c, dtype=np.float64)
    return (d2 + np.diag(k ** 2 - k0 ** 2)) / k0 ** 2


def dense_rational(X: np.ndarray, u: np.ndarray, C: complex, a, b) -> np.ndarray:
    """C prod_j (1 + a_j X)(1 + b_j X)^{-1} u by dense solves (no eigendecomposition)."""
    out = np.asarray(u, dtype=np.complex128)
    eye = np.eye(X.shape[0])
    for aj, bj in zip(a, b):
        out = (eye + aj * X) @ np.linalg.solve(eye + bj * X, out)
    return C * out
