"""Normal-mode starter and normal-mode reference field (Sec. 3.2, initial conditions).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see oracle/__init__.py).

Sec. 3.2 starts the march from the normal-mode solution of a point source at depth zs:
u(r0, z) = sqrt(2 pi) sum_m Psi_m(zs) Psi_m(z) / sqrt(kappa_m), with the mode functions
Psi_m and horizontal wavenumbers kappa_m of the depth (Sturm-Liouville) problem
    d_z^2 Psi + (k^2(z) - kappa^2) Psi = 0          (the printed "+ kappa^2" is garbled)
under the waveguide's boundary conditions.  In the spectral basis of the method this is an
eigenproblem of the same vertical operator X = k0^-2 (d_z^2 + k^2 - k0^2) that the range
step propagates: k0^2 (X + 1) Psi = kappa^2 Psi.

Readings (the paper gives no discretisation of the starter):
  * X as a dense matrix in the Dirichlet sine basis, T diag(x) T + diag(v) with T the
    orthonormal DST-I (its eigenvectors are the mode functions on the grid);
  * modes are the propagating ones, kappa_m^2 > 0, ordered by decreasing kappa (the
    first is the lowest mode); max_modes caps their number;
  * Psi_m is normalised to unit L2 norm over depth: the unit eigenvector y_m gives
    Psi_m(z_n) = y_m[n] / sqrt(dz), and Psi_m(zs) between grid points comes from the
    basis expansion Psi_m(z) = sum_l a_lm sqrt(2/H) sin(l pi z/H), a = T y (exact for the
    sine basis);
  * the starter is real; the normal-mode field at range r replaces 1/sqrt(kappa_m) by
    e^{i kappa_m r}/sqrt(kappa_m) (one-way, far-field form of the modal sum).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from .bases import orthonormal_matrix, wavenumbers


def depth_modes(nz: int, depth: float, freq: float, c0: float, c: np.ndarray,
                max_modes: Optional[int] = None):
    """Propagating modes of the Dirichlet waveguide: (kappa [M], Y [Nz][M] unit eigenvectors,
    A [Nz][M] sine-basis coefficients), ordered by decreasing kappa."""
    k0 = 2.0 * math.pi * freq / c0
    T = orthonormal_matrix("dirichlet", nz)
    x = -(wavenumbers("dirichlet", nz, depth) / k0) ** 2
    v = (c0 / np.asarray(c, dtype=np.float64)) ** 2 - 1.0
    X = T @ np.diag(x) @ T + np.diag(v)
    lam, Y = np.linalg.eigh(X)
    order = np.argsort(lam)[::-1]
    lam, Y = lam[order], Y[:, order]
    keep = lam > -1.0
    if max_modes is not None:
        keep &= np.arange(nz) < max_modes
    lam, Y = lam[keep], Y[:, keep]
    kappa = k0 * np.sqrt(1.0 + lam)
    return kappa, Y, T @ Y


def _mode_values(A: np.ndarray, depth: float, zs: float) -> np.ndarray:
    nz = A.shape[0]
    phi = math.sqrt(2.0 / depth) * np.sin(np.arange(1, nz + 1) * math.pi * zs / depth)
    return phi @ A


def modal_field(nz: int, depth: float, freq: float, c0: float, c: np.ndarray, zs: float,
                ranges, max_modes: Optional[int] = None) -> np.ndarray:
    """Normal-mode field sqrt(2 pi) sum_m Psi_m(zs) Psi_m(z_n) e^{i kappa_m r}/sqrt(kappa_m)
    on the grid, [len(ranges)][Nz] complex; r = 0 is the modal starter."""
    kappa, Y, A = depth_modes(nz, depth, freq, c0, c, max_modes)
    dz = depth / (nz + 1)
    w = math.sqrt(2.0 * math.pi) * _mode_values(A, depth, zs) / (math.sqrt(dz) * np.sqrt(kappa))
    return np.array([Y @ (w * np.exp(1j * kappa * r)) for r in np.atleast_1d(ranges)])


def modal_starter(nz: int, depth: float, freq: float, c0: float, c: np.ndarray, zs: float,
                  max_modes: Optional[int] = None) -> np.ndarray:
    """The modal starter u(0, z_n) (complex128 [Nz], real-valued)."""
    return modal_field(nz, depth, freq, c0, c, zs, [0.0], max_modes)[0]
