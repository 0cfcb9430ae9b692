"""Transform bases of the three boundary conditions of Sec. 3.1.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see oracle/__init__.py).

Sec. 3.1 pairs each homogeneous boundary condition at z = 0 and z = H with the transform
that satisfies it: the discrete Fourier transform for periodic boundaries (the setting of
the derivation in Sec. 3), the sine transform for Dirichlet and a cosine transform for
Neumann boundaries.  The paper does not fix the grids or the cosine transform's type; the
readings taken here are the grids whose samples of the continuous eigenfunctions the
transform diagonalises exactly:

  dirichlet  z_n = n H/(Nz+1), n = 1..Nz (interior points), orthonormal DST-I,
             eigenfunctions sin(l pi z/H), kappa_l = l pi/H, l = 1..Nz
  neumann    z_n = n H/(Nz-1), n = 0..Nz-1 (both boundaries on the grid), orthonormal
             DCT-I, eigenfunctions cos(l pi z/H), kappa_l = l pi/H, l = 0..Nz-1
  periodic   z_n = n H/Nz, n = 0..Nz-1, orthonormal DFT (forward e^{-2 pi i l n/Nz}),
             eigenfunctions e^{2 pi i l z/H}, kappa_l = 2 pi l'/H with l' = l for
             l <= Nz/2 and l - Nz above (the symbol of d_z^2, -kappa^2, is even in l',
             so the Nyquist index of an even Nz is unambiguous)

In each basis d_z^2 is diagonal with eigenvalues -kappa_l^2, so the isovelocity inverse
of Sec. 3 is inverse(diag(1/(1 + b_j x_l)) forward(u)) with x_l = -(kappa_l/k0)^2.

The orthonormal DCT-I is C_{kn} = sqrt(2/(Nz-1)) e_k e_n cos(pi k n/(Nz-1)) with
e_0 = e_{Nz-1} = 1/sqrt(2) and e = 1 elsewhere: symmetric and its own inverse, like the
DST-I.  Its columns are the sampled cosines with the two boundary samples scaled by
1/sqrt(2), so the Neumann transform pair acts on grid values f through that weighting:
forward(f) = C (e f), inverse(a) = (C a)/e.  Coefficient-space 2-norms are then the
trapezoidal norm ||e f|| of the grid values (Parseval); the series' stopping rule uses
that norm (weights(bc)).  The forward DFT is F_{kn} = e^{-2 pi i k n/Nz}/sqrt(Nz), its
inverse the conjugate transpose.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from .dst import dst, dst_matrix

BCS = ("dirichlet", "neumann", "periodic")


def check_bc(bc: str) -> str:
    if bc not in BCS:
        raise ValueError(f"boundary condition must be one of {BCS}, got {bc!r}")
    return bc


def grid(bc: str, nz: int, depth: float) -> np.ndarray:
    """Depth points of the grid of boundary condition bc (float64 [Nz])."""
    check_bc(bc)
    if bc == "dirichlet":
        return depth / (nz + 1) * np.arange(1, nz + 1, dtype=np.float64)
    if bc == "neumann":
        return depth / (nz - 1) * np.arange(nz, dtype=np.float64)
    return depth / nz * np.arange(nz, dtype=np.float64)


def wavenumbers(bc: str, nz: int, depth: float) -> np.ndarray:
    """kappa_l (rad/m) of the basis functions in transform order; d_z^2 -> -kappa_l^2."""
    check_bc(bc)
    if bc == "dirichlet":
        return np.arange(1, nz + 1, dtype=np.float64) * math.pi / depth
    if bc == "neumann":
        return np.arange(nz, dtype=np.float64) * math.pi / depth
    ell = np.arange(nz, dtype=np.float64)
    ell = np.where(ell <= nz / 2, ell, ell - nz)
    return 2.0 * math.pi * ell / depth


def _real_parts(f, u):
    u = np.asarray(u)
    if np.iscomplexobj(u):
        return f(u.real) + 1j * f(u.imag)
    return f(u)


def dct1(u: np.ndarray) -> np.ndarray:
    """Orthonormal DCT-I along the last axis (library routine, FP64)."""
    return _real_parts(lambda a: sfft.dct(a, type=1, norm="ortho", axis=-1), u)


def weights(bc: str, nz: int) -> np.ndarray:
    """Grid weights e of the transform pair (1/sqrt(2) at the two Neumann boundary points,
    1 elsewhere); ||e f|| is the coefficient-space norm of grid values f."""
    check_bc(bc)
    e = np.ones(nz)
    if bc == "neumann":
        e[0] = e[-1] = 1.0 / math.sqrt(2.0)
    return e


def forward(bc: str, u: np.ndarray) -> np.ndarray:
    """Physical grid values -> basis coefficients."""
    check_bc(bc)
    if bc == "dirichlet":
        return dst(u)
    if bc == "neumann":
        u = np.asarray(u)
        return dct1(weights(bc, u.shape[-1]) * u)
    return np.fft.fft(np.asarray(u, dtype=np.complex128), norm="ortho", axis=-1)


def inverse(bc: str, a: np.ndarray) -> np.ndarray:
    """Basis coefficients -> physical grid values."""
    check_bc(bc)
    if bc == "dirichlet":
        return dst(a)
    if bc == "neumann":
        a = np.asarray(a)
        return dct1(a) / weights(bc, a.shape[-1])
    return np.fft.ifft(np.asarray(a, dtype=np.complex128), norm="ortho", axis=-1)


def orthonormal_matrix(bc: str, nz: int) -> np.ndarray:
    """The orthonormal transform of bc written out from its definition (DST-I, DCT-I with
    its endpoint factors, DFT), for small Nz checks."""
    check_bc(bc)
    if bc == "dirichlet":
        return dst_matrix(nz)
    n = np.arange(nz)
    if bc == "neumann":
        e = weights(bc, nz)
        return math.sqrt(2.0 / (nz - 1)) * np.outer(e, e) * np.cos(math.pi * np.outer(n, n) / (nz - 1))
    return np.exp(-2j * math.pi * np.outer(n, n) / nz) / math.sqrt(nz)


def forward_matrix(bc: str, nz: int) -> np.ndarray:
    """The forward transform as a matrix acting on grid values."""
    return orthonormal_matrix(bc, nz) * weights(bc, nz)[None, :]
