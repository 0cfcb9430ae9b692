"""Orthonormal type-I discrete sine transform (homogeneous Dirichlet boundaries).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see oracle/__init__.py).

Sec. 3.1 (boundary conditions): with u(0) = u(H) = 0 the Fourier transform of the
isovelocity inverse is replaced by a sine transform.  On the interior grid
z_n = n H/(Nz+1), n = 1..Nz, the orthonormal DST-I is

    (S u)_l = sqrt(2/(Nz+1)) * sum_{n=1..Nz} u_n sin(pi l n / (Nz+1)),   l = 1..Nz,

which is symmetric and its own inverse (S S = I), and diagonalises the second
derivative: d_z^2 sin(l pi z / H) = -(l pi / H)^2 sin(l pi z / H).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def dst(u: np.ndarray) -> np.ndarray:
    """Orthonormal DST-I along the last axis (library routine, FP64/complex128)."""
    u = np.asarray(u)
    if np.iscomplexobj(u):
        return (sfft.dst(u.real, type=1, norm="ortho", axis=-1)
                + 1j * sfft.dst(u.imag, type=1, norm="ortho", axis=-1))
    return sfft.dst(u, type=1, norm="ortho", axis=-1)


idst = dst  # orthonormal DST-I is an involution


def dst_matrix(nz: int) -> np.ndarray:
    """The DST-I matrix written out from its definition (for small Nz checks)."""
    n = np.arange(1, nz + 1)
    return np.sqrt(2.0 / (nz + 1)) * np.sin(np.pi * np.outer(n, n) / (nz + 1))


def dst_direct(u: np.ndarray) -> np.ndarray:
    """O(Nz^2) evaluation of the definition, for pinning the library routine."""
    u = np.asarray(u)
    return u @ dst_matrix(u.shape[-1]).T
