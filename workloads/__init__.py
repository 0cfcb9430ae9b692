"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module generates *inputs only*: depth grids, sound-speed samples, starters and
workload descriptions.  It contains none of the propagation arithmetic (no Pade
coefficients, no transforms, no Neumann series, no range step); both the FP64 oracle and
the HIP library receive what this module produces and compute everything else on their
own.

Environments follow the paper's numerical section:
  * Munk profile, Sec. 4.1 eq. (Munk): c(z) = 1500 (1 + 0.00737 (eta + exp(-eta) - 1)),
    eta = 2 (z - 1300 m) / 1300 m.
  * Range-dependent eddy: the paper's parameterised eddy (Sec. 4.2, eq. (Eddy), Table 1)
    is garbled in its depth factor, so the eddy used here is a Gaussian perturbation
    dc(r, z) = -20 exp(-((r - 50 km)/25 km)^2 - ((z - 800 m)/500 m)^2) m/s added to the
    Munk profile.
  * Starters: Sec. 3.2 lists modal, self- and Greene starters; the Gaussian starter used
    here, sqrt(k0) [exp(-k0^2 (z-zs)^2 / 2) - exp(-k0^2 (z+zs)^2 / 2)], is the plain
    Gaussian form with an image term so that it vanishes at the Dirichlet surface.

The grid convention: Nz interior unknowns, dz = H / (Nz + 1), z_n = n dz for n = 1..Nz
(homogeneous Dirichlet values at z = 0 and z = H are not stored).  The other boundary
conditions of Sec. 3.1 use z_n = n H/(Nz - 1), n = 0..Nz-1 (Neumann, both boundaries on the
grid) and z_n = n H/Nz, n = 0..Nz-1 (periodic).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional

import numpy as np

SEED = 20251103

# ----------------------------------------------------------------------------------------
# grids and environments
# ----------------------------------------------------------------------------------------


def depth_grid(nz: int, depth: float, bc: str = "dirichlet") -> np.ndarray:
    """Depth points of the grid (float64): interior points n H/(Nz+1), n = 1..Nz, for
    Dirichlet boundaries; n H/(Nz-1), n = 0..Nz-1, for Neumann; n H/Nz for periodic."""
    if bc == "dirichlet":
        return depth / (nz + 1) * np.arange(1, nz + 1, dtype=np.float64)
    if bc == "neumann":
        return depth / (nz - 1) * np.arange(nz, dtype=np.float64)
    if bc == "periodic":
        return depth / nz * np.arange(nz, dtype=np.float64)
    raise ValueError(f"unknown boundary condition {bc!r}")


def munk(z: np.ndarray) -> np.ndarray:
    """Munk sound-speed profile in m/s (Sec. 4.1, eq. Munk)."""
    eta = 2.0 * (np.asarray(z, dtype=np.float64) - 1300.0) / 1300.0
    return 1500.0 * (1.0 + 0.00737 * (eta + np.exp(-eta) - 1.0))


@dataclass(frozen=True)
class Eddy:
    """Gaussian synoptic-eddy perturbation dc = -amp exp(-((r-r0)/rr)^2 - ((z-z0)/rz)^2)."""
    amp: float = 20.0
    r0: float = 50_000.0
    rr: float = 25_000.0
    z0: float = 800.0
    rz: float = 500.0

    def dc(self, r: float, z: np.ndarray) -> np.ndarray:
        z = np.asarray(z, dtype=np.float64)
        return -self.amp * np.exp(-((r - self.r0) / self.rr) ** 2 - ((z - self.z0) / self.rz) ** 2)


def sound_speed(kind: str, z: np.ndarray, r: float = 0.0, c_const: float = 1500.0,
                eddy: Optional[Eddy] = None) -> np.ndarray:
    """Sampled c(r, z) for the environment `kind` in {"iso", "munk", "munk+eddy"}."""
    if kind == "iso":
        return np.full(np.shape(z), c_const, dtype=np.float64)
    if kind == "munk":
        return munk(z)
    if kind == "munk+eddy":
        return munk(z) + (eddy or Eddy()).dc(r, z)
    raise ValueError(f"unknown environment {kind!r}")


def profile_steps(kind: str, nz: int, depth: float, dr: float, step0: int, nsteps: int,
                  eddy: Optional[Eddy] = None, bc: str = "dirichlet") -> np.ndarray:
    """c(r, z) for range steps step0+1 .. step0+nsteps, each sampled at the step's mid-range
    r = (n - 1/2) dr, shape [nsteps][Nz] float64."""
    z = depth_grid(nz, depth, bc)
    out = np.empty((nsteps, nz), dtype=np.float64)
    for i in range(nsteps):
        n = step0 + i + 1
        out[i] = sound_speed(kind, z, r=(n - 0.5) * dr, eddy=eddy)
    return out


def absorbing_layer(nz: int, depth: float, thickness: float, strength: float,
                    bc: str = "dirichlet") -> np.ndarray:
    """Imaginary part eta(z) of a complex absorbing potential in a bottom layer: zero above
    H - thickness, rising as strength ((z - (H - thickness))/thickness)^2 to `strength` at
    z = H (float64 [Nz])."""
    z = depth_grid(nz, depth, bc)
    t = np.clip((z - (depth - thickness)) / thickness, 0.0, None)
    return strength * t * t


# ----------------------------------------------------------------------------------------
# starters
# ----------------------------------------------------------------------------------------


def gaussian_starter(nz: int, depth: float, freq: float, c0: float, zs: float,
                     bc: str = "dirichlet") -> np.ndarray:
    """Gaussian starter with a surface image term, complex128 [Nz]: the image is subtracted
    for Dirichlet boundaries (zero at z = 0), added for Neumann (zero slope at z = 0) and
    left out for periodic ones."""
    k0 = 2.0 * math.pi * freq / c0
    z = depth_grid(nz, depth, bc)
    sign = {"dirichlet": -1.0, "neumann": 1.0, "periodic": 0.0}[bc]
    g = np.exp(-0.5 * (k0 * (z - zs)) ** 2) + sign * np.exp(-0.5 * (k0 * (z + zs)) ** 2)
    return (math.sqrt(k0) * g).astype(np.complex128)


def random_field(nz: int, seed: int) -> np.ndarray:
    """A seeded complex Gaussian vector (for transform and kernel parity cases)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(nz) + 1j * rng.standard_normal(nz)


def source_depths(count: int, lo: float, hi: float, seed: int = SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=count)


# ----------------------------------------------------------------------------------------
# workload descriptions
# ----------------------------------------------------------------------------------------


@dataclass
class Solve:
    """One propagation problem: everything the library's plan and march need."""
    nz: int
    depth: float
    freq: float
    c0: float
    dr: float
    pade_order: int
    neumann_max: int
    tol: float
    nsteps: int
    zs: float
    env: str = "munk"              # "iso" | "munk" | "munk+eddy"
    rotation: float = 0.0          # branch-cut rotation angle (rad); 0 = standard Pade
    out_every: int = 1
    eddy: Optional[Eddy] = None
    bc: str = "dirichlet"          # "dirichlet" | "neumann" | "periodic" (Sec. 3.1)

    @property
    def k0(self) -> float:
        return 2.0 * math.pi * self.freq / self.c0

    def starter(self) -> np.ndarray:
        return gaussian_starter(self.nz, self.depth, self.freq, self.c0, self.zs, self.bc)

    def profile(self, step0: int = 0, nsteps: Optional[int] = None) -> np.ndarray:
        """c for steps step0+1..step0+nsteps ([nsteps][Nz]); range-independent
        environments return a single row [1][Nz]."""
        if self.env != "munk+eddy":
            z = depth_grid(self.nz, self.depth, self.bc)
            return sound_speed(self.env, z, c_const=self.c0)[None, :]
        return profile_steps(self.env, self.nz, self.depth, self.dr, step0,
                             self.nsteps if nsteps is None else nsteps, self.eddy or Eddy(),
                             self.bc)

    def updates(self) -> int:
        return self.nz * self.nsteps


def first_experiment(nsteps: int = 250, zs: float = 1100.0, nz: int = 8001) -> Solve:
    """Sec. 4.1's range-independent set-up: Munk profile in a 4 km waveguide, source at
    1100 m, 8001 depth points, range step 100 m, [4/4] Pade at 100 Hz, the series cut at
    M = 2 terms (the paper's largest M of the experiment; tol never reached), TL every
    10 steps (1 km).  The starter of the experiment is the normal-mode starter; starter()
    returns the Gaussian one."""
    return Solve(nz=nz, depth=4000.0, freq=100.0, c0=1500.0, dr=100.0, pade_order=4,
                 neumann_max=2, tol=1e-10, nsteps=nsteps, zs=zs, env="munk", out_every=10)


def homogeneous_waveguide(nsteps: int = 1000, zs: float = 50.0) -> Solve:
    """Range-independent homogeneous waveguide: H = 200 m, c = c0 = 1500 m/s, 100 Hz,
    Nz = 256, rotated [4/4] Pade (alpha = pi/16), dr = 5 m, V = 0."""
    return Solve(nz=256, depth=200.0, freq=100.0, c0=1500.0, dr=5.0, pade_order=4,
                 neumann_max=0, tol=1e-10, nsteps=nsteps, zs=zs, env="iso",
                 rotation=math.pi / 16, out_every=10)


def munk_deep(nsteps: int = 4000, zs: float = 1000.0, neumann_max: int = 48,
              nz: int = 4096) -> Solve:
    """Range-independent deep-ocean Munk waveguide: H = 5000 m, c0 = 1500 m/s, 50 Hz,
    Nz = 4096, [6/6] Pade, dr = 25 m, 4000 steps (100 km), Neumann tol 1e-10."""
    return Solve(nz=nz, depth=5000.0, freq=50.0, c0=1500.0, dr=25.0, pade_order=6,
                 neumann_max=neumann_max, tol=1e-10, nsteps=nsteps, zs=zs, env="munk",
                 out_every=4)


def munk_eddy(nsteps: int = 10_000, zs: float = 1000.0, nz: int = 16384,
              neumann_max: int = 12) -> Solve:
    """Range-dependent Munk + Gaussian eddy: H = 5000 m, c0 = 1500 m/s, 200 Hz,
    Nz = 16384, [8/8] Pade, Neumann <= 12, dr = 20 m, 10^4 steps (200 km)."""
    return Solve(nz=nz, depth=5000.0, freq=200.0, c0=1500.0, dr=20.0, pade_order=8,
                 neumann_max=neumann_max, tol=1e-10, nsteps=nsteps, zs=zs,
                 env="munk+eddy", out_every=5, eddy=Eddy())


def broadband(count: int = 256, nsteps: int = 2000) -> List[Solve]:
    """256 frequencies uniformly in 50..300 Hz on the Munk profile, Nz = round(16 H f /
    1500) clamped to 2048..16384, [6/6], dr = 25 m, 2000 steps (50 km)."""
    out = []
    for i in range(count):
        f = 50.0 + 250.0 * i / (count - 1) if count > 1 else 50.0
        nz = int(min(16384, max(2048, round(16 * 5000.0 * f / 1500.0))))
        out.append(Solve(nz=nz, depth=5000.0, freq=f, c0=1500.0, dr=25.0, pade_order=6,
                         neumann_max=48, tol=1e-10, nsteps=nsteps, zs=1000.0, env="munk",
                         out_every=40))
    return out


@dataclass
class Request:
    arrival: float
    solve: Solve


def serving_requests(rate: float = 200.0, duration: float = 60.0, seed: int = SEED,
                     nz_cap: int = 16384) -> List[Request]:
    """Poisson arrivals of mixed solves: f ~ U[25, 400] Hz, Nz a power of two in
    [max(512, 2^ceil(log2(4 H f / 1500))), nz_cap], range U[10, 100] km, Munk or Munk+eddy,
    zs ~ U[50, 2000] m, [6/6], dr = max(25 m, 5/k0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out: List[Request] = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        f = rng.uniform(25.0, 400.0)
        lo = max(512, 1 << int(math.ceil(math.log2(4 * 5000.0 * f / 1500.0))))
        sizes = [1 << k for k in range(9, 15) if lo <= (1 << k) <= nz_cap] or [nz_cap]
        nz = int(rng.choice(sizes))
        k0 = 2 * math.pi * f / 1500.0
        dr = max(25.0, 5.0 / k0)
        rng_m = rng.uniform(10_000.0, 100_000.0)
        env = "munk" if rng.random() < 0.5 else "munk+eddy"
        zs = rng.uniform(50.0, 2000.0)
        out.append(Request(t, Solve(nz=nz, depth=5000.0, freq=f, c0=1500.0, dr=dr,
                                    pade_order=6, neumann_max=48, tol=1e-10,
                                    nsteps=int(round(rng_m / dr)), zs=zs, env=env,
                                    out_every=max(1, int(round(rng_m / dr)) // 50),
                                    eddy=Eddy() if env == "munk+eddy" else None)))
    return out
