"""Write the stored oracle references used by the full-size GPU parity tests.

Calls only oracle/ and workloads/.  Each fixture is the FP64 oracle's field at a few output
ranges of a full-length march; storing it lets the GPU test compare the whole range without
re-running minutes of FP64 work on the GPU machine.

    python tests/golden/make_golden.py munk4096
    python tests/golden/make_golden.py eddy16384
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import Plan  # noqa: E402


def munk4096():
    # deep Munk waveguide at its full size and range: Nz = 4096, 4000 steps (100 km)
    s = W.munk_deep()
    keep_every = 400                       # store every 400th step (10 km)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    res = pl.march(s.starter(), s.nsteps, s.profile(), out_every=keep_every)
    np.savez_compressed(os.path.join(HERE, "munk4096_zs1000.npz"),
                        field=res.field.astype(np.complex128), ranges=res.ranges,
                        status=res.status, iterations=res.iterations.sum(axis=0),
                        out_every=keep_every, nsteps=s.nsteps)


def eddy16384():
    # Munk + eddy at its full size (200 Hz, Nz = 16384, [8/8], Neumann <= 12, dr = 20 m),
    # 3000 steps (60 km, through the eddy core at 50 km)
    s = W.munk_eddy(nsteps=3000)
    keep_every = 600                       # store every 600th step (12 km)
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    res = pl.march(s.starter(), s.nsteps, s.profile(), out_every=keep_every)
    np.savez_compressed(os.path.join(HERE, "eddy16384_zs1000.npz"),
                        field=res.field.astype(np.complex128), ranges=res.ranges,
                        status=res.status, iterations=res.iterations.sum(axis=0),
                        not_converged=int((res.residuals > s.tol).sum()),
                        out_every=keep_every, nsteps=s.nsteps)


if __name__ == "__main__":
    {"munk4096": munk4096, "eddy16384": eddy16384}[sys.argv[1]]()
