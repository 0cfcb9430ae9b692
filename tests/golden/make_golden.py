"""Write the stored oracle references used by the full-size GPU parity tests.

Calls only oracle/ and workloads/.  Each fixture is the FP64 oracle's field at a few output
ranges of a full-length march; storing it lets the GPU test compare the whole range without
re-running minutes of FP64 work on the GPU machine.

    python tests/golden/make_golden.py munk4096
    python tests/golden/make_golden.py eddy16384
    python tests/golden/make_golden.py eddy16384_full
    python tests/golden/make_golden.py broadband <frequency index> [...]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import Plan  # noqa: E402

# frequency indices of the broadband set whose full march is stored: FFT lengths 8192
# (indices 0 .. 27), 16384 (28 .. 106) and the split length 32768 (107 .. 255)
BROADBAND_SAMPLES = (0, 20, 28, 64, 106, 107, 180, 255)


def _single_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


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


def eddy16384_full():
    # the same environment over its whole range: 10^4 steps (200 km), a stored row every
    # 1000 steps (20 km); the sound speed of each step is passed in chunks so that the
    # [steps][Nz] table is never held whole
    _single_thread()
    s = W.munk_eddy()
    keep_every, chunk = 1000, 500
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    psi, rows, ranges, iters, nc, status = s.starter(), [], [], np.zeros(s.pade_order, np.int64), 0, 0
    for n0 in range(0, s.nsteps, chunk):
        res = pl.march(psi, chunk, s.profile(n0, chunk), out_every=0, r0=n0 * s.dr)
        psi = res.final
        iters += res.iterations.sum(axis=0)
        nc += int((res.residuals > s.tol).sum())
        status = max(status, res.status) if res.status >= 0 else res.status
        if res.status < 0:
            break
        if (n0 + chunk) % keep_every == 0:
            rows.append(psi.copy())
            ranges.append((n0 + chunk) * s.dr)
        print(f"eddy16384_full: step {n0 + chunk} of {s.nsteps}", flush=True)
    np.savez_compressed(os.path.join(HERE, "eddy16384_full_zs1000.npz"),
                        field=np.array(rows).astype(np.complex64), ranges=np.array(ranges),
                        status=status, iterations=iters, not_converged=nc,
                        out_every=keep_every, nsteps=s.nsteps)


def broadband(index):
    # one frequency of the broadband set at its full range (2000 steps, 50 km), the field
    # stored at 25 km and 50 km
    _single_thread()
    s = W.broadband()[index]
    keep_every = 1000
    pl = Plan(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    res = pl.march(s.starter(), s.nsteps, s.profile(), out_every=keep_every)
    np.savez_compressed(os.path.join(HERE, f"broadband_f{index:03d}.npz"),
                        field=res.field.astype(np.complex64), ranges=res.ranges,
                        status=res.status, iterations=res.iterations.sum(axis=0),
                        not_converged=int((res.residuals > s.tol).sum()),
                        out_every=keep_every, nsteps=s.nsteps, freq=s.freq, nz=s.nz)
    print(f"broadband {index}: f = {s.freq:.3f} Hz, Nz = {s.nz}, status {res.status}", flush=True)


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "broadband":
        for i in (sys.argv[2:] or BROADBAND_SAMPLES):
            broadband(int(i))
    else:
        {"munk4096": munk4096, "eddy16384": eddy16384, "eddy16384_full": eddy16384_full}[what]()
