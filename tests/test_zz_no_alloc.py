"""ssp_march_device_noalloc (the device march for callers that cannot allocate) against
ssp_march_device through the C ABI: the same kernels on the same inputs, so the fields, step
counters, TL rows and statistics must be bitwise equal, on two calls in a row (the second
with a smaller batch, reusing the fixed scratch), for an unsplit and a split FFT length;
a batch whose scratch exceeds the fixed array is rejected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _plan(ssp, s, stream):
    pl = ssp.ssp_plan_create(s.nz, s.depth, s.freq, s.c0, s.dr, s.pade_order, s.neumann_max, s.tol)
    ssp.ssp_plan_set_option(pl, ssp.SSP_OPT_OUT_EVERY, s.out_every)
    ssp.ssp_set_profile(pl, 0, -1, s.profile()[0])
    ssp.ssp_plan_set_stream(pl, stream.cuda_stream)
    return pl


def _run(ssp, torch, pl, s, psi, nsteps, noalloc, with_stats):
    B = psi.shape[0]
    d_psi = torch.from_numpy(psi.astype(np.complex64)).cuda()
    d_step = torch.arange(B, dtype=torch.int64, device="cuda") % 3   # counters differ per solve
    d_tl = torch.full((B, nsteps // s.out_every + 1, s.nz), -7.0, dtype=torch.float32, device="cuda")
    d_stats = torch.zeros((B, 48), dtype=torch.uint8, device="cuda") if with_stats else None
    ssp.ssp_to_sine(pl, B, d_psi.data_ptr(), d_psi.data_ptr())
    fn = ssp.ssp_march_device_noalloc if noalloc else ssp.ssp_march_device
    fn(pl, B, d_psi.data_ptr(), d_step.data_ptr(), nsteps, d_tl.data_ptr(),
       d_stats.data_ptr() if with_stats else 0)
    torch.cuda.synchronize()
    return (d_psi.cpu().numpy(), d_step.cpu().numpy(), d_tl.cpu().numpy(),
            None if d_stats is None else d_stats.cpu().numpy())


@pytest.mark.parametrize("nz,freq", [(1000, 50.0), (9000, 170.0)])
def test_noalloc_march_equals_device_march_twice(ssp, gpu, nz, freq):
    torch = gpu
    s = W.munk_deep(nz=nz)
    s.freq, s.out_every = freq, 3
    stream = torch.cuda.Stream()
    pl = _plan(ssp, s, stream)
    try:
        with torch.cuda.stream(stream):
            for call, (B, nsteps, with_stats) in enumerate([(12, 7, True), (5, 4, False)]):
                zs = W.source_depths(B, 50.0, 2000.0, seed=W.SEED + call)
                psi = np.stack([W.gaussian_starter(s.nz, s.depth, s.freq, s.c0, z) for z in zs])
                ref = _run(ssp, torch, pl, s, psi, nsteps, noalloc=False, with_stats=with_stats)
                got = _run(ssp, torch, pl, s, psi, nsteps, noalloc=True, with_stats=with_stats)
                print(f"[noalloc] nz={nz} call={call} B={B} steps={nsteps}", flush=True)
                for a, b in zip(ref, got):
                    if a is not None:
                        assert np.array_equal(a, b)
                assert (ref[2][:, 0] != -7.0).all()   # the first output row was written
    finally:
        ssp.ssp_plan_destroy(pl)


def test_noalloc_rejects_a_batch_above_the_scratch(ssp, gpu):
    torch = gpu
    s = W.munk_deep(nz=4096)
    stream = torch.cuda.Stream()
    pl = _plan(ssp, s, stream)
    try:
        B = 1024  # 5 x 4096 x 1024 complex values of state alone: 160 MiB
        d_psi = torch.zeros((B, s.nz), dtype=torch.complex64, device="cuda")
        d_step = torch.zeros(B, dtype=torch.int64, device="cuda")
        with pytest.raises(ssp.SspError) as e:
            ssp.ssp_march_device_noalloc(pl, B, d_psi.data_ptr(), d_step.data_ptr(), 4)
        assert e.value.status == ssp.SSP_E_INVAL and "scratch" in str(e.value)
        assert d_step.cpu().numpy().max() == 0   # nothing ran
    finally:
        ssp.ssp_plan_destroy(pl)
