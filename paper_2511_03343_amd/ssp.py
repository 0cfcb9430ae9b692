"""Thin ctypes binding of libssp.so (include/ssp.h): argument marshalling only.

Every function keeps the C name and argument order; arrays are numpy arrays (host) or
integers holding device addresses (e.g. torch_tensor.data_ptr()).  Statuses < 0 raise
SspError; the warning SSP_W_NOT_CONVERGED is returned.  There is no fallback: if the
library is missing, loading raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssp.so")

SSP_OK = 0
SSP_W_NOT_CONVERGED = 1
SSP_E_INVAL = -1
SSP_E_NOMEM = -2
SSP_E_DEVICE = -3
SSP_E_DIVERGED = -4
SSP_E_UNSTABLE = -5
SSP_E_STATE = -6
SSP_E_UNIMPL = -7

SSP_OPT_ROTATION = 1
SSP_OPT_OUT_EVERY = 2
SSP_OPT_STREAM = 3
SSP_OPT_ENGINE = 4
SSP_OPT_GRAPH = 5
SSP_OPT_VARIANT = 6
SSP_OPT_PLAIN = 7
SSP_OPT_FORM = 8
SSP_OPT_GAIN_LIMIT = 9
SSP_OPT_CONTRACTION_CHECK = 10

SSP_ENGINE_FFT = 0
SSP_ENGINE_DENSE = 1
SSP_ENGINE_AUTO = 2
SSP_FORM_PRODUCT = 0
SSP_FORM_SUM = 1

SSP_BC_DIRICHLET = 0
SSP_BC_NEUMANN = 1
SSP_BC_PERIODIC = 2
BC_CODES = {"dirichlet": SSP_BC_DIRICHLET, "neumann": SSP_BC_NEUMANN, "periodic": SSP_BC_PERIODIC}


class ssp_stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("step_index", C.c_int64),
                ("neumann_terms", C.c_int64), ("neumann_max_used", C.c_int32),
                ("not_converged", C.c_int32), ("max_residual", C.c_double),
                ("status", C.c_int32), ("pad_", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class ssp_env(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("munk_c1", "munk_eps", "munk_z1", "eddy_amp",
                                          "eddy_r0", "eddy_rr", "eddy_z0", "eddy_rz")]


class SspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None
_DP = C.POINTER(C.c_double)
_FP = C.POINTER(C.c_float)
_VP = C.c_void_p


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname); if
        # torch is importable it is loaded first so that libssp binds to that runtime and
        # device pointers and streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        S = C.c_int
        sig = {
            "ssp_plan_create": (S, [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_int, C.c_int, C.c_double, C.POINTER(_VP)]),
            "ssp_plan_create_bc": (S, [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_int, C.c_int, C.c_double, C.c_int, C.POINTER(_VP)]),
            "ssp_plan_destroy": (None, [_VP]),
            "ssp_plan_set_option": (S, [_VP, C.c_int, C.c_double]),
            "ssp_plan_set_stream": (S, [_VP, _VP]),
            "ssp_plan_info": (S, [_VP, _DP, _DP, _DP, _DP, _DP, _DP, _DP]),
            "ssp_max_nz": (C.c_int, []),
            "ssp_plan_engine": (S, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "ssp_pade_coefficients": (S, [C.c_double, C.c_int, C.c_double, _DP, _DP, _DP, _DP, _DP]),
            "ssp_set_profile": (S, [_VP, C.c_int, C.c_int, _DP]),
            "ssp_set_profile_analytic": (S, [_VP, C.POINTER(ssp_env)]),
            "ssp_set_absorber": (S, [_VP, _DP]),
            "ssp_modal_starter": (S, [_VP, _DP, C.c_int, _DP, C.c_int, _DP, _DP, C.POINTER(C.c_int)]),
            "ssp_set_field": (S, [_VP, _DP]),
            "ssp_get_field": (S, [_VP, _DP]),
            "ssp_march": (S, [_VP, _DP, C.c_int, _DP, _FP, C.POINTER(ssp_stats)]),
            "ssp_count_outputs": (C.c_int, [_VP, C.c_int]),
            "ssp_march_batch": (S, [C.POINTER(_VP), C.c_int, C.c_int, C.POINTER(_DP),
                                    C.POINTER(_FP), C.POINTER(ssp_stats)]),
            "ssp_march_batch_steps": (S, [C.POINTER(_VP), C.c_int, C.POINTER(C.c_int), C.POINTER(_DP),
                                          C.POINTER(_FP), C.POINTER(ssp_stats)]),
            "ssp_march_device": (S, [_VP, C.c_int, _VP, _VP, C.c_int, _VP, _VP]),
            "ssp_march_device_noalloc": (S, [_VP, C.c_int, _VP, _VP, C.c_int, _VP, _VP]),
            "ssp_march_batch_async": (S, [C.POINTER(_VP), C.c_int, C.POINTER(C.c_int), C.POINTER(_FP)]),
            "ssp_batch_stats": (S, [C.POINTER(_VP), C.c_int, C.POINTER(ssp_stats)]),
            "ssp_plan_contraction": (S, [_VP, C.c_int, _DP, _DP]),
            "ssp_to_sine": (S, [_VP, C.c_int, _VP, _VP]),
            "ssp_from_sine": (S, [_VP, C.c_int, _VP, _VP, _VP]),
            "ssp_dst_device": (S, [_VP, C.c_int, _VP, _VP]),
            "ssp_dst_dense_device": (S, [_VP, C.c_int, _VP, _VP]),
            "ssp_max_dense_nz": (C.c_int, []),
            "ssp_status_string": (C.c_char_p, [C.c_int]),
            "ssp_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st < 0:
        L = lib()
        raise SspError(st, f"{L.ssp_status_string(st).decode()}: {L.ssp_last_error().decode()}")
    return st


def _dp(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _fp(a):
    return None if a is None else a.ctypes.data_as(_FP)


def _c128(a, n):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != (n,):
        raise ValueError(f"expected {n} complex values, got shape {a.shape}")
    return a.view(np.float64)


# ------------------------------------------------------------------------- C-named calls
def ssp_plan_create(Nz, H, f, c0, dr, pade_order, neumann_max, tol):
    out = _VP()
    _check(lib().ssp_plan_create(int(Nz), float(H), float(f), float(c0), float(dr),
                                 int(pade_order), int(neumann_max), float(tol), C.byref(out)))
    return out.value


def ssp_plan_create_bc(Nz, H, f, c0, dr, pade_order, neumann_max, tol, bc):
    """bc: SSP_BC_* code or one of "dirichlet", "neumann", "periodic"."""
    code = BC_CODES[bc] if isinstance(bc, str) else int(bc)
    out = _VP()
    _check(lib().ssp_plan_create_bc(int(Nz), float(H), float(f), float(c0), float(dr),
                                    int(pade_order), int(neumann_max), float(tol), code,
                                    C.byref(out)))
    return out.value


def ssp_plan_destroy(plan):
    lib().ssp_plan_destroy(plan)


def ssp_plan_set_option(plan, key, value):
    return _check(lib().ssp_plan_set_option(plan, int(key), float(value)))


def ssp_plan_set_stream(plan, stream_ptr):
    return _check(lib().ssp_plan_set_stream(plan, stream_ptr))


def ssp_max_nz():
    return lib().ssp_max_nz()


def ssp_plan_engine(plan):
    """(layout, threads per workgroup, FFT length) of the plan's fused march."""
    v, t, p = C.c_int(), C.c_int(), C.c_int()
    _check(lib().ssp_plan_engine(plan, C.byref(v), C.byref(t), C.byref(p)))
    return v.value, t.value, p.value


def ssp_pade_coefficients(sigma, pade_order, alpha=0.0):
    p = int(pade_order)
    b, g, d = (np.zeros(2 * p) for _ in range(3))
    Cc, d0 = np.zeros(2), np.zeros(2)
    _check(lib().ssp_pade_coefficients(float(sigma), p, float(alpha), _dp(b), _dp(g), _dp(Cc),
                                       _dp(d0), _dp(d)))
    cx = lambda a: a[0::2] + 1j * a[1::2]
    return {"b": cx(b), "g": cx(g), "C": complex(Cc[0], Cc[1]), "d0": complex(d0[0], d0[1]),
            "d": cx(d)}


def ssp_plan_info(plan, p):
    sig, k0 = C.c_double(), C.c_double()
    b, g, d = (np.zeros(2 * p) for _ in range(3))
    Cc, d0 = np.zeros(2), np.zeros(2)
    _check(lib().ssp_plan_info(plan, C.byref(sig), C.byref(k0), _dp(b), _dp(g), _dp(Cc),
                               _dp(d0), _dp(d)))
    cx = lambda a: a[0::2] + 1j * a[1::2]
    return {"sigma": sig.value, "k0": k0.value, "b": cx(b), "g": cx(g),
            "C": complex(Cc[0], Cc[1]), "d0": complex(d0[0], d0[1]), "d": cx(d)}


def ssp_set_profile(plan, step0, nsteps, c):
    c = np.ascontiguousarray(c, dtype=np.float64)
    return _check(lib().ssp_set_profile(plan, int(step0), int(nsteps), _dp(c)))


def ssp_set_profile_analytic(plan, munk=(1500.0, 0.00737, 1300.0), eddy=None):
    e = ssp_env()
    e.munk_c1, e.munk_eps, e.munk_z1 = munk
    if eddy is not None:
        e.eddy_amp, e.eddy_r0, e.eddy_rr, e.eddy_z0, e.eddy_rz = eddy
    return _check(lib().ssp_set_profile_analytic(plan, C.byref(e)))


def ssp_set_absorber(plan, eta=None):
    """eta: [Nz] imaginary part of the potential (None removes the absorber)."""
    arr = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
    return _check(lib().ssp_set_absorber(plan, _dp(arr)))


def ssp_modal_starter(plan, c, zs, max_modes=0):
    """Normal-mode starters for sound speed c [Nz] and source depth(s) zs (a number or a
    sequence): (psi0 complex128 [Nz] or [nsrc][Nz], kappa [modes])."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    nz = c.shape[0]
    single = np.ndim(zs) == 0
    zarr = np.ascontiguousarray(np.atleast_1d(zs), dtype=np.float64)
    out = np.zeros((len(zarr), nz), dtype=np.complex128)
    kap = np.zeros(nz, dtype=np.float64)
    n = C.c_int(0)
    _check(lib().ssp_modal_starter(plan, _dp(c), len(zarr), _dp(zarr), int(max_modes),
                                   _dp(out.view(np.float64)), _dp(kap), C.byref(n)))
    return (out[0] if single else out), kap[:n.value].copy()


def ssp_set_field(plan, psi0, nz):
    return _check(lib().ssp_set_field(plan, _dp(_c128(psi0, nz))))


def ssp_get_field(plan, nz):
    out = np.zeros(nz, dtype=np.complex128)
    _check(lib().ssp_get_field(plan, _dp(out.view(np.float64))))
    return out


def ssp_count_outputs(plan, nsteps):
    return lib().ssp_count_outputs(plan, int(nsteps))


def ssp_march(plan, nz, psi0, nsteps, want_field=True, want_tl=True):
    """Returns (status, field [nout][Nz] complex128 or None, tl [nout][Nz] or None, stats).
    A starter (psi0) is installed first with ssp_set_field, which resets the step counter,
    so that the output count is known before the march."""
    if psi0 is not None:
        ssp_set_field(plan, psi0, nz)
    nout = ssp_count_outputs(plan, nsteps)
    fld = np.zeros((nout, nz), dtype=np.complex128) if want_field else None
    tl = np.zeros((nout, nz), dtype=np.float32) if want_tl else None
    st = ssp_stats()
    status = _check(lib().ssp_march(plan, None, int(nsteps),
                                    None if fld is None else _dp(fld.view(np.float64)),
                                    _fp(tl), C.byref(st)))
    return status, fld, tl, st.as_dict()


def _check_batch(st, stats):
    """A batch's returned status: a failure that belongs to individual plans (their own
    status in the statistics, e.g. one diverged series) is returned with the other plans'
    results; any other failure raises."""
    if st < 0 and not any(x.status == st for x in stats):
        _check(st)
    return st


def ssp_march_batch(plans, nzs, nsteps, want_field=True, want_tl=True):
    """Returns (status, fields, tls, stats); per-plan failures (status < 0 in that plan's
    stats) do not raise."""
    n = len(plans)
    arr = (_VP * n)(*plans)
    fl = [np.zeros((ssp_count_outputs(pl, nsteps), nz), dtype=np.complex128) if want_field else None
          for pl, nz in zip(plans, nzs)]
    tl = [np.zeros((ssp_count_outputs(pl, nsteps), nz), dtype=np.float32) if want_tl else None
          for pl, nz in zip(plans, nzs)]
    fptr = (_DP * n)(*[None if f is None else _dp(f.view(np.float64)) for f in fl])
    tptr = (_FP * n)(*[None if t is None else _fp(t) for t in tl])
    stats = (ssp_stats * n)()
    status = _check_batch(lib().ssp_march_batch(arr, n, int(nsteps), fptr, tptr, stats), stats)
    return status, fl, tl, [s.as_dict() for s in stats]


def ssp_march_batch_steps(plans, nzs, nsteps, want_field=True, want_tl=True):
    """Like ssp_march_batch with a step count per plan (nsteps: sequence of n ints)."""
    n = len(plans)
    arr = (_VP * n)(*plans)
    ns = (C.c_int * n)(*[int(k) for k in nsteps])
    fl = [np.zeros((ssp_count_outputs(pl, k), nz), dtype=np.complex128) if want_field else None
          for pl, nz, k in zip(plans, nzs, nsteps)]
    tl = [np.zeros((ssp_count_outputs(pl, k), nz), dtype=np.float32) if want_tl else None
          for pl, nz, k in zip(plans, nzs, nsteps)]
    fptr = (_DP * n)(*[None if f is None else _dp(f.view(np.float64)) for f in fl])
    tptr = (_FP * n)(*[None if t is None else _fp(t) for t in tl])
    stats = (ssp_stats * n)()
    status = _check_batch(lib().ssp_march_batch_steps(arr, n, ns, fptr, tptr, stats), stats)
    return status, fl, tl, [s.as_dict() for s in stats]


def ssp_march_batch_async(plans, nsteps, d_tl=None):
    """nsteps: sequence of n ints; d_tl: sequence of n device addresses (0/None: no TL rows)
    or None."""
    n = len(plans)
    arr = (_VP * n)(*plans)
    ns = (C.c_int * n)(*[int(k) for k in nsteps])
    tptr = None if d_tl is None else (_FP * n)(*[C.cast(C.c_void_p(a), _FP) if a else None for a in d_tl])
    return _check(lib().ssp_march_batch_async(arr, n, ns, tptr))


def ssp_batch_stats(plans):
    """(worst status, [stats dict per plan]); per-plan failures do not raise."""
    n = len(plans)
    arr = (_VP * n)(*plans)
    stats = (ssp_stats * n)()
    st = _check_batch(lib().ssp_batch_stats(arr, n, stats), stats)
    return st, [s.as_dict() for s in stats]


def ssp_plan_contraction(plan, p, iterations=40):
    """(bound [p], estimate [p]) of every Pade factor's Neumann operator."""
    b, e = np.zeros(p), np.zeros(p)
    _check(lib().ssp_plan_contraction(plan, int(iterations), _dp(b), _dp(e)))
    return b, e


def ssp_march_device(plan, B, d_psi, d_step, nsteps, d_tl=0, d_stats=0):
    return _check(lib().ssp_march_device(plan, int(B), d_psi, d_step, int(nsteps), d_tl or None,
                                         d_stats or None))


def ssp_march_device_noalloc(plan, B, d_psi, d_step, nsteps, d_tl=0, d_stats=0):
    return _check(lib().ssp_march_device_noalloc(plan, int(B), d_psi, d_step, int(nsteps), d_tl or None,
                                                 d_stats or None))


def ssp_to_sine(plan, B, d_phys, d_sine):
    return _check(lib().ssp_to_sine(plan, int(B), d_phys, d_sine))


def ssp_from_sine(plan, B, d_sine, d_step, d_phys):
    return _check(lib().ssp_from_sine(plan, int(B), d_sine, d_step, d_phys))


def ssp_dst_device(plan, B, d_in, d_out):
    return _check(lib().ssp_dst_device(plan, int(B), d_in, d_out))


def ssp_dst_dense_device(plan, B, d_in, d_out):
    return _check(lib().ssp_dst_dense_device(plan, int(B), d_in, d_out))


def ssp_max_dense_nz():
    return lib().ssp_max_dense_nz()


def ssp_status_string(s):
    return lib().ssp_status_string(int(s)).decode()


def ssp_last_error():
    return lib().ssp_last_error().decode()


def header_functions(header_path=None):
    """Names of the functions declared in include/ssp.h."""
    import re
    header_path = header_path or os.path.join(os.path.dirname(_HERE), "include", "ssp.h")
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ssp_[a-z_]+)\s*\(", txt)))
