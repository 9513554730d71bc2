"""Python binding of libite, the MI355X (gfx950) implicit imaginary-time
evolution library for matrix product states.

Every function here marshals arguments for the C entry point of the same name
declared in ``include/ite.h`` and raises ``IteError`` on a non-zero status.
All computation happens in the HIP library; there is no Python or CPU fallback.
PyTorch only provides device memory (its caching allocator) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libite.so")

ITE_OK, ITE_EINVAL, ITE_ENOMEM, ITE_EDEVICE, ITE_ESTATE, ITE_ENONFINITE = 0, -1, -2, -3, -4, -5
SCHEME_TRAP, SCHEME_BE, SCHEME_GL = 0, 1, 2
SHIFT_FIXED, SHIFT_TRACK = 0, 1
PREC_FP64, PREC_FP32_IR, PREC_BF16_IR = 0, 1, 2
GUESS_PSI, GUESS_B = 0, 1
RHS_PROJECT, RHS_MPS = 0, 1
FLAG_BUDGET_EXHAUSTED, FLAG_BREAKDOWN, FLAG_REFINE_LIMIT = 1, 2, 4


class IteError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class ite_allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("user", C.c_void_p)]


class ite_step_opts(C.Structure):
    _fields_ = [("scheme", C.c_int), ("shift_mode", C.c_int), ("shift", C.c_double),
                ("chi_max", C.c_int), ("cutoff", C.c_double), ("tie_rel", C.c_double),
                ("krylov_dim", C.c_int), ("max_cycles", C.c_int), ("tol_loc", C.c_double),
                ("nsweeps", C.c_int), ("precision", C.c_int), ("max_refine", C.c_int),
                ("tol_refine", C.c_double), ("init_guess", C.c_int), ("gl_nodes", C.c_int),
                ("rhs_mode", C.c_int)]


class ite_step_report(C.Structure):
    _fields_ = [("tau", C.c_double), ("dtau", C.c_double), ("h", C.c_double), ("shift", C.c_double),
                ("energy", C.c_double), ("norm_before", C.c_double), ("max_chi", C.c_int),
                ("flags", C.c_int), ("max_disc", C.c_double), ("sum_disc", C.c_double),
                ("max_res_rel", C.c_double), ("mean_res_rel", C.c_double),
                ("matvecs_fp64", C.c_longlong), ("matvecs_lo", C.c_longlong),
                ("ms_total", C.c_double), ("ms_rhs", C.c_double), ("ms_solve", C.c_double),
                ("ms_split", C.c_double), ("ms_env", C.c_double), ("rhs_disc", C.c_double),
                ("aux_max_chi", C.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ite_server_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("workers", C.c_int), ("max_active", C.c_int), ("mem_cap", C.c_double)]


class ite_request(C.Structure):
    _fields_ = [("L", C.c_int), ("d", C.POINTER(C.c_int)), ("w", C.POINTER(C.c_int)),
                ("W", C.POINTER(C.POINTER(C.c_double))), ("spinors", C.POINTER(C.POINTER(C.c_double))),
                ("chi_max", C.c_int), ("pad_full", C.c_int),
                ("tau0", C.c_double), ("tau1", C.c_double), ("ratio", C.c_double),
                ("opts", ite_step_opts)]


class ite_request_info(C.Structure):
    _fields_ = [("status", C.c_int), ("error", C.c_int), ("worker", C.c_int), ("n_steps", C.c_int),
                ("n_grid", C.c_int), ("tau", C.c_double), ("energy", C.c_double), ("footprint", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


REQ_PENDING, REQ_ACTIVE, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_PI = C.POINTER(C.c_int)
_PD = C.POINTER(C.c_double)
_PPD = C.POINTER(C.POINTER(C.c_double))

# name -> (restype, argtypes); mirrors include/ite.h
_SIGNATURES = {
    "ite_version": (C.c_char_p, []),
    "ite_default_opts": (None, [C.POINTER(ite_step_opts)]),
    "ite_ctx_create": (_I, [_I, _P, C.POINTER(ite_allocator), C.POINTER(_P)]),
    "ite_ctx_destroy": (_I, [_P]),
    "ite_last_error": (C.c_char_p, [_P]),
    "ite_ctx_profile": (_I, [_P, _I]),
    "ite_ctx_profile_read": (_I, [_P, C.POINTER(C.c_longlong), _PD, _PD]),
    "ite_ctx_profile_kernel": (_I, [_P, _I, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong), _PD, _PD, _PD]),
    "ite_mpo_load": (_I, [_P, _I, _PI, _PI, _PPD, C.POINTER(_P)]),
    "ite_mpo_destroy": (_I, [_P]),
    "ite_mps_create": (_I, [_P, _I, _PI, _PPD, _I, _I, C.POINTER(_P)]),
    "ite_mps_load": (_I, [_P, _I, _PI, _PI, _PPD, _I, C.POINTER(_P)]),
    "ite_mps_export": (_I, [_P, _PI, _PPD]),
    "ite_mps_destroy": (_I, [_P]),
    "ite_mps_get_tau": (_I, [_P, _PD]),
    "ite_mps_set_tau": (_I, [_P, _D]),
    "ite_imag_step": (_I, [_P, _P, _D, C.POINTER(ite_step_opts), C.POINTER(ite_step_report)]),
    "ite_evolve_loggrid": (_I, [_P, _P, _D, _D, _D, C.POINTER(ite_step_opts),
                                C.POINTER(ite_step_report), _I, _PI]),
    "ite_evolve_grid": (_I, [_P, _P, _PD, _I, C.POINTER(ite_step_opts),
                             C.POINTER(ite_step_report), _I, _PI]),
    "ite_measure_energy": (_I, [_P, _P, _PD]),
    "ite_mpo_apply": (_I, [_P, _P, _I, _D, _D, C.POINTER(_P), _PD]),
    "ite_mps_sample": (_I, [_P, _I, _I, _PD, _PI]),
    "ite_mps_sample_noalloc": (_I, [_P, _I, _I, _P, _P]),
    "ite_mps_expect_site": (_I, [_P, _I, _PD, _PD]),
    "ite_step_batch": (_I, [_P, _I, C.POINTER(_P), C.POINTER(_P), _PD, C.POINTER(C.POINTER(ite_step_opts)),
                            C.POINTER(ite_step_report), _PI]),
    "ite_ctx_set_graphs": (_I, [_P, _I]),
    "ite_ctx_batch_stats": (_I, [_P, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "ite_metts_chain": (_I, [_P, _PI, _I, _D, _D, _D, C.POINTER(ite_step_opts), _I, _PD, _I, _I, _PD, _PI, _PD,
                             _PD]),
    "ite_dmrg_sweeps": (_I, [_P, _P, _I, _I, _D, _D, _I, _I, _D, _PD, _PD, _PD, C.POINTER(C.c_longlong)]),
    "ite_mps_overlap": (_I, [_P, _P, _PD]),
    "ite_mps_norm": (_I, [_P, _PD]),
    "ite_loggrid": (_I, [_D, _D, _D, _PD, _I, _PI]),
    "ite_panel_grid": (_I, [_D, _I, _I, _PD, _I, _PI]),
    "ite_gl_coefficients": (_I, [_I, _PD, _PD, _PD, _PD, _PD]),
    "ite_debug_gemm": (_I, [_P, _I, _I, _I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _P, _I, _I]),
    "ite_debug_heff_apply": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _I, _P, _PD, _PD, _P, _P,
                                  _D, _D, _P, _I]),
    "ite_debug_heff_time": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _I, _P, _PD, _PD, _P, _P,
                                 _D, _D, _P, _I, _I, _PD]),
    "ite_debug_env_update": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _I, _P, _P, _PD, _P, _P]),
    "ite_debug_svd_split": (_I, [_P, _I, _I, _I, _I, _I, _P, _I, _D, _D, _P, _P, _PD, _PI, _PD]),
    "ite_debug_local_solve": (_I, [_P, _I, _I, _I, _I, _I, _I, _I, _P, _PD, _PD, _P, _D, _D, _P, _P,
                                   _I, _I, _D, _I, _I, _D, _P, _PI, _PD]),
    "ite_debug_mfma_probe": (_I, [_P, _I, _PD]),
    "ite_server_create": (_I, [C.POINTER(ite_server_opts), C.POINTER(_P)]),
    "ite_server_destroy": (_I, [_P]),
    "ite_server_submit": (_I, [_P, C.POINTER(ite_request), C.POINTER(C.c_longlong)]),
    "ite_server_wait": (_I, [_P, C.c_longlong, _D, C.POINTER(ite_request_info)]),
    "ite_server_info": (_I, [_P, C.c_longlong, C.POINTER(ite_request_info)]),
    "ite_server_reports": (_I, [_P, C.c_longlong, C.POINTER(ite_step_report), _I, _PI]),
    "ite_server_state": (_I, [_P, C.c_longlong, _PI, _PPD]),
    "ite_server_release": (_I, [_P, C.c_longlong]),
    "ite_server_clock": (_D, [_P]),
    "ite_server_error": (_I, [_P, C.c_longlong, C.c_char_p, _I]),
    "ite_request_footprint": (_D, [_I, _PI, _PI, _I, _I]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libite.so (built by ``paper_2606_02930_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_2606_02930_amd.build)")
    # torch first: its HIP runtime is then the one the library binds to, so
    # that a process holds one runtime whichever of the two is used first
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, ctx=None):
    if rc != ITE_OK:
        msg = load_library().ite_last_error(ctx).decode() if ctx else ""
        raise IteError(rc, msg or "error")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _ptr_array(arrays):
    arr = (C.POINTER(C.c_double) * len(arrays))()
    for i, a in enumerate(arrays):
        arr[i] = a.ctypes.data_as(_PD)
    return arr


def _ints(v):
    return (C.c_int * len(v))(*[int(x) for x in v])


# ---------------------------------------------------------------------------
# Context (device memory from torch's caching allocator on torch's stream)
# ---------------------------------------------------------------------------

@dataclass
class Ctx:
    handle: int
    device: int
    stream: object
    _keep: tuple = ()


def ite_version() -> str:
    return load_library().ite_version().decode()


def ite_default_opts(**overrides) -> ite_step_opts:
    o = ite_step_opts()
    load_library().ite_default_opts(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def ite_ctx_create(device: int = 0, stream=None, allocator: str = "torch") -> Ctx:
    """Create a context on ``device``.  stream: a torch.cuda.Stream (default:
    torch's current stream).  allocator: "torch" (caching allocator) or
    "hip" (plain hipMalloc inside the library)."""
    lib = load_library()
    import torch
    if not torch.cuda.is_available():
        raise IteError(ITE_EDEVICE, "no GPU visible to torch")
    torch.cuda.set_device(device)
    s = stream if stream is not None else torch.cuda.current_stream(device)
    keep = ()
    alloc_p = None
    if allocator == "torch":
        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, s)
            except Exception:
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        fa = ite_allocator._fields_[0][1](_alloc)
        ff = ite_allocator._fields_[1][1](_free)
        al = ite_allocator(fa, ff, None)
        keep = (fa, ff, al)
        alloc_p = C.byref(al)
    elif allocator != "hip":
        raise ValueError(allocator)
    h = _P()
    rc = lib.ite_ctx_create(device, C.c_void_p(s.cuda_stream), alloc_p, C.byref(h))
    if rc != ITE_OK:
        raise IteError(rc, "ite_ctx_create failed")
    return Ctx(h.value, device, s, keep)


def ite_ctx_destroy(ctx: Ctx) -> None:
    _check(load_library().ite_ctx_destroy(ctx.handle))


def ite_last_error(ctx: Ctx) -> str:
    return load_library().ite_last_error(ctx.handle).decode()


def ite_ctx_profile(ctx: Ctx, enable: bool) -> None:
    _check(load_library().ite_ctx_profile(ctx.handle, int(bool(enable))), ctx.handle)


def ite_ctx_profile_read(ctx: Ctx) -> tuple[int, float, float]:
    """(GEMM launches, summed device ms, summed algorithmic flops)."""
    n = C.c_longlong()
    ms = C.c_double()
    fl = C.c_double()
    _check(load_library().ite_ctx_profile_read(ctx.handle, C.byref(n), C.byref(ms), C.byref(fl)), ctx.handle)
    return n.value, ms.value, fl.value


PROBE_GEMM, PROBE_GRAM, PROBE_INNER, PROBE_ROTATE = 0, 1, 2, 3


def ite_ctx_profile_kernel(ctx: Ctx, kind: int) -> dict:
    """Launch profile of one kernel kind since the last enable: launches,
    timed launches, their summed device ms, algorithmic flops and bytes of all
    launches."""
    n, t = C.c_longlong(), C.c_longlong()
    ms, fl, by = C.c_double(), C.c_double(), C.c_double()
    _check(load_library().ite_ctx_profile_kernel(ctx.handle, int(kind), C.byref(n), C.byref(t), C.byref(ms),
                                                 C.byref(fl), C.byref(by)), ctx.handle)
    return {"launches": n.value, "timed": t.value, "ms_timed": ms.value, "flops": fl.value, "bytes": by.value}


# ---------------------------------------------------------------------------
# Hamiltonian and states
# ---------------------------------------------------------------------------

def ite_mpo_load(ctx: Ctx, Ws) -> int:
    """Ws[i]: array [w_i][w_(i+1)][d_i][d_i] (out, in)."""
    Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
    L = len(Ws)
    d = [W.shape[2] for W in Ws]
    w = [Ws[0].shape[0]] + [W.shape[1] for W in Ws]
    h = _P()
    _check(load_library().ite_mpo_load(ctx.handle, L, _ints(d), _ints(w), _ptr_array(Ws), C.byref(h)),
           ctx.handle)
    return h.value


def ite_mpo_destroy(mpo: int) -> None:
    _check(load_library().ite_mpo_destroy(mpo))


def ite_mps_create(ctx: Ctx, spinors, chi_max: int, pad_full: bool = False) -> int:
    sp = [np.ascontiguousarray(s, dtype=np.float64) for s in spinors]
    h = _P()
    _check(load_library().ite_mps_create(ctx.handle, len(sp), _ints([len(s) for s in sp]), _ptr_array(sp),
                                         int(chi_max), int(bool(pad_full)), C.byref(h)), ctx.handle)
    return h.value


def ite_mps_load(ctx: Ctx, tensors, chi_max: int) -> int:
    A = [np.ascontiguousarray(a, dtype=np.float64) for a in tensors]
    L = len(A)
    d = [a.shape[1] for a in A]
    chi = [A[0].shape[0]] + [a.shape[2] for a in A]
    h = _P()
    _check(load_library().ite_mps_load(ctx.handle, L, _ints(d), _ints(chi), _ptr_array(A), int(chi_max),
                                       C.byref(h)), ctx.handle)
    return h.value


def ite_mps_export(ctx: Ctx, psi: int, d) -> list[np.ndarray]:
    L = len(d)
    chi = (C.c_int * (L + 1))()
    lib = load_library()
    _check(lib.ite_mps_export(psi, chi, None), ctx.handle)
    out = [np.empty((chi[i], d[i], chi[i + 1])) for i in range(L)]
    _check(lib.ite_mps_export(psi, chi, _ptr_array(out)), ctx.handle)
    return out


def ite_mps_destroy(psi: int) -> None:
    _check(load_library().ite_mps_destroy(psi))


def ite_mps_get_tau(psi: int) -> float:
    t = C.c_double()
    _check(load_library().ite_mps_get_tau(psi, C.byref(t)))
    return t.value


def ite_mps_set_tau(psi: int, tau: float) -> None:
    _check(load_library().ite_mps_set_tau(psi, float(tau)))


# ---------------------------------------------------------------------------
# The method
# ---------------------------------------------------------------------------

def ite_imag_step(ctx: Ctx, psi: int, mpo: int, h: float, opts: ite_step_opts) -> dict:
    rep = ite_step_report()
    _check(load_library().ite_imag_step(psi, mpo, float(h), C.byref(opts), C.byref(rep)), ctx.handle)
    return rep.as_dict()


def ite_step_batch(ctx: Ctx, psis, mpos, hs, opts) -> tuple[list[dict], list[int]]:
    """One implicit step of every state as a batch; opts: one ite_step_opts
    or a list.  Returns (reports, statuses); raises on the first failure."""
    n = len(psis)
    if isinstance(opts, ite_step_opts):
        opts = [opts] * n
    P = (_P * n)(*psis)
    Hm = (_P * n)(*mpos)
    h = np.ascontiguousarray(hs, dtype=np.float64)
    keep = [C.pointer(o) for o in opts]
    O = (C.POINTER(ite_step_opts) * n)(*keep)
    reps = (ite_step_report * n)()
    st = (C.c_int * n)()
    rc = load_library().ite_step_batch(ctx.handle, n, P, Hm, _dptr(h), O, reps, st)
    _check(rc, ctx.handle)
    return [reps[i].as_dict() for i in range(n)], list(st)


def ite_ctx_set_graphs(ctx: Ctx, enable: bool) -> None:
    _check(load_library().ite_ctx_set_graphs(ctx.handle, int(bool(enable))), ctx.handle)


def ite_ctx_batch_stats(ctx: Ctx) -> dict:
    a, b, c = C.c_longlong(), C.c_longlong(), C.c_longlong()
    _check(load_library().ite_ctx_batch_stats(ctx.handle, C.byref(a), C.byref(b), C.byref(c)), ctx.handle)
    return {"solves": a.value, "captures": b.value, "replays": c.value}


def ite_evolve_loggrid(ctx: Ctx, psi: int, mpo: int, tau0: float, tau1: float, ratio: float,
                       opts: ite_step_opts, max_steps: int = 100000) -> list[dict]:
    n = C.c_int()
    cap = int(min(max_steps, 4096))
    reps = (ite_step_report * cap)()
    rc = load_library().ite_evolve_loggrid(psi, mpo, float(tau0), float(tau1), float(ratio), C.byref(opts),
                                           reps, cap, C.byref(n))
    _check(rc, ctx.handle)
    return [reps[i].as_dict() for i in range(min(n.value, cap))]


def ite_evolve_grid(ctx: Ctx, psi: int, mpo: int, taus, opts: ite_step_opts) -> list[dict]:
    t = np.ascontiguousarray(taus, dtype=np.float64)
    n = C.c_int()
    cap = len(t)
    reps = (ite_step_report * cap)()
    _check(load_library().ite_evolve_grid(psi, mpo, _dptr(t), len(t), C.byref(opts), reps, cap, C.byref(n)),
           ctx.handle)
    return [reps[i].as_dict() for i in range(n.value)]


def ite_dmrg_sweeps(ctx: Ctx, psi: int, mpo: int, nsweeps: int, chi_max: int, cutoff: float = 0.0,
                    tie_rel: float = 1e-10, krylov_dim: int = 10, max_cycles: int = 1, tol: float = 0.0) -> dict:
    e, res, disc, mv = C.c_double(), C.c_double(), C.c_double(), C.c_longlong()
    _check(load_library().ite_dmrg_sweeps(psi, mpo, int(nsweeps), int(chi_max), float(cutoff), float(tie_rel),
                                          int(krylov_dim), int(max_cycles), float(tol), C.byref(e), C.byref(res),
                                          C.byref(disc), C.byref(mv)), ctx.handle)
    return {"energy": e.value, "max_res_rel": res.value, "max_disc": disc.value, "matvecs": mv.value}


def ite_mps_sample(ctx: Ctx, psi: int, uniforms) -> np.ndarray:
    """uniforms [L][nsamples] in [0, 1); returns configs [nsamples][L]."""
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.ndim != 2:
        raise ValueError("uniforms must be a [L][nsamples] array")
    L, S = u.shape
    cfg = np.zeros((S, L), dtype=np.int32)
    _check(load_library().ite_mps_sample(psi, S, L, _dptr(u), cfg.ctypes.data_as(_PI)), ctx.handle)
    return cfg


def ite_mps_expect_site(ctx: Ctx, psi: int, site: int, op) -> float:
    """<psi|O_site|psi> / <psi|psi>; op [d][d] (out, in)."""
    o = np.ascontiguousarray(op, dtype=np.float64)
    out = C.c_double()
    _check(load_library().ite_mps_expect_site(psi, int(site), _dptr(o), C.byref(out)), ctx.handle)
    return out.value


def ite_metts_chain(ctx: Ctx, mpo: int, start, chi_max: int, beta: float, tau0: float, ratio: float,
                    opts: ite_step_opts, site: int, op, uniforms):
    """uniforms [nsamples][L]; returns (configs [nsamples][L], energies,
    observables)."""
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.ndim != 2:
        raise ValueError("uniforms must be a [nsamples][L] array")
    n, L = u.shape
    st = np.ascontiguousarray(start, dtype=np.int32)
    if st.shape != (L,):
        raise ValueError("start must have L entries")
    o = np.ascontiguousarray(op, dtype=np.float64)
    cfg = np.zeros((n, L), dtype=np.int32)
    en = np.zeros(n)
    ob = np.zeros(n)
    _check(load_library().ite_metts_chain(mpo, st.ctypes.data_as(_PI), int(chi_max), float(beta), float(tau0),
                                          float(ratio), C.byref(opts), int(site), _dptr(o), n, L, _dptr(u),
                                          cfg.ctypes.data_as(_PI), _dptr(en), _dptr(ob)), ctx.handle)
    return cfg, en, ob


def ite_mps_sample_noalloc(ctx: Ctx, psi: int, uniforms, configs) -> None:
    """uniforms: device tensor [L][nsamples] (float64); configs: device tensor
    [nsamples][L] (int32), written in place.  No allocation in the library."""
    if uniforms.dim() != 2 or configs.dim() != 2:
        raise ValueError("uniforms [L][nsamples] and configs [nsamples][L] must be 2-d")
    L, S = uniforms.shape
    if tuple(configs.shape) != (S, L):
        raise ValueError("configs must be [nsamples][L]")
    if not (uniforms.is_contiguous() and configs.is_contiguous()):
        raise ValueError("uniforms and configs must be contiguous")
    import torch
    if uniforms.dtype != torch.float64 or configs.dtype != torch.int32:
        raise ValueError("uniforms must be float64 and configs int32")
    _check(load_library().ite_mps_sample_noalloc(psi, S, L, _tp(uniforms), _tp(configs)), ctx.handle)


def ite_mpo_apply(ctx: Ctx, mpo: int, psi: int, chi_max: int, cutoff: float = 0.0,
                  tie_rel: float = 1e-13) -> tuple[int, float]:
    """O psi by the density-matrix product; returns (new MPS handle, largest
    discarded-weight fraction)."""
    out = _P()
    disc = C.c_double()
    _check(load_library().ite_mpo_apply(mpo, psi, int(chi_max), float(cutoff), float(tie_rel), C.byref(out),
                                        C.byref(disc)), ctx.handle)
    return out.value, disc.value


def ite_measure_energy(ctx: Ctx, psi: int, mpo: int) -> float:
    e = C.c_double()
    _check(load_library().ite_measure_energy(psi, mpo, C.byref(e)), ctx.handle)
    return e.value


def ite_mps_overlap(ctx: Ctx, a: int, b: int) -> float:
    o = C.c_double()
    _check(load_library().ite_mps_overlap(a, b, C.byref(o)), ctx.handle)
    return o.value


def ite_mps_norm(ctx: Ctx, psi: int) -> float:
    o = C.c_double()
    _check(load_library().ite_mps_norm(psi, C.byref(o)), ctx.handle)
    return o.value


def ite_loggrid(tau0: float, tau1: float, ratio: float) -> np.ndarray:
    lib = load_library()
    n = C.c_int()
    lib.ite_loggrid(float(tau0), float(tau1), float(ratio), None, 0, C.byref(n))
    if n.value <= 0:
        raise IteError(ITE_EINVAL, "ite_loggrid: bad parameters")
    out = np.empty(n.value)
    _check(lib.ite_loggrid(float(tau0), float(tau1), float(ratio), _dptr(out), n.value, C.byref(n)))
    return out


def ite_gl_coefficients(p: int) -> dict:
    """Nodes c, weights b, collocation matrix A, end weights w and r_inf of a
    p-node Gauss-Legendre panel, as the library's panel step uses them."""
    c, b, w = (np.zeros(p) for _ in range(3))
    A = np.zeros((p, p))
    r = C.c_double()
    _check(load_library().ite_gl_coefficients(int(p), _dptr(c), _dptr(b), _dptr(A), _dptr(w), C.byref(r)))
    return {"c": c, "b": b, "A": A, "w": w, "r_inf": r.value}


def ite_panel_grid(tau_max: float, P: int, n: int) -> np.ndarray:
    lib = load_library()
    m = C.c_int()
    lib.ite_panel_grid(float(tau_max), int(P), int(n), None, 0, C.byref(m))
    if m.value <= 0:
        raise IteError(ITE_EINVAL, "ite_panel_grid: bad parameters")
    out = np.empty(m.value)
    _check(lib.ite_panel_grid(float(tau_max), int(P), int(n), _dptr(out), m.value, C.byref(m)))
    return out


# ---------------------------------------------------------------------------
# Building blocks for parity tests (torch CUDA tensors in, device pointers out)
# ---------------------------------------------------------------------------

def _tp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def ite_debug_gemm(ctx: Ctx, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, Cm, ldc, D, ldd, prec=0):
    _check(load_library().ite_debug_gemm(ctx.handle, int(transA), int(transB), M, N, K, float(alpha), _tp(A), lda,
                                         _tp(B), ldb, float(beta), _tp(Cm), ldc, _tp(D), ldd, int(prec)), ctx.handle)


def ite_debug_heff_apply(ctx: Ctx, L, W1, W2, R, theta, alpha, beta, y, prec=0):
    W1 = np.ascontiguousarray(W1, dtype=np.float64)
    W2 = np.ascontiguousarray(W2, dtype=np.float64)
    Dxl, w0, Dyl = L.shape
    Dxr, w2, Dyr = R.shape
    d1, d2 = W1.shape[2], W2.shape[2]
    _check(load_library().ite_debug_heff_apply(ctx.handle, Dxl, Dyl, Dxr, Dyr, d1, d2, w0, W1.shape[1], w2,
                                               _tp(L), _dptr(W1), _dptr(W2), _tp(R), _tp(theta), float(alpha),
                                               float(beta), _tp(y), int(prec)), ctx.handle)


def ite_debug_heff_time(ctx: Ctx, L, W1, W2, R, theta, alpha, beta, y, prec=0, reps=10):
    """Mean device milliseconds of one H_eff product as a local solve runs it."""
    W1 = np.ascontiguousarray(W1, dtype=np.float64)
    W2 = np.ascontiguousarray(W2, dtype=np.float64)
    Dxl, w0, Dyl = L.shape
    Dxr, w2, Dyr = R.shape
    d1, d2 = W1.shape[2], W2.shape[2]
    ms = C.c_double(0.0)
    _check(load_library().ite_debug_heff_time(ctx.handle, Dxl, Dyl, Dxr, Dyr, d1, d2, w0, W1.shape[1], w2,
                                              _tp(L), _dptr(W1), _dptr(W2), _tp(R), _tp(theta), float(alpha),
                                              float(beta), _tp(y), int(prec), int(reps), C.byref(ms)),
           ctx.handle)
    return ms.value


def ite_debug_env_update(ctx: Ctx, direction, E, X, W, Y, Eout):
    Wn = None if W is None else np.ascontiguousarray(W, dtype=np.float64)
    if direction == 0:
        Dxa, Dya = X.shape[0], Y.shape[0]
        Dxb, Dyb = X.shape[2], Y.shape[2]
    else:
        Dxa, Dya = X.shape[2], Y.shape[2]
        Dxb, Dyb = X.shape[0], Y.shape[0]
    d = X.shape[1]
    wl, wr = (1, 1) if Wn is None else (Wn.shape[0], Wn.shape[1])
    _check(load_library().ite_debug_env_update(ctx.handle, int(direction), Dxa, Dya, Dxb, Dyb, d, wl, wr, _tp(E),
                                               _tp(X), None if Wn is None else _dptr(Wn), _tp(Y), _tp(Eout)),
           ctx.handle)


def ite_debug_svd_split(ctx: Ctx, direction, theta, chi_max, cutoff, tie_rel, A1, A2):
    Dl, d1, d2, Dr = theta.shape
    r = min(Dl * d1, d2 * Dr)
    sig = np.zeros(r)
    k = C.c_int()
    disc = C.c_double()
    _check(load_library().ite_debug_svd_split(ctx.handle, int(direction), Dl, d1, d2, Dr, _tp(theta), int(chi_max),
                                              float(cutoff), float(tie_rel), _tp(A1), _tp(A2), _dptr(sig),
                                              C.byref(k), C.byref(disc)), ctx.handle)
    return k.value, sig, disc.value


def ite_debug_local_solve(ctx: Ctx, L, W1, W2, R, alpha, beta, b, x0, x, krylov_dim=10, max_cycles=1, tol=0.0,
                          precision=0, max_refine=1, tol_refine=0.0):
    W1 = np.ascontiguousarray(W1, dtype=np.float64)
    W2 = np.ascontiguousarray(W2, dtype=np.float64)
    Dl, w0, _ = L.shape
    Dr, w2, _ = R.shape
    d1, d2 = W1.shape[2], W2.shape[2]
    mv = C.c_int()
    res = C.c_double()
    _check(load_library().ite_debug_local_solve(ctx.handle, Dl, Dr, d1, d2, w0, W1.shape[1], w2, _tp(L), _dptr(W1),
                                                _dptr(W2), _tp(R), float(alpha), float(beta), _tp(b), _tp(x0),
                                                int(krylov_dim), int(max_cycles), float(tol), int(precision),
                                                int(max_refine), float(tol_refine), _tp(x), C.byref(mv),
                                                C.byref(res)), ctx.handle)
    return mv.value, res.value


def ite_debug_mfma_probe(ctx: Ctx, kind: int = 0) -> np.ndarray:
    out = np.zeros(256)
    _check(load_library().ite_debug_mfma_probe(ctx.handle, int(kind), _dptr(out)), ctx.handle)
    return out


# ---------------------------------------------------------------------------
# Serving: many independent evolutions on one device
# ---------------------------------------------------------------------------

def ite_server_create(device: int = 0, workers: int = 4, max_active: int = 2, mem_cap: float = 200e9) -> int:
    """A server with ``workers`` host threads / streams; ``mem_cap`` bytes of
    admission budget."""
    o = ite_server_opts(int(device), int(workers), int(max_active), float(mem_cap))
    h = _P()
    _check(load_library().ite_server_create(C.byref(o), C.byref(h)))
    return h.value


def ite_server_destroy(srv: int) -> None:
    _check(load_library().ite_server_destroy(srv))


def ite_server_submit(srv: int, Ws, spinors, chi_max: int, tau0: float, tau1: float, ratio: float,
                      opts: ite_step_opts, pad_full: bool = False) -> int:
    """Queue one evolution (MPO tensors Ws as ite_mpo_load, product state as
    ite_mps_create, geometric grid as ite_evolve_loggrid); returns its id."""
    Ws = [np.ascontiguousarray(W, dtype=np.float64) for W in Ws]
    sp = [np.ascontiguousarray(x, dtype=np.float64) for x in spinors]
    L = len(Ws)
    d = _ints([W.shape[2] for W in Ws])
    w = _ints([Ws[0].shape[0]] + [W.shape[1] for W in Ws])
    req = ite_request(L, d, w, _ptr_array(Ws), _ptr_array(sp), int(chi_max), int(bool(pad_full)),
                      float(tau0), float(tau1), float(ratio), opts)
    rid = C.c_longlong()
    _check(load_library().ite_server_submit(srv, C.byref(req), C.byref(rid)))
    return rid.value


def ite_server_wait(srv: int, rid: int, timeout: float = -1.0) -> dict:
    info = ite_request_info()
    rc = load_library().ite_server_wait(srv, C.c_longlong(rid), float(timeout), C.byref(info))
    if rc not in (ITE_OK, ITE_ESTATE):
        _check(rc)
    return info.as_dict()


def ite_server_info(srv: int, rid: int) -> dict:
    info = ite_request_info()
    _check(load_library().ite_server_info(srv, C.c_longlong(rid), C.byref(info)))
    return info.as_dict()


def ite_server_reports(srv: int, rid: int) -> list[dict]:
    lib = load_library()
    n = C.c_int()
    _check(lib.ite_server_reports(srv, C.c_longlong(rid), None, 0, C.byref(n)))
    out = (ite_step_report * max(1, n.value))()
    _check(lib.ite_server_reports(srv, C.c_longlong(rid), out, n.value, C.byref(n)))
    return [out[i].as_dict() for i in range(n.value)]


def ite_server_state(srv: int, rid: int, d) -> list[np.ndarray]:
    L = len(d)
    chi = (C.c_int * (L + 1))()
    lib = load_library()
    _check(lib.ite_server_state(srv, C.c_longlong(rid), chi, None))
    out = [np.empty((chi[i], d[i], chi[i + 1])) for i in range(L)]
    _check(lib.ite_server_state(srv, C.c_longlong(rid), chi, _ptr_array(out)))
    return out


def ite_server_release(srv: int, rid: int) -> None:
    _check(load_library().ite_server_release(srv, C.c_longlong(rid)))


def ite_server_clock(srv: int) -> float:
    return load_library().ite_server_clock(srv)


def ite_server_error(srv: int, rid: int) -> str:
    buf = C.create_string_buffer(1024)
    _check(load_library().ite_server_error(srv, C.c_longlong(rid), buf, 1024))
    return buf.value.decode()


def ite_request_footprint(d, w, chi_max: int, krylov_dim: int = 10) -> float:
    return load_library().ite_request_footprint(len(d), _ints(d), _ints(w), int(chi_max), int(krylov_dim))
