"""ctypes binding of librh (names follow include/rh.h).

Argument marshalling only: every computation happens in the library.  The
binding refuses to run without the built library (no fallback).  PyTorch is
imported first so that the library shares PyTorch's HIP runtime (device
pointers and streams from PyTorch are then valid in librh).
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "librh.so"

RH_OK, RH_EINVAL, RH_ENOMEM, RH_ENOCONV, RH_ESINGULAR, RH_ESTATE, RH_EDEVICE, RH_EBUSY = (
    0, -1, -2, -3, -4, -5, -6, -7)
RH_FP64, RH_FP32_REFINED = 0, 1

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class rh_network_desc(ctypes.Structure):
    _fields_ = [
        ("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32), ("n_gen", ctypes.c_int32),
        ("br_from", _i32p), ("br_to", _i32p),
        ("br_r", _f64p), ("br_x", _f64p), ("br_b", _f64p),
        ("bus_type", _i32p),
        ("Pd", _f64p), ("Qd", _f64p),
        ("gen_bus", _i32p),
        ("Pg", _f64p), ("Vg", _f64p), ("c2", _f64p), ("c1", _f64p), ("c0", _f64p),
    ]


class rh_tile(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32), ("dirs_per_group", ctypes.c_int32),
        ("block_rows", ctypes.c_int32), ("wave_steps", ctypes.c_int32),
        ("ms_per_hessian", ctypes.c_double), ("source", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


RH_TUNE_MEASURE, RH_TUNE_NO_CACHE = 1, 2


class rh_report(ctypes.Structure):
    _fields_ = [
        ("n_x", ctypes.c_int32), ("n_p", ctypes.c_int32),
        ("nnz_gx", ctypes.c_int64), ("nnz_l", ctypes.c_int64), ("nnz_u", ctypes.c_int64),
        ("levels_l", ctypes.c_int32), ("levels_u", ctypes.c_int32),
        ("steps_l", ctypes.c_int32), ("steps_u", ctypes.c_int32),
        ("newton_iters", ctypes.c_int32),
        ("newton_resid", ctypes.c_double),
        ("last_k", ctypes.c_int32), ("last_launches", ctypes.c_int32),
        ("dirs_per_group", ctypes.c_int32),
        ("last_kernel_ms", ctypes.c_double),
        ("phase_us", ctypes.c_double * 7),
        ("tile", rh_tile * 2),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_us"] = list(self.phase_us)
        d["tile"] = [t.as_dict() for t in self.tile]
        return d


class rh_tracking_info(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double), ("tries", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("grad_inf", ctypes.c_double), ("step_inf", ctypes.c_double),
        ("ms_gradient", ctypes.c_double), ("ms_hessian", ctypes.c_double),
        ("ms_solve", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class RhError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"librh status {status}: {msg}")
        self.status = status


_lib = None

# symbol -> (restype, argtypes)
_SIGS = {
    "rh_context_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "rh_context_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rh_context_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rh_context_set_refinement": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rh_context_set_refinement_tol": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "rh_network_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rh_network_desc),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "rh_network_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rh_network_dims": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p]),
    "rh_network_index_maps": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p, _i32p, _i32p]),
    "rh_set_parameters": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_get_parameters": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_set_loads": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p]),
    "rh_set_initial_state": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_solve_powerflow": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                          _i32p, _f64p]),
    "rh_solve_powerflow_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                                 _i32p, _f64p]),
    "rh_get_factors": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p]),
    "rh_get_state": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_objective": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_condition_estimate": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_reduced_gradient": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "rh_hvp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, ctypes.c_int64, _f64p,
                              ctypes.c_int64, ctypes.c_int]),
    "rh_hvp_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_void_p]),
    "rh_hvp_device_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int, ctypes.c_void_p]),
    "rh_reduced_hessian": (ctypes.c_int, [ctypes.c_void_p, _f64p, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_int]),
    "rh_reduced_hessian_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                                 ctypes.c_void_p]),
    "rh_hvp_batch_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p), _i32p,
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_int64), _i32p,
                                           ctypes.c_int, ctypes.c_void_p]),
    "rh_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p), _i32p,
                                       ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_int64), _i32p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "rh_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rh_batch_info": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i32p, _i32p]),
    "rh_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rh_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                   ctypes.POINTER(rh_tile)]),
    "rh_get_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(rh_tile)]),
    "rh_last_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rh_report)]),
    "rh_network_device_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "rh_refinement_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, _i32p, _f64p,
                                            _i32p]),
    "rh_context_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rh_report)]),
    "rh_reduced_gradient_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rh_cholesky_solve_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int32, ctypes.c_void_p, _i32p]),
    "rh_tracking_step_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                               _f64p, _f64p, _f64p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.POINTER(rh_tracking_info)]),
    "rh_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rh_last_error": (ctypes.c_char_p, []),
}

SYMBOLS = tuple(_SIGS)


def load(path: str | os.PathLike | None = None):
    """Load librh (after PyTorch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime librh links against)

    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"librh is not built ({p}); run __graft_entry__.build()")
    lib = ctypes.CDLL(str(p))
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != RH_OK:
        raise RhError(status, _lib.rh_last_error().decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a: np.ndarray, typ):
    return a.ctypes.data_as(typ)


def _ld(t) -> int:
    """Leading dimension of a row-major (k, ld) device tensor (PyTorch reports
    an arbitrary stride for a dimension of size one)."""
    return max(int(t.stride(0)), int(t.shape[1])) if t.shape[0] == 1 else int(t.stride(0))


# ---- thin wrappers with the C names -------------------------------------
def rh_context_create(device: int) -> ctypes.c_void_p:
    lib = load()
    h = ctypes.c_void_p()
    _check(lib.rh_context_create(int(device), ctypes.byref(h)))
    return h


def rh_context_destroy(ctx) -> None:
    _check(load().rh_context_destroy(ctx))


def rh_context_set_timing(ctx, level) -> None:
    """0 off, 1 launch events, 2 also in-kernel phase stamps."""
    _check(load().rh_context_set_timing(ctx, int(level)))


def rh_context_set_refinement(ctx, steps: int) -> None:
    _check(load().rh_context_set_refinement(ctx, int(steps)))


def rh_context_set_refinement_tol(ctx, tol: float) -> None:
    _check(load().rh_context_set_refinement_tol(ctx, float(tol)))


def rh_network_create(ctx, grid):
    """``grid`` carries the description arrays (see rh_network_desc)."""
    lib = load()
    keep = dict(
        br_from=_i32(grid.br_from), br_to=_i32(grid.br_to), br_r=_f64(grid.br_r),
        br_x=_f64(grid.br_x), br_b=_f64(grid.br_b), bus_type=_i32(grid.bus_type),
        Pd=_f64(grid.Pd), Qd=_f64(grid.Qd), gen_bus=_i32(grid.gen_bus), Pg=_f64(grid.Pg),
        Vg=_f64(grid.Vg), c2=_f64(grid.c2), c1=_f64(grid.c1), c0=_f64(grid.c0),
    )
    d = rh_network_desc()
    d.n_bus = int(grid.n_bus)
    d.n_branch = int(keep["br_from"].size)
    d.n_gen = int(keep["gen_bus"].size)
    for k, v in keep.items():
        setattr(d, k, _p(v, _i32p if v.dtype == np.int32 else _f64p))
    h = ctypes.c_void_p()
    _check(lib.rh_network_create(ctx, ctypes.byref(d), ctypes.byref(h)))
    return h


def rh_network_destroy(net) -> None:
    _check(load().rh_network_destroy(net))


def rh_network_dims(net):
    nx, np_ = ctypes.c_int32(), ctypes.c_int32()
    _check(load().rh_network_dims(net, ctypes.byref(nx), ctypes.byref(np_)))
    return nx.value, np_.value


def rh_network_index_maps(net):
    nx, npar = rh_network_dims(net)
    xb, xk = np.zeros(nx, np.int32), np.zeros(nx, np.int32)
    pb, pk = np.zeros(npar, np.int32), np.zeros(npar, np.int32)
    _check(load().rh_network_index_maps(net, _p(xb, _i32p), _p(xk, _i32p), _p(pb, _i32p),
                                        _p(pk, _i32p)))
    return xb, xk, pb, pk


def rh_set_parameters(net, p) -> None:
    p = _f64(p)
    _check(load().rh_set_parameters(net, _p(p, _f64p)))


def rh_get_parameters(net) -> np.ndarray:
    _, npar = rh_network_dims(net)
    p = np.zeros(npar)
    _check(load().rh_get_parameters(net, _p(p, _f64p)))
    return p


def rh_set_loads(net, Pd, Qd) -> None:
    Pd, Qd = _f64(Pd), _f64(Qd)
    _check(load().rh_set_loads(net, _p(Pd, _f64p), _p(Qd, _f64p)))


def rh_set_initial_state(net, x0=None) -> None:
    if x0 is None:
        _check(load().rh_set_initial_state(net, None))
    else:
        x0 = _f64(x0)
        _check(load().rh_set_initial_state(net, _p(x0, _f64p)))


def rh_solve_powerflow(net, tol=1e-13, max_iter=30):
    it, r = ctypes.c_int32(), ctypes.c_double()
    _check(load().rh_solve_powerflow(net, float(tol), int(max_iter), ctypes.byref(it),
                                     ctypes.byref(r)))
    return it.value, r.value


def rh_solve_powerflow_device(net, tol=1e-13, max_iter=30):
    it, r = ctypes.c_int32(), ctypes.c_double()
    _check(load().rh_solve_powerflow_device(net, float(tol), int(max_iter), ctypes.byref(it),
                                            ctypes.byref(r)))
    return it.value, r.value


def rh_get_factors(net, nnz_l, nnz_u):
    lv, uv = np.zeros(nnz_l), np.zeros(nnz_u)
    _check(load().rh_get_factors(net, _p(lv, _f64p), _p(uv, _f64p)))
    return lv, uv


def rh_get_state(net) -> np.ndarray:
    nx, _ = rh_network_dims(net)
    x = np.zeros(nx)
    _check(load().rh_get_state(net, _p(x, _f64p)))
    return x


def rh_objective(net) -> float:
    f = ctypes.c_double()
    _check(load().rh_objective(net, ctypes.byref(f)))
    return f.value


def rh_condition_estimate(net) -> float:
    c = ctypes.c_double()
    _check(load().rh_condition_estimate(net, ctypes.byref(c)))
    return c.value


def rh_reduced_gradient(net) -> np.ndarray:
    _, npar = rh_network_dims(net)
    g = np.zeros(npar)
    _check(load().rh_reduced_gradient(net, _p(g, _f64p)))
    return g


def rh_hvp(net, W, prec=RH_FP64) -> np.ndarray:
    _, npar = rh_network_dims(net)
    W = np.asfortranarray(W, dtype=np.float64)
    if W.ndim != 2 or W.shape[0] != npar:
        raise ValueError("W must be n_p x k")
    k = W.shape[1]
    HW = np.zeros((npar, k), order="F")
    _check(load().rh_hvp(net, k, _p(W, _f64p), npar, _p(HW, _f64p), npar, int(prec)))
    return HW


def rh_hvp_device(net, k, dW_ptr, ldw, dHW_ptr, ldhw, prec=RH_FP64, stream=None) -> None:
    _check(load().rh_hvp_device(net, int(k), ctypes.c_void_p(dW_ptr), int(ldw),
                                ctypes.c_void_p(dHW_ptr), int(ldhw), int(prec),
                                ctypes.c_void_p(stream or 0)))


def rh_hvp_device_noalloc(net, k, dW_ptr, ldw, dHW_ptr, ldhw, prec=RH_FP64, stream=None) -> None:
    _check(load().rh_hvp_device_noalloc(net, int(k), ctypes.c_void_p(dW_ptr), int(ldw),
                                        ctypes.c_void_p(dHW_ptr), int(ldhw), int(prec),
                                        ctypes.c_void_p(stream or 0)))


def rh_reduced_hessian(net, k_block=0, prec=RH_FP64) -> np.ndarray:
    _, npar = rh_network_dims(net)
    H = np.zeros((npar, npar), order="F")
    _check(load().rh_reduced_hessian(net, _p(H, _f64p), npar, int(k_block), int(prec)))
    return H


def rh_reduced_hessian_device(net, dH_ptr, ldh, k_block=0, prec=RH_FP64, stream=None) -> None:
    _check(load().rh_reduced_hessian_device(net, ctypes.c_void_p(dH_ptr), int(ldh), int(k_block),
                                            int(prec), ctypes.c_void_p(stream or 0)))


def rh_hvp_batch_device(ctx, nets, ks, dWs, ldws, dHWs, ldhws, identity_from=None,
                        prec=RH_FP64, stream=None) -> None:
    n = len(nets)
    arr_v = ctypes.c_void_p * n
    arr_l = ctypes.c_int64 * n
    kk = np.ascontiguousarray(ks, dtype=np.int32)
    idf = None if identity_from is None else np.ascontiguousarray(identity_from, dtype=np.int32)
    _check(load().rh_hvp_batch_device(
        ctx, n, arr_v(*[nn.value if isinstance(nn, ctypes.c_void_p) else nn for nn in nets]),
        _p(kk, _i32p), arr_v(*[w or None for w in dWs]), arr_l(*ldws), arr_v(*dHWs),
        arr_l(*ldhws), None if idf is None else _p(idf, _i32p), int(prec),
        ctypes.c_void_p(stream or 0)))


def rh_batch_create(ctx, nets, ks, dWs, ldws, dHWs, ldhws, identity_from=None, prec=RH_FP64):
    n = len(nets)
    arr_v = ctypes.c_void_p * n
    arr_l = ctypes.c_int64 * n
    kk = np.ascontiguousarray(ks, dtype=np.int32)
    idf = None if identity_from is None else np.ascontiguousarray(identity_from, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(load().rh_batch_create(
        ctx, n, arr_v(*[nn.value if isinstance(nn, ctypes.c_void_p) else nn for nn in nets]),
        _p(kk, _i32p), arr_v(*[w or None for w in dWs]), arr_l(*ldws), arr_v(*dHWs), arr_l(*ldhws),
        None if idf is None else _p(idf, _i32p), int(prec), ctypes.byref(h)))
    return h


def rh_batch_launch(batch, stream=None) -> None:
    _check(load().rh_batch_launch(batch, ctypes.c_void_p(stream or 0)))


def rh_batch_info(batch):
    c, g, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().rh_batch_info(batch, ctypes.byref(c), ctypes.byref(g), ctypes.byref(d)))
    return {"dirs_per_group": c.value, "workgroups": g.value, "directions": d.value}


def rh_batch_destroy(batch) -> None:
    _check(load().rh_batch_destroy(batch))


def rh_autotune(net, prec=RH_FP64, flags=0) -> dict:
    t = rh_tile()
    _check(load().rh_autotune(net, int(prec), int(flags), ctypes.byref(t)))
    return t.as_dict()


def rh_get_tile(net, prec=RH_FP64) -> dict:
    t = rh_tile()
    _check(load().rh_get_tile(net, int(prec), ctypes.byref(t)))
    return t.as_dict()


def rh_context_report(ctx) -> dict:
    r = rh_report()
    _check(load().rh_context_report(ctx, ctypes.byref(r)))
    return r.as_dict()


def rh_last_report(net) -> dict:
    r = rh_report()
    _check(load().rh_last_report(net, ctypes.byref(r)))
    return r.as_dict()


def rh_network_device_bytes(net, prec=RH_FP64):
    """(resident bytes, launch scratch bytes per direction) of a network."""
    r, d = ctypes.c_int64(), ctypes.c_int64()
    _check(load().rh_network_device_bytes(net, int(prec), ctypes.byref(r), ctypes.byref(d)))
    return r.value, d.value


def rh_refinement_report(net, n: int) -> dict:
    """Per-column backward errors and correction counts of the last refined call."""
    bz, bp = np.zeros(n), np.zeros(n)
    kz, kp = np.zeros(n, np.int32), np.zeros(n, np.int32)
    _check(load().rh_refinement_report(net, int(n), _p(bz, _f64p), _p(kz, _i32p), _p(bp, _f64p),
                                       _p(kp, _i32p)))
    return {"berr_z": bz, "steps_z": kz, "berr_psi": bp, "steps_psi": kp}


def rh_reduced_gradient_device(net, dgrad_ptr, stream=None) -> None:
    _check(load().rh_reduced_gradient_device(net, dgrad_ptr, stream))


def rh_cholesky_solve_device(ctx, n, dA_ptr, lda, dB_ptr, ldb, nrhs, stream=None) -> int:
    """Returns -1, or raises RhError (RH_ESINGULAR) whose .failed_col is the
    column whose leading minor is not positive definite."""
    bad = ctypes.c_int32(-1)
    s = load().rh_cholesky_solve_device(ctx, int(n), dA_ptr, int(lda), dB_ptr, int(ldb), int(nrhs),
                                        stream, ctypes.byref(bad))
    if s != RH_OK:
        e = RhError(s, _lib.rh_last_error().decode())
        e.failed_col = bad.value
        raise e
    return bad.value


def rh_tracking_step_device(net, k_block=0, shift=0.0, lo=None, hi=None, ramp=None, dd_ptr=None,
                            stream=None) -> dict:
    arrs = [None if a is None else _f64(a) for a in (lo, hi, ramp)]
    ptrs = [None if a is None else _p(a, _f64p) for a in arrs]
    info = rh_tracking_info()
    _check(load().rh_tracking_step_device(net, int(k_block), float(shift), *ptrs, dd_ptr, stream,
                                          ctypes.byref(info)))
    return info.as_dict()


def rh_status_string(s: int) -> str:
    return load().rh_status_string(int(s)).decode()


def rh_last_error() -> str:
    return load().rh_last_error().decode()


# ---- convenience object ---------------------------------------------------
class Context:
    def __init__(self, device: int = 0):
        self.h = rh_context_create(device)
        self.device = device

    def set_timing(self, level=1):
        rh_context_set_timing(self.h, int(level))

    def set_refinement(self, steps: int):
        rh_context_set_refinement(self.h, steps)

    def set_refinement_tol(self, tol: float):
        rh_context_set_refinement_tol(self.h, tol)

    def report(self):
        return rh_context_report(self.h)

    def cholesky_solve_device(self, A, B, stream=None):
        """A: torch float64 CUDA tensor (n, n) whose row j is column j of the
        matrix (only entries A[j, i] with i >= j are read; they receive L);
        B: (nrhs, n), row q a right-hand side, overwritten by the solution."""
        n = A.shape[0]
        return rh_cholesky_solve_device(self.h, n, A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                                        B.shape[0], stream)

    def hvp_batch_device(self, nets, Ws, HWs, stream=None, prec=RH_FP64):
        """nets: Network objects; Ws/HWs: torch float64 CUDA tensors (k_i, n_p_i)."""
        rh_hvp_batch_device(self.h, [n.h for n in nets], [W.shape[0] for W in Ws],
                            [W.data_ptr() for W in Ws], [_ld(W) for W in Ws],
                            [H.data_ptr() for H in HWs], [_ld(H) for H in HWs], None, prec,
                            stream)

    def batch(self, nets, Ws, HWs, prec=RH_FP64):
        """A recorded batched launch over torch float64 CUDA tensors (k_i, n_p_i)."""
        return Batch(self, nets, Ws, HWs, prec)

    def close(self):
        if self.h:
            rh_context_destroy(self.h)
            self.h = None


class Batch:
    """rh_batch: the batched launch recorded once, replayed by launch()."""

    def __init__(self, ctx, nets, Ws, HWs, prec=RH_FP64):
        self.keep = (list(nets), list(Ws), list(HWs))  # the bound buffers stay alive
        self.h = rh_batch_create(ctx.h, [n.h for n in nets], [W.shape[0] for W in Ws],
                                 [W.data_ptr() for W in Ws], [_ld(W) for W in Ws],
                                 [H.data_ptr() for H in HWs], [_ld(H) for H in HWs], None, prec)

    def launch(self, stream=None):
        rh_batch_launch(self.h, stream)

    def info(self):
        return rh_batch_info(self.h)

    def close(self):
        if self.h:
            rh_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    """One network handle; methods mirror the C calls."""

    def __init__(self, ctx: Context, grid):
        self.ctx = ctx
        self.h = rh_network_create(ctx.h, grid)
        self.n_x, self.n_p = rh_network_dims(self.h)
        v0 = getattr(grid, "v0", None)
        if v0 is not None:  # Newton starts at angles 0 and the grid's magnitude guess
            xb, xk, _, _ = rh_network_index_maps(self.h)
            x0 = np.where(xk == 1, np.asarray(v0, dtype=np.float64)[xb], 0.0)
            rh_set_initial_state(self.h, x0)

    def close(self):
        if self.h:
            rh_network_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    index_maps = lambda self: rh_network_index_maps(self.h)  # noqa: E731
    set_parameters = lambda self, p: rh_set_parameters(self.h, p)  # noqa: E731
    get_parameters = lambda self: rh_get_parameters(self.h)  # noqa: E731
    set_loads = lambda self, Pd, Qd: rh_set_loads(self.h, Pd, Qd)  # noqa: E731
    set_initial_state = lambda self, x0=None: rh_set_initial_state(self.h, x0)  # noqa: E731
    solve = lambda self, tol=1e-13, max_iter=30: rh_solve_powerflow(self.h, tol, max_iter)  # noqa
    state = lambda self: rh_get_state(self.h)  # noqa: E731
    solve_device = lambda self, tol=1e-13, max_iter=30: rh_solve_powerflow_device(self.h, tol, max_iter)  # noqa

    def factors(self):
        """(L values, U values) of the solved operating point (see rh_get_factors)."""
        r = self.report()
        return rh_get_factors(self.h, r["nnz_l"], r["nnz_u"])
    objective = lambda self: rh_objective(self.h)  # noqa: E731
    condition_estimate = lambda self: rh_condition_estimate(self.h)  # noqa: E731
    reduced_gradient = lambda self: rh_reduced_gradient(self.h)  # noqa: E731
    hvp = lambda self, W, prec=RH_FP64: rh_hvp(self.h, W, prec)  # noqa: E731
    reduced_hessian = lambda self, k_block=0, prec=RH_FP64: rh_reduced_hessian(self.h, k_block, prec)  # noqa
    report = lambda self: rh_last_report(self.h)  # noqa: E731
    refinement_report = lambda self, n: rh_refinement_report(self.h, n)  # noqa: E731
    device_bytes = lambda self, prec=RH_FP64: rh_network_device_bytes(self.h, prec)  # noqa: E731
    autotune = lambda self, prec=RH_FP64, flags=0: rh_autotune(self.h, prec, flags)  # noqa: E731
    tile = lambda self, prec=RH_FP64: rh_get_tile(self.h, prec)  # noqa: E731

    def hvp_device(self, W, HW, stream=None, prec=RH_FP64):
        """W, HW: torch float64 CUDA tensors of shape (k, n_p) (row j = direction j)."""
        k = W.shape[0]
        rh_hvp_device(self.h, k, W.data_ptr(), _ld(W), HW.data_ptr(), _ld(HW), prec, stream)

    def hvp_device_noalloc(self, W, HW, stream=None, prec=RH_FP64):
        """As hvp_device, with the library's fixed scratch (no allocation)."""
        k = W.shape[0]
        rh_hvp_device_noalloc(self.h, k, W.data_ptr(), _ld(W), HW.data_ptr(), _ld(HW), prec, stream)

    def reduced_hessian_device(self, H, k_block=0, stream=None, prec=RH_FP64):
        """H: torch float64 CUDA tensor (n_p, n_p); row j receives column j of the Hessian."""
        rh_reduced_hessian_device(self.h, H.data_ptr(), _ld(H), k_block, prec, stream)

    def reduced_gradient_device(self, g, stream=None):
        """g: torch float64 CUDA tensor of n_p values."""
        rh_reduced_gradient_device(self.h, g.data_ptr(), stream)

    def tracking_step_device(self, k_block=0, shift=0.0, lo=None, hi=None, ramp=None, d=None,
                             stream=None):
        """One tracking update; d (optional torch float64 CUDA tensor, n_p)
        receives the step.  Returns the rh_tracking_info figures."""
        return rh_tracking_step_device(self.h, k_block, shift, lo, hi, ramp,
                                       None if d is None else d.data_ptr(), stream)
