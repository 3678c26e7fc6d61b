"""Python binding of the WaveHoltz C ABI (``include/wh.h``).

Argument marshalling only: every function here has the name of the C entry
point it calls and every step of the computation runs in ``libwh.so``'s HIP
kernels.  PyTorch supplies device memory (the workspace and the grid
functions) and the stream.  If the HIP library is missing the import fails;
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwh.so")

WH_OK, WH_EINVAL, WH_ENOMEM, WH_EDEVICE, WH_EUNSTABLE, WH_ENOTCONV, WH_ENONFINITE, WH_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
WH_FP64, WH_FP32_STATE = 0, 1
WH_SOLVER_FPI, WH_SOLVER_GMRES, WH_SOLVER_CG = 0, 1, 2
WH_MAX_RESTART = 4096
WH_KERNEL_AUTO, WH_KERNEL_NODE, WH_KERNEL_BLOCKED_2D, WH_KERNEL_ZCOL_3D, WH_KERNEL_BLOCKED_3D = 0, 1, 2, 3, 4
KERNEL_NAMES = {0: "auto", 1: "node", 2: "blocked_2d", 3: "zcol_3d", 4: "blocked_3d"}
KERNEL_IDS = {v: k for k, v in KERNEL_NAMES.items()}


class WhError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status)} ({status}): {message}")
        self.status = status


class wh_time_params(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("periods", ctypes.c_int32), ("dt", ctypes.c_double),
                ("omega", ctypes.c_double), ("omega_e", ctypes.c_double), ("alpha", ctypes.c_double),
                ("cfl", ctypes.c_double), ("c2max", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


WH_ITER_CALLBACK = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p)


class wh_solve_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("rtol", ctypes.c_double), ("on_iter", WH_ITER_CALLBACK),
                ("user", ctypes.c_void_p)]


class wh_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("applies", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("scaled_res", ctypes.c_double), ("cr_last", ctypes.c_double), ("cr_avg", ctypes.c_double),
                ("ecr", ctypes.c_double), ("mu_pred", ctypes.c_double), ("seconds", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("point_steps", ctypes.c_double),
                ("rel_res_recursive", ctypes.c_double), ("ritz_min", ctypes.c_double),
                ("ritz_max", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class wh_profile(ctypes.Structure):
    _fields_ = [("applies", ctypes.c_int64), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("point_steps", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_I64x3 = ctypes.c_int64 * 3
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run `python -m paper_2504_03074_amd.build`)")
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "wh_version": (ctypes.c_int32, []),
        "wh_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
        "wh_compute_time_params": (st, [ctypes.c_int32, _I64x3, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(wh_time_params)]),
        "wh_create": (st, [ctypes.POINTER(_vp), ctypes.c_int32, _vp]),
        "wh_destroy": (None, [_vp]),
        "wh_last_error": (ctypes.c_char_p, [_vp]),
        "wh_set_grid": (st, [_vp, ctypes.c_int32, _I64x3, ctypes.c_int32, ctypes.c_int32]),
        "wh_workspace_size": (st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
        "wh_bind_workspace": (st, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32]),
        "wh_set_c2": (st, [_vp, _vp, ctypes.c_int32]),
        "wh_set_c2_constant": (st, [_vp, ctypes.c_double]),
        "wh_set_source": (st, [_vp, _vp, ctypes.c_int32]),
        "wh_set_frequency": (st, [_vp, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                  ctypes.c_double]),
        "wh_get_time_params": (st, [_vp, ctypes.POINTER(wh_time_params)]),
        "wh_run_periods": (st, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
        "wh_apply": (st, [_vp, _vp, _vp, ctypes.c_int32]),
        "wh_apply_A": (st, [_vp, _vp, _vp]),
        "wh_apply_A_noalloc": (st, [_vp, _vp, _vp]),
        "wh_filter_spectrum": (st, [_vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
        "wh_solve": (st, [_vp, ctypes.POINTER(wh_solve_opts), _vp, ctypes.POINTER(wh_solve_info)]),
        "wh_solve_rhs": (st, [_vp, ctypes.POINTER(wh_solve_opts), _vp, _vp, ctypes.POINTER(wh_solve_info)]),
        "wh_solve_mixed": (st, [_vp, _vp, ctypes.POINTER(wh_solve_opts), ctypes.POINTER(wh_solve_opts), _vp,
                                ctypes.POINTER(wh_solve_info)]),
        "wh_helmholtz_residual": (st, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
        "wh_dot": (st, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
        "wh_stream_bandwidth": (st, [ctypes.c_int32, _vp, _vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                     _vp, ctypes.POINTER(ctypes.c_double)]),
        "wh_set_tuning": (st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "wh_get_tuning": (st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)]),
        "wh_profile_enable": (st, [_vp, ctypes.c_int32]),
        "wh_autotune": (st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
        "wh_profile_read": (st, [_vp, ctypes.POINTER(wh_profile)]),
        "wh_select_deflation": (st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double)]),
        "wh_deflation_workspace_size": (st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
        "wh_set_deflation": (st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _vp, ctypes.c_size_t]),
        "wh_set_implicit": (st, [_vp, ctypes.c_int32, ctypes.c_double]),
        "wh_implicit_workspace_size": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "wh_bind_implicit_workspace": (st, [_vp, _vp, ctypes.c_size_t]),
        "wh_implicit_stats": (st, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "wh_adjoint_workspace_size": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "wh_bind_adjoint_workspace": (st, [_vp, _vp, ctypes.c_size_t]),
        "wh_gradient": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "wh_solve_adjoint": (st, [_vp, ctypes.POINTER(wh_solve_opts), _vp, _vp, ctypes.POINTER(wh_solve_info)]),
        "wh_receiver_misfit": (st, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _vp]),
        "wh_batch_create": (st, [ctypes.POINTER(_vp), ctypes.c_int32, _vp]),
        "wh_batch_destroy": (None, [_vp]),
        "wh_batch_last_error": (ctypes.c_char_p, [_vp]),
        "wh_batch_add": (st, [_vp, _vp, ctypes.POINTER(ctypes.c_int32)]),
        "wh_batch_set_tuning": (st, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "wh_batch_workspace_size": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "wh_batch_finalize": (st, [_vp, _vp, ctypes.c_size_t]),
        "wh_batch_autotune": (st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
        "wh_batch_get_tuning": (st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
        "wh_batch_apply": (st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32]),
        "wh_batch_solve": (st, [_vp, ctypes.POINTER(wh_solve_opts), ctypes.POINTER(_vp),
                                ctypes.POINTER(wh_solve_info)]),
        "wh_batch_solve_rhs": (st, [_vp, ctypes.POINTER(wh_solve_opts), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                    ctypes.POINTER(wh_solve_info)]),
        "wh_batch_solve_mixed": (st, [_vp, _vp, ctypes.POINTER(wh_solve_opts), ctypes.POINTER(wh_solve_opts),
                                      ctypes.POINTER(_vp), ctypes.POINTER(wh_solve_info)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises ImportError if it was not built)."""
    return _load()


def status_name(status: int) -> str:
    return _load().wh_status_string(int(status)).decode()


def _check(ctx, status):
    if status != WH_OK:
        msg = _load().wh_last_error(ctx).decode() if ctx else ""
        raise WhError(status, msg)


def _n3(n):
    n = list(int(x) for x in n) + [0] * (3 - len(n))
    return _I64x3(*n[:3])


# --------------------------------------------------------------------------
# thin wrappers, one per C entry point
# --------------------------------------------------------------------------
def wh_version() -> int:
    return int(_load().wh_version())


def wh_status_string(status: int) -> str:
    return status_name(status)


def wh_compute_time_params(dim, n, order, c2max, omega, periods=1, cfl_frac=0.9, nt_override=0,
                           alpha=-1.0) -> wh_time_params:
    out = wh_time_params()
    st = _load().wh_compute_time_params(int(dim), _n3(n), int(order), float(c2max), float(omega), int(periods),
                                        float(cfl_frac), int(nt_override), float(alpha), ctypes.byref(out))
    if st != WH_OK:
        raise WhError(st, "wh_compute_time_params rejected its arguments")
    return out


def wh_create(device: int = 0, stream: int | None = None):
    ctx = _vp()
    st = _load().wh_create(ctypes.byref(ctx), int(device), _vp(stream) if stream else None)
    if st != WH_OK:
        raise WhError(st, f"wh_create(device={device}) failed")
    return ctx


def wh_destroy(ctx):
    _load().wh_destroy(ctx)


def wh_last_error(ctx) -> str:
    return _load().wh_last_error(ctx).decode()


def wh_set_grid(ctx, dim, n, order, precision=WH_FP64):
    _check(ctx, _load().wh_set_grid(ctx, int(dim), _n3(n), int(order), int(precision)))


def wh_workspace_size(ctx, restart=0) -> int:
    out = ctypes.c_size_t()
    _check(ctx, _load().wh_workspace_size(ctx, int(restart), ctypes.byref(out)))
    return int(out.value)


def wh_bind_workspace(ctx, ptr: int, nbytes: int, restart=0):
    _check(ctx, _load().wh_bind_workspace(ctx, _vp(ptr), int(nbytes), int(restart)))


def wh_set_c2(ctx, ptr: int | None, on_device: bool):
    _check(ctx, _load().wh_set_c2(ctx, _vp(ptr) if ptr else None, int(bool(on_device))))


def wh_set_c2_constant(ctx, c2: float):
    _check(ctx, _load().wh_set_c2_constant(ctx, float(c2)))


def wh_set_source(ctx, ptr: int, on_device: bool):
    _check(ctx, _load().wh_set_source(ctx, _vp(ptr), int(bool(on_device))))


def wh_set_frequency(ctx, omega, periods=1, cfl_frac=0.9, nt_override=0, alpha=-1.0):
    _check(ctx, _load().wh_set_frequency(ctx, float(omega), int(periods), float(cfl_frac), int(nt_override),
                                         float(alpha)))


def wh_get_time_params(ctx) -> wh_time_params:
    out = wh_time_params()
    _check(ctx, _load().wh_get_time_params(ctx, ctypes.byref(out)))
    return out


def wh_run_periods(ctx, w0: int, with_forcing: bool, w_final: int | None, filtered: int | None):
    _check(ctx, _load().wh_run_periods(ctx, _vp(w0), int(bool(with_forcing)), _vp(w_final) if w_final else None,
                                       _vp(filtered) if filtered else None))


def wh_apply(ctx, v: int, out: int, with_forcing: bool):
    _check(ctx, _load().wh_apply(ctx, _vp(v), _vp(out), int(bool(with_forcing))))


def wh_apply_A(ctx, v: int, Av: int):
    _check(ctx, _load().wh_apply_A(ctx, _vp(v), _vp(Av)))


def wh_filter_spectrum(ctx, c2: float):
    """(min, max) of 1 - beta_d over the sine modes for constant c2, and the
    wave numbers of the mode closest to resonance."""
    lo, hi, k = ctypes.c_double(), ctypes.c_double(), (ctypes.c_int32 * 3)()
    _check(ctx, _load().wh_filter_spectrum(ctx, float(c2), ctypes.byref(lo), ctypes.byref(hi), k))
    return float(lo.value), float(hi.value), tuple(int(x) for x in k)


def wh_apply_A_noalloc(ctx, v: int, Av: int):
    _check(ctx, _load().wh_apply_A_noalloc(ctx, _vp(v), _vp(Av)))


def wh_solve(ctx, opts: wh_solve_opts, v: int) -> tuple[int, wh_solve_info]:
    """Returns (status, info); WH_ENOTCONV is returned, not raised, so the
    caller can inspect the last iterate."""
    info = wh_solve_info()
    st = _load().wh_solve(ctx, ctypes.byref(opts), _vp(v), ctypes.byref(info))
    if st not in (WH_OK, WH_ENOTCONV):
        _check(ctx, st)
    return st, info


def wh_solve_rhs(ctx, opts: wh_solve_opts, b: int, v: int) -> tuple[int, wh_solve_info]:
    info = wh_solve_info()
    st = _load().wh_solve_rhs(ctx, ctypes.byref(opts), _vp(b), _vp(v), ctypes.byref(info))
    if st not in (WH_OK, WH_ENOTCONV):
        _check(ctx, st)
    return st, info


def wh_solve_mixed(hi, lo, outer: wh_solve_opts, inner: wh_solve_opts, v: int) -> tuple[int, wh_solve_info]:
    info = wh_solve_info()
    st = _load().wh_solve_mixed(hi, lo, ctypes.byref(outer), ctypes.byref(inner), _vp(v), ctypes.byref(info))
    if st not in (WH_OK, WH_ENOTCONV):
        _check(hi, st)
    return st, info


def make_opts(method="cg", rtol=1e-8, maxit=1000, restart=2, callback=None):
    """wh_solve_opts (and the ctypes callback object that must outlive the call)."""
    opts = wh_solve_opts()
    opts.method = {"gmres": WH_SOLVER_GMRES, "fpi": WH_SOLVER_FPI, "cg": WH_SOLVER_CG}[method]
    opts.restart = int(restart)
    opts.maxit = int(maxit)
    opts.flags = 0
    opts.rtol = float(rtol)
    cb = None
    if callback is not None:
        cb = WH_ITER_CALLBACK(lambda k, r, u: callback(k, r))
        opts.on_iter = cb
    opts.user = None
    return opts, cb


def wh_helmholtz_residual(ctx, u: int, res: int | None) -> float:
    rel = ctypes.c_double()
    _check(ctx, _load().wh_helmholtz_residual(ctx, _vp(u), _vp(res) if res else None, ctypes.byref(rel)))
    return float(rel.value)


def wh_dot(ctx, x: int, y: int) -> float:
    out = ctypes.c_double()
    _check(ctx, _load().wh_dot(ctx, _vp(x), _vp(y), ctypes.byref(out)))
    return float(out.value)


def wh_stream_bandwidth(kind: int, src: int, dst: int, nbytes: int, groups: int = 0, reps: int = 10,
                        stream: int = 0) -> float:
    """Average milliseconds per launch of the library's streaming kernel
    (kind 0 copy, 1 read, 2 write) over `nbytes` of device memory, or (kind
    3) of the FP32 blocked pass's per-node traffic over nbytes / 36 nodes."""
    ms = ctypes.c_double()
    st = _load().wh_stream_bandwidth(int(kind), _vp(src) if src else None, _vp(dst) if dst else None,
                                     int(nbytes), int(groups), int(reps), _vp(stream) if stream else None,
                                     ctypes.byref(ms))
    if st != 0:
        raise WhError(st, "wh_stream_bandwidth rejected its arguments or a launch failed")
    return float(ms.value)


def wh_set_tuning(ctx, kernel=WH_KERNEL_AUTO, kblock=0, tile=0):
    _check(ctx, _load().wh_set_tuning(ctx, int(kernel), int(kblock), int(tile)))


def wh_get_tuning(ctx):
    """(kernel, kblock, tile, owned_x, owned_y) actually used."""
    out = [ctypes.c_int32() for _ in range(5)]
    _check(ctx, _load().wh_get_tuning(ctx, *[ctypes.byref(o) for o in out]))
    return tuple(int(o.value) for o in out)


def wh_autotune(ctx, applies=3):
    """(kernel, kblock, tile, ms per application) chosen."""
    k, kb, t, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(ctx, _load().wh_autotune(ctx, int(applies), ctypes.byref(k), ctypes.byref(kb), ctypes.byref(t),
                                    ctypes.byref(ms)))
    return int(k.value), int(kb.value), int(t.value), float(ms.value)


def wh_profile_enable(ctx, enable=True):
    _check(ctx, _load().wh_profile_enable(ctx, int(bool(enable))))


def wh_profile_read(ctx) -> wh_profile:
    out = wh_profile()
    _check(ctx, _load().wh_profile_read(ctx, ctypes.byref(out)))
    return out

def wh_select_deflation(ctx, count: int, dim: int):
    """(modes as a list of dim-tuples, predicted deflated rate)."""
    arr = (ctypes.c_int32 * max(count * dim, 1))()
    mu = ctypes.c_double()
    _check(ctx, _load().wh_select_deflation(ctx, int(count), arr, ctypes.byref(mu)))
    return [tuple(arr[q * dim + m] for m in range(dim)) for q in range(count)], mu.value


def wh_deflation_workspace_size(ctx, count: int) -> int:
    out = ctypes.c_size_t()
    _check(ctx, _load().wh_deflation_workspace_size(ctx, int(count), ctypes.byref(out)))
    return out.value


def wh_set_deflation(ctx, modes, ptr, nbytes):
    modes = list(modes)
    dim = len(modes[0]) if modes else 1
    arr = (ctypes.c_int32 * max(len(modes) * dim, 1))(*[int(k) for m in modes for k in m])
    _check(ctx, _load().wh_set_deflation(ctx, arr, len(modes), _vp(ptr) if ptr else None, int(nbytes)))


def wh_set_implicit(ctx, nits: int, inner_rtol: float):
    _check(ctx, _load().wh_set_implicit(ctx, int(nits), float(inner_rtol)))


def wh_implicit_workspace_size(ctx) -> int:
    out = ctypes.c_size_t()
    _check(ctx, _load().wh_implicit_workspace_size(ctx, ctypes.byref(out)))
    return out.value


def wh_bind_implicit_workspace(ctx, ptr, nbytes):
    _check(ctx, _load().wh_bind_implicit_workspace(ctx, _vp(ptr) if ptr else None, int(nbytes)))


def wh_implicit_stats(ctx) -> dict:
    steps, iters = ctypes.c_int64(), ctypes.c_int64()
    mx, lv = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, _load().wh_implicit_stats(ctx, ctypes.byref(steps), ctypes.byref(iters), ctypes.byref(mx),
                                          ctypes.byref(lv)))
    return dict(steps=steps.value, inner_iters=iters.value, max_inner=mx.value, levels=lv.value)


def wh_adjoint_workspace_size(ctx) -> int:
    out = ctypes.c_size_t()
    _check(ctx, _load().wh_adjoint_workspace_size(ctx, ctypes.byref(out)))
    return out.value


def wh_bind_adjoint_workspace(ctx, ptr, nbytes):
    _check(ctx, _load().wh_bind_adjoint_workspace(ctx, _vp(ptr) if ptr else None, int(nbytes)))


def wh_gradient(ctx, v: int, lam: int, grad_c2, grad_f, grad_v):
    _check(ctx, _load().wh_gradient(ctx, _vp(v), _vp(lam), _vp(grad_c2) if grad_c2 else None,
                                    _vp(grad_f) if grad_f else None, _vp(grad_v) if grad_v else None))


def wh_solve_adjoint(ctx, opts: wh_solve_opts, g: int, lam: int) -> tuple[int, wh_solve_info]:
    info = wh_solve_info()
    st = _load().wh_solve_adjoint(ctx, ctypes.byref(opts), _vp(g), _vp(lam), ctypes.byref(info))
    if st not in (WH_OK, WH_ENOTCONV):
        _check(ctx, st)
    return st, info


def wh_receiver_misfit(ctx, u: int, idx: int, data: int, nrec: int, grad) -> float:
    J = ctypes.c_double()
    _check(ctx, _load().wh_receiver_misfit(ctx, _vp(u), _vp(idx) if idx else None, _vp(data) if data else None,
                                           int(nrec), ctypes.byref(J), _vp(grad) if grad else None))
    return J.value


def _bcheck(batch, status):
    if status != WH_OK:
        msg = _load().wh_batch_last_error(batch).decode() if batch else ""
        raise WhError(status, msg)


def _ptrs(ptrs):
    arr = (_vp * max(len(ptrs), 1))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def wh_batch_create(device: int = 0, stream: int | None = None):
    b = _vp()
    st = _load().wh_batch_create(ctypes.byref(b), int(device), _vp(stream) if stream else None)
    if st != WH_OK:
        raise WhError(st, f"wh_batch_create(device={device}) failed")
    return b


def wh_batch_destroy(batch):
    _load().wh_batch_destroy(batch)


def wh_batch_last_error(batch) -> str:
    return _load().wh_batch_last_error(batch).decode()


def wh_batch_add(batch, ctx) -> int:
    idx = ctypes.c_int32()
    _bcheck(batch, _load().wh_batch_add(batch, ctx, ctypes.byref(idx)))
    return idx.value


def wh_batch_set_tuning(batch, kblock=0, tile=0):
    _bcheck(batch, _load().wh_batch_set_tuning(batch, int(kblock), int(tile)))


def wh_batch_workspace_size(batch) -> int:
    out = ctypes.c_size_t()
    _bcheck(batch, _load().wh_batch_workspace_size(batch, ctypes.byref(out)))
    return out.value


def wh_batch_finalize(batch, ptr: int, nbytes: int):
    _bcheck(batch, _load().wh_batch_finalize(batch, _vp(ptr), nbytes))


def wh_batch_autotune(batch, applies=3):
    k, t, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _bcheck(batch, _load().wh_batch_autotune(batch, int(applies), ctypes.byref(k), ctypes.byref(t),
                                             ctypes.byref(ms)))
    return k.value, t.value, ms.value


def wh_batch_get_tuning(batch):
    k, t = ctypes.c_int32(), ctypes.c_int32()
    _bcheck(batch, _load().wh_batch_get_tuning(batch, ctypes.byref(k), ctypes.byref(t)))
    return k.value, t.value


def wh_batch_apply(batch, v: list, out: list, with_forcing: bool):
    _bcheck(batch, _load().wh_batch_apply(batch, _ptrs(v), _ptrs(out), int(bool(with_forcing))))


def wh_batch_solve(batch, opts: wh_solve_opts, x: list) -> tuple[int, list]:
    """Returns (status, [wh_solve_info per problem]); WH_ENOTCONV is returned."""
    infos = (wh_solve_info * max(len(x), 1))()
    st = _load().wh_batch_solve(batch, ctypes.byref(opts), _ptrs(x), infos)
    if st not in (WH_OK, WH_ENOTCONV):
        _bcheck(batch, st)
    return st, [infos[i] for i in range(len(x))]


def wh_batch_solve_rhs(batch, opts: wh_solve_opts, b: list, x: list) -> tuple[int, list]:
    """Batched CG with given right-hand sides; (status, infos)."""
    infos = (wh_solve_info * max(len(x), 1))()
    st = _load().wh_batch_solve_rhs(batch, ctypes.byref(opts), _ptrs(b), _ptrs(x), infos)
    if st not in (WH_OK, WH_ENOTCONV):
        _bcheck(batch, st)
    return st, [infos[i] for i in range(len(x))]


def wh_batch_solve_mixed(hi, lo, outer: wh_solve_opts, inner: wh_solve_opts, x: list) -> tuple[int, list]:
    """Batched residual correction (FP64 hi, FP32-state lo); (status, infos)."""
    infos = (wh_solve_info * max(len(x), 1))()
    st = _load().wh_batch_solve_mixed(hi, lo, ctypes.byref(outer), ctypes.byref(inner), _ptrs(x), infos)
    if st not in (WH_OK, WH_ENOTCONV):
        _bcheck(hi, st)
    return st, [infos[i] for i in range(len(x))]


# --------------------------------------------------------------------------
# convenience objects over torch tensors
# --------------------------------------------------------------------------
class Solver:
    """One WaveHoltz problem on one GPU, with torch-owned device memory.

    Grid functions are float64 torch tensors of node shape
    (n_y+1, n_x+1) or (n_z+1, n_y+1, n_x+1) on the solver's device.
    """

    def __init__(self, dim, n, order=2, precision="fp64", restart=0, device=0, stream=None):
        import torch
        self._torch = torch
        if isinstance(n, int):
            n = (n,) * dim
        self.dim, self.n, self.order = int(dim), tuple(int(x) for x in n), int(order)
        self.precision = WH_FP32_STATE if precision in ("fp32", WH_FP32_STATE) else WH_FP64
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = wh_create(device, self.stream.cuda_stream)
        wh_set_grid(self.ctx, self.dim, self.n, self.order, self.precision)
        self.restart = int(restart)
        nbytes = wh_workspace_size(self.ctx, self.restart)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        wh_bind_workspace(self.ctx, self.workspace.data_ptr(), nbytes, self.restart)
        self._keep = []

    @property
    def shape(self):
        return tuple(k + 1 for k in reversed(self.n))

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                wh_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def _dev(self, a, name):
        t = self._torch
        if not isinstance(a, t.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if a.dtype != t.float64 or tuple(a.shape) != self.shape or not a.is_contiguous() or a.device != self.device:
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {self.shape} on {self.device}")
        return a.data_ptr()

    def _any(self, a, name):
        """(pointer, on_device, keepalive) for a torch tensor or numpy array."""
        t = self._torch
        if isinstance(a, t.Tensor):
            if a.device.type == "cuda":
                return self._dev(a, name), True, a
            a = a.detach().numpy()
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != self.shape:
            raise ValueError(f"{name} must have shape {self.shape}")
        return a.ctypes.data, False, a

    def new(self):
        return self._torch.zeros(self.shape, dtype=self._torch.float64, device=self.device)

    def set_c2(self, c2):
        if isinstance(c2, (int, float)):
            wh_set_c2_constant(self.ctx, float(c2))
        else:
            ptr, on_dev, keep = self._any(c2, "c2")
            wh_set_c2(self.ctx, ptr, on_dev)

    def set_source(self, f):
        ptr, on_dev, keep = self._any(f, "f")
        wh_set_source(self.ctx, ptr, on_dev)

    def set_frequency(self, omega, periods=1, cfl_frac=0.9, nt=0, alpha=-1.0):
        wh_set_frequency(self.ctx, omega, periods, cfl_frac, nt, alpha)
        return self.time_params

    @property
    def time_params(self):
        return wh_get_time_params(self.ctx).as_dict()

    def set_tuning(self, kernel="auto", kblock=0, tile=0):
        """kernel: "auto", "node", "blocked_2d", "zcol_3d" or "blocked_3d"."""
        wh_set_tuning(self.ctx, KERNEL_IDS[kernel] if isinstance(kernel, str) else int(kernel), kblock, tile)

    def tuning(self):
        """dict(kernel, kblock, tile, owned=(x, y)) actually used."""
        k, kb, t, ox, oy = wh_get_tuning(self.ctx)
        return dict(kernel=KERNEL_NAMES[k], kblock=kb, tile=t, owned=(ox, oy))

    def autotune(self, applies=3):
        """Time every kernel variant on this problem and keep the fastest."""
        k, kb, t, ms = wh_autotune(self.ctx, applies)
        return dict(kernel=KERNEL_NAMES[k], kblock=kb, tile=t, ms_per_apply=ms)

    def apply(self, v, with_forcing=True, out=None):
        out = self.new() if out is None else out
        wh_apply(self.ctx, self._dev(v, "v"), self._dev(out, "out"), with_forcing)
        return out

    def apply_A(self, v, out=None):
        out = self.new() if out is None else out
        wh_apply_A(self.ctx, self._dev(v, "v"), self._dev(out, "out"))
        return out

    def filter_spectrum(self, c2=1.0):
        """(min, max) of 1 - beta_d over the sine modes for constant c2 and the
        mode closest to resonance (host computation)."""
        return wh_filter_spectrum(self.ctx, c2)

    def apply_A_noalloc(self, v, out):
        """A v with the library's fixed device scratch (no workspace levels)."""
        wh_apply_A_noalloc(self.ctx, self._dev(v, "v"), self._dev(out, "out"))
        return out

    def run_periods(self, w0, with_forcing=True, want_final=True, want_filtered=True):
        fin = self.new() if want_final else None
        fil = self.new() if want_filtered else None
        wh_run_periods(self.ctx, self._dev(w0, "w0"), with_forcing, fin.data_ptr() if fin is not None else None,
                       fil.data_ptr() if fil is not None else None)
        return fin, fil

    def solve(self, method="gmres", rtol=1e-8, maxit=1000, restart=None, v0=None, callback=None, b=None):
        """Solve (I - S_h) v = b, b = W_h(0, f) unless given (device tensor)."""
        v = self.new() if v0 is None else v0.clone()
        opts, cb = make_opts(method, rtol, maxit, self.restart if restart is None else restart, callback)
        if b is None:
            st, info = wh_solve(self.ctx, opts, self._dev(v, "v"))
        else:
            st, info = wh_solve_rhs(self.ctx, opts, self._dev(b, "b"), self._dev(v, "v"))
        d = info.as_dict()
        d["converged"] = st == WH_OK
        return v, d

    def solve_mixed(self, lo, rtol=1e-8, maxit=50, inner_method="cg", inner_rtol=1e-3, inner_maxit=2000,
                    v0=None, callback=None):
        """Residual correction: FP64 residuals on this solver, corrections
        from `lo` (a Solver of the same problem, normally precision="fp32")."""
        v = self.new() if v0 is None else v0.clone()
        outer, cb = make_opts("cg", rtol, maxit, 2, callback)
        inner, _ = make_opts(inner_method, inner_rtol, inner_maxit, max(lo.restart, 2))
        st, info = wh_solve_mixed(self.ctx, lo.ctx, outer, inner, self._dev(v, "v"))
        d = info.as_dict()
        d["converged"] = st == WH_OK
        return v, d

    def helmholtz_residual(self, u, want_field=False):
        res = self.new() if want_field else None
        rel = wh_helmholtz_residual(self.ctx, self._dev(u, "u"), res.data_ptr() if res is not None else None)
        return (rel, res) if want_field else rel

    def dot(self, x, y):
        return wh_dot(self.ctx, self._dev(x, "x"), self._dev(y, "y"))

    # ---- deflation (constant c^2) ----
    def select_deflation(self, count):
        """The `count` slowest-converging sine modes and the deflated rate."""
        return wh_select_deflation(self.ctx, count, self.dim)

    def set_deflation(self, modes=None, count=None):
        """Deflate the given modes (list of wave-number tuples), or the
        `count` slowest ones; returns (modes, predicted deflated rate or None).
        modes=[] / count=0 clears deflation."""
        mu = None
        if modes is None:
            modes, mu = self.select_deflation(int(count or 0))
        modes = [tuple(int(k) for k in m) for m in modes]
        if not modes:
            wh_set_deflation(self.ctx, [], None, 0)
            self._defl_ws = None
            return [], mu
        need = wh_deflation_workspace_size(self.ctx, len(modes))
        self._defl_ws = self._torch.empty(need, dtype=self._torch.uint8, device=self.device)
        wh_set_deflation(self.ctx, modes, self._defl_ws.data_ptr(), need)
        return modes, mu

    # ---- implicit time stepping (2-D, FP64 state) ----
    def set_implicit(self, nits=10, rtol=1e-12):
        """Implicit steps (nits >= 5 per period, multigrid-preconditioned CG to
        rtol per step), or explicit again with nits = 0.  Call set_frequency
        afterwards."""
        wh_set_implicit(self.ctx, nits, rtol)
        if nits == 0:
            wh_bind_implicit_workspace(self.ctx, None, 0)
            self._imp_ws = None
            return
        need = wh_implicit_workspace_size(self.ctx)
        ws = getattr(self, "_imp_ws", None)
        if ws is None or ws.numel() < need:
            self._imp_ws = self._torch.empty(need, dtype=self._torch.uint8, device=self.device)
        wh_bind_implicit_workspace(self.ctx, self._imp_ws.data_ptr(), self._imp_ws.numel())

    def implicit_stats(self):
        return wh_implicit_stats(self.ctx)

    # ---- discrete adjoint (FP64 state) ----
    def _adjoint_ready(self):
        need = wh_adjoint_workspace_size(self.ctx)
        ws = getattr(self, "_adj_ws", None)
        if ws is None or ws.numel() < need:
            self._adj_ws = self._torch.empty(need, dtype=self._torch.uint8, device=self.device)
            wh_bind_adjoint_workspace(self.ctx, self._adj_ws.data_ptr(), need)

    def gradient(self, v, lam, c2=True, f=True, v_grad=False):
        """Sensitivities of lam . W_h(v, f) to c^2, f and v (dict of tensors)."""
        self._adjoint_ready()
        out = {}
        if c2:
            out["c2"] = self.new()
        if f:
            out["f"] = self.new()
        if v_grad:
            out["v"] = self.new()
        p = lambda k: out[k].data_ptr() if k in out else None
        wh_gradient(self.ctx, self._dev(v, "v"), self._dev(lam, "lam"), p("c2"), p("f"), p("v"))
        return out

    def solve_adjoint(self, g, method="cg", rtol=1e-8, maxit=1000, restart=None, lam0=None):
        """lam with (I - S_h)^T lam = g (device tensor)."""
        lam = self.new() if lam0 is None else lam0.clone()
        opts, _ = make_opts(method, rtol, maxit, self.restart if restart is None else restart)
        st, info = wh_solve_adjoint(self.ctx, opts, self._dev(g, "g"), self._dev(lam, "lam"))
        d = info.as_dict()
        d["converged"] = st == WH_OK
        return lam, d

    def receiver_misfit(self, u, idx, data, want_grad=True):
        """(J, dJ/du) for flat receiver indices idx (int64 device tensor)."""
        t = self._torch
        if idx.dtype != t.int64 or idx.device != self.device or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 tensor on the solver's device")
        if data.dtype != t.float64 or data.device != self.device or data.numel() != idx.numel():
            raise ValueError("data must be a float64 tensor on the solver's device, one value per receiver")
        data = data.contiguous()
        g = self.new() if want_grad else None
        J = wh_receiver_misfit(self.ctx, self._dev(u, "u"), idx.data_ptr(), data.data_ptr(), idx.numel(),
                               g.data_ptr() if g is not None else None)
        return J, g

    def profile_enable(self, enable=True):
        wh_profile_enable(self.ctx, enable)

    def profile_read(self):
        return wh_profile_read(self.ctx).as_dict()


class Batch:
    """Independent 2-D problems (configured Solvers with restart >= 2, same
    order and precision) advanced together: one launch per blocked pass of
    all problems, the CG iteration captured in a HIP graph."""

    def __init__(self, solvers, kblock=0, tile=0, device=0, stream=None):
        import torch
        self._torch = torch
        self.solvers = list(solvers)
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.batch = wh_batch_create(device, self.stream.cuda_stream)
        for s in self.solvers:
            wh_batch_add(self.batch, s.ctx)
        if kblock or tile:
            wh_batch_set_tuning(self.batch, kblock, tile)
        nbytes = wh_batch_workspace_size(self.batch)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        wh_batch_finalize(self.batch, self.workspace.data_ptr(), nbytes)

    def __len__(self):
        return len(self.solvers)

    def __del__(self):
        b = getattr(self, "batch", None)
        if b:
            try:
                wh_batch_destroy(b)
            except Exception:
                pass
            self.batch = None

    def autotune(self, applies=3):
        """Time every (kblock, tile) choice on the batch and keep the fastest."""
        k, t, ms = wh_batch_autotune(self.batch, applies)
        return dict(kblock=k, tile=t, ms_per_apply=ms)

    def tuning(self):
        k, t = wh_batch_get_tuning(self.batch)
        return dict(kblock=k, tile=t)

    def apply(self, vs, with_forcing=True, outs=None):
        outs = [s.new() for s in self.solvers] if outs is None else outs
        wh_batch_apply(self.batch, [s._dev(v, "v") for s, v in zip(self.solvers, vs)],
                       [s._dev(o, "out") for s, o in zip(self.solvers, outs)], with_forcing)
        return outs

    def solve(self, rtol=1e-8, maxit=1000, x0=None, callback=None, b=None):
        """CG on every problem (right-hand sides W_h(0, f_i), or the device
        tensors b); returns (list of x, list of info dicts)."""
        xs = [s.new() for s in self.solvers] if x0 is None else [x.clone() for x in x0]
        opts, cb = make_opts("cg", rtol, maxit, 2, callback)
        xp = [s._dev(x, "x") for s, x in zip(self.solvers, xs)]
        if b is None:
            st, infos = wh_batch_solve(self.batch, opts, xp)
        else:
            st, infos = wh_batch_solve_rhs(self.batch, opts, [s._dev(bb, "b") for s, bb in zip(self.solvers, b)], xp)
        out = []
        for inf in infos:
            d = inf.as_dict()
            d["converged"] = d["rel_res"] <= rtol
            out.append(d)
        return xs, out

    def solve_mixed(self, lo, rtol=1e-8, maxit=50, inner_rtol=1e-3, inner_maxit=5000, x0=None, callback=None):
        """Residual correction: FP64 residuals on this batch (FP64 solvers),
        corrections by the batched CG on `lo`, a Batch of the same problems
        with FP32 state; returns (list of x, list of info dicts)."""
        xs = [s.new() for s in self.solvers] if x0 is None else [x.clone() for x in x0]
        outer, cb = make_opts("cg", rtol, maxit, 2, callback)
        inner, _ = make_opts("cg", inner_rtol, inner_maxit, 2)
        st, infos = wh_batch_solve_mixed(self.batch, lo.batch, outer, inner,
                                         [s._dev(x, "x") for s, x in zip(self.solvers, xs)])
        out = []
        for inf in infos:
            d = inf.as_dict()
            d["converged"] = d["rel_res"] <= rtol
            out.append(d)
        return xs, out
