"""ctypes binding of ``libgpr.so`` (the C-ABI declared in include/gpr.h).

Argument marshalling only: every function here has the name of its C entry point,
converts torch tensors to device pointers and raises ``GprError`` on a non-zero
status.  All arithmetic happens in the HIP kernels behind the C-ABI; if the
library is not built, importing the entry points fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpr.so")

GPR_OK, GPR_ERR_ARG, GPR_ERR_SHAPE, GPR_ERR_NOT_SPD, GPR_ERR_OOM, GPR_ERR_HIP, GPR_ERR_WORKSPACE = range(7)
GPR_FP64, GPR_FP32, GPR_BF16X3, GPR_BF16X6 = range(4)
PRECISIONS = {"fp64": GPR_FP64, "fp32": GPR_FP32, "bf16x3": GPR_BF16X3, "bf16x6": GPR_BF16X6}


class GprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpr error {code}: {msg}")
        self.code = code


KERNELS = {"se": 0, "matern12": 1, "matern32": 2, "matern52": 3}


class GprHyper(ctypes.Structure):
    _fields_ = [("lengthscale", ctypes.c_double), ("signal_var", ctypes.c_double), ("noise_var", ctypes.c_double),
                ("kernel", ctypes.c_int32)]


_vp, _i64, _int, _dbl, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "gpr_version": ([], _int),
    "gpr_last_error": ([], ctypes.c_char_p),
    "gpr_init": ([_i64, _i64, _i64, _int], _int),
    "gpr_set_lookahead": ([_int], _int),
    "gpr_set_schedule": ([_int], _int),
    "gpr_dag_check": ([_i64, _i64, _int, _i64, _dbl, ctypes.POINTER(_i64)], _int),
    "gpr_tiles_bytes": ([_i64, _i64, _int, ctypes.POINTER(_sz)], _int),
    "gpr_workspace_size": ([_i64, _i64, _i64, _i64, _int, ctypes.POINTER(_sz)], _int),
    "gpr_assemble": ([_vp, _i64, _i64, GprHyper, _i64, _int, _vp, _vp], _int),
    "gpr_cholesky": ([_vp, _i64, _i64, _int, _vp, _sz, ctypes.POINTER(_i64), _vp], _int),
    "gpr_solve": ([_vp, _vp, _i64, _i64, GprHyper, _i64, _int, _vp, _vp, _int, _vp, _sz, _vp], _int),
    "gpr_predict": ([_vp, _i64, _vp, _i64, _i64, GprHyper, _vp, _vp, _vp, _sz, _vp], _int),
    "gpr_predict_noalloc": ([_vp, _i64, _vp, _i64, _i64, GprHyper, _vp, _vp, _vp], _int),
    "gpr_predict_var": ([_vp, _i64, _vp, _i64, _i64, GprHyper, _vp, _i64, _int, _int, _int, _vp, _vp, _sz, _vp], _int),
    "gpr_nlml": ([_vp, _i64, _i64, _int, _vp, _vp, _vp, _vp], _int),
    "gpr_nlml_grad": ([_vp, _i64, _i64, GprHyper, _vp, _i64, _int, _vp, ctypes.POINTER(_int), _vp, _vp, _sz, _vp], _int),
    "gpr_optimize": ([_vp, _vp, _i64, _i64, _i64, _int, _int, ctypes.POINTER(_dbl), ctypes.POINTER(_int), _int, _dbl, _dbl,
                      _dbl, _dbl, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _vp, _vp, _sz, _vp], _int),
    "gpr_cholesky_census": ([_i64, ctypes.POINTER(_i64)], _int),
    "gpr_cholesky_schedule_check": ([_i64, _i64, _int, _i64, ctypes.POINTER(_i64)], _int),
    "gpr_timing_enable": ([_int], _int),
    "gpr_split_bf16x3": ([_vp, _i64, _vp, _vp, _vp, _vp], _int),
    "gpr_stats_workspace": ([_i64, ctypes.POINTER(_sz)], _int),
    "gpr_summary_stats": ([_vp, _vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _sz, _vp], _int),
    "gpr_mlp_nparams": ([], _int),
    "gpr_mlp_workspace": ([_i64, ctypes.POINTER(_sz)], _int),
    "gpr_mlp_forward": ([_vp, _vp, _i64, _vp, _vp, _sz, _vp], _int),
    "gpr_mlp_loss_grad": ([_vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp], _int),
    "gpr_mlp_train_step": ([_vp, _vp, _vp, _int, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, _vp, _vp, _sz, _vp], _int),
    "gpr_timing_read": ([_int, ctypes.POINTER(_i64), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)], _int),
}
_EXTRA_SIGS = {}

_lib = None


def load():
    """The loaded library (built in-tree by ``paper_2505_00136_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_00136_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in {**_SIGS, **_EXTRA_SIGS}.items():
            fn = getattr(lib, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def exported_symbols():
    lib = load()
    return [n for n in list(_SIGS) + list(_EXTRA_SIGS) if hasattr(lib, n)]


def _check(rc: int):
    if rc != GPR_OK:
        raise GprError(rc, load().gpr_last_error().decode())


def _ptr(x):
    """Device (or host) address of a tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _kernel(k) -> int:
    return KERNELS[k] if isinstance(k, str) else int(k)


def hyper(h) -> GprHyper:
    """(l, nu, sigma^2) or (l, nu, sigma^2, kernel), or an object with those attributes;
    kernel is a name of KERNELS or its number (default: squared exponential)."""
    if isinstance(h, GprHyper):
        return h
    if hasattr(h, "lengthscale"):
        return GprHyper(h.lengthscale, h.signal_var, h.noise_var, _kernel(getattr(h, "kernel", 0)))
    if len(h) == 4:
        l, nu, s2, k = h
        return GprHyper(float(l), float(nu), float(s2), _kernel(k))
    l, nu, s2 = h
    return GprHyper(float(l), float(nu), float(s2), 0)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ---------------------------------------------------------------- entry points
def gpr_version() -> int:
    return load().gpr_version()


def gpr_init(n=0, m=0, tile=1, prec="fp64"):
    _check(load().gpr_init(n, m, tile, _prec(prec)))


def gpr_set_lookahead(on: bool):
    _check(load().gpr_set_lookahead(int(on)))


SCHEDULES = {"stream": 0, "lookahead": 1, "device": 2}


def gpr_set_schedule(mode):
    """'stream', 'lookahead' (the default) or 'device' (the task graph on the device)."""
    _check(load().gpr_set_schedule(SCHEDULES[mode] if isinstance(mode, str) else int(mode)))


DAG_REPORT = ("tasks", "items", "edges", "items_run", "violations", "aborted", "timed_out", "threads_returned",
              "unordered_conflicts")


def gpr_dag_check(n, tile, threads, withhold=-1, limit_ms=1000.0):
    r = (_i64 * 9)()
    _check(load().gpr_dag_check(n, tile, threads, withhold, limit_ms, r))
    return dict(zip(DAG_REPORT, list(r)))


def gpr_tiles_bytes(n, tile, prec) -> int:
    out = _sz()
    _check(load().gpr_tiles_bytes(n, tile, _prec(prec), ctypes.byref(out)))
    return out.value


def gpr_workspace_size(n, m, d, tile, prec) -> int:
    out = _sz()
    _check(load().gpr_workspace_size(n, m, d, tile, _prec(prec), ctypes.byref(out)))
    return out.value


def gpr_assemble(Z, n, d, h, tile, prec, K_tiles, stream=None):
    _check(load().gpr_assemble(_ptr(Z), n, d, hyper(h), tile, _prec(prec), _ptr(K_tiles), _stream(stream)))


def gpr_cholesky(K_tiles, n, tile, prec, ws, ws_bytes, want_info=True, stream=None):
    """Returns the LAPACK-style info (0 or the 1-based failing column) when want_info."""
    info = _i64(0)
    rc = load().gpr_cholesky(_ptr(K_tiles), n, tile, _prec(prec), _ptr(ws), ws_bytes,
                             ctypes.byref(info) if want_info else None, _stream(stream))
    if rc == GPR_ERR_NOT_SPD:
        return int(info.value)
    _check(rc)
    return int(info.value)


def gpr_solve(L_tiles, Z, n, d, h, tile, prec, y, alpha, refine_sweeps, ws, ws_bytes, stream=None):
    _check(load().gpr_solve(_ptr(L_tiles), _ptr(Z), n, d, hyper(h), tile, _prec(prec), _ptr(y), _ptr(alpha),
                            refine_sweeps, _ptr(ws), ws_bytes, _stream(stream)))


def gpr_predict(Z, n, Zs, m, d, h, alpha, mean, ws, ws_bytes, stream=None):
    _check(load().gpr_predict(_ptr(Z), n, _ptr(Zs), m, d, hyper(h), _ptr(alpha), _ptr(mean), _ptr(ws), ws_bytes,
                              _stream(stream)))


def gpr_predict_noalloc(Z, n, Zs, m, d, h, alpha, mean, stream=None):
    _check(load().gpr_predict_noalloc(_ptr(Z), n, _ptr(Zs), m, d, hyper(h), _ptr(alpha), _ptr(mean),
                                      _stream(stream)))


def gpr_predict_var(Z, n, Zs, m, d, h, L_tiles, tile, prec, full_cov, add_noise, out, ws, ws_bytes, stream=None):
    _check(load().gpr_predict_var(_ptr(Z), n, _ptr(Zs), m, d, hyper(h), _ptr(L_tiles), tile, _prec(prec),
                                  int(full_cov), int(add_noise), _ptr(out), _ptr(ws), ws_bytes, _stream(stream)))


def gpr_nlml(L_tiles, n, tile, prec, y, alpha, nlml, stream=None):
    _check(load().gpr_nlml(_ptr(L_tiles), n, tile, _prec(prec), _ptr(y), _ptr(alpha), _ptr(nlml), _stream(stream)))


def gpr_nlml_grad(Z, n, d, h, L_tiles, tile, prec, alpha, trainable, grad_log, ws, ws_bytes, stream=None):
    tr = (_int * 3)(*[int(t) for t in (trainable if trainable is not None else (1, 1, 1))])
    _check(load().gpr_nlml_grad(_ptr(Z), n, d, hyper(h), _ptr(L_tiles), tile, _prec(prec), _ptr(alpha), tr,
                                _ptr(grad_log), _ptr(ws), ws_bytes, _stream(stream)))


def gpr_optimize(Z, y, n, d, tile, prec, theta_log, trainable, steps, lr, beta1, beta2, eps, adam_state, K_tiles,
                 ws, ws_bytes, stream=None, kernel="se"):
    """Returns (theta_log[3], adam_state[7], nlml_trace[steps+1]) as Python lists."""
    th = (_dbl * 3)(*[float(t) for t in theta_log])
    tr = (_int * 3)(*[int(t) for t in (trainable if trainable is not None else (1, 1, 1))])
    st = (_dbl * 7)(*([float(x) for x in adam_state] if adam_state is not None else [0.0] * 7))
    trace = (_dbl * (steps + 1))()
    _check(load().gpr_optimize(_ptr(Z), _ptr(y), n, d, tile, _prec(prec), _kernel(kernel), th, tr, steps, lr, beta1,
                               beta2, eps, st, trace, _ptr(K_tiles), _ptr(ws), ws_bytes, _stream(stream)))
    return list(th), list(st), list(trace)


def gpr_cholesky_census(T):
    c = (_i64 * 4)()
    _check(load().gpr_cholesky_census(T, c))
    return dict(potrf=c[0], trsm=c[1], syrk=c[2], gemm=c[3])


SCHEDULE_REPORT = ("launches", "launches_main", "launches_aux", "waits", "concurrent_pairs", "conflicts",
                   "unannotated", "early_waits")


def gpr_cholesky_schedule_check(n, tile, prec, omit_event=-1):
    r = (_i64 * 8)()
    _check(load().gpr_cholesky_schedule_check(n, tile, _prec(prec), omit_event, r))
    return dict(zip(SCHEDULE_REPORT, list(r)))


def gpr_timing_enable(on: bool):
    _check(load().gpr_timing_enable(int(on)))


def gpr_split_bf16x3(x, count, hi, mid, lo, stream=None):
    _check(load().gpr_split_bf16x3(_ptr(x), count, _ptr(hi), _ptr(mid), _ptr(lo), _stream(stream)))


def gpr_stats_workspace(nsub) -> int:
    out = _sz()
    _check(load().gpr_stats_workspace(nsub, ctypes.byref(out)))
    return out.value


def gpr_summary_stats(Z_raw, Z_std, y_raw, n, d, sub_idx, nsub, stats64, stats32, ws, ws_bytes, stream=None):
    _check(load().gpr_summary_stats(_ptr(Z_raw), _ptr(Z_std), _ptr(y_raw), n, d, _ptr(sub_idx), nsub, _ptr(stats64),
                                    _ptr(stats32), _ptr(ws), ws_bytes, _stream(stream)))


def gpr_mlp_nparams() -> int:
    return load().gpr_mlp_nparams()


def gpr_mlp_workspace(batch) -> int:
    out = _sz()
    _check(load().gpr_mlp_workspace(batch, ctypes.byref(out)))
    return out.value


def gpr_mlp_forward(params, X, batch, out, ws, ws_bytes, stream=None):
    _check(load().gpr_mlp_forward(_ptr(params), _ptr(X), batch, _ptr(out), _ptr(ws), ws_bytes, _stream(stream)))


def gpr_mlp_loss_grad(params, X, Y, batch, loss, grad, ws, ws_bytes, stream=None):
    _check(load().gpr_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(Y), batch, _ptr(loss), _ptr(grad), _ptr(ws),
                                    ws_bytes, _stream(stream)))


def gpr_mlp_train_step(params, adam_m, adam_v, t, X, Y, batch, lr, beta1, beta2, eps, loss, ws, ws_bytes,
                       stream=None):
    _check(load().gpr_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), t, _ptr(X), _ptr(Y), batch, lr, beta1,
                                     beta2, eps, _ptr(loss), _ptr(ws), ws_bytes, _stream(stream)))


TIMING_KINDS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "fp64_trtri": 4, "fp32_trtri": 5,
                "fp64_trace": 6, "fp32_trace": 7, "bf16x3_trtri": 8, "bf16x6_trtri": 9, "bf16x3_trace": 10,
                "bf16x6_trace": 11}


def gpr_timing_read(kind="fp64"):
    """(launches, total_ms, algorithmic_flops) of one kind of timed tile-GEMM launch since the last read."""
    n, ms, fl = _i64(), _dbl(), _dbl()
    k = TIMING_KINDS[kind] if isinstance(kind, str) else int(kind)
    _check(load().gpr_timing_read(k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)))
    return int(n.value), float(ms.value), float(fl.value)
