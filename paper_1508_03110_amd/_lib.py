"""ctypes binding of libalsncg (include/alsncg.h): argument marshalling only.

Every function here has the name of the C entry point it calls and forwards
its arguments unchanged (tensors become device pointers, the stream defaults
to torch's current stream).  No arithmetic of the method happens here: if the
library is missing, loading fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libalsncg.so")

F64, F32, BF16 = 0, 1, 2
OK, E_INVAL, E_HIP, E_NOT_SPD, E_NONFINITE, E_NOMEM, E_BUDGET = 0, -1, -2, -3, -4, -5, -6
INT64_MAX = (1 << 63) - 1


class AlsError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (fn, strerror(status), status))


class Csr(ctypes.Structure):
    """als_csr: one orientation of R, device pointers."""
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    """als_server_config."""
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("split", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_csrp = ctypes.POINTER(Csr)

_SIGS = {
    "als_ctx_create": (_i, [ctypes.POINTER(_vp), _i]),
    "als_ctx_destroy": (None, [_vp]),
    "als_strerror": (ctypes.c_char_p, [_i]),
    "als_ctx_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "als_plan_create": (_i, [_vp, _csrp, _i64, ctypes.POINTER(_vp)]),
    "als_plan_destroy": (None, [_vp]),
    "als_plan_set_grid": (_i, [_vp, _i64, _i64]),
    "als_plan_info": (_i, [_vp, ctypes.POINTER(_i64)]),
    "als_plan_set_dual": (_i, [_vp, _i64]),
    "als_plan_create_sliced": (_i, [_vp, _csrp, _i64, _i64, ctypes.POINTER(_vp)]),
    "als_plan_set_split_copy": (_i, [_vp, _i]),
    "als_sweep": (_i, [_vp, _vp, _csrp, _vp, _vp, _i, _i, _d, _i, _vp, _vp, _vp, _vp]),
    "als_sweep_mixed": (_i, [_vp, _vp, _csrp, _vp, _vp, _vp, _vp, _i, _i, _d, _i, _vp, _vp]),
    "als_to_bf16": (_i, [_vp, _i64, _vp, _vp, _vp]),
    "ncg_gradient": (_i, [_vp, _vp, _csrp, _vp, _csrp, _vp, _vp, _i, _i, _d, _i, _vp, _vp, _vp,
                          _vp]),
    "linesearch_coeffs": (_i, [_vp, _vp, _csrp, _csrp, _vp, _vp, _vp, _vp, _i, _i, _d, _i, _vp,
                               _vp]),
    "linesearch_coeffs_noalloc": (_i, [_vp, _vp, _csrp, _csrp, _vp, _vp, _vp, _vp, _i, _i, _d,
                                       _i, _vp, _vp]),
    "linesearch_coeffs_noalloc_max_chunks": (ctypes.c_size_t, []),
    "ncg_backtrack": (_i, [_vp, _vp, _d, _d, _d, _i, _vp, _vp, _vp, _vp]),
    "ncg_axpy": (_i, [_vp, _i64, _vp, _vp, _vp, _i, _vp]),
    "ncg_axpby": (_i, [_vp, _i64, _d, _vp, _d, _vp, _i, _vp]),
    "ncg_direction": (_i, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp]),
    "ncg_linesearch_step": (_i, [_vp, _vp, _csrp, _csrp, _vp, _vp, _vp, _i, _i, _d, _i, _i, _d, _d,
                                 _d, _i, _vp, _vp]),
    "ncg_linesearch_exact": (_i, [_vp, _vp, _d, _vp, _vp, _vp, _vp]),
    "ncg_direction_dev": (_i, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp]),
    "fold_in": (_i, [_vp, _vp, _i64, _i, _i, _d, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rank_top_t": (_i, [_vp, _vp, _vp, _i64, _i64, _i, _i, _i, _i, _vp, _vp]),
    "rank_accuracy": (_i, [_vp, _vp, _vp, _i64, _i64, _i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "als_server_create": (_i, [_vp, _vp, _i64, _i, _i, _d, _i, ctypes.POINTER(ServerConfig),
                               ctypes.POINTER(_vp)]),
    "als_server_destroy": (None, [_vp]),
    "als_server_submit": (_i, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "als_server_poll": (_i, [_vp, _i64, _vp, _vp, _vp, ctypes.POINTER(_i64)]),
    "als_server_pending": (_i64, [_vp]),
    "als_server_replay": (_i, [_vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
}
EXPORTS = tuple(_SIGS)

_lib = None


def load():
    """Load libalsncg.so (built in-tree by paper_1508_03110_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libalsncg.so is not built (%s): run paper_1508_03110_amd/build.py" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load().als_strerror(int(status)).decode()


def _ptr(t):
    """Device pointer of a tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(fn, rc):
    if rc != OK:
        raise AlsError(fn, rc)
    return rc


def dtype_code(dtype) -> int:
    import torch
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise ValueError("unsupported factor dtype %s" % dtype)


# ---------------------------------------------------------------- context / plans

def als_ctx_create(device: int = 0):
    out = _vp()
    _check("als_ctx_create", load().als_ctx_create(ctypes.byref(out), int(device)))
    return out.value


def als_ctx_destroy(ctx):
    load().als_ctx_destroy(ctx)


def als_ctx_workspace_bytes(ctx) -> int:
    return int(load().als_ctx_workspace_bytes(ctx))


def als_plan_create(ctx, R: Csr, chunk: int = 0):
    out = _vp()
    _check("als_plan_create", load().als_plan_create(ctx, ctypes.byref(R), int(chunk), ctypes.byref(out)))
    return out.value


def als_plan_create_sliced(ctx, R: Csr, chunk: int, n_slices: int):
    out = _vp()
    _check("als_plan_create_sliced", load().als_plan_create_sliced(
        ctx, ctypes.byref(R), int(chunk), int(n_slices), ctypes.byref(out)))
    return out.value


def als_plan_set_split_copy(plan, mode):
    return _check("als_plan_set_split_copy", load().als_plan_set_split_copy(plan, int(mode)))


def als_plan_destroy(plan):
    load().als_plan_destroy(plan)


def als_plan_set_grid(plan, sweep_grid, pass_grid=0):
    return _check("als_plan_set_grid", load().als_plan_set_grid(plan, int(sweep_grid), int(pass_grid)))


def als_plan_set_dual(plan, max_len):
    return _check("als_plan_set_dual", load().als_plan_set_dual(plan, int(max_len)))


def als_plan_info(plan) -> dict:
    a = (_i64 * 8)()
    _check("als_plan_info", load().als_plan_info(plan, a))
    keys = ("n_rows", "nnz", "n_chunks", "split_rows", "split_chunks", "chunk", "max_row",
            "dual_rows")
    return dict(zip(keys, [int(v) for v in a]))


# ---------------------------------------------------------------- hot path

def als_sweep(ctx, plan, R: Csr, Y, X, n_f, ld, lam, dt, X_at=None, grad_out=None, bad_row=None,
              stream=None):
    return _check("als_sweep", load().als_sweep(ctx, plan, ctypes.byref(R), _ptr(Y), _ptr(X), int(n_f),
                                                int(ld), float(lam), int(dt), _ptr(X_at),
                                                _ptr(grad_out), _ptr(bad_row), _stream(stream)))


def als_sweep_mixed(ctx, plan, R: Csr, Y16, Y32, X32, X16, n_f, ld, lam, refine, bad_row=None,
                    stream=None):
    return _check("als_sweep_mixed", load().als_sweep_mixed(
        ctx, plan, ctypes.byref(R), _ptr(Y16), _ptr(Y32), _ptr(X32), _ptr(X16), int(n_f), int(ld),
        float(lam), 1 if refine else 0, _ptr(bad_row), _stream(stream)))


def als_to_bf16(ctx, n, x, y, stream=None):
    return _check("als_to_bf16", load().als_to_bf16(ctx, int(n), _ptr(x), _ptr(y), _stream(stream)))


def ncg_gradient(ctx, plan_R, R: Csr, plan_Rt, Rt: Csr, U, M, n_f, ld, lam, dt, gU=None, gM=None,
                 out2=None, stream=None):
    return _check("ncg_gradient", load().ncg_gradient(ctx, plan_R, ctypes.byref(R), plan_Rt,
                                                      ctypes.byref(Rt), _ptr(U), _ptr(M), int(n_f),
                                                      int(ld), float(lam), int(dt), _ptr(gU),
                                                      _ptr(gM), _ptr(out2), _stream(stream)))


def linesearch_coeffs(ctx, plan_R, R: Csr, Rt: Csr, U, M, pU, pM, n_f, ld, lam, dt, coeffs,
                      stream=None):
    return _check("linesearch_coeffs", load().linesearch_coeffs(
        ctx, plan_R, ctypes.byref(R), ctypes.byref(Rt), _ptr(U), _ptr(M), _ptr(pU), _ptr(pM),
        int(n_f), int(ld), float(lam), int(dt), _ptr(coeffs), _stream(stream)))


def linesearch_coeffs_noalloc(ctx, plan_R, R: Csr, Rt: Csr, U, M, pU, pM, n_f, ld, lam, dt, coeffs,
                              stream=None):
    return _check("linesearch_coeffs_noalloc", load().linesearch_coeffs_noalloc(
        ctx, plan_R, ctypes.byref(R), ctypes.byref(Rt), _ptr(U), _ptr(M), _ptr(pU), _ptr(pM),
        int(n_f), int(ld), float(lam), int(dt), _ptr(coeffs), _stream(stream)))


def linesearch_coeffs_noalloc_max_chunks():
    return int(load().linesearch_coeffs_noalloc_max_chunks())


def ncg_backtrack(ctx, coeffs, alpha0, tau, c, max_trials, alpha_out, trials_out=None, q_out=None,
                  stream=None):
    return _check("ncg_backtrack", load().ncg_backtrack(ctx, _ptr(coeffs), float(alpha0), float(tau),
                                                        float(c), int(max_trials), _ptr(alpha_out),
                                                        _ptr(trials_out), _ptr(q_out),
                                                        _stream(stream)))


def ncg_axpy(ctx, n, x, p, alpha, dt, stream=None):
    return _check("ncg_axpy", load().ncg_axpy(ctx, int(n), _ptr(x), _ptr(p), _ptr(alpha), int(dt),
                                              _stream(stream)))


def ncg_axpby(ctx, n, a, x, b, y, dt, stream=None):
    return _check("ncg_axpby", load().ncg_axpby(ctx, int(n), float(a), _ptr(x), float(b), _ptr(y),
                                                int(dt), _stream(stream)))


def ncg_direction(ctx, n, x, xbar, g_new, g_old, p, scal, restart, pr_plus, dt, stream=None):
    return _check("ncg_direction", load().ncg_direction(ctx, int(n), _ptr(x), _ptr(xbar), _ptr(g_new),
                                                        _ptr(g_old), _ptr(p), _ptr(scal),
                                                        int(restart), int(pr_plus), int(dt),
                                                        _stream(stream)))


def ncg_linesearch_step(ctx, plan_R, R: Csr, Rt: Csr, x, p, gbar, n_f, ld, lam, dt, search, alpha0,
                        tau, c, max_trials, state, stream=None):
    return _check("ncg_linesearch_step", load().ncg_linesearch_step(
        ctx, plan_R, ctypes.byref(R), ctypes.byref(Rt), _ptr(x), _ptr(p), _ptr(gbar), int(n_f),
        int(ld), float(lam), int(dt), int(search), float(alpha0), float(tau), float(c),
        int(max_trials), _ptr(state), _stream(stream)))


def ncg_linesearch_exact(ctx, coeffs, c, alpha_out, trials_out=None, q_out=None, stream=None):
    return _check("ncg_linesearch_exact", load().ncg_linesearch_exact(
        ctx, _ptr(coeffs), float(c), _ptr(alpha_out), _ptr(trials_out), _ptr(q_out),
        _stream(stream)))


def ncg_direction_dev(ctx, n, x, xbar, g_new, g_old, p, scal, restart_flag, pr_plus, dt, stream=None):
    return _check("ncg_direction_dev", load().ncg_direction_dev(
        ctx, int(n), _ptr(x), _ptr(xbar), _ptr(g_new), _ptr(g_old), _ptr(p), _ptr(scal),
        _ptr(restart_flag), int(pr_plus), int(dt), _stream(stream)))


def fold_in(ctx, M, n_items, n_f, ld, lam, dt, n_req, req_indptr, req_items, req_vals, U_out,
            req_status=None, stream=None):
    return _check("fold_in", load().fold_in(ctx, _ptr(M), int(n_items), int(n_f), int(ld), float(lam),
                                            int(dt), int(n_req), _ptr(req_indptr), _ptr(req_items),
                                            _ptr(req_vals), _ptr(U_out), _ptr(req_status),
                                            _stream(stream)))


# ---------------------------------------------------------------- ranking accuracy

def rank_top_t(ctx, U, M, n_u, n_m, n_f, ld, dt, t, top, stream=None):
    return _check("rank_top_t", load().rank_top_t(ctx, _ptr(U), _ptr(M), int(n_u), int(n_m), int(n_f),
                                                  int(ld), int(dt), int(t), _ptr(top),
                                                  _stream(stream)))


def rank_accuracy(ctx, U, M, n_u, n_m, n_f, ld, dt, t, top, swaps=None, mean_q=None, stream=None):
    return _check("rank_accuracy", load().rank_accuracy(ctx, _ptr(U), _ptr(M), int(n_u), int(n_m),
                                                        int(n_f), int(ld), int(dt), int(t), _ptr(top),
                                                        _ptr(swaps), _ptr(mean_q), _stream(stream)))


# ---------------------------------------------------------------- fold-in server

def _hp(a):
    """Host pointer of a contiguous numpy array (or None)."""
    return None if a is None else a.ctypes.data


def als_server_create(ctx, M, n_items, n_f, ld, lam, dt, cfg: ServerConfig):
    out = _vp()
    _check("als_server_create", load().als_server_create(ctx, _ptr(M), int(n_items), int(n_f), int(ld),
                                                         float(lam), int(dt), ctypes.byref(cfg),
                                                         ctypes.byref(out)))
    return out.value


def als_server_destroy(srv):
    load().als_server_destroy(srv)


def als_server_submit(srv, ids, indptr, items, vals):
    return _check("als_server_submit", load().als_server_submit(srv, int(len(ids)), _hp(ids), _hp(indptr),
                                                                _hp(items), _hp(vals)))


def als_server_poll(srv, max_done, done_ids, done_status, done_U):
    n = _i64(0)
    _check("als_server_poll", load().als_server_poll(srv, int(max_done), _hp(done_ids), _hp(done_status),
                                                     _hp(done_U), ctypes.byref(n)))
    return int(n.value)


def als_server_pending(srv) -> int:
    return int(load().als_server_pending(srv))


def als_server_replay(srv, arrival_ns, pool_row, pool_indptr, pool_items, pool_vals, completion_ns,
                      status=None, U_out=None):
    return _check("als_server_replay", load().als_server_replay(
        srv, int(len(arrival_ns)), _hp(arrival_ns), _hp(pool_row), int(len(pool_indptr) - 1),
        _hp(pool_indptr), _hp(pool_items), _hp(pool_vals), _hp(completion_ns), _hp(status),
        _hp(U_out)))
