"""ALS (Algorithm 1) and ALS-NCG (Algorithm 2) driven through libalsncg.

Device memory comes from PyTorch; every arithmetic step runs in the HIP
library through the C ABI (``_lib``).  The host only sequences the calls
and, once per ALS-NCG iteration of step(), reads back 16 scalars (the
quartic coefficients, the step and Q(step), beta, norms) to take the
restart and safeguard decisions; step_device() takes them on the device.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import _lib as L

TAU, C_ARMIJO, ALPHA0, MAX_TRIALS = 0.9, 0.5, 10.0, 400  # Section V-C
# sufficient-decrease constant of the exact search: the tolerance of the
# paper's serial line search (Section IV); with c = 0.5 the exact minimiser of
# a nearly quadratic Q would sit on the boundary of the test
C_EXACT = 1e-4

# layout of the per-solver FP64 scalar block on the device
S_DEN, S_BETA, S_GG, S_NUM = 0, 1, 2, 3
S_COEF = 4          # 4..8: C0..C4
S_ALPHA = 9
S_F, S_GN = 10, 11  # ncg_gradient out2
S_Q = 12            # Q(alpha) = f(x + alpha p) of the accepted step


class Context:
    """Owns an als_ctx on one device."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the ALS-NCG library needs an MI355X (gfx950)")
        self.device = int(device)
        self.handle = L.als_ctx_create(self.device)
        self.torch_device = torch.device("cuda", self.device)

    def close(self):
        if getattr(self, "handle", None):
            L.als_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return L.als_ctx_workspace_bytes(self.handle)


class DeviceCsr:
    """One orientation of R resident in HBM, with its row plan."""

    def __init__(self, ctx: Context, indptr, indices, values, n_cols: int, chunk: int = 0):
        dev = ctx.torch_device

        def put(a, npt, tt):
            if isinstance(a, torch.Tensor):  # already on the device: no host round trip
                return a.to(device=dev, dtype=tt).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a, dtype=npt)).to(dev)

        self.indptr = put(indptr, np.int64, torch.int64)
        self.indices = put(indices, np.int32, torch.int32)
        self.values = put(values, np.float32, torch.float32)
        self.n_rows = int(self.indptr.numel() - 1)
        self.n_cols = int(n_cols)
        self.nnz = int(self.indices.numel())
        self.csr = L.Csr(self.n_rows, self.n_cols, self.nnz, self.indptr.data_ptr(),
                         self.indices.data_ptr() if self.nnz else 0,
                         self.values.data_ptr() if self.nnz else 0)
        self.ctx = ctx
        self.plan = L.als_plan_create(ctx.handle, self.csr, int(chunk))

    @classmethod
    def from_host(cls, ctx, A, chunk: int = 0):
        """A: any object with n_rows, n_cols, indptr, indices, values (host arrays)."""
        return cls(ctx, A.indptr, A.indices, A.values, A.n_cols, chunk)

    def info(self) -> dict:
        d = L.als_plan_info(self.plan)
        d["grid"] = getattr(self, "grid", 0)
        d["grid_pass"] = getattr(self, "grid_pass", 0)
        return d

    def replan(self, chunk: int = 0, grid: int = 0, grid_pass: int = 0):
        """Rebuild the row plan with another chunk size and set its launch
        grids (the dual-form bins are kept)."""
        if self.plan:
            L.als_plan_destroy(self.plan)
            self.plan = None
        self.plan = L.als_plan_create(self.ctx.handle, self.csr, int(chunk))
        self.set_grid(grid, grid_pass)
        if getattr(self, "dual_max", 0):
            L.als_plan_set_dual(self.plan, self.dual_max)
        if getattr(self, "split_copy", -1) != -1:
            L.als_plan_set_split_copy(self.plan, self.split_copy)

    def set_dual(self, max_len: int):
        """Solve rows of 1..max_len ratings (max_len <= 94) in the dual form
        of the half-sweep (an n_i x n_i system); 0 turns it off."""
        L.als_plan_set_dual(self.plan, int(max_len))
        self.dual_max = int(max_len)

    def set_split_copy(self, mode: int):
        """FP32 half-sweep over a split copy of the fixed side: 1 on, 0 off,
        -1 on when its rows are no wider than the factor rows (default)."""
        L.als_plan_set_split_copy(self.plan, int(mode))
        self.split_copy = int(mode)

    def set_grad_slices(self, n_slices: int, chunk: int = 0):
        """Give the gradient pass its own plan with every row cut at n_slices
        column slices (one slice per die of the device at a time, so that
        the gathered rows of each slice stay in that die's L2); 0 drops it."""
        if getattr(self, "grad_plan", None):
            L.als_plan_destroy(self.grad_plan)
            self.grad_plan = None
        self.grad_slices = int(n_slices)
        if n_slices > 0:
            self.grad_plan = L.als_plan_create_sliced(self.ctx.handle, self.csr, int(chunk), int(n_slices))

    def set_grid(self, grid: int, grid_pass: int = 0):
        """Persistent grids of the half-sweep and of the streaming passes (0: one
        workgroup per chunk)."""
        L.als_plan_set_grid(self.plan, int(grid), int(grid_pass))
        self.grid, self.grid_pass = int(grid), int(grid_pass)

    def close(self):
        if getattr(self, "plan", None):
            L.als_plan_destroy(self.plan)
            self.plan = None
        if getattr(self, "grad_plan", None):
            L.als_plan_destroy(self.grad_plan)
            self.grad_plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceProblem:
    """R (users x items) and R^T on the device plus n_f, lambda and the factor type."""

    def __init__(self, ctx: Context, R, Rt, n_f: int, lam: float, dtype=torch.float32,
                 chunk: int = 0, chunk_t: Optional[int] = None, ld: Optional[int] = None):
        self.ctx = ctx
        self.R = R if isinstance(R, DeviceCsr) else DeviceCsr.from_host(ctx, R, chunk)
        self.Rt = Rt if isinstance(Rt, DeviceCsr) else DeviceCsr.from_host(
            ctx, Rt, chunk if chunk_t is None else chunk_t)
        if self.R.n_rows != self.Rt.n_cols or self.R.n_cols != self.Rt.n_rows or self.R.nnz != self.Rt.nnz:
            raise ValueError("R and R^T shapes disagree")
        self.n_u, self.n_m = self.R.n_rows, self.R.n_cols
        self.n_f, self.lam = int(n_f), float(lam)
        self.ld = int(ld or n_f)
        self.dtype = dtype
        self.dt = L.dtype_code(dtype)
        self.N = (self.n_u + self.n_m) * self.ld

    # -- helpers over a flat [U; M] buffer
    def zeros(self, n=None):
        return torch.zeros(self.N if n is None else n, dtype=self.dtype, device=self.ctx.torch_device)

    def U(self, x):
        return x[: self.n_u * self.ld].view(self.n_u, self.ld)

    def M(self, x):
        return x[self.n_u * self.ld:].view(self.n_m, self.ld)

    def pack(self, U, M):
        x = self.zeros()
        for dst, a in ((self.U(x), U), (self.M(x), M)):
            t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
            dst[:, : self.n_f] = t.to(device=x.device, dtype=self.dtype)
        return x

    # -- single ABI calls
    def sweep(self, side: str, Y, X, X_at=None, grad_out=None, bad_row=None):
        A = self.R if side == "U" else self.Rt
        L.als_sweep(self.ctx.handle, A.plan, A.csr, Y, X, self.n_f, self.ld, self.lam, self.dt,
                    X_at, grad_out, bad_row)

    def sweep_mixed(self, side: str, Y16, Y32, X32, X16=None, refine: bool = True, bad_row=None):
        """Reduced-precision half-sweep: Gram from the BF16 copy Y16, solve in
        FP32, optional refinement against Y32 (FP32 factors only)."""
        A = self.R if side == "U" else self.Rt
        L.als_sweep_mixed(self.ctx.handle, A.plan, A.csr, Y16, Y32, X32, X16, self.n_f, self.ld,
                          self.lam, refine, bad_row)

    def bf16_rows(self, n_rows: int):
        return torch.empty((n_rows, self.ld), dtype=torch.bfloat16, device=self.ctx.torch_device)

    def to_bf16(self, X32, X16):
        L.als_to_bf16(self.ctx.handle, X32.numel(), X32, X16)

    def gradient(self, U, M, gU=None, gM=None, out2=None):
        L.ncg_gradient(self.ctx.handle, getattr(self.R, "grad_plan", None) or self.R.plan, self.R.csr,
                       getattr(self.Rt, "grad_plan", None) or self.Rt.plan, self.Rt.csr, U, M,
                       self.n_f, self.ld, self.lam, self.dt, gU, gM, out2)

    def coeffs(self, U, M, pU, pM, out):
        L.linesearch_coeffs(self.ctx.handle, self.R.plan, self.R.csr, self.Rt.csr, U, M, pU, pM,
                            self.n_f, self.ld, self.lam, self.dt, out)

    def loss_and_gnorm(self, x, g=None):
        """(f(x), ||grad f(x)||) by one gradient pass per orientation (FP64 reductions)."""
        out = torch.zeros(2, dtype=torch.float64, device=self.ctx.torch_device)
        g = self.zeros() if g is None else g
        self.gradient(self.U(x), self.M(x), self.U(g), self.M(g), out)
        f, gg = out.cpu().tolist()
        return f, math.sqrt(max(gg, 0.0))


def _check_precision(prob: DeviceProblem, precision: str):
    if precision not in ("fp", "bf16"):
        raise ValueError("precision must be 'fp' (the factor type) or 'bf16'")
    if precision == "bf16" and prob.dtype != torch.float32:
        raise ValueError("the bf16 form keeps FP32 factors next to their BF16 copies")


class Als:
    """Algorithm 1: U half-sweep from M, then M half-sweep from the new U.

    precision="bf16": the half-sweeps build their Gram matrices from BF16
    copies of the fixed side (refined against the FP32 factors when
    `refine`); the factors themselves stay FP32."""

    def __init__(self, prob: DeviceProblem, x0=None, precision: str = "fp", refine: bool = True):
        _check_precision(prob, precision)
        self.p = prob
        self.x = prob.zeros() if x0 is None else x0
        self.k = 0
        self.precision, self.refine = precision, refine
        if precision == "bf16":
            self.u16 = prob.bf16_rows(prob.n_u)
            self.m16 = prob.bf16_rows(prob.n_m)
            prob.to_bf16(prob.M(self.x), self.m16)

    def sweep(self):
        P = self.p
        if self.precision == "bf16":
            P.sweep_mixed("U", self.m16, P.M(self.x), P.U(self.x), self.u16, self.refine)
            P.sweep_mixed("M", self.u16, P.U(self.x), P.M(self.x), self.m16, self.refine)
        else:
            P.sweep("U", P.M(self.x), P.U(self.x))
            P.sweep("M", P.U(self.x), P.M(self.x))
        self.k += 1


class AlsNcg:
    """Algorithm 2 (ALS-NCG) with the preconditioned beta of Eq. (8) and the
    one-pass quartic backtracking line search of Section V-C (search="exact":
    the exact minimiser of the same quartic instead).

    Safeguards (the paper is silent on failures): a direction with
    g^T p >= 0 is reset to -gbar; if the line search still fails, the ALS
    point P(x_k) is taken and the next direction restarts (beta = 0).
    """

    def __init__(self, prob: DeviceProblem, safeguard: bool = True, pr_plus: bool = False,
                 alpha0: float = ALPHA0, tau: float = TAU, c: float = C_ARMIJO,
                 max_trials: int = MAX_TRIALS, precision: str = "fp", refine: bool = True,
                 search: str = "backtracking"):
        _check_precision(prob, precision)
        if search not in ("backtracking", "exact"):
            raise ValueError("search must be 'backtracking' (Algorithm 4) or 'exact'")
        self.search = search
        if search == "exact" and c == C_ARMIJO:
            c = C_EXACT
        self.p = prob
        self.precision, self.refine = precision, refine
        if precision == "bf16":
            self.u16 = prob.bf16_rows(prob.n_u)   # BF16 copy of U(P(x))
            self.m16 = prob.bf16_rows(prob.n_m)   # BF16 copy of M(x)
        self.safeguard, self.pr_plus = safeguard, pr_plus
        self.alpha0, self.tau, self.c, self.max_trials = alpha0, tau, c, max_trials
        dev = prob.ctx.torch_device
        self.x = prob.zeros()
        self.pdir = prob.zeros()
        self.xbar = prob.zeros()      # P(x); after the direction update it holds gbar
        self.g_new = prob.zeros()
        self.g_old = prob.zeros()
        self.scal = torch.zeros(16, dtype=torch.float64, device=dev)
        self.trials = torch.zeros(1, dtype=torch.int32, device=dev)
        self.k = 0
        self.restarts = self.safeguards = 0
        self.f = float("nan")
        self.alpha = float("nan")
        self.n_trials = 0
        self.coef = None
        self.timers = None  # {phase: [(start, end) torch.cuda.Event pairs]} when timing
        # device-side step control (ncg_linesearch_step): decisions in `state`
        self.state = torch.zeros(32, dtype=torch.float64, device=dev)
        self.graphs = None

    def enable_timing(self, on: bool = True):
        """Record HIP events (on torch's current stream, where the library
        launches) around every phase of each iteration."""
        self.timers = {} if on else None

    def _mark(self, name):
        if self.timers is None:
            return None
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        self.timers.setdefault(name, []).append([e, None])
        return name

    def _done(self, name):
        if name is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.timers[name][-1][1] = e

    def phase_ms(self) -> dict:
        """Mean milliseconds per launch of each timed phase (synchronises)."""
        torch.cuda.synchronize()
        return {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in (self.timers or {}).items()}

    # -- pieces
    def _precondition_and_gradient(self):
        """xbar = P(x) (two half-sweeps); g_new = grad f(x): the U block fused
        into the U half-sweep, the M block by one pass over R^T."""
        P = self.p
        if self.precision == "bf16":
            # the gradient cannot come from the BF16 Gram: both blocks by passes
            t = self._mark("to_bf16")
            P.to_bf16(P.M(self.x), self.m16)
            self._done(t)
            t = self._mark("sweep_U")
            P.sweep_mixed("U", self.m16, P.M(self.x), P.U(self.xbar), self.u16, self.refine)
            self._done(t)
            t = self._mark("sweep_M")
            P.sweep_mixed("M", self.u16, P.U(self.xbar), P.M(self.xbar), None, self.refine)
            self._done(t)
            t = self._mark("gradient")
            P.gradient(P.U(self.x), P.M(self.x), P.U(self.g_new), P.M(self.g_new), None)
            self._done(t)
            return
        t = self._mark("sweep_U")
        P.sweep("U", P.M(self.x), P.U(self.xbar), X_at=P.U(self.x), grad_out=P.U(self.g_new))
        self._done(t)
        t = self._mark("sweep_M")
        P.sweep("M", P.U(self.xbar), P.M(self.xbar))
        self._done(t)
        t = self._mark("gradient_M")
        P.gradient(P.U(self.x), P.M(self.x), None, P.M(self.g_new), None)
        self._done(t)

    def _direction(self, restart: bool):
        P = self.p
        t = self._mark("direction")
        L.ncg_direction(P.ctx.handle, P.N, self.x, self.xbar, self.g_new, self.g_old, self.pdir,
                        self.scal, 1 if restart else 0, 1 if self.pr_plus else 0, P.dt)
        self._done(t)
        self.g_new, self.g_old = self.g_old, self.g_new

    def _line_search(self):
        P = self.p
        coef = self.scal[S_COEF:S_COEF + 5]
        t = self._mark("linesearch_coeffs")
        P.coeffs(P.U(self.x), P.M(self.x), P.U(self.pdir), P.M(self.pdir), coef)
        self._done(t)
        alpha_d, q_d = self.scal[S_ALPHA:S_ALPHA + 1], self.scal[S_Q:S_Q + 1]
        if self.search == "exact":
            L.ncg_linesearch_exact(P.ctx.handle, coef, self.c, alpha_d, self.trials, q_d)
        else:
            L.ncg_backtrack(P.ctx.handle, coef, self.alpha0, self.tau, self.c, self.max_trials,
                            alpha_d, self.trials, q_d)
        host = self.scal.cpu().numpy()
        n = int(self.trials.cpu().item())
        C = host[S_COEF:S_COEF + 5].copy()
        alpha = float(host[S_ALPHA]) if n >= 0 else None
        return C, alpha, n, float(host[S_Q])

    # -- Algorithm 2
    def init(self, U0, M0):
        self.x = self.p.pack(U0, M0)
        self._precondition_and_gradient()
        self._direction(restart=True)       # p_0 = -gbar_0
        self.k = 0
        return self

    def step(self):
        P = self.p
        C, alpha, n, q = self._line_search()
        if self.safeguard and (C[1] >= 0.0 or alpha is None):
            L.ncg_axpby(P.ctx.handle, P.N, -1.0, self.xbar, 0.0, self.pdir, P.dt)  # p = -gbar
            self.restarts += 1
            C, alpha, n, q = self._line_search()
        restart = False
        if alpha is None or (self.safeguard and C[1] >= 0.0):
            if not self.safeguard:
                raise RuntimeError("line search failed at iteration %d" % self.k)
            L.ncg_axpby(P.ctx.handle, P.N, -1.0, self.xbar, 1.0, self.x, P.dt)  # x = x - gbar = P(x)
            self.safeguards += 1
            restart = True
            self.f, self.alpha = float("nan"), float("nan")
        else:
            L.ncg_axpy(P.ctx.handle, P.N, self.x, self.pdir, self.scal[S_ALPHA:S_ALPHA + 1], P.dt)
            self.alpha = alpha
            self.f = q  # Q(alpha), evaluated on the device
        self.coef, self.n_trials = C, n
        self._precondition_and_gradient()
        self._direction(restart=restart)
        self.k += 1
        return self

    # -- Algorithm 2 with every decision on the device (no host read per step)
    def step_device(self):
        """One iteration as a fixed launch sequence: device-side line search,
        restart and safeguard (same decisions as step()), preconditioner,
        gradient, direction.  Host-visible results via read_state()."""
        if not self.safeguard:
            raise ValueError("device-side control implements the safeguarded iteration")
        P = self.p
        t = self._mark("linesearch")
        L.ncg_linesearch_step(P.ctx.handle, P.R.plan, P.R.csr, P.Rt.csr, self.x, self.pdir,
                              self.xbar, P.n_f, P.ld, P.lam, P.dt,
                              1 if self.search == "exact" else 0, self.alpha0, self.tau, self.c,
                              self.max_trials, self.state)
        self._done(t)
        self._precondition_and_gradient()
        t = self._mark("direction")
        L.ncg_direction_dev(P.ctx.handle, P.N, self.x, self.xbar, self.g_new, self.g_old, self.pdir,
                            self.scal, self.state[24:25], 1 if self.pr_plus else 0, P.dt)
        self._done(t)
        self.g_new, self.g_old = self.g_old, self.g_new
        self.k += 1
        return self

    def read_state(self):
        """Copy the device step state to the host attributes (synchronises)."""
        st = self.state.cpu().numpy()
        self.coef = st[16:21].copy()
        self.alpha = float(st[21]) if st[24] == 0 else float("nan")
        self.n_trials = int(st[22])
        self.f = float(st[25])
        self.restarts, self.safeguards = int(st[26]), int(st[27])
        return self

    def capture(self):
        """Capture one device-controlled iteration as a HIP graph, twice: the
        gradient buffers alternate between iterations, so graph k % 2 runs
        iteration k.  The workspace must already have its final size (run one
        step_device() first)."""
        timers, self.timers = self.timers, None
        graphs = []
        for _ in range(2):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.step_device()
            graphs.append(g)
        self.k -= 2
        self.timers = timers
        self.graphs = graphs
        self._graph_base = self.k
        return self

    def replay(self):
        """Run the next iteration from the captured graphs (the buffers the
        graphs were captured with; do not re-init after capturing)."""
        self.graphs[(self.k - self._graph_base) % 2].replay()
        self.g_new, self.g_old = self.g_old, self.g_new
        self.k += 1
        return self

    def gnorm(self) -> float:
        """||g(x_k)|| from the last direction update (no extra pass)."""
        return math.sqrt(max(float(self.scal[S_GG].item()), 0.0))


def fold_in(ctx: Context, M, lam: float, req, n_f: int, ld: Optional[int] = None):
    """Batched fold-in of host request CSR `req` against device factors M
    [n_items, ld]; returns (U [n_req, ld] device tensor, status int32)."""
    ld = int(ld or n_f)
    dev = ctx.torch_device
    ip = torch.as_tensor(np.ascontiguousarray(req.indptr, dtype=np.int64)).to(dev)
    it = torch.as_tensor(np.ascontiguousarray(req.indices, dtype=np.int32)).to(dev)
    va = torch.as_tensor(np.ascontiguousarray(req.values, dtype=np.float32)).to(dev)
    n_req = ip.numel() - 1
    U = torch.zeros((n_req, ld), dtype=M.dtype, device=dev)
    st = torch.zeros(n_req, dtype=torch.int32, device=dev)
    L.fold_in(ctx.handle, M, M.shape[0], n_f, ld, lam, L.dtype_code(M.dtype), n_req, ip, it, va, U, st)
    return U, st


def rank_top_t(ctx: Context, U, M, t: int, n_f: Optional[int] = None):
    """Top-t items of every user's ranking by U . M^T (Section IV), device
    int32 [n_u, t].  U [n_u, ld], M [n_m, ld] device factors."""
    n_f = int(n_f or U.shape[1])
    top = torch.empty((U.shape[0], int(t)), dtype=torch.int32, device=ctx.torch_device)
    L.rank_top_t(ctx.handle, U, M, U.shape[0], M.shape[0], n_f, U.shape[1], L.dtype_code(U.dtype),
                 int(t), top)
    return top


def rank_accuracy(ctx: Context, U, M, top, n_f: Optional[int] = None, swaps: bool = False):
    """Ranking accuracy of Section IV of (U, M) against reference top-t lists
    `top` (device int32 [n_u, t]): device double [1] holding the mean of
    q_i = 1 - s_i / s_max, and with swaps=True also the device int64 s_i."""
    n_f = int(n_f or U.shape[1])
    dev = ctx.torch_device
    mean_q = torch.empty(1, dtype=torch.float64, device=dev)
    s = torch.empty(U.shape[0], dtype=torch.int64, device=dev) if swaps else None
    L.rank_accuracy(ctx.handle, U, M, U.shape[0], M.shape[0], n_f, U.shape[1], L.dtype_code(U.dtype),
                    top.shape[1], top, s, mean_q)
    return (mean_q, s) if swaps else mean_q


class FoldInServer:
    """Continuous-batching fold-in server (als_server_*) against device item
    factors M [n_items, ld]; host numpy in, host numpy out."""

    def __init__(self, ctx: Context, M, lam: float, n_f: int, budget_bytes: int = 16 << 30,
                 max_inflight: int = 4, max_batch: int = 4096, split: int = 256):
        self.ctx, self.M, self.n_f = ctx, M, int(n_f)
        self.np_dtype = np.float64 if M.dtype == torch.float64 else np.float32
        cfg = L.ServerConfig(int(budget_bytes), int(max_inflight), int(max_batch), int(split))
        self.handle = L.als_server_create(ctx.handle, M, M.shape[0], n_f, M.shape[1], lam,
                                          L.dtype_code(M.dtype), cfg)

    def close(self):
        if getattr(self, "handle", None):
            L.als_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, ids, req):
        """Queue the rows of host CSR `req` with the given ids."""
        L.als_server_submit(self.handle, np.ascontiguousarray(ids, dtype=np.int64),
                            np.ascontiguousarray(req.indptr, dtype=np.int64),
                            np.ascontiguousarray(req.indices, dtype=np.int32),
                            np.ascontiguousarray(req.values, dtype=np.float32))

    def poll(self, max_done: int = 4096):
        ids = np.empty(max_done, np.int64)
        st = np.empty(max_done, np.int32)
        U = np.empty((max_done, self.n_f), self.np_dtype)
        n = L.als_server_poll(self.handle, max_done, ids, st, U)
        return ids[:n], st[:n], U[:n]

    def pending(self) -> int:
        return L.als_server_pending(self.handle)

    def drain(self, timeout_s: float = 60.0):
        """Poll until nothing is queued or in flight; returns all results."""
        import time
        out_ids, out_st, out_U = [], [], []
        t0 = time.time()
        while True:
            ids, st, U = self.poll()
            out_ids.append(ids); out_st.append(st); out_U.append(U)
            if self.pending() == 0 and len(ids) == 0:
                break
            if time.time() - t0 > timeout_s:
                raise TimeoutError("fold-in server did not drain")
        return np.concatenate(out_ids), np.concatenate(out_st), np.concatenate(out_U)

    def replay(self, arrival_ns, pool_row, pool, want_U: bool = False):
        """Open-loop replay (als_server_replay); returns (completion_ns, status, U|None)."""
        n = len(arrival_ns)
        comp = np.empty(n, np.int64)
        st = np.empty(n, np.int32)
        U = np.empty((n, self.n_f), self.np_dtype) if want_U else None
        L.als_server_replay(self.handle, np.ascontiguousarray(arrival_ns, dtype=np.int64),
                            np.ascontiguousarray(pool_row, dtype=np.int32),
                            np.ascontiguousarray(pool.indptr, dtype=np.int64),
                            np.ascontiguousarray(pool.indices, dtype=np.int32),
                            np.ascontiguousarray(pool.values, dtype=np.float32), comp, st, U)
        return comp, st, U
