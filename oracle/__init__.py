"""Plain FP64 CPU oracle for the ALS / ALS-NCG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this package; the product library never
does, and this package never imports the product.  The per-row arithmetic
lives in ``als_oracle.c`` (plain C, double precision); this module adds the
outer algorithms in numpy float64:

* ``als_sweep``      -- one ALS iteration P(x), Algorithm 1 (Section III-A);
* ``mixed_half_sweep`` -- the row solve of Eq. (3) on bfloat16 copies of the
                        fixed factor, with an optional refinement step
                        against the FP32 normal equations;
* ``backtrack``      -- backtracking line search on the quartic, Algorithm 4
                        with tau = 0.9, c = 0.5, alpha_0 = 10 (Section V-C);
* ``NcgOracle``      -- ALS-NCG, Algorithm 2 with the preconditioned
                        Polak-Ribiere beta of Eq. (8) (Section III-B);
* ``ncg_loop``       -- the same iteration with pluggable P, gradient and line
                        search (used to check the PCG equivalence the paper
                        states for convex quadratics).

The submodule ``ranking`` holds the top-t ranking accuracy of Section IV (a
modified Kendall tau distance between the top-t rankings of two solutions).

Every function cites the passage it implements.  Parity is pinned by the CPU
tests (brute-force least squares, block-gradient zero, monotone ALS, quartic
against direct evaluation, finite differences, closed forms).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Callable, Optional

import numpy as np

from . import ranking  # noqa: E402,F401  (Section IV ranking accuracy)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "als_oracle.c")
_LIB = os.environ.get("ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

# line-search constants of Section V-C (tau, c, alpha_0)
TAU = 0.9
C_ARMIJO = 0.5
ALPHA0 = 10.0
MAX_TRIALS = 400


def build(force: bool = False) -> str:
    """Compile als_oracle.c with gcc (double precision, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        # ORACLE_CFLAGS (e.g. "-O3 -march=native") only changes code generation;
        # -ffp-contract=off keeps every product and sum separately rounded.
        extra = os.environ.get("ORACLE_CFLAGS", "-O2").split()
        subprocess.check_call(["gcc"] + extra + ["-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_half_sweep.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_int,
                                       ctypes.c_double, _f64p, _i64p]
        lib.orc_half_sweep.restype = ctypes.c_int
        lib.orc_loss.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p,
                                 ctypes.c_int, ctypes.c_double]
        lib.orc_loss.restype = ctypes.c_double
        lib.orc_gradient.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int64, _i64p,
                                     _i32p, _f64p, _f64p, _f64p, ctypes.c_int, ctypes.c_double,
                                     _f64p, _f64p]
        lib.orc_gradient.restype = None
        lib.orc_quartic.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p, _f64p,
                                    _f64p, _f64p, _f64p, ctypes.c_int, ctypes.c_double, _f64p]
        lib.orc_quartic.restype = None
        _lib = lib
    return _lib


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (n > 0); returns the count now in effect."""
    return _load().orc_set_threads(int(n))


def _p(a, t):
    return a.ctypes.data_as(t)


class _Csr64:
    """The CSR with float64 values, kept alive for the C calls."""

    def __init__(self, A):
        self.n_rows, self.n_cols = int(A.n_rows), int(A.n_cols)
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.values = np.ascontiguousarray(A.values, dtype=np.float64)


def _c(A):
    return A if isinstance(A, _Csr64) else _Csr64(A)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# per-call oracles (plain definitions)
# ----------------------------------------------------------------------------

def half_sweep(A, Y: np.ndarray, lam: float, raise_on_bad: bool = True) -> np.ndarray:
    """Eq. (3) / Eq. (4): x_i = (Y_I^T Y_I + lam n_i I)^-1 Y_I^T r_i for every row."""
    A = _c(A)
    Y = _f64(Y)
    n_f = Y.shape[1]
    X = np.empty((A.n_rows, n_f), dtype=np.float64)
    bad = ctypes.c_int64(-1)
    rc = _load().orc_half_sweep(A.n_rows, _p(A.indptr, _i64p), _p(A.indices, _i32p),
                                _p(A.values, _f64p), _p(Y, _f64p), n_f, float(lam),
                                _p(X, _f64p), ctypes.byref(bad))
    if rc != 0 and raise_on_bad:
        raise np.linalg.LinAlgError("row %d: normal equations not SPD" % bad.value)
    return X


def fold_in(M: np.ndarray, requests, lam: float) -> np.ndarray:
    """Fold-in of new users against fixed M: Eq. (3) applied to request rows."""
    return half_sweep(requests, M, lam)


def loss(R, U: np.ndarray, M: np.ndarray, lam: float) -> float:
    """f of Eq. (1)."""
    R = _c(R)
    U, M = _f64(U), _f64(M)
    return _load().orc_loss(R.n_rows, R.n_cols, _p(R.indptr, _i64p), _p(R.indices, _i32p),
                            _p(R.values, _f64p), _p(U, _f64p), _p(M, _f64p), U.shape[1], float(lam))


def gradient(R, Rt, U: np.ndarray, M: np.ndarray, lam: float):
    """(g_U, g_M): the gradient of Eq. (1) (Section III-A, Section V-C)."""
    R, Rt = _c(R), _c(Rt)
    U, M = _f64(U), _f64(M)
    gU = np.empty_like(U)
    gM = np.empty_like(M)
    _load().orc_gradient(R.n_rows, _p(R.indptr, _i64p), _p(R.indices, _i32p), _p(R.values, _f64p),
                         Rt.n_rows, _p(Rt.indptr, _i64p), _p(Rt.indices, _i32p),
                         _p(Rt.values, _f64p), _p(U, _f64p), _p(M, _f64p), U.shape[1],
                         float(lam), _p(gU, _f64p), _p(gM, _f64p))
    return gU, gM


def quartic(R, U, M, PU, PM, lam: float) -> np.ndarray:
    """C[0..4] with f(x + alpha p) = sum_n C[n] alpha^n (Section V-C)."""
    R = _c(R)
    U, M, PU, PM = _f64(U), _f64(M), _f64(PU), _f64(PM)
    C = np.zeros(5, dtype=np.float64)
    _load().orc_quartic(R.n_rows, R.n_cols, _p(R.indptr, _i64p), _p(R.indices, _i32p),
                        _p(R.values, _f64p), _p(U, _f64p), _p(M, _f64p), _p(PU, _f64p),
                        _p(PM, _f64p), U.shape[1], float(lam), _p(C, _f64p))
    return C


# ----------------------------------------------------------------------------
# reduced-precision half-sweep (the row solve of Eq. (3) on bfloat16 copies)
# ----------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Nearest bfloat16 value of each FP32 input, ties to even, as float64.

    bfloat16 is the upper half of an IEEE binary32 word (sign, 8 exponent
    bits, 7 stored mantissa bits).  Rounding adds half a unit of the dropped
    16 bits, plus one when the kept part is odd and the dropped part is
    exactly half (round half to even); a mantissa carry moves into the
    exponent, as it should.  Inputs must be finite."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    half = np.uint64(0x7FFF) + ((a >> np.uint64(16)) & np.uint64(1))
    kept = ((a + half) >> np.uint64(16)) << np.uint64(16)
    return kept.astype(np.uint32).view(np.float32).astype(np.float64)


def mixed_half_sweep(A, Y32: np.ndarray, lam: float, refine: bool) -> np.ndarray:
    """Row solve of Eq. (3) (Eq. (4) for R^T) on bfloat16 copies, in FP64.

    For each row i with ratings (j, r_ij):
        At = sum_j yt_j yt_j^T + lam n_i I,   vt = sum_j bf16(r_ij) yt_j,
        x0 = At^{-1} vt                         (yt_j = bf16(Y32[j]))
    and with refine, one refinement step against the unrounded normal
    equations A x = v of Eq. (3):
        x1 = x0 + At^{-1} (v - A x0),  v - A x0 = sum_j (r_ij - y_j.x0) y_j - lam n_i x0.
    Rows without ratings are 0.  Dense per-row solves (numpy); tiny inputs only."""
    Y = _f64(np.asarray(Y32, dtype=np.float32))
    Yt = bf16_round(Y32).reshape(Y.shape)
    n_f = Y.shape[1]
    X = np.zeros((A.n_rows, n_f), dtype=np.float64)
    for i in range(A.n_rows):
        lo, hi = int(A.indptr[i]), int(A.indptr[i + 1])
        n = hi - lo
        if n == 0:
            continue
        ids = np.asarray(A.indices[lo:hi])
        r = np.asarray(A.values[lo:hi], dtype=np.float32)
        Gt = Yt[ids].T @ Yt[ids] + lam * n * np.eye(n_f)
        x = np.linalg.solve(Gt, Yt[ids].T @ bf16_round(r))
        if refine:
            Yi = Y[ids]
            res = Yi.T @ (r.astype(np.float64) - Yi @ x) - lam * n * x
            x = x + np.linalg.solve(Gt, res)
        X[i] = x
    return X


# ----------------------------------------------------------------------------
# Algorithm 1 and Algorithm 4
# ----------------------------------------------------------------------------

def als_sweep(R, Rt, M: np.ndarray, lam: float):
    """One ALS iteration, Algorithm 1: all u_i from M, then all m_j from the new U.
    This is the preconditioner P of Section III-B; it ignores the incoming U."""
    U = half_sweep(R, M, lam)
    return U, half_sweep(Rt, U, lam)


def backtrack(C, alpha0: float = ALPHA0, tau: float = TAU, c: float = C_ARMIJO,
              max_trials: int = MAX_TRIALS):
    """Backtracking line search, Algorithm 4, on Q(alpha) = sum C[n] alpha^n.

    The sufficient-decrease test Q(alpha) - Q(0) <= alpha c g^T p with
    g^T p = C[1] is divided by alpha > 0 so the two large C[0] terms never
    meet: accept alpha when (1 - c) C1 + alpha (C2 + alpha (C3 + alpha C4)) <= 0.
    Step lengths follow alpha <- tau alpha from alpha_0.  Returns
    (alpha, trials) with trials = number of rejected steps, or (None, trials)
    when max_trials steps were all rejected.
    """
    C = [float(x) for x in C]
    alpha = float(alpha0)
    for n in range(max_trials):
        t = (1.0 - c) * C[1] + alpha * (C[2] + alpha * (C[3] + alpha * C[4]))
        if t <= 0.0:
            return alpha, n
        alpha = tau * alpha
    return None, max_trials


# sufficient-decrease tolerance of the paper's serial line search (Section IV)
C_EXACT = 1e-4


def quartic_min(C, c: float = C_EXACT):
    """Exact line search on the same quartic (the stronger search the paper's
    serial runs use, Section IV, here on the Section V-C polynomial): the
    global minimiser over alpha > 0 of Q(alpha) = sum C[n] alpha^n, from the
    real roots of Q'(alpha) = C1 + 2 C2 alpha + 3 C3 alpha^2 + 4 C4 alpha^3
    (numpy.roots).  Returned only when it also passes the sufficient-decrease
    test of Algorithm 4 (divided by alpha, as in backtrack); else None.  None
    when C1 >= 0 (not a descent direction) or Q has no minimiser on alpha > 0."""
    C = [float(x) for x in C]
    if not C[1] < 0.0:
        return None
    der = [4.0 * C[4], 3.0 * C[3], 2.0 * C[2], C[1]]
    while der and der[0] == 0.0:
        der = der[1:]
    if len(der) < 2:
        return None
    roots = np.roots(der)
    cand = [r.real for r in roots if abs(r.imag) <= 1e-12 * max(1.0, abs(r.real)) and r.real > 0.0]
    if not cand:
        return None
    q = lambda a: C[0] + a * (C[1] + a * (C[2] + a * (C[3] + a * C[4])))  # noqa: E731
    best = min(cand, key=q)
    if (1.0 - c) * C[1] + best * (C[2] + best * (C[3] + best * C[4])) > 0.0:
        return None
    return best


# ----------------------------------------------------------------------------
# Algorithm 2 with pluggable pieces
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class NcgState:
    x: np.ndarray        # current iterate x_k (flat)
    p: np.ndarray        # search direction p_k
    g: np.ndarray        # true gradient g_k
    gbar: np.ndarray     # preconditioned gradient x_k - P(x_k)
    xbar: np.ndarray     # P(x_k), kept for the safeguard step
    k: int = 0
    f: float = float("nan")
    alpha: float = float("nan")
    trials: int = 0
    restarts: int = 0
    safeguards: int = 0


def ncg_init(x0, P: Callable, grad: Callable) -> NcgState:
    """Algorithm 2 set-up: gbar_0 = x_0 - P(x_0), p_0 = -gbar_0."""
    xbar = P(x0)
    gbar = x0 - xbar
    return NcgState(x=x0.copy(), p=-gbar, g=grad(x0), gbar=gbar, xbar=xbar)


def ncg_step(s: NcgState, P: Callable, grad: Callable, line_search: Callable,
             safeguard: bool = True, pr_plus: bool = False) -> NcgState:
    """One pass through the loop body of Algorithm 2.

    line_search(x, p) -> (alpha or None, trials, f(x + alpha p) or nan,
    g^T p).  Safeguard (a reading: the paper is silent on failures): when
    g^T p >= 0 the direction is reset to -gbar_k; when that is still not a
    descent direction, or the line search fails, x_{k+1} = P(x_k) (the ALS
    step) is taken and the next direction restarts (beta = 0).
    """
    restart = False
    alpha, trials, fnew, gtp = line_search(s.x, s.p)
    if safeguard and (gtp >= 0.0 or alpha is None):
        s.p = -s.gbar
        s.restarts += 1
        alpha, trials, fnew, gtp = line_search(s.x, s.p)
    if alpha is None or (safeguard and gtp >= 0.0):
        if not safeguard:
            raise RuntimeError("line search failed")
        x_new = s.xbar
        s.safeguards += 1
        restart = True
        alpha, fnew = float("nan"), float("nan")
    else:
        x_new = s.x + alpha * s.p
    xbar = P(x_new)
    gbar_new = x_new - xbar
    g_new = grad(x_new)
    den = float(s.gbar @ s.g)
    beta = float(gbar_new @ (g_new - s.g)) / den if (den != 0.0 and np.isfinite(den)) else 0.0
    if not np.isfinite(beta) or restart:
        beta = 0.0
    if pr_plus:
        beta = max(beta, 0.0)
    s.p = -gbar_new + beta * s.p
    s.x, s.g, s.gbar, s.xbar = x_new, g_new, gbar_new, xbar
    s.k += 1
    s.alpha, s.trials, s.f = alpha, trials, fnew
    return s


def ncg_loop(x0, P, grad, line_search, n_iter: int, stop: Optional[Callable] = None):
    """Algorithm 2 for n_iter iterations (or until stop(state) is true)."""
    s = ncg_init(x0, P, grad)
    hist = [s.x.copy()]
    for _ in range(n_iter):
        if stop is not None and stop(s):
            break
        ncg_step(s, P, grad, line_search)
        hist.append(s.x.copy())
    return s, hist


class NcgOracle:
    """ALS-NCG (Algorithm 2) for the loss of Eq. (1) on one ratings problem.

    x = [u_1 .. u_nu, m_1 .. m_nm] as in Eq. (5), flat float64.  P is one ALS
    iteration, the line search is Algorithm 4 on the quartic of Section V-C.
    """

    def __init__(self, R, Rt, n_f: int, lam: float, alpha0: float = ALPHA0, tau: float = TAU,
                 c: float = C_ARMIJO, max_trials: int = MAX_TRIALS, safeguard: bool = True,
                 pr_plus: bool = False):
        self.R, self.Rt = _c(R), _c(Rt)
        self.n_u, self.n_m, self.n_f, self.lam = self.R.n_rows, self.R.n_cols, n_f, float(lam)
        self.nU = self.n_u * n_f
        # Algorithm 4's constants (Section V-C: alpha_0 = 10, tau = 0.9, c = 0.5)
        # and the trial cap of the safeguard reading
        self.alpha0, self.tau, self.c, self.max_trials = float(alpha0), float(tau), float(c), int(max_trials)
        self.safeguard, self.pr_plus = bool(safeguard), bool(pr_plus)

    def split(self, x):
        return x[: self.nU].reshape(self.n_u, self.n_f), x[self.nU:].reshape(self.n_m, self.n_f)

    def join(self, U, M):
        return np.concatenate([np.asarray(U, np.float64).reshape(-1), np.asarray(M, np.float64).reshape(-1)])

    def P(self, x):
        _, M = self.split(x)
        U2, M2 = als_sweep(self.R, self.Rt, M, self.lam)
        return self.join(U2, M2)

    def grad(self, x):
        U, M = self.split(x)
        gU, gM = gradient(self.R, self.Rt, U, M, self.lam)
        return self.join(gU, gM)

    def f(self, x):
        U, M = self.split(x)
        return loss(self.R, U, M, self.lam)

    def coeffs(self, x, p):
        U, M = self.split(x)
        PU, PM = self.split(p)
        return quartic(self.R, U, M, PU, PM, self.lam)

    def line_search(self, x, p):
        C = self.coeffs(x, p)
        self.last_coeffs = C
        if C[1] >= 0.0:
            return None, 0, float("nan"), float(C[1])
        alpha, n = backtrack(C, self.alpha0, self.tau, self.c, self.max_trials)
        fnew = float("nan") if alpha is None else float(np.polyval(C[::-1], alpha))
        return alpha, n, fnew, float(C[1])

    def init(self, U0, M0) -> NcgState:
        return ncg_init(self.join(U0, M0), self.P, self.grad)

    def step(self, s: NcgState, **kw) -> NcgState:
        kw.setdefault("safeguard", self.safeguard)
        kw.setdefault("pr_plus", self.pr_plus)
        return ncg_step(s, self.P, self.grad, self.line_search, **kw)


def als_run(R, Rt, M0, lam: float, n_sweeps: int, U0=None):
    """Algorithm 1 for n_sweeps sweeps; returns (U, M, [f after each sweep])."""
    R, Rt = _c(R), _c(Rt)
    M = _f64(M0)
    fs = []
    U = U0
    for _ in range(n_sweeps):
        U, M = als_sweep(R, Rt, M, lam)
        fs.append(loss(R, U, M, lam))
    return U, M, fs


def als_ncg_run(R, Rt, U0, M0, lam: float, n_iter: int):
    """Algorithm 2 for n_iter iterations; returns (state, [f(x_k) for k=1..])."""
    o = NcgOracle(R, Rt, U0.shape[1], lam)
    s = o.init(U0, M0)
    fs = []
    for _ in range(n_iter):
        o.step(s)
        fs.append(o.f(s.x))
    return s, fs
