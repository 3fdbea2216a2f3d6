"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with a retyped copy of itself: each check is
a brute-force solve, a closed form, an invariant, a worked example or an
identity between two different formulas.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small(seed=3, n_u=40, n_m=30, n_f=4, lam=0.05, **kw):
    P = synth.random_problem(n_u, n_m, n_f=n_f, lam=lam, seed=seed, density=0.3,
                             x0_sigma=1.0, **kw)
    return P


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- worked example

def test_hand_worked_example():
    """Every per-call oracle on a 2x2, n_f=1 problem worked by hand (fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "hand_2x2.json")))
    R = synth.csr_from_pairs(np.array(g["rows"]), np.array(g["cols"]), np.array(g["values"]),
                             g["n_u"], g["n_m"])
    Rt = synth.transpose(R)
    U, M = np.array(g["U"]), np.array(g["M"])
    lam = g["lambda"]
    assert oracle.loss(R, U, M, lam) == pytest.approx(g["f"], rel=1e-15)
    gU, gM = oracle.gradient(R, Rt, U, M, lam)
    np.testing.assert_allclose(gU, g["gU"], rtol=1e-15)
    np.testing.assert_allclose(gM, g["gM"], rtol=1e-15)
    np.testing.assert_allclose(oracle.half_sweep(R, M, lam), g["U_from_M"], rtol=1e-15)
    np.testing.assert_allclose(oracle.half_sweep(Rt, U, lam), g["M_from_U"], rtol=1e-15)
    C = oracle.quartic(R, U, M, np.array(g["pU"]), np.array(g["pM"]), lam)
    np.testing.assert_allclose(C, g["quartic"], rtol=0, atol=1e-14)
    alpha, n = oracle.backtrack(C)
    assert n == g["backtrack_trials"]
    assert alpha == pytest.approx(g["backtrack_alpha"], rel=1e-14)


# ---------------------------------------------------------------- P1 brute force

@pytest.mark.parametrize("n_f", [1, 3, 8])
def test_half_sweep_matches_lstsq(n_f):
    """P1: each row solve is the ridge least-squares problem
    min ||Y_I u - r||^2 + lam n_i ||u||^2, solved by numpy lstsq on the
    stacked system [Y_I; sqrt(lam n_i) I] u = [r; 0]."""
    P = small(n_f=n_f, long_rows=1, empty_rows=2)
    Y = np.random.default_rng(1).normal(size=(P.n_m, n_f))
    X = oracle.half_sweep(P.R, Y, P.lam)
    for i in range(P.n_u):
        a, b = P.R.indptr[i], P.R.indptr[i + 1]
        if a == b:
            assert np.all(X[i] == 0.0)
            continue
        Yi = Y[P.R.indices[a:b]]
        r = P.R.values[a:b].astype(np.float64)
        S = np.vstack([Yi, math.sqrt(P.lam * (b - a)) * np.eye(n_f)])
        t = np.concatenate([r, np.zeros(n_f)])
        ref = np.linalg.lstsq(S, t, rcond=None)[0]
        assert rel(X[i], ref) < 1e-12


def test_fold_in_is_a_row_solve():
    """Fold-in of a request equals the lstsq solve of that request's row."""
    rng = np.random.default_rng(5)
    M = rng.normal(size=(50, 6))
    req = synth.fold_in_requests(8, 50, seed=2, max_len=40)
    X = oracle.fold_in(M, req, 0.05)
    for i in range(8):
        a, b = req.indptr[i], req.indptr[i + 1]
        S = np.vstack([M[req.indices[a:b]], math.sqrt(0.05 * (b - a)) * np.eye(6)])
        t = np.concatenate([req.values[a:b].astype(np.float64), np.zeros(6)])
        assert rel(X[i], np.linalg.lstsq(S, t, rcond=None)[0]) < 1e-12


# ---------------------------------------------------------------- P2 / P3 invariants

def test_block_gradient_zero_after_half_sweep():
    """P2: a half-sweep is an exact block minimiser, so the gradient block of
    the updated side vanishes (relative to the size of its data term)."""
    P = small(n_f=5)
    U = oracle.half_sweep(P.R, P.M0, P.lam)
    gU, _ = oracle.gradient(P.R, P.Rt, U, P.M0, P.lam)
    scale = np.linalg.norm(2 * P.M0.T @ np.ones(P.n_m)) + 1.0
    assert np.linalg.norm(gU) < 1e-10 * scale
    M = oracle.half_sweep(P.Rt, U, P.lam)
    _, gM = oracle.gradient(P.R, P.Rt, U, M, P.lam)
    assert np.linalg.norm(gM) < 1e-10 * (np.linalg.norm(U) + 1.0)


def test_als_monotone_on_tiny_planted(c0):
    """P3: f never increases across ALS half-sweeps (Algorithm 1)."""
    U, M = c0.U0, c0.M0
    prev = oracle.loss(c0.R, U, M, c0.lam)
    for _ in range(10):
        U = oracle.half_sweep(c0.R, M, c0.lam)
        f1 = oracle.loss(c0.R, U, M, c0.lam)
        assert f1 <= prev * (1 + 1e-14)
        M = oracle.half_sweep(c0.Rt, U, c0.lam)
        f2 = oracle.loss(c0.R, U, M, c0.lam)
        assert f2 <= f1 * (1 + 1e-14)
        prev = f2


# ---------------------------------------------------------------- P4 quartic

def test_quartic_matches_direct_evaluation():
    """P4: Q(alpha) equals f(x + alpha p) evaluated directly at 5 step sizes;
    solving the 5x5 Vandermonde system recovers C0..C4; C0 = f(x), C1 = g^T p."""
    P = small(n_f=6)
    rng = np.random.default_rng(7)
    U, M = P.U0, P.M0
    PU, PM = rng.normal(size=U.shape), rng.normal(size=M.shape)
    C = oracle.quartic(P.R, U, M, PU, PM, P.lam)
    alphas = np.array([0.0, 0.3, 1.0, 2.5, 10.0])
    fd = np.array([oracle.loss(P.R, U + a * PU, M + a * PM, P.lam) for a in alphas])
    q = np.polyval(C[::-1], alphas)
    assert rel(q, fd) < 1e-13
    V = np.vander(alphas, 5, increasing=True)
    assert rel(np.linalg.solve(V, fd), C) < 1e-9
    assert C[0] == pytest.approx(oracle.loss(P.R, U, M, P.lam), rel=1e-14)
    gU, gM = oracle.gradient(P.R, P.Rt, U, M, P.lam)
    assert C[1] == pytest.approx(float(np.sum(gU * PU) + np.sum(gM * PM)), rel=1e-12)
    assert C[4] >= 0.0


# ---------------------------------------------------------------- P5 gradient

def test_gradient_matches_five_point_difference():
    """P5: f is a quartic along any line, so the 5-point central difference
    is exact up to rounding (not O(h^4)): it pins the directional derivative;
    coordinate directions pin single gradient entries."""
    P = small(n_f=3, n_u=15, n_m=12)
    U, M = P.U0, P.M0
    gU, gM = oracle.gradient(P.R, P.Rt, U, M, P.lam)
    rng = np.random.default_rng(11)
    h = 1e-2

    def dd(DU, DM):
        f = lambda t: oracle.loss(P.R, U + t * DU, M + t * DM, P.lam)
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    for _ in range(3):
        DU, DM = rng.normal(size=U.shape), rng.normal(size=M.shape)
        assert dd(DU, DM) == pytest.approx(np.sum(gU * DU) + np.sum(gM * DM), rel=1e-9, abs=1e-9)
    for (i, k) in [(0, 0), (3, 2), (14, 1)]:
        DU = np.zeros_like(U); DU[i, k] = 1.0
        assert dd(DU, np.zeros_like(M)) == pytest.approx(gU[i, k], rel=1e-8, abs=1e-8)
    for (j, k) in [(0, 1), (11, 2)]:
        DM = np.zeros_like(M); DM[j, k] = 1.0
        assert dd(np.zeros_like(U), DM) == pytest.approx(gM[j, k], rel=1e-8, abs=1e-8)


def test_gradient_u_block_is_normal_equation_residual():
    """g_U = 2 (A_i u_i - v_i) with A_i, v_i the normal-equation terms of Eq. (3)."""
    P = small(n_f=4)
    U, M = P.U0, P.M0
    gU, _ = oracle.gradient(P.R, P.Rt, U, M, P.lam)
    for i in range(P.n_u):
        a, b = P.R.indptr[i], P.R.indptr[i + 1]
        Y = M[P.R.indices[a:b]]
        A = Y.T @ Y + P.lam * (b - a) * np.eye(4)
        v = Y.T @ P.R.values[a:b].astype(np.float64)
        np.testing.assert_allclose(gU[i], 2 * (A @ U[i] - v), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P6 f forms

def test_loss_per_row_equals_per_rating_form():
    """P6: because the regulariser weights are the counts, Eq. (1) equals
    sum over ratings of (r - u.m)^2 + lam (||u_i||^2 + ||m_j||^2)."""
    P = small(n_f=5, empty_rows=3)
    U, M = P.U0, P.M0
    rows = np.repeat(np.arange(P.n_u), P.R.counts())
    cols = P.R.indices.astype(np.int64)
    e = P.R.values - np.sum(U[rows] * M[cols], axis=1)
    per_rating = np.sum(e * e + P.lam * (np.sum(U[rows] ** 2, 1) + np.sum(M[cols] ** 2, 1)))
    assert oracle.loss(P.R, U, M, P.lam) == pytest.approx(per_rating, rel=1e-13)
    assert oracle.loss(P.R, np.zeros_like(U), np.zeros_like(M), P.lam) == pytest.approx(
        float(np.sum(P.R.values.astype(np.float64) ** 2)), rel=1e-15)


# ---------------------------------------------------------------- P7 n_f = 1

def test_nf1_closed_form():
    """P7: with n_f = 1, u_i = sum_j r_ij m_j / (sum_j m_j^2 + lam n_i)."""
    P = small(n_f=1)
    M = P.M0
    U = oracle.half_sweep(P.R, M, P.lam)
    for i in range(P.n_u):
        a, b = P.R.indptr[i], P.R.indptr[i + 1]
        m = M[P.R.indices[a:b], 0]
        r = P.R.values[a:b].astype(np.float64)
        ref = np.sum(r * m) / (np.sum(m * m) + P.lam * (b - a)) if b > a else 0.0
        assert U[i, 0] == pytest.approx(ref, rel=1e-14, abs=1e-300)


# ---------------------------------------------------------------- P8 dense optimum

def test_dense_global_optimum_svd_shrinkage():
    """P8: with every rating observed the minimum of Eq. (1) has the closed form
    sum_{k>n_f} s_k^2 + sum_{k<=n_f} (s_k > t ? 2 t s_k - t^2 : s_k^2),
    t = lam sqrt(n_u n_m), s_k the singular values of R (variational form of
    the nuclear norm).  ALS and ALS-NCG both reach it."""
    n_u, n_m, n_f, lam = 20, 15, 3, 0.05
    P = synth.dense_problem(n_u, n_m, n_f=n_f, lam=lam, seed=4, rank=3, noise=0.3)
    Rd = np.zeros((n_u, n_m))
    rows = np.repeat(np.arange(n_u), P.R.counts())
    Rd[rows, P.R.indices] = P.R.values
    s = np.linalg.svd(Rd, compute_uv=False)
    t = lam * math.sqrt(n_u * n_m)
    fstar = float(np.sum(s[n_f:] ** 2) + sum((2 * t * x - t * t) if x > t else x * x for x in s[:n_f]))
    U, M, fs = oracle.als_run(P.R, P.Rt, P.M0, lam, 600)
    assert fs[-1] == pytest.approx(fstar, rel=1e-10)
    st, fn = oracle.als_ncg_run(P.R, P.Rt, P.U0, P.M0, lam, 60)
    assert min(fn) == pytest.approx(fstar, rel=1e-10)


# ---------------------------------------------------------------- P9 PCG equivalence

def test_ncg_loop_is_pcg_on_convex_quadratic():
    """P9: on phi(x) = x^T A x / 2 - b^T x with P(x) = x - B (A x - b) and an exact
    line search, Algorithm 2 with beta of Eq. (8) is preconditioned CG with
    preconditioner B (Section III-B); it matches textbook PCG iterate by
    iterate and terminates in at most n steps."""
    rng = np.random.default_rng(0)
    n = 25
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T
    b = rng.normal(size=n)
    Bp = np.diag(1.0 / np.diag(A))
    grad = lambda x: A @ x - b
    P = lambda x: x - Bp @ (A @ x - b)

    def exact(x, p):
        g = grad(x)
        return -float(g @ p) / float(p @ A @ p), 0, float("nan"), float(g @ p)

    x0 = rng.normal(size=n)
    st, hist = oracle.ncg_loop(x0, P, grad, exact, n_iter=n,
                               stop=lambda s: np.linalg.norm(s.g) < 1e-12 * np.linalg.norm(b))
    # textbook preconditioned CG
    x = x0.copy(); r = A @ x - b; y = Bp @ r; p = -y
    ref = [x.copy()]
    for _ in range(len(hist) - 1):
        Ap = A @ p
        a = float(r @ y) / float(p @ Ap)
        x = x + a * p
        rn = r + a * Ap
        yn = Bp @ rn
        beta = float(rn @ yn) / float(r @ y)
        p = -yn + beta * p
        r, y = rn, yn
        ref.append(x.copy())
    for k in range(min(len(hist), 12)):
        assert rel(hist[k], ref[k]) < 1e-9
    assert len(hist) - 1 <= n
    assert np.linalg.norm(A @ hist[-1] - b) < 1e-8 * np.linalg.norm(b)


# ---------------------------------------------------------------- P10 conditioning

def test_normal_equation_conditioning_bound():
    """P10: lam n_i <= eig(A_i) <= n_i (max_j ||m_j||^2 + lam), so
    cond(A_i) <= 1 + max_j ||m_j||^2 / lam whatever n_i is."""
    P = small(n_f=6)
    M = P.M0
    mx = float(np.max(np.sum(M * M, axis=1)))
    for i in range(P.n_u):
        a, b = P.R.indptr[i], P.R.indptr[i + 1]
        if a == b:
            continue
        Y = M[P.R.indices[a:b]]
        w = np.linalg.eigvalsh(Y.T @ Y + P.lam * (b - a) * np.eye(6))
        assert w[0] >= P.lam * (b - a) * (1 - 1e-12)
        assert w[-1] <= (b - a) * (mx + P.lam) * (1 + 1e-12)
        assert w[-1] / w[0] <= 1 + mx / P.lam + 1e-9


# ---------------------------------------------------------------- Algorithm 4

def test_backtracking_first_armijo_step():
    """Algorithm 4: the accepted step is the first alpha_0 tau^n whose direct
    evaluation satisfies Q(alpha) - Q(0) <= alpha c Q'(0); every earlier one fails."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        C = np.array([5.0, -abs(rng.normal()) - 0.1, rng.normal(), rng.normal(), abs(rng.normal())])
        alpha, n = oracle.backtrack(C)
        q = lambda a: float(np.polyval(C[::-1], a))
        a = 10.0
        for k in range(n):
            assert q(a) - q(0.0) > a * 0.5 * C[1] - 1e-12 * abs(C[0])
            a *= 0.9
        assert a == alpha
        assert q(alpha) - q(0.0) <= alpha * 0.5 * C[1] + 1e-12 * abs(C[0])
    assert oracle.backtrack([1.0, 1.0, 0.0, 0.0, 1.0])[0] is None  # ascent direction never accepted


@pytest.mark.parametrize("c", [0.1, 0.9])
def test_backtracking_other_sufficient_decrease_constants(c):
    """Algorithm 4 with c != 1/2 (so c and 1 - c cannot be confused) and other tau."""
    C = np.array([3.0, -2.0, -1.0, 0.5, 0.7])
    alpha, n = oracle.backtrack(C, alpha0=4.0, tau=0.5, c=c)
    q = lambda a: float(np.polyval(C[::-1], a))
    assert q(alpha) - q(0.0) <= alpha * c * C[1]
    if n:
        assert q(2 * alpha) - q(0.0) > 2 * alpha * c * C[1]
    assert alpha == 4.0 * 0.5 ** n


# ---------------------------------------------------------------- Algorithm 2 invariants

def test_als_ncg_decreases_f_and_q_matches_f(c0):
    """Along ALS-NCG (Algorithm 2) with backtracking, every accepted step obeys
    sufficient decrease, so f(x_k) strictly decreases; Q(alpha_k) reproduces
    f(x_{k+1}); the result beats ALS's first sweep."""
    o = oracle.NcgOracle(c0.R, c0.Rt, c0.n_f, c0.lam)
    s = o.init(c0.U0, c0.M0)
    f_prev = o.f(s.x)
    for _ in range(8):
        o.step(s)
        f_now = o.f(s.x)
        assert s.safeguards == 0
        assert f_now < f_prev
        assert s.f == pytest.approx(f_now, rel=1e-12)
        f_prev = f_now
    _, _, fa = oracle.als_run(c0.R, c0.Rt, c0.M0, c0.lam, 1)
    assert f_prev < fa[0]


# ---------------------------------------------------------------- safeguards of Algorithm 2

# The paper says nothing about a line search that fails or a direction that
# is not a descent direction.  The reading taken here: when g^T p >= 0 or the
# search fails, p is reset to -gbar_k and the search is run again (a
# restart); if that fails too, the ALS point x_{k+1} = P(x_k) is taken and the
# next direction restarts (beta = 0).  Each pin below compares ncg_step with
# quantities formed separately: P from oracle.als_sweep, g from
# oracle.gradient, steps from oracle.quartic and oracle.backtrack.

def _ncg_parts(P):
    o = oracle.NcgOracle(P.R, P.Rt, P.n_f, P.lam)

    def als_point(x):
        _, M = o.split(x)
        U2, M2 = oracle.als_sweep(P.R, P.Rt, M, P.lam)
        return o.join(U2, M2)

    def grad(x):
        U, M = o.split(x)
        return o.join(*oracle.gradient(P.R, P.Rt, U, M, P.lam))
    return o, als_point, grad


def _advanced_state(o, P, k=3):
    """An ALS-NCG state a few iterations in, so beta and p are generic."""
    s = o.init(P.U0, P.M0)
    for _ in range(k):
        o.step(s)
    assert s.safeguards == 0
    return s


def test_safeguard_failed_search_takes_the_als_point(c0):
    """A line search that never accepts: the step must restart once, then take
    x_{k+1} = P(x_k) (the ALS iteration, formed here by its own call), and the
    next direction must be -gbar_{k+1} exactly (beta reset), with
    gbar_{k+1} = x_{k+1} - P(x_{k+1})."""
    o, als_point, grad = _ncg_parts(c0)
    s = _advanced_state(o, c0)
    x_k = s.x.copy()
    r0 = s.restarts
    calls = []

    def never(x, p):
        calls.append(p.copy())
        return None, 400, float("nan"), float(grad(x) @ p)

    oracle.ncg_step(s, o.P, o.grad, never)
    assert len(calls) == 2                                 # first search, then the restarted one
    np.testing.assert_array_equal(calls[1], -(x_k - als_point(x_k)))  # restart on -gbar_k
    assert (s.restarts - r0, s.safeguards) == (1, 1)
    assert rel(s.x, als_point(x_k)) <= 1e-15
    gbar_new = s.x - als_point(s.x)
    assert rel(s.p, -gbar_new) <= 1e-15                     # beta = 0 after the ALS point
    assert rel(s.g, grad(s.x)) <= 1e-15
    assert math.isnan(s.alpha) and math.isnan(s.f)
    # f does not increase: the ALS point minimises each block in turn
    assert o.f(s.x) <= o.f(x_k)


def test_safeguard_ascent_direction_is_restarted_on_minus_gbar(c0):
    """A direction with g^T p > 0 is replaced by -gbar_k before any step is
    taken: with a line search that accepts any direction at a fixed alpha,
    x_{k+1} = x_k - alpha gbar_k (not x_k + alpha p_k), one restart, no ALS
    point, and beta of Eq. (8) is kept for the next direction."""
    o, als_point, grad = _ncg_parts(c0)
    s = _advanced_state(o, c0)
    x_k, g_k = s.x.copy(), grad(s.x)
    r0 = s.restarts
    gbar_k = x_k - als_point(x_k)
    s.p = g_k.copy()                                         # ascent: g^T p = ||g||^2 > 0
    alpha = 0.37

    def fixed(x, p):
        return alpha, 0, float("nan"), float(grad(x) @ p)

    oracle.ncg_step(s, o.P, o.grad, fixed)
    assert (s.restarts - r0, s.safeguards) == (1, 0)
    assert rel(s.x, x_k - alpha * gbar_k) <= 1e-15
    gbar_new = s.x - als_point(s.x)
    g_new = grad(s.x)
    beta = float(gbar_new @ (g_new - g_k)) / float(gbar_k @ g_k)
    assert beta != 0.0
    assert rel(s.p, -gbar_new + beta * (-gbar_k)) <= 1e-13


def test_safeguard_restart_still_ascent_takes_the_als_point(c0):
    """When -gbar_k is not a descent direction either (a line search that
    reports g^T p >= 0 for everything), the ALS point is taken."""
    o, als_point, grad = _ncg_parts(c0)
    s = _advanced_state(o, c0)
    x_k = s.x.copy()
    r0 = s.restarts

    def uphill(x, p):
        return 1.0, 0, float("nan"), 1.0

    oracle.ncg_step(s, o.P, o.grad, uphill)
    assert (s.restarts - r0, s.safeguards) == (1, 1)
    assert rel(s.x, als_point(x_k)) <= 1e-15
    assert rel(s.p, -(s.x - als_point(s.x))) <= 1e-15


def test_safeguard_first_search_fails_restart_succeeds(c0):
    """Backtracking with a cap too small for the first direction: the restarted
    search on -gbar_k is Algorithm 4 on the quartic along -gbar_k (formed by
    oracle.quartic and oracle.backtrack here), and its step is taken."""
    o, als_point, grad = _ncg_parts(c0)
    s = _advanced_state(o, c0)
    x_k = s.x.copy()
    r0 = s.restarts
    gbar_k = x_k - als_point(x_k)
    U, M = o.split(x_k)
    PU, PM = o.split(-gbar_k)
    C = oracle.quartic(c0.R, U, M, PU, PM, c0.lam)
    a_ref, n_ref = oracle.backtrack(C)
    assert a_ref is not None
    seen = []

    def first_fails(x, p):
        Ux, Mx = o.split(x)
        Pu, Pm = o.split(p)
        Cp = oracle.quartic(c0.R, Ux, Mx, Pu, Pm, c0.lam)
        if not seen:
            seen.append(1)
            return None, 0, float("nan"), float(Cp[1])
        a, n = oracle.backtrack(Cp)
        return a, n, float(np.polyval(Cp[::-1], a)), float(Cp[1])

    oracle.ncg_step(s, o.P, o.grad, first_fails)
    assert (s.restarts - r0, s.safeguards) == (1, 0)
    assert s.trials == n_ref
    assert rel(s.x, x_k - a_ref * gbar_k) <= 1e-15


def test_safeguards_along_a_run_with_a_tight_trial_cap():
    """NcgOracle with alpha_0 = 1e3 and at most 60 trials (alpha >= 1e3 * 0.9^59
    = 2.0): many first searches fail.  Every iteration must then either take an
    Armijo step along p_k or -gbar_k, or the ALS point P(x_k); f never increases;
    and the counters count exactly those events."""
    P = synth.random_problem(80, 60, n_f=6, lam=0.05, seed=21, density=0.25, x0_sigma=0.5)
    o = oracle.NcgOracle(P.R, P.Rt, P.n_f, P.lam, alpha0=1e3, max_trials=60)
    _, als_point, grad = _ncg_parts(P)
    s = o.init(P.U0, P.M0)
    f_prev = o.f(s.x)
    restarts = safeguards = 0
    for _ in range(12):
        x_k, p_k = s.x.copy(), s.p.copy()
        gbar_k = x_k - als_point(x_k)
        o.step(s)
        f_now = o.f(s.x)
        assert f_now <= f_prev * (1 + 1e-14)
        if s.safeguards > safeguards:
            assert rel(s.x, als_point(x_k)) <= 1e-15
            restarts += 1
            safeguards += 1
        else:
            d = p_k if s.restarts == restarts else -gbar_k
            restarts = s.restarts
            assert s.alpha == pytest.approx(1e3 * 0.9 ** s.trials, rel=1e-12)
            assert rel(s.x, x_k + s.alpha * d) <= 1e-14
        assert (s.restarts, s.safeguards) == (restarts, safeguards)
        f_prev = f_now
    assert restarts > 0 and safeguards > 0


# ---------------------------------------------------------------- reduced precision

def test_bf16_round_matches_torch_and_hand_values():
    """bf16_round against torch's float32 -> bfloat16 conversion (round to
    nearest even, an independent implementation) on random magnitudes over 40
    decades, and hand-rounded values: 1 + 2^-8 is a tie between 1 and
    1 + 2^-7 and goes to the even mantissa (1); 1 + 3 2^-8 is a tie that goes
    up to 1 + 2^-6 (1.015625); 65504 (the largest FP16) rounds to 65536."""
    import torch
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200_000) * 10.0 ** rng.integers(-20, 20, 200_000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(oracle.bf16_round(x), ref)
    hand = {1.0: 1.0, 1 + 2**-8: 1.0, 1 + 3 * 2**-8: 1.015625, 1 + 2**-8 + 2**-20: 1 + 2**-7,
            -2.5: -2.5, 65504.0: 65536.0, 0.1: 0.10009765625}
    got = oracle.bf16_round(np.array(list(hand), dtype=np.float32))
    np.testing.assert_array_equal(got, np.array(list(hand.values())))


def test_mixed_half_sweep_on_bf16_exact_inputs_is_the_plain_row_solve():
    """With factors and ratings that bfloat16 represents exactly (8 significant
    bits), rounding changes nothing and the unrefined reduced-precision solve
    is the plain row solve of Eq. (3) computed by the C oracle; the refinement
    step then adds a zero residual."""
    P = small(seed=11, n_f=5)
    M = oracle.bf16_round(P.M0.astype(np.float32)).reshape(P.M0.shape)
    ref = oracle.half_sweep(P.R, M, P.lam)
    assert rel(oracle.mixed_half_sweep(P.R, M, P.lam, refine=False), ref) < 1e-12
    assert rel(oracle.mixed_half_sweep(P.R, M, P.lam, refine=True), ref) < 1e-12


def test_mixed_refinement_error_identity():
    """One refinement step obeys x1 - x* = (I - At^{-1} A)(x0 - x*), x* the
    exact row solve (C oracle), A the FP32 normal matrix and At its bfloat16
    counterpart: x1 = x0 + At^{-1}(v - A x0) and v = A x*.  A dropped term, a
    sign or a transposed operand in the refinement breaks the identity; the
    step must also shrink the error."""
    P = small(seed=12, n_f=6, n_u=25)
    M = P.M0.astype(np.float32)
    xs = oracle.half_sweep(P.R, M.astype(np.float64), P.lam)
    x0 = oracle.mixed_half_sweep(P.R, M, P.lam, refine=False)
    x1 = oracle.mixed_half_sweep(P.R, M, P.lam, refine=True)
    Mt = oracle.bf16_round(M).reshape(M.shape)
    Md = M.astype(np.float64)
    e0 = e1 = 0.0
    for i in range(P.R.n_rows):
        lo, hi = P.R.indptr[i], P.R.indptr[i + 1]
        ids = P.R.indices[lo:hi]
        if hi == lo:
            continue
        n = hi - lo
        A = Md[ids].T @ Md[ids] + P.lam * n * np.eye(P.n_f)
        At = Mt[ids].T @ Mt[ids] + P.lam * n * np.eye(P.n_f)
        pred = (np.eye(P.n_f) - np.linalg.solve(At, A)) @ (x0[i] - xs[i])
        np.testing.assert_allclose(x1[i] - xs[i], pred, rtol=0, atol=1e-10 * np.abs(xs[i]).max())
        e0 = max(e0, np.abs(x0[i] - xs[i]).max())
        e1 = max(e1, np.abs(x1[i] - xs[i]).max())
    assert e0 > 1e-4 and e1 < 0.05 * e0


def test_quartic_min_is_the_global_minimiser_on_a_dense_grid():
    """The exact line search returns the global minimiser of Q over alpha > 0:
    checked against dense evaluation of Q on [0, 3 alpha*] for random quartics
    with C1 < 0 and C4 > 0 (including double-well shapes), and None for an
    ascent direction."""
    rng = np.random.default_rng(13)
    for _ in range(200):
        C = rng.normal(size=5)
        C[1] = -abs(C[1]) - 0.1
        C[4] = abs(C[4]) + 0.05
        a = oracle.quartic_min(C, c=1e-4)
        q = lambda t: np.polyval(C[::-1], t)  # noqa: E731
        grid = np.linspace(0.0, 3.0 * (a or 10.0), 200001)
        gmin = q(grid).min()
        if a is None:
            assert q(grid).min() > C[0] + 1e-4 * grid[np.argmin(q(grid))] * C[1] - 1e-12
            continue
        assert q(a) <= gmin + 1e-9 * (1.0 + abs(gmin))
    assert oracle.quartic_min([1.0, 0.5, 1.0, 0.0, 1.0]) is None
