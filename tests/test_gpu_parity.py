"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances (derivations in the design notes):
  * FP64 path: per call <= 1e-12 relative (1e-11 for reductions of many terms);
    f after 20 ALS sweeps / 20 ALS-NCG iterations on the tiny planted problem
    <= 1e-10 relative;
  * FP32 path: half-sweep rows <= 1e-4 relative per row and <= 2e-5 on the whole
    factor; quartic coefficients and gradient <= 1e-5 of their scale; f after
    20 sweeps <= 1e-5 relative.
"""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    from paper_1508_03110_amd.solver import Context
    c = Context(0)
    yield c
    c.close()


def dev_problem(ctx, P, dtype, chunk=0, chunk_t=None, ld=None):
    from paper_1508_03110_amd.solver import DeviceProblem
    return DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, dtype, chunk=chunk, chunk_t=chunk_t, ld=ld)


def to_dev(a, dtype, ctx):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(ctx.torch_device)


def host(t, n_f=None):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[:, :n_f] if n_f is not None and a.ndim == 2 else a


def rowrel(a, b):
    """max over rows of ||a_i - b_i|| / max(||b_i||, tiny)."""
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float(np.max(num / den)) if a.shape[0] else 0.0


def fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


TOL = {torch.float64: dict(row=1e-11, fro=1e-12), torch.float32: dict(row=1e-4, fro=2e-5)}


# ---------------------------------------------------------------- half-sweep

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("chunk", [0, 8])
def test_sweep_tiny_planted(ctx, c0, dtype, chunk):
    """Both half-sweeps of the tiny planted problem, unsplit and split-K."""
    DP = dev_problem(ctx, c0, dtype, chunk=chunk, chunk_t=chunk)
    M0 = c0.M0 if dtype == torch.float64 else r32(c0.M0)
    Md = to_dev(M0, dtype, ctx)
    Ud = torch.zeros((c0.n_u, c0.n_f), dtype=dtype, device=ctx.torch_device)
    DP.sweep("U", Md, Ud)
    Uref = oracle.half_sweep(c0.R, M0, c0.lam)
    Ug = host(Ud)
    assert rowrel(Ug, Uref) <= TOL[dtype]["row"] and fro(Ug, Uref) <= TOL[dtype]["fro"]
    Mout = torch.zeros_like(Md)
    DP.sweep("M", Ud, Mout)
    Mref = oracle.half_sweep(c0.Rt, Ug, c0.lam)
    Mg = host(Mout)
    assert rowrel(Mg, Mref) <= TOL[dtype]["row"] and fro(Mg, Mref) <= TOL[dtype]["fro"]


NF64 = [1, 2, 10, 16, 31, 32, 50, 64, 95]
# FP32 n_f = 32..35 and 48..55 put 1..4 (1..8) real slots in the last 16-wide
# block column, which then runs on 4x4 MFMA blocks (one or two column
# groups); 36 and 56 are the first sizes past it
NF32 = [1, 2, 10, 15, 16, 32, 35, 36, 48, 50, 51, 52, 55, 56, 64, 96, 100, 127, 128, 143]


@pytest.mark.parametrize("dtype,n_f", [(torch.float64, n) for n in NF64] +
                         [(torch.float32, n) for n in NF32])
def test_sweep_random_shapes(ctx, dtype, n_f):
    """Random pattern with empty rows and very long rows (split and unsplit),
    n_f across 1..9 tile blocks and ragged tails."""
    P = synth.random_problem(70, 300, n_f=n_f, lam=0.1, seed=100 + n_f, density=0.08,
                             long_rows=3, long_len=290, empty_rows=4, x0_sigma=0.5)
    Y = P.M0 if dtype == torch.float64 else r32(P.M0)
    ref = oracle.half_sweep(P.R, Y, P.lam)
    for chunk in (0, 64):
        DP = dev_problem(ctx, P, dtype, chunk=chunk)
        X = torch.full((P.n_u, n_f), float("nan"), dtype=dtype, device=ctx.torch_device)
        DP.sweep("U", to_dev(Y, dtype, ctx), X)
        Xg = host(X)
        empty = P.R.counts() == 0
        assert np.all(Xg[empty] == 0.0)
        assert rowrel(Xg[~empty], ref[~empty]) <= TOL[dtype]["row"], chunk
        assert fro(Xg, ref) <= TOL[dtype]["fro"], chunk


@pytest.mark.parametrize("dtype,n_f,ld", [(torch.float64, 10, 13), (torch.float64, 50, 53),
                                         (torch.float32, 100, 101), (torch.float32, 100, 104),
                                         (torch.float32, 64, 66)])
def test_sweep_padded_leading_dimension(ctx, dtype, n_f, ld):
    """ld > n_f: padding columns are neither read nor written (ld % 4 == 0
    takes the vector-gather path for FP32, other strides the scalar one)."""
    P = synth.random_problem(50, 40, n_f=n_f, lam=0.05, seed=9, density=0.3, x0_sigma=0.5)
    Y = np.full((P.n_m, ld), 7.0)
    Y[:, :n_f] = P.M0 if dtype == torch.float64 else r32(P.M0)
    X = torch.full((P.n_u, ld), -3.0, dtype=dtype, device=ctx.torch_device)
    DP = dev_problem(ctx, P, dtype, ld=ld)
    G = torch.full((P.n_u, ld), -5.0, dtype=dtype, device=ctx.torch_device)
    Xat = torch.zeros((P.n_u, ld), dtype=dtype, device=ctx.torch_device)
    Xat[:, :n_f] = to_dev(P.U0 if dtype == torch.float64 else r32(P.U0), dtype, ctx)
    DP.sweep("U", to_dev(Y, dtype, ctx), X, X_at=Xat, grad_out=G)
    Xg, Gg = host(X), host(G)
    assert np.all(Xg[:, n_f:] == -3.0) and np.all(Gg[:, n_f:] == -5.0)
    Yr = Y[:, :n_f]
    assert fro(Xg[:, :n_f], oracle.half_sweep(P.R, Yr, P.lam)) <= TOL[dtype]["fro"]
    gU, _ = oracle.gradient(P.R, P.Rt, host(Xat)[:, :n_f], Yr, P.lam)
    assert fro(Gg[:, :n_f], gU) <= (1e-12 if dtype == torch.float64 else 2e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_gradient_of_sweep(ctx, c0, dtype):
    """grad_out = 2 (A_i x_i - v_i) at X_at equals the U block of the gradient."""
    DP = dev_problem(ctx, c0, dtype, chunk=16)
    U0 = c0.U0 if dtype == torch.float64 else r32(c0.U0)
    M0 = c0.M0 if dtype == torch.float64 else r32(c0.M0)
    Ud = to_dev(U0, dtype, ctx)
    X = torch.zeros_like(Ud)
    G = torch.zeros_like(Ud)
    DP.sweep("U", to_dev(M0, dtype, ctx), X, X_at=Ud, grad_out=G)
    gU, _ = oracle.gradient(c0.R, c0.Rt, U0, M0, c0.lam)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert fro(host(G), gU) <= tol
    assert fro(host(X), oracle.half_sweep(c0.R, M0, c0.lam)) <= TOL[dtype]["fro"]


def test_sweep_not_spd_reports_row(ctx):
    """lambda = 0 and a row whose Gram is rank deficient: bad_row names it, NaN output."""
    rows = np.array([0, 0, 1, 1, 1, 2, 2])
    cols = np.array([0, 1, 0, 1, 2, 1, 2])
    R = synth.csr_from_pairs(rows, cols, np.ones(7), 3, 3)
    Rt = synth.transpose(R)
    P = synth.Problem("tiny", R, Rt, 3, 0.0, np.zeros((3, 3)), np.eye(3), 0)
    DP = dev_problem(ctx, P, torch.float64)
    X = torch.zeros((3, 3), dtype=torch.float64, device=ctx.torch_device)
    bad = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    DP.sweep("U", to_dev(np.eye(3), torch.float64, ctx), X, bad_row=bad)
    assert int(bad.item()) == 0
    Xg = host(X)
    assert np.all(np.isnan(Xg[0])) and np.all(np.isnan(Xg[2]))
    np.testing.assert_allclose(Xg[1], [1.0, 1.0, 1.0], rtol=1e-14)
    DP2 = dev_problem(ctx, dataclasses.replace(P, lam=0.1), torch.float64)
    DP2.sweep("U", to_dev(np.eye(3), torch.float64, ctx), X, bad_row=bad)
    assert int(bad.item()) == (1 << 63) - 1


def test_sweep_is_deterministic(ctx, c0):
    DP = dev_problem(ctx, c0, torch.float32, chunk=8, chunk_t=8)
    Md = to_dev(r32(c0.M0), torch.float32, ctx)
    outs = []
    for _ in range(2):
        U = torch.zeros((c0.n_u, c0.n_f), dtype=torch.float32, device=ctx.torch_device)
        DP.sweep("U", Md, U)
        M = torch.zeros_like(Md)
        DP.sweep("M", U, M)
        outs.append((U.cpu().numpy(), M.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------- gradient and f

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("chunk", [0, 8])
@pytest.mark.parametrize("n_f", [20, 50, 65, 100, 128, 140])
def test_gradient_and_loss(ctx, dtype, chunk, n_f):
    """Both gradient blocks and f; FP32 n_f = 20 and 100 take the 4-wide
    gather with 8 lanes per rating (the last vector of a lane clamped inside
    the row), 128 the same with every vector real, 140 the 4-wide gather with
    16 lanes, n_f = 50 the one-element gather with 8 lanes and 65 with 16;
    FP64 n_f = 65, 100, 128 and 140 the one-element gather with 16 lanes."""
    P = synth.random_problem(90, 70, n_f=n_f, lam=0.07, seed=21, density=0.15, long_rows=2,
                             empty_rows=3, x0_sigma=0.5)
    U0 = P.U0 if dtype == torch.float64 else r32(P.U0)
    M0 = P.M0 if dtype == torch.float64 else r32(P.M0)
    DP = dev_problem(ctx, P, dtype, chunk=chunk, chunk_t=chunk)
    x = DP.pack(U0, M0)
    g = DP.zeros()
    out = torch.zeros(2, dtype=torch.float64, device=ctx.torch_device)
    DP.gradient(DP.U(x), DP.M(x), DP.U(g), DP.M(g), out)
    gU, gM = oracle.gradient(P.R, P.Rt, U0, M0, P.lam)
    f = oracle.loss(P.R, U0, M0, P.lam)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert fro(host(DP.U(g)), gU) <= tol
    assert fro(host(DP.M(g)), gM) <= tol
    fg, gg = out.cpu().tolist()
    assert fg == pytest.approx(f, rel=1e-12 if dtype == torch.float64 else 1e-6)
    assert gg == pytest.approx(float(np.sum(gU ** 2) + np.sum(gM ** 2)),
                               rel=1e-11 if dtype == torch.float64 else 1e-5)


# ---------------------------------------------------------------- quartic coefficients

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n_f", [3, 16, 65, 100, 128, 140])
def test_linesearch_coefficients(ctx, dtype, n_f):
    P = synth.random_problem(80, 60, n_f=n_f, lam=0.05, seed=30 + n_f, density=0.2,
                             long_rows=2, empty_rows=2, x0_sigma=0.3)
    rng = np.random.default_rng(n_f)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    U0, M0 = cast(P.U0), cast(P.M0)
    PU, PM = cast(rng.normal(0, 0.1, P.U0.shape)), cast(rng.normal(0, 0.1, P.M0.shape))
    ref = oracle.quartic(P.R, U0, M0, PU, PM, P.lam)
    for chunk in (0, 16):
        DP = dev_problem(ctx, P, dtype, chunk=chunk)
        x, p = DP.pack(U0, M0), DP.pack(PU, PM)
        C = torch.zeros(5, dtype=torch.float64, device=ctx.torch_device)
        DP.coeffs(DP.U(x), DP.M(x), DP.U(p), DP.M(p), C)
        Cg = C.cpu().numpy()
        scale = np.max(np.abs(ref))
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        assert np.max(np.abs(Cg - ref)) <= tol * scale, (chunk, Cg, ref)


def test_backtracking_matches_oracle_decisions(ctx):
    """Same coefficients in, same trial count and bitwise the same step out."""
    from paper_1508_03110_amd import _lib as L
    rng = np.random.default_rng(4)
    C = torch.zeros(5, dtype=torch.float64, device=ctx.torch_device)
    a = torch.zeros(1, dtype=torch.float64, device=ctx.torch_device)
    n = torch.zeros(1, dtype=torch.int32, device=ctx.torch_device)
    q = torch.zeros(1, dtype=torch.float64, device=ctx.torch_device)
    for k in range(200):
        c = np.array([3.0, -abs(rng.normal()) * 10 ** rng.uniform(-3, 1), rng.normal(),
                      rng.normal() * 0.1, abs(rng.normal()) * 0.01])
        if k % 50 == 0:
            c[1] = abs(c[1])  # not a descent direction
        C.copy_(torch.as_tensor(c))
        L.ncg_backtrack(ctx.handle, C, 10.0, 0.9, 0.5, 400, a, n, q)
        alpha, trials = oracle.backtrack(c)
        if c[1] >= 0.0:  # not a descent direction: the device refuses (documented)
            alpha = None
        if alpha is None:
            assert int(n.item()) == -1 and float(a.item()) == 0.0 and math.isnan(q.item())
        else:
            assert int(n.item()) == trials and float(a.item()) == alpha
            # Q(alpha) by Horner without contraction: the host's polyval, bit for bit
            assert float(q.item()) == float(np.polyval(c[::-1], alpha))


# ---------------------------------------------------------------- vector layer

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vector_layer(ctx, dtype):
    from paper_1508_03110_amd import _lib as L
    rng = np.random.default_rng(8)
    n = 100_003
    dt = L.dtype_code(dtype)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    xh, xbh, gnh, goh, ph = [cast(rng.normal(size=n)) for _ in range(5)]
    x, xb, gn, go, p = [to_dev(a, dtype, ctx) for a in (xh, xbh, gnh, goh, ph)]
    scal = torch.zeros(4, dtype=torch.float64, device=ctx.torch_device)
    scal[0] = 2.5
    L.ncg_direction(ctx.handle, n, x, xb, gn, go, p, scal, 0, 0, dt)
    gb = xh - xbh
    beta = float(gb @ (gnh - goh)) / 2.5
    s = scal.cpu().numpy()
    rt = 1e-12 if dtype == torch.float64 else 1e-6
    assert s[1] == pytest.approx(beta, rel=rt)
    assert s[0] == pytest.approx(float(gb @ gnh), rel=rt)
    assert s[2] == pytest.approx(float(gnh @ gnh), rel=rt)
    tol = 1e-15 if dtype == torch.float64 else 1e-6
    assert fro(host(xb), gb) <= tol
    assert fro(host(p), -gb + beta * ph) <= max(tol, 1e-12)
    alpha = torch.tensor([0.37], dtype=torch.float64, device=ctx.torch_device)
    L.ncg_axpy(ctx.handle, n, x, p, alpha, dt)
    assert fro(host(x), xh + 0.37 * host(p)) <= tol
    L.ncg_axpby(ctx.handle, n, -1.0, xb, 0.0, p, dt)
    assert np.array_equal(host(p), -host(xb))


# ---------------------------------------------------------------- fold-in

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fold_in_alone_and_in_the_mix(ctx, dtype):
    """Each request's result equals the oracle's and is bitwise the same
    whether solved alone or in a mixed batch; empty requests are rejected."""
    from paper_1508_03110_amd.solver import fold_in
    rng = np.random.default_rng(3)
    n_m, n_f = 500, 32 if dtype == torch.float64 else 100
    M = rng.normal(0, 0.3, (n_m, n_f))
    M = M if dtype == torch.float64 else r32(M)
    req = synth.fold_in_requests(40, n_m, seed=5, max_len=400)
    Md = to_dev(M, dtype, ctx)
    U, st = fold_in(ctx, Md, 0.05, req, n_f)
    ref = oracle.fold_in(M, req, 0.05)
    assert np.all(st.cpu().numpy() == 0)
    assert rowrel(host(U), ref) <= TOL[dtype]["row"]
    for q in (0, 7, 39):
        a, b = req.indptr[q], req.indptr[q + 1]
        one = synth.Csr(1, n_m, np.array([0, b - a]), req.indices[a:b], req.values[a:b])
        U1, _ = fold_in(ctx, Md, 0.05, one, n_f)
        assert np.array_equal(U1.cpu().numpy()[0], U.cpu().numpy()[q])
    empty = synth.Csr(2, n_m, np.array([0, 0, 3]), np.array([1, 2, 3], np.int32),
                      np.array([1.0, 2.0, 3.0], np.float32))
    U2, st2 = fold_in(ctx, Md, 0.05, empty, n_f)
    assert st2.cpu().tolist() == [-1, 0]
    assert np.all(U2.cpu().numpy()[0] == 0)


# ---------------------------------------------------------------- whole algorithms

def test_als_20_sweeps_fp64_tiny_planted(ctx, c0):
    """Algorithm 1, 20 sweeps, FP64: f within 1e-10 of the oracle's after each sweep."""
    from paper_1508_03110_amd.solver import Als
    DP = dev_problem(ctx, c0, torch.float64)
    als = Als(DP, DP.pack(c0.U0, c0.M0))
    _, _, fref = oracle.als_run(c0.R, c0.Rt, c0.M0, c0.lam, 20)
    for k in range(20):
        als.sweep()
        f, _ = DP.loss_and_gnorm(als.x)
        assert f == pytest.approx(fref[k], rel=1e-10), k


def test_als_20_sweeps_fp32_tiny_planted(ctx, c0):
    from paper_1508_03110_amd.solver import Als
    DP = dev_problem(ctx, c0, torch.float32)
    als = Als(DP, DP.pack(c0.U0, c0.M0))
    _, _, fref = oracle.als_run(c0.R, c0.Rt, r32(c0.M0), c0.lam, 20)
    for _ in range(20):
        als.sweep()
    f, _ = DP.loss_and_gnorm(als.x)
    assert f == pytest.approx(fref[-1], rel=1e-5)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_als_ncg_20_iterations_lockstep(ctx, c0, dtype, tol):
    """Algorithm 2, 20 iterations, run in lockstep with the oracle: the same
    trial count each iteration and f(x_k) within tol.  A trial-count flip is
    allowed only when the Armijo test was within rounding of its boundary;
    the oracle is then re-seeded from the GPU state."""
    from paper_1508_03110_amd.solver import AlsNcg
    DP = dev_problem(ctx, c0, dtype)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    U0, M0 = cast(c0.U0), cast(c0.M0)
    gpu = AlsNcg(DP).init(U0, M0)
    o = oracle.NcgOracle(c0.R, c0.Rt, c0.n_f, c0.lam)
    s = o.init(U0, M0)
    flips = 0
    for k in range(20):
        gpu.step()
        o.step(s)
        if gpu.n_trials != s.trials:
            C = o.last_coeffs
            a = 10.0 * 0.9 ** min(gpu.n_trials, s.trials)
            margin = 0.5 * C[1] + a * (C[2] + a * (C[3] + a * C[4]))
            assert abs(margin) <= 1e-6 * (abs(C[1]) + abs(C[2]) * a), (k, margin)
            flips += 1
            xs = gpu.x.cpu().numpy().astype(np.float64)
            s = o.init(*o.split(xs))
            continue
        fo = o.f(s.x)
        assert gpu.f == pytest.approx(fo, rel=tol), (k, gpu.f, fo)
    assert gpu.safeguards == 0 and flips <= 2
    _, _, fa = oracle.als_run(c0.R, c0.Rt, M0, c0.lam, 20)
    assert gpu.f < fa[-1]  # ALS-NCG ahead of ALS after the same number of iterations


@pytest.mark.parametrize("dtype,ld,tol", [(torch.float64, 16, 1e-10), (torch.float32, 16, 1e-5)])
@pytest.mark.parametrize("mode", ["host", "device", "graph"])
def test_als_ncg_with_padded_rows(ctx, c0, dtype, ld, tol, mode):
    """Algorithm 2 with factor rows padded past n_f (n_f = 10, ld = 16, as the
    billion-rating benchmark pads n_f = 50 to 64): every NCG vector carries
    the padding columns, which must stay zero and out of every dot product;
    f(x_k) tracks the oracle for 8 iterations driven from the host, from the
    device, and as replays of the captured iteration."""
    from paper_1508_03110_amd.solver import AlsNcg
    DP = dev_problem(ctx, c0, dtype, ld=ld)
    assert DP.ld == ld
    cast = (lambda a: a) if dtype == torch.float64 else r32
    U0, M0 = cast(c0.U0), cast(c0.M0)
    gpu = AlsNcg(DP).init(U0, M0)
    o = oracle.NcgOracle(c0.R, c0.Rt, c0.n_f, c0.lam)
    s = o.init(U0, M0)
    for k in range(8):
        if mode == "host":
            gpu.step()
        elif mode == "device" or k == 0:
            gpu.step_device()  # (graph mode: the eager step sizes the workspace)
            gpu.read_state()
        else:
            if k == 1:
                gpu.capture()
            gpu.replay()
            gpu.read_state()
        o.step(s)
        assert gpu.n_trials == s.trials, k
        assert gpu.f == pytest.approx(o.f(s.x), rel=tol), k
    X = gpu.x.view(-1, ld).cpu().numpy()
    assert np.all(X[:, c0.n_f:] == 0.0)


def test_exact_quartic_minimiser_matches_oracle(ctx):
    """ncg_linesearch_exact against oracle.quartic_min (numpy's polynomial
    roots) on random quartics, double wells, a vanishing quartic term and an
    ascent direction."""
    from paper_1508_03110_amd import _lib as L
    rng = np.random.default_rng(17)
    cases = []
    for _ in range(300):
        C = rng.normal(size=5) * 10.0 ** rng.integers(-3, 4, 5)
        C[1] = -abs(C[1])
        C[4] = abs(C[4])
        cases.append(C)
    cases += [np.array([1.0, -2.0, 1.0, 0.0, 0.0]), np.array([5.0, -1.0, -3.0, 0.5, 0.3]),
              np.array([1.0, 0.5, 1.0, 0.0, 1.0]), np.array([1.0, -1.0, -1.0, -1.0, 0.0])]
    dev = ctx.torch_device
    for C in cases:
        cd = torch.as_tensor(C, dtype=torch.float64, device=dev)
        a = torch.zeros(1, dtype=torch.float64, device=dev)
        n = torch.zeros(1, dtype=torch.int32, device=dev)
        q = torch.zeros(1, dtype=torch.float64, device=dev)
        L.ncg_linesearch_exact(ctx.handle, cd, 1e-4, a, n, q)
        ref = oracle.quartic_min(C, c=1e-4)
        if ref is None:
            assert int(n.item()) == -1 and float(a.item()) == 0.0, C
            assert math.isnan(q.item()), C
        else:
            assert int(n.item()) == 0, C
            assert float(a.item()) == pytest.approx(ref, rel=1e-10), C
            assert float(q.item()) == float(np.polyval(C[::-1], float(a.item()))), C


def test_als_ncg_exact_search_lockstep(ctx, c0):
    """Algorithm 2 with the exact minimiser of the same quartic, FP64, 15
    iterations in lockstep with the oracle using oracle.quartic_min: f(x_k)
    within 1e-10 relative at every iteration."""
    from paper_1508_03110_amd.solver import AlsNcg
    DP = dev_problem(ctx, c0, torch.float64)
    gpu = AlsNcg(DP, search="exact").init(c0.U0, c0.M0)
    o = oracle.NcgOracle(c0.R, c0.Rt, c0.n_f, c0.lam)

    def exact_ls(x, p):
        C = o.coeffs(x, p)
        a = oracle.quartic_min(C)
        fnew = float("nan") if a is None else float(np.polyval(C[::-1], a))
        return a, (0 if a is not None else -1), fnew, float(C[1])

    s = o.init(c0.U0, c0.M0)
    for k in range(15):
        gpu.step()
        oracle.ncg_step(s, o.P, o.grad, exact_ls)
        assert gpu.f == pytest.approx(o.f(s.x), rel=1e-10), k
    assert gpu.safeguards == 0


@pytest.mark.parametrize("mode", ["host", "device"])
@pytest.mark.parametrize("problem,max_trials", [("c0", 60), ("c0", 64), ("random", 62)])
def test_als_ncg_safeguards_lockstep_with_oracle(ctx, c0, mode, problem, max_trials):
    """The restart and ALS-point branch of Algorithm 2 with Algorithm 4 (the
    safeguard reading: p = -gbar when g^T p >= 0 or no trial passes, then the
    ALS point P(x_k) with beta = 0 next), forced by alpha0 = 1e3 and a cap of
    60-64 trials (smallest alpha 2.0-1.6), FP64, in lockstep with the
    oracle run with the same constants: every iteration the same trial
    count, restart and safeguard counters, x_k within 1e-10 and f(x_k)
    within 1e-10 relative (both NaN on an ALS-point step).  With the cap 60
    every restart also fails (8 ALS points on the planted problem); with 64
    and 62 some restarted searches succeed.  step() decides on the host,
    step_device() on the device."""
    from paper_1508_03110_amd.solver import AlsNcg
    P = c0 if problem == "c0" else synth.random_problem(80, 60, n_f=6, lam=0.05, seed=21,
                                                         density=0.25, x0_sigma=0.5)
    DP = dev_problem(ctx, P, torch.float64)
    kw = dict(alpha0=1e3, max_trials=max_trials)
    gpu = AlsNcg(DP, **kw).init(P.U0, P.M0)
    o = oracle.NcgOracle(P.R, P.Rt, P.n_f, P.lam, **kw)
    s = o.init(P.U0, P.M0)
    for k in range(12):
        if mode == "host":
            gpu.step()
        else:
            gpu.step_device()
            gpu.read_state()
        o.step(s)
        assert (gpu.restarts, gpu.safeguards) == (s.restarts, s.safeguards), k
        xs = gpu.x.cpu().numpy()
        assert np.linalg.norm(xs - s.x) <= 1e-10 * np.linalg.norm(s.x), k
        if math.isnan(s.alpha):           # ALS point taken
            assert math.isnan(gpu.f), k
        else:
            assert gpu.n_trials == s.trials, k
            assert gpu.f == pytest.approx(o.f(s.x), rel=1e-10), k
    assert s.restarts > 0 and s.safeguards > 0, (s.restarts, s.safeguards)


# ---------------------------------------------------------------- device-side control, graphs

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_device_controlled_step_matches_host_step(ctx, dtype):
    """step_device() takes every line-search, restart and safeguard decision
    on the device; from the same start it must reproduce step() bit for bit
    (same kernels, same inputs), including forced restarts and ALS-point
    steps: with alpha0 = 1e3 and 60 trials the search fails on some
    iterations."""
    from paper_1508_03110_amd.solver import AlsNcg
    P = synth.random_problem(80, 60, n_f=6, lam=0.05, seed=21, density=0.25, x0_sigma=0.5)
    DP = dev_problem(ctx, P, dtype)
    U0 = P.U0 if dtype == torch.float64 else r32(P.U0)
    M0 = P.M0 if dtype == torch.float64 else r32(P.M0)
    for kw in ({}, dict(alpha0=1e3, max_trials=60), dict(search="exact")):
        a = AlsNcg(DP, **kw).init(U0, M0)
        b = AlsNcg(DP, **kw).init(U0, M0)
        for k in range(12):
            a.step()
            b.step_device()
            b.read_state()
            assert torch.equal(a.x, b.x), (kw, k)
            assert torch.equal(a.pdir, b.pdir), (kw, k)
            assert (a.restarts, a.safeguards) == (b.restarts, b.safeguards), (kw, k)
            if math.isnan(a.f):
                assert math.isnan(b.f)
            else:
                assert a.f == b.f and a.n_trials == b.n_trials, (kw, k)
        if "alpha0" in kw:  # the FP64 oracle takes 7 restarts and 7 ALS points here
            assert b.restarts > 0 and 0 < b.safeguards < 12


def test_graph_replays_match_eager(ctx, c0):
    """One ALS-NCG iteration captured as a HIP graph (two graphs, alternating
    gradient buffers): six replays with eager work and synchronisations in
    between, each compared bit for bit with an eager device-controlled run."""
    from paper_1508_03110_amd.solver import AlsNcg
    DP = dev_problem(ctx, c0, torch.float32, chunk=64, chunk_t=64)
    U0, M0 = r32(c0.U0), r32(c0.M0)
    ref = AlsNcg(DP).init(U0, M0)
    g = AlsNcg(DP).init(U0, M0)
    ref.step_device()
    g.step_device()
    g.capture()
    for k in range(6):
        ref.step_device()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=ctx.torch_device).sum().item()  # eager work between replays
        assert torch.equal(ref.x, g.x), k
        assert torch.equal(ref.pdir, g.pdir), k
        assert torch.equal(ref.state, g.state), k
        assert torch.equal(ref.scal, g.scal), k
