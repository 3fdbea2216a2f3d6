"""GPU parity of the length-binned half-sweep: rows of 1..max_len ratings
solved in the dual form x = Y_I^T (Y_I Y_I^T + lambda n I)^{-1} r, the
others in the n_f x n_f form of Eq. (3).

Every row is compared with the FP64 oracle's row solve (which follows
Eq. (3) directly) at the half-sweep tolerances of the plain path, with the
dual bins on and off; the fused gradient against the oracle's gradient;
the bins themselves against the row lengths; lambda = 0 must fall back to
the n_f x n_f form; and ALS-NCG with the bins on must track the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL = {torch.float64: dict(row=1e-11, fro=1e-12), torch.float32: dict(row=1e-4, fro=2e-5)}


@pytest.fixture(scope="module")
def ctx():
    from paper_1508_03110_amd.solver import Context
    c = Context(0)
    yield c
    c.close()


def r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rowrel(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float(np.max(num / den)) if a.shape[0] else 0.0


def fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ragged_problem(n_f, seed, lam=0.05):
    """Users with every length 0..110 (each bin of 16 and its edges, empty
    rows, rows longer than any dual system) over 140 items."""
    rng = np.random.default_rng(seed)
    n_m = 140
    lens = np.concatenate([np.arange(0, 111), rng.integers(1, 95, 60), [140, 139, 96, 95, 94, 93]])
    rows, cols = [], []
    for u, L in enumerate(lens):
        c = rng.choice(n_m, size=int(L), replace=False)
        rows.append(np.full(L, u))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    vals = rng.integers(1, 11, rows.size) / 2.0
    R = synth.csr_from_pairs(rows, cols, vals, len(lens), n_m)
    U0 = rng.normal(0, 0.3, (len(lens), n_f))
    M0 = rng.normal(0, 0.3, (n_m, n_f))
    return synth.Problem("ragged", R, synth.transpose(R), n_f, lam, U0, M0, seed, {})


def sweep(ctx, P, dtype, dual, chunk=0, ld=None, grad=False, X_at=None):
    from paper_1508_03110_amd.solver import DeviceProblem
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, dtype, chunk=chunk, ld=ld)
    DP.R.set_dual(dual)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    Y = DP.pack(np.zeros((P.n_u, P.n_f)), cast(P.M0))
    X = torch.full((P.n_u, DP.ld), float("nan"), dtype=dtype, device=ctx.torch_device)
    G = None
    Xa = None
    if grad:
        G = torch.full_like(X, float("nan"))
        Xa = torch.zeros_like(X)
        Xa[:, :P.n_f] = torch.as_tensor(cast(X_at), dtype=dtype)
    DP.sweep("U", DP.M(Y), X, X_at=Xa, grad_out=G)
    torch.cuda.synchronize()
    out = X[:, :P.n_f].cpu().numpy().astype(np.float64)
    g = G[:, :P.n_f].cpu().numpy().astype(np.float64) if grad else None
    return out, g, DP.R.info()


@pytest.mark.parametrize("dtype,n_f", [(torch.float32, 100), (torch.float32, 64),
                                       (torch.float32, 50), (torch.float32, 10),
                                       (torch.float32, 127), (torch.float64, 50),
                                       (torch.float64, 10)])
def test_dual_bins_match_the_oracle(ctx, dtype, n_f):
    """Every length 1..94 in its bin (and the rest in the n_f x n_f form)
    against the oracle's row solve; the dual-form rows also against the
    bins-off result of the same kernels' n_f x n_f path."""
    P = ragged_problem(n_f, seed=n_f)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    ref = oracle.half_sweep(P.R, cast(P.M0), P.lam)
    lens = P.R.counts()
    got, _, info = sweep(ctx, P, dtype, 94)
    assert info["dual_rows"] == int(np.sum((lens >= 1) & (lens <= 94)))
    off, _, info0 = sweep(ctx, P, dtype, 0)
    assert info0["dual_rows"] == 0
    nz = lens > 0
    assert np.all(got[~nz] == 0.0)
    for X in (got, off):
        assert rowrel(X[nz], ref[nz]) <= TOL[dtype]["row"]
        assert fro(X, ref) <= TOL[dtype]["fro"]
    # rows above the bound are bitwise the n_f x n_f result
    big = lens > 94
    assert np.array_equal(got[big], off[big])


@pytest.mark.parametrize("dual", [14, 30, 46, 62, 78])
def test_each_bound_splits_the_rows_at_it(ctx, dual):
    """FP32, n_f = 100: with bound m the rows of length <= m take the dual
    form, the others are bitwise the bins-off result."""
    P = ragged_problem(100, seed=5)
    lens = P.R.counts()
    got, _, info = sweep(ctx, P, torch.float32, dual)
    off, _, _ = sweep(ctx, P, torch.float32, 0)
    assert info["dual_rows"] == int(np.sum((lens >= 1) & (lens <= dual)))
    assert np.array_equal(got[lens > dual], off[lens > dual])
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    sel = (lens >= 1) & (lens <= dual)
    assert rowrel(got[sel], ref[sel]) <= 1e-4


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("at", ["X_at", "X"])
def test_dual_fused_gradient(ctx, dtype, at):
    """The U block of the gradient at (X_at, Y) fused into the half-sweep,
    dual rows and n_f x n_f rows, against the oracle's gradient."""
    n_f = 50
    P = ragged_problem(n_f, seed=11)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    Xat = cast(np.random.default_rng(3).normal(0, 0.3, (P.n_u, n_f)))
    from paper_1508_03110_amd.solver import DeviceProblem
    DP = DeviceProblem(ctx, P.R, P.Rt, n_f, P.lam, dtype)
    DP.R.set_dual(94)
    M = torch.as_tensor(cast(P.M0), dtype=dtype).to(ctx.torch_device)
    G = torch.full((P.n_u, n_f), float("nan"), dtype=dtype, device=ctx.torch_device)
    if at == "X_at":
        X = torch.zeros((P.n_u, n_f), dtype=dtype, device=ctx.torch_device)
        DP.sweep("U", M, X, X_at=torch.as_tensor(Xat, dtype=dtype).to(ctx.torch_device), grad_out=G)
    else:  # gradient at the output's old contents
        X = torch.as_tensor(Xat, dtype=dtype).to(ctx.torch_device).clone()
        DP.sweep("U", M, X, grad_out=G)
    gU, _ = oracle.gradient(P.R, P.Rt, Xat, cast(P.M0), P.lam)
    g = G.cpu().numpy().astype(np.float64)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert fro(g, gU) <= tol
    ref = oracle.half_sweep(P.R, cast(P.M0), P.lam)
    nz = P.R.counts() > 0
    assert rowrel(X.cpu().numpy().astype(np.float64)[nz], ref[nz]) <= TOL[dtype]["row"]


def test_dual_bound_is_capped_by_the_chunk_and_padded_rows(ctx):
    """chunk 32: rows above 32 are split and stay in the n_f x n_f form, the
    bound is capped at 32; ld = 104 > n_f = 100 (padding neither read into
    the result nor written)."""
    P = ragged_problem(100, seed=8)
    lens = P.R.counts()
    got, _, info = sweep(ctx, P, torch.float32, 94, chunk=32, ld=104)
    assert info["dual_rows"] == int(np.sum((lens >= 1) & (lens <= 32)))
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    nz = lens > 0
    assert rowrel(got[nz], ref[nz]) <= 1e-4


def test_lambda_zero_keeps_the_primal_form(ctx):
    """With lambda = 0 the dual bins are ignored: rows with fewer ratings
    than n_f have a singular n_f x n_f system and are reported, as without
    the bins."""
    from paper_1508_03110_amd.solver import DeviceProblem
    P = ragged_problem(20, seed=2, lam=0.0)
    DP = DeviceProblem(ctx, P.R, P.Rt, 20, 0.0, torch.float32)
    DP.R.set_dual(94)
    M = torch.as_tensor(r32(P.M0), dtype=torch.float32).to(ctx.torch_device)
    outs = []
    for dual in (94, 0):
        DP.R.set_dual(dual)
        X = torch.zeros((P.n_u, 20), dtype=torch.float32, device=ctx.torch_device)
        bad = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
        DP.sweep("U", M, X, bad_row=bad)
        torch.cuda.synchronize()
        outs.append((X.cpu().numpy(), int(bad.item())))
    assert np.array_equal(outs[0][0], outs[1][0], equal_nan=True)
    assert outs[0][1] == outs[1][1] < P.n_u


def test_als_ncg_with_dual_bins_tracks_the_oracle(ctx, c0):
    """Algorithm 2 on the tiny planted problem, FP64, n_f = 10, with the dual
    bound at 30 for users (17..49 ratings: 181 of 600 rows) and 46 for items
    (32..66: 116 of 400): f(x_k) within 1e-10 of the oracle for 10
    iterations, and ALS within 1e-10 after each of 10 sweeps."""
    from paper_1508_03110_amd.solver import Als, AlsNcg, DeviceProblem
    DP = DeviceProblem(ctx, c0.R, c0.Rt, c0.n_f, c0.lam, torch.float64)
    DP.R.set_dual(30)
    DP.Rt.set_dual(46)
    assert DP.R.info()["dual_rows"] == 181 and DP.Rt.info()["dual_rows"] == 116
    gpu = AlsNcg(DP).init(c0.U0, c0.M0)
    o = oracle.NcgOracle(c0.R, c0.Rt, c0.n_f, c0.lam)
    s = o.init(c0.U0, c0.M0)
    for k in range(10):
        gpu.step()
        o.step(s)
        assert gpu.n_trials == s.trials, k
        assert gpu.f == pytest.approx(o.f(s.x), rel=1e-10), k
    als = Als(DP, DP.pack(c0.U0, c0.M0))
    _, _, fref = oracle.als_run(c0.R, c0.Rt, c0.M0, c0.lam, 10)
    for k in range(10):
        als.sweep()
        assert DP.loss_and_gnorm(als.x)[0] == pytest.approx(fref[k], rel=1e-10), k
