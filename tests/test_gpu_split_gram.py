"""GPU parity of the FP32 half-sweep's Gram on FP16 MFMAs (two-term splits of
the rows scaled by a power of two chosen from max |Y| and each chunk's
largest rating) against the FP64 oracle's row solve of Eq. (3).

The scale must keep every split value inside the FP16 range and its low
part normal whatever the magnitudes: factor entries from 1e-6 to 1e4,
ratings from 1e-3 to 1e5, chunks of one row with very different ratings
(each chunk picks its own scale, the partial Grams are summed unscaled),
the augmented rating slot at every lane position (n_f = 16 b + k), and
fold-in against fixed item factors.  Tolerances are the FP32 ones of the
other half-sweep tests: 1e-4 per row, 2e-5 on the whole factor.
"""
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


def r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rowrel(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-300)
    return float(np.max(num / den)) if a.shape[0] else 0.0


def fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(n_f, seed, y_scale=1.0, r_scale=1.0, n_u=90, n_m=300, lam=0.05, long_rows=False):
    """Users with 1..200 ratings (a few with 260..300 when long_rows) over
    n_m items; factors N(0, 0.3) * y_scale, ratings in {0.5 .. 5} * r_scale."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 201, n_u)
    if long_rows:
        lens[:6] = rng.integers(260, 301, 6)
    rows, cols = [], []
    for u, L in enumerate(lens):
        rows.append(np.full(L, u))
        cols.append(rng.choice(n_m, size=int(L), replace=False))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    vals = rng.integers(1, 11, rows.size) / 2.0 * r_scale
    R = synth.csr_from_pairs(rows, cols, vals, n_u, n_m)
    U0 = rng.normal(0, 0.3, (n_u, n_f)) * y_scale
    M0 = rng.normal(0, 0.3, (n_m, n_f)) * y_scale
    return synth.Problem("split", R, synth.transpose(R), n_f, lam, U0, M0, seed, {})


def sweep_u(ctx, P, chunk=0, ld=None):
    from paper_1508_03110_amd.solver import DeviceProblem
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32, chunk=chunk, ld=ld)
    Y = DP.pack(np.zeros((P.n_u, P.n_f)), r32(P.M0))
    X = torch.full((P.n_u, DP.ld), float("nan"), dtype=torch.float32, device=ctx.torch_device)
    DP.sweep("U", DP.M(Y), X)
    torch.cuda.synchronize()
    return X[:, :P.n_f].cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("y_scale,r_scale", [(1.0, 1.0), (1e-6, 1.0), (1e4, 1.0), (1.0, 1e5),
                                             (1e-3, 1e-3), (1e3, 1e-3)])
def test_magnitudes(ctx, y_scale, r_scale):
    """Factor and rating magnitudes far from 1 in both directions (lambda
    scaled with y_scale^2 so the regulariser keeps its weight)."""
    P = problem(100, seed=3, y_scale=y_scale, r_scale=r_scale)
    P.lam = 0.05 * y_scale * y_scale
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    got = sweep_u(ctx, P)
    assert np.all(np.isfinite(got))
    assert rowrel(got, ref) <= 1e-4 and fro(got, ref) <= 2e-5


@pytest.mark.parametrize("n_f", [1, 15, 16, 17, 31, 47, 48, 50, 63, 95, 100, 111, 112, 127, 143])
def test_rating_slot_at_every_lane(ctx, n_f):
    """n_f = 16 b + k puts the augmented rating at lane k of the last block
    (k = 15: the last block holds only the rating)."""
    P = problem(n_f, seed=n_f)
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    got = sweep_u(ctx, P)
    assert rowrel(got, ref) <= 1e-4 and fro(got, ref) <= 2e-5


@pytest.mark.parametrize("chunk", [32, 40, 100])
def test_split_rows_with_different_scales(ctx, chunk):
    """Rows split over chunks whose ratings differ by 1e4 (each chunk scales
    by its own largest rating) and padded rows (ld = 104)."""
    P = problem(100, seed=7, long_rows=True)
    vals = P.R.values.copy()
    for u in range(6):  # the long rows: the first 64 ratings 1e4 times larger
        b = P.R.indptr[u]
        vals[b:b + 64] *= 1e4
    R = synth.Csr(P.R.n_rows, P.R.n_cols, P.R.indptr, P.R.indices, vals.astype(np.float32))
    P = synth.Problem("split", R, synth.transpose(R), P.n_f, P.lam, P.U0, P.M0, 7, {})
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    got = sweep_u(ctx, P, chunk=chunk, ld=104)
    assert rowrel(got, ref) <= 1e-4 and fro(got, ref) <= 2e-5
    # the same rows without splitting agree to the same tolerance
    whole = sweep_u(ctx, P)
    assert rowrel(whole, ref) <= 1e-4


def test_fold_in_against_large_item_factors(ctx):
    """fold_in (no plan: the scale of M is taken in the same call) with item
    factors of magnitude 1e3."""
    from paper_1508_03110_amd.solver import fold_in
    P = problem(64, seed=5, y_scale=1e3, n_u=40)
    lam = 0.05 * 1e6
    M = torch.as_tensor(r32(P.M0), dtype=torch.float32).to(ctx.torch_device)
    U, st = fold_in(ctx, M, lam, P.R, P.n_f)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    ref = oracle.fold_in(r32(P.M0), P.R, lam)
    got = U[:, :P.n_f].cpu().numpy().astype(np.float64)
    assert rowrel(got, ref) <= 1e-4


def test_non_finite_factor_row_stays_local(ctx):
    """An item row holding NaN and one holding infinity: the users who rated
    them get NaN rows and are reported by bad_row; every other user matches
    the oracle (the non-finite entries do not set the scale of the others)."""
    from paper_1508_03110_amd.solver import DeviceProblem
    P = problem(100, seed=13)
    M = r32(P.M0)
    M[7, 3] = np.nan
    M[11, 50] = np.inf
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32)
    X = torch.zeros((P.n_u, P.n_f), dtype=torch.float32, device=ctx.torch_device)
    bad = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    DP.sweep("U", torch.as_tensor(M, dtype=torch.float32).to(ctx.torch_device), X, bad_row=bad)
    got = X.cpu().numpy().astype(np.float64)
    touched = np.zeros(P.n_u, dtype=bool)
    for u in range(P.n_u):
        items = P.R.indices[P.R.indptr[u]:P.R.indptr[u + 1]]
        touched[u] = np.any((items == 7) | (items == 11))
    assert touched.any() and (~touched).any()
    assert np.all(~np.isfinite(got[touched]).all(axis=1))
    assert int(bad.item()) == int(np.flatnonzero(touched)[0])
    clean = r32(P.M0)
    ref = oracle.half_sweep(P.R, clean, P.lam)
    assert rowrel(got[~touched], ref[~touched]) <= 1e-4


def test_not_spd_row_fp32(ctx):
    """lambda = 0 and rank-deficient rows in the FP32 path (FP16-split Gram,
    hardware reciprocal square root on the pivots): bad_row names the first
    one, its output is NaN, the full-rank row is solved."""
    rows = np.array([0, 0, 1, 1, 1, 2, 2])
    cols = np.array([0, 1, 0, 1, 2, 1, 2])
    R = synth.csr_from_pairs(rows, cols, np.ones(7), 3, 3)
    P = synth.Problem("tiny", R, synth.transpose(R), 3, 0.0, np.zeros((3, 3)), np.eye(3), 0)
    from paper_1508_03110_amd.solver import DeviceProblem
    DP = DeviceProblem(ctx, P.R, P.Rt, 3, 0.0, torch.float32)
    X = torch.zeros((3, 3), dtype=torch.float32, device=ctx.torch_device)
    bad = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    DP.sweep("U", torch.eye(3, dtype=torch.float32, device=ctx.torch_device), X, bad_row=bad)
    assert int(bad.item()) == 0
    Xg = X.cpu().numpy()
    assert np.all(np.isnan(Xg[0])) and np.all(np.isnan(Xg[2]))
    np.testing.assert_allclose(Xg[1], [1.0, 1.0, 1.0], rtol=1e-6)


@pytest.mark.parametrize("n_f,ld", [(15, 15), (16, 16), (40, 40), (50, 64), (63, 63), (70, 72),
                                    (90, 90), (100, 100), (100, 104), (127, 128), (143, 144)])
def test_split_copy_matches_the_split_in_the_loop(ctx, n_f, ld):
    """A planned FP32 half-sweep splits the fixed side once into a copy;
    fold-in (no plan) splits each gathered row in the Gram loop.  Whole rows
    (no chunk splits, no dual bins) give the same bits either way, including
    positions past the end of a chunk (rows of 1..200 ratings)."""
    from paper_1508_03110_amd.solver import DeviceProblem, fold_in
    P = problem(n_f, seed=60 + n_f, n_u=70)
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32, ld=ld)
    assert DP.R.info()["split_rows"] == 0
    DP.R.set_split_copy(1)
    Y = DP.pack(np.zeros((P.n_u, P.n_f)), r32(P.M0))
    X = torch.full((P.n_u, ld), float("nan"), dtype=torch.float32, device=ctx.torch_device)
    DP.sweep("U", DP.M(Y), X)
    M = DP.M(Y)[:, :n_f].contiguous()
    U, st = fold_in(ctx, M, P.lam, P.R, n_f)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    assert torch.equal(X[:, :n_f], U[:, :n_f])
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    assert rowrel(X[:, :n_f].cpu().numpy().astype(np.float64), ref) <= 1e-4


@pytest.mark.parametrize("n_f", [50, 100])
@pytest.mark.parametrize("chunk,dual", [(0, 0), (32, 0), (40, 30), (0, 62)])
def test_split_copy_on_and_off_agree_bitwise(ctx, n_f, chunk, dual):
    """The planned half-sweep with and without the split copy: rows cut over
    chunks (partial Grams summed by the second stage), dual-form bins beside
    the n_f x n_f launch, the fused gradient; every output bit equal."""
    from paper_1508_03110_amd.solver import DeviceProblem
    P = problem(n_f, seed=80 + n_f, long_rows=True)
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32, chunk=chunk)
    if dual:
        DP.R.set_dual(dual)
    x = DP.pack(r32(P.U0), r32(P.M0))
    outs = []
    for mode in (0, 1):
        DP.R.set_split_copy(mode)
        X = torch.full((P.n_u, DP.ld), float("nan"), dtype=torch.float32, device=ctx.torch_device)
        G = torch.zeros((P.n_u, DP.ld), dtype=torch.float32, device=ctx.torch_device)
        DP.sweep("U", DP.M(x), X, X_at=DP.U(x), grad_out=G)
        outs.append((X, G))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    ref = oracle.half_sweep(P.R, r32(P.M0), P.lam)
    assert rowrel(outs[1][0][:, :n_f].cpu().numpy().astype(np.float64), ref) <= 1e-4
