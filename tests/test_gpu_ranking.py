"""GPU parity of the ranking-accuracy calls (Section IV) against the oracle.

Both sides form predicted ratings in FP64 from the same factor values, so the
top-t lists and swap counts are compared exactly; ties (integer factors,
zero rows) are decided by item id on both sides.  The mean accuracy agrees to
rounding (the library divides the exact integer sum once).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ranking as rk

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    from paper_1508_03110_amd.solver import Context
    c = Context(0)
    yield c
    c.close()


def dev(a, dtype, ctx, ld=None):
    a = np.asarray(a, np.float64)
    if ld is not None and ld > a.shape[1]:
        pad = np.full((a.shape[0], ld - a.shape[1]), np.nan)  # padding is never read
        a = np.concatenate([a, pad], axis=1)
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(ctx.torch_device)


def factors(n_u, n_m, n_f, seed, dtype):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n_u, n_f)) / np.sqrt(n_f)
    M = rng.standard_normal((n_m, n_f)) / np.sqrt(n_f)
    if dtype == torch.float32:  # the oracle sees the values the library sees
        U, M = U.astype(np.float32).astype(np.float64), M.astype(np.float32).astype(np.float64)
    return U, M


CASES = [  # n_u, n_m, n_f, dtype, t, ld
    (600, 400, 10, torch.float64, 20, None),     # tiny planted shape
    (37, 130, 5, torch.float32, 1, None),
    (100, 257, 100, torch.float32, 20, None),    # 16-byte loads, ragged item tile
    (70, 300, 50, torch.float32, 32, 52),        # n_f not a multiple of 4, padded rows
    (65, 64, 128, torch.float64, 7, None),       # one full item tile, ragged user block
    (129, 31, 16, torch.float32, 31, 20),
    (3, 20, 112, torch.float32, 20, None),       # t = n_m
    (1, 2, 1, torch.float64, 1, None),           # smallest problem
]


@pytest.mark.parametrize("n_u,n_m,n_f,dtype,t,ld", CASES)
def test_top_t_matches_oracle(ctx, n_u, n_m, n_f, dtype, t, ld):
    from paper_1508_03110_amd.solver import rank_top_t
    U, M = factors(n_u, n_m, n_f, 100 + n_u, dtype)
    top = rank_top_t(ctx, dev(U, dtype, ctx, ld), dev(M, dtype, ctx, ld), t, n_f=n_f)
    torch.cuda.synchronize()
    assert np.array_equal(top.cpu().numpy(), rk.top_t(U, M, t))


@pytest.mark.parametrize("n_u,n_m,n_f,dtype,t,ld", CASES)
def test_swaps_and_accuracy_match_oracle(ctx, n_u, n_m, n_f, dtype, t, ld):
    from paper_1508_03110_amd.solver import rank_accuracy
    Ur, Mr = factors(n_u, n_m, n_f, 200 + n_u, dtype)
    ref = rk.top_t(Ur, Mr, t)
    rng = np.random.default_rng(7)
    U = Ur + 0.3 * rng.standard_normal(Ur.shape) / np.sqrt(n_f)
    M = Mr + 0.3 * rng.standard_normal(Mr.shape) / np.sqrt(n_f)
    if dtype == torch.float32:
        U, M = U.astype(np.float32).astype(np.float64), M.astype(np.float32).astype(np.float64)
    top = torch.as_tensor(ref).to(ctx.torch_device)
    mean_q, s = rank_accuracy(ctx, dev(U, dtype, ctx, ld), dev(M, dtype, ctx, ld), top, n_f=n_f,
                              swaps=True)
    torch.cuda.synchronize()
    want = rk.swaps(ref, U, M)
    assert np.array_equal(s.cpu().numpy(), want)
    assert mean_q.item() == pytest.approx(rk.accuracy(ref, U, M), abs=1e-13)


def test_ties_decided_by_item_id(ctx):
    """Integer factors: every predicted rating is exact, with many ties,
    zero rows (unrated items) and duplicated rows."""
    from paper_1508_03110_amd.solver import rank_accuracy, rank_top_t
    rng = np.random.default_rng(3)
    U = rng.integers(-2, 3, size=(90, 6)).astype(np.float64)
    M = rng.integers(-2, 3, size=(150, 6)).astype(np.float64)
    M[::7] = 0.0
    M[100:110] = M[10:20]
    for dtype in (torch.float32, torch.float64):
        Ud, Md = dev(U, dtype, ctx), dev(M, dtype, ctx)
        top = rank_top_t(ctx, Ud, Md, 25)
        torch.cuda.synchronize()
        assert np.array_equal(top.cpu().numpy(), rk.top_t(U, M, 25))
        U2 = U + rng.integers(-1, 2, size=U.shape)
        ref = rk.top_t(U2, M, 25)
        _, s = rank_accuracy(ctx, Ud, Md, torch.as_tensor(ref).to(ctx.torch_device), swaps=True)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), rk.swaps(ref, U, M))


def test_extremes_and_chaining(ctx):
    """Own top-t: every swap count 0 and accuracy exactly 1; negated users
    (reversed rankings, no ties): every count s_max and accuracy exactly 0."""
    from paper_1508_03110_amd.solver import rank_accuracy, rank_top_t
    U, M = factors(200, 500, 64, 9, torch.float32)
    Ud, Md = dev(U, torch.float32, ctx), dev(M, torch.float32, ctx)
    top = rank_top_t(ctx, Ud, Md, 20)
    q, s = rank_accuracy(ctx, Ud, Md, top, swaps=True)
    torch.cuda.synchronize()
    assert q.item() == 1.0 and int(s.abs().max()) == 0
    q, s = rank_accuracy(ctx, -Ud, Md, top, swaps=True)
    torch.cuda.synchronize()
    assert q.item() == 0.0 and bool((s == rk.s_max(500, 20)).all())


def test_ml20m_shape_sampled_users(ctx):
    """138,493 users x 26,744 items, n_f = 100, t = 20, in the launch the
    benchmark uses; the oracle checks 48 users spread over the range,
    including the first and the last."""
    from paper_1508_03110_amd.solver import rank_accuracy, rank_top_t
    n_u, n_m, n_f, t = 138_493, 26_744, 100, 20
    g = torch.Generator(device=ctx.torch_device).manual_seed(5)
    U = torch.randn((n_u, n_f), generator=g, device=ctx.torch_device) / 10
    M = torch.randn((n_m, n_f), generator=g, device=ctx.torch_device) / 10
    U2 = U + 0.05 * torch.randn((n_u, n_f), generator=g, device=ctx.torch_device)
    top = rank_top_t(ctx, U, M, t)
    q, s = rank_accuracy(ctx, U2, M, top, swaps=True)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, n_u - 1], np.linspace(1, n_u - 2, 46).astype(np.int64)]))
    Uh, U2h, Mh = (a.cpu().numpy().astype(np.float64) for a in (U, U2, M))
    top_h = top.cpu().numpy()
    assert np.array_equal(top_h[rows], rk.top_t(Uh, Mh, t, rows=rows))
    assert np.array_equal(s.cpu().numpy()[rows], rk.swaps(top_h, U2h, Mh, rows=rows))
    s_all = s.cpu().numpy()
    assert q.item() == pytest.approx(1.0 - s_all.sum() / (n_u * rk.s_max(n_m, t)), abs=1e-15)


def test_argument_errors(ctx):
    from paper_1508_03110_amd import _lib as L
    U = torch.zeros((4, 8), dtype=torch.float32, device=ctx.torch_device)
    M = torch.zeros((10, 8), dtype=torch.float32, device=ctx.torch_device)
    top = torch.zeros((4, 33), dtype=torch.int32, device=ctx.torch_device)
    h = ctx.handle
    bad = [
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 8, L.F32, 0, top),      # t = 0
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 8, L.F32, 33, top),     # t > 32
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 8, L.F32, 11, top),     # t > n_m
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 7, L.F32, 5, top),      # ld < n_f
        lambda: L.rank_top_t(h, U, M, 4, 10, 129, 129, L.F32, 5, top),  # n_f > 128
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 8, L.BF16, 5, top),     # dtype
        lambda: L.rank_top_t(h, U, M, 4, 10, 8, 8, L.F32, 5, None),     # NULL output
        lambda: L.rank_accuracy(h, U, M, 0, 10, 8, 8, L.F32, 5, top),   # no users
        lambda: L.rank_accuracy(h, U, M, 4, 1, 8, 8, L.F32, 1, top),    # n_m < 2
    ]
    for f in bad:
        with pytest.raises(L.AlsError) as e:
            f()
        assert e.value.status == L.E_INVAL
    L.rank_top_t(h, U, M, 0, 10, 8, 8, L.F32, 5, top)  # no users: nothing to do
