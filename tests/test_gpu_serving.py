"""Fold-in server (continuous batching) against the oracle and against itself."""
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


def setup(ctx, n_m=600, n_f=100, dtype=torch.float32, seed=0):
    rng = np.random.default_rng(seed)
    M = rng.normal(0, 0.3, (n_m, n_f))
    if dtype == torch.float32:
        M = M.astype(np.float32).astype(np.float64)
    Md = torch.as_tensor(M, dtype=dtype).to(ctx.torch_device)
    return M, Md


def rowrel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-30)))


@pytest.mark.parametrize("split", [0, 64])
def test_server_matches_oracle_and_fold_in(ctx, split):
    """Served solutions equal the oracle's row solves, and bitwise the
    one-shot fold_in call's (no split) whatever the batching."""
    from paper_1508_03110_amd.solver import FoldInServer, fold_in
    M, Md = setup(ctx)
    req = synth.fold_in_requests(300, M.shape[0], seed=7, max_len=500)
    srv = FoldInServer(ctx, Md, 0.05, 100, max_inflight=3, max_batch=37, split=split)
    ids = np.arange(300) * 10 + 1
    srv.submit(ids[:150], synth.Csr(150, M.shape[0], req.indptr[:151], req.indices, req.values))
    got_ids, st, U = srv.drain()
    srv.submit(ids[150:], synth.Csr(150, M.shape[0], req.indptr[150:] - req.indptr[150],
                                     req.indices[req.indptr[150]:], req.values[req.indptr[150]:]))
    i2, s2, U2 = srv.drain()
    got_ids, st, U = np.concatenate([got_ids, i2]), np.concatenate([st, s2]), np.concatenate([U, U2])
    assert sorted(got_ids.tolist()) == sorted(ids.tolist())
    assert np.all(st == 0)
    order = np.argsort(got_ids)
    U = U[order].astype(np.float64)
    ref = oracle.fold_in(M, req, 0.05)
    assert rowrel(U, ref) < 1e-4
    if split == 0:
        Uf, _ = fold_in(ctx, Md, 0.05, req, 100)
        assert np.array_equal(U.astype(np.float32), Uf.cpu().numpy())
    srv.close()


def test_server_alone_vs_in_the_mix(ctx):
    """A request's result does not depend on the batch it shares."""
    from paper_1508_03110_amd.solver import FoldInServer
    M, Md = setup(ctx)
    req = synth.fold_in_requests(120, M.shape[0], seed=9, max_len=1500)
    mix = FoldInServer(ctx, Md, 0.05, 100, max_inflight=2, max_batch=64, split=128)
    mix.submit(np.arange(120), req)
    ids, st, U = mix.drain()
    U = U[np.argsort(ids)]
    alone = FoldInServer(ctx, Md, 0.05, 100, max_inflight=1, max_batch=1, split=128)
    for q in (0, 5, 77, 119):
        a, b = req.indptr[q], req.indptr[q + 1]
        one = synth.Csr(1, M.shape[0], np.array([0, b - a]), req.indices[a:b], req.values[a:b])
        alone.submit(np.array([q]), one)
        i1, s1, U1 = alone.drain()
        assert i1.tolist() == [q] and s1.tolist() == [0]
        assert np.array_equal(U1[0], U[q])
    mix.close()
    alone.close()


def test_server_budget_and_bad_requests(ctx):
    """Tiny HBM budget: requests that fit are served (deferred, never lost),
    one that can never fit is answered with ALS_E_BUDGET; empty requests and
    out-of-range item ids are answered with ALS_E_INVAL."""
    from paper_1508_03110_amd import _lib as L
    from paper_1508_03110_amd.solver import FoldInServer
    n_m = 3000
    M, Md = setup(ctx, n_m=n_m, n_f=16)
    lens = [5, 0, 40, 3000, 7, 12]
    rng = np.random.default_rng(1)
    items, vals, ip = [], [], [0]
    for n in lens:
        n_eff = n
        items.append(rng.choice(n_m, size=n_eff, replace=False).astype(np.int32))
        vals.append(rng.integers(1, 11, size=n_eff).astype(np.float32) / 2)
        ip.append(ip[-1] + n_eff)
    items = np.concatenate(items)
    items[ip[4]] = n_m  # request 4: item id out of range
    req = synth.Csr(len(lens), n_m, np.array(ip), items, np.concatenate(vals))
    # budget: two slots of about 1000 ratings each (2 rows x 112 B + 8 KiB
    # alignment slack + 8 B per rating): the 3000-rating request never fits
    srv = FoldInServer(ctx, Md, 0.05, 16, budget_bytes=2 * (2 * 112 + 32 * 256 + 8000),
                       max_inflight=2, max_batch=2, split=0)
    srv.submit(np.arange(len(lens)), req)
    ids, st, U = srv.drain()
    got = dict(zip(ids.tolist(), st.tolist()))
    assert sorted(got) == list(range(len(lens)))
    assert got[1] == L.E_INVAL and got[4] == L.E_INVAL and got[3] == L.E_BUDGET
    for q in (0, 2, 5):
        assert got[q] == 0
    ref = oracle.fold_in(M, synth.Csr(1, n_m, np.array([0, lens[2]]), items[ip[2]:ip[3]],
                                      req.values[ip[2]:ip[3]]), 0.05)
    assert rowrel(U[ids.tolist().index(2)][None].astype(np.float64), ref) < 1e-4
    srv.close()


def test_server_replay_open_loop(ctx):
    """Open-loop replay answers every arrival once, in time order of arrival
    or later, with the same solutions as the oracle."""
    from paper_1508_03110_amd.solver import FoldInServer
    M, Md = setup(ctx)
    pool = synth.fold_in_requests(64, M.shape[0], seed=3, max_len=800)
    rng = np.random.default_rng(2)
    n = 2000
    arrival = np.cumsum(rng.exponential(1e9 / 50_000, size=n)).astype(np.int64)
    pool_row = rng.integers(0, 64, size=n).astype(np.int32)
    srv = FoldInServer(ctx, Md, 0.05, 100, max_inflight=4, max_batch=512, split=256)
    comp, st, U = srv.replay(arrival, pool_row, pool, want_U=True)
    assert np.all(st == 0)
    assert np.all(comp >= arrival)
    ref = oracle.fold_in(M, pool, 0.05)
    assert rowrel(U.astype(np.float64), ref[pool_row]) < 1e-4
    srv.close()
