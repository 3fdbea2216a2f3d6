"""Launch shapes and the billion-rating configuration.

* A persistent grid (workgroups striding over the chunks) must give results
  bit-identical to one workgroup per chunk: every chunk reduces into its own
  slot in a fixed order.
* At the full 10M x 1M, 1e9-rating shape (n_f = 50) both half-sweeps run in
  the launch configuration the benchmark uses; sampled rows (random users,
  the longest user, random items and the most-rated item, which is split
  over many chunks) are recomputed one by one by the FP64 oracle from the
  same FP32 inputs.  FP32 tolerance: 1e-4 relative per row.
* At the 20M-rating shape (n_f = 100): sampled half-sweep rows the same way,
  ten ALS-NCG iterations against the FP64 oracle's stored trajectory of f,
  and one full coefficient pass and gradient against the oracle.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def ctx():
    from paper_1508_03110_amd.solver import Context
    c = Context(0)
    yield c
    c.close()


def n_cu():
    return torch.cuda.get_device_properties(0).multi_processor_count


def test_persistent_grid_is_bit_identical(ctx):
    from paper_1508_03110_amd.solver import AlsNcg, DeviceProblem
    P = synth.random_problem(300, 200, n_f=20, lam=0.05, seed=41, density=0.05, long_rows=4,
                             long_len=190, empty_rows=5, x0_sigma=0.5)
    U0, M0 = P.U0.astype(np.float32), P.M0.astype(np.float32)
    runs = []
    for grid in (0, 7, 64):
        DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32, chunk=32)
        DP.R.set_grid(grid, grid)
        DP.Rt.set_grid(grid, grid)
        s = AlsNcg(DP).init(U0, M0)
        for _ in range(5):
            s.step()
        runs.append((s.x.clone(), s.pdir.clone(), s.f))
    for x, p, f in runs[1:]:
        assert torch.equal(x, runs[0][0]) and torch.equal(p, runs[0][1]) and f == runs[0][2]


@pytest.mark.timeout(600)
def test_billion_rating_half_sweeps_sampled(ctx):
    from paper_1508_03110_amd.solver import DeviceCsr, DeviceProblem
    from synth import scale
    print("generating 1e9 ratings", flush=True)
    R, U0, M0 = scale.generate(device=ctx.torch_device, log=lambda m: print(m, flush=True))
    Rd = DeviceCsr(ctx, R.indptr, R.indices, R.values, R.n_m)
    Rtd = DeviceCsr(ctx, R.indptr_t, R.indices_t, R.values_t, R.n_u)
    DP = DeviceProblem(ctx, Rd, Rtd, 50, 0.05, torch.float32)
    DP.R.set_grid(8 * n_cu())
    DP.Rt.set_grid(8 * n_cu())
    assert DP.R.nnz == 1_000_000_000 and DP.n_u == 10_000_000 and DP.n_m == 1_000_000
    U = torch.empty((DP.n_u, 50), dtype=torch.float32, device=ctx.torch_device)
    M = torch.empty((DP.n_m, 50), dtype=torch.float32, device=ctx.torch_device)
    bad = torch.zeros(1, dtype=torch.int64, device=ctx.torch_device)
    DP.sweep("U", M0, U, bad_row=bad)
    DP.sweep("M", U, M, bad_row=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == (1 << 63) - 1
    check_sampled(ctx, R.indptr, R.indices, R.values, R.indptr_t, R.indices_t, R.values_t,
                  M0, U, M, DP.n_u, DP.n_m, 50, 0.05, seed=9, n_users=24, n_items=12)
    # the benchmark's length bins (users with 1..46 ratings in the dual form,
    # 9.2M rows in bins of 1..3 tiles) and one workgroup per chunk; users
    # sampled among the short rows as well
    DP.R.set_grid(0)
    DP.Rt.set_grid(0)
    DP.R.set_dual(46)
    DP.Rt.set_dual(46)
    print("dual rows", DP.R.info()["dual_rows"], DP.Rt.info()["dual_rows"], flush=True)
    DP.sweep("U", M0, U, bad_row=bad)
    DP.sweep("M", U, M, bad_row=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == (1 << 63) - 1
    check_sampled(ctx, R.indptr, R.indices, R.values, R.indptr_t, R.indices_t, R.values_t,
                  M0, U, M, DP.n_u, DP.n_m, 50, 0.05, seed=10, n_users=48, n_items=12)


def check_sampled(ctx, ip_u, ix_u, va_u, ip_m, ix_m, va_m, M0, U, M, n_u, n_m, n_f, lam, seed,
                  n_users, n_items, tol=1e-4):
    """Sampled rows of both half-sweeps (random rows plus the longest row of
    each orientation) recomputed by the FP64 oracle from the same FP32 inputs."""
    dev = ctx.torch_device
    rng = np.random.default_rng(seed)
    lens_u = ip_u[1:] - ip_u[:-1]
    lens_m = ip_m[1:] - ip_m[:-1]
    users = sorted(set(rng.integers(0, n_u, n_users).tolist()) | {int(torch.argmax(lens_u))})
    items = sorted(set(rng.integers(0, n_m, n_items).tolist()) | {int(torch.argmax(lens_m))})
    for side, rows, ip, ix, va, Y, X in (("U", users, ip_u, ix_u, va_u, M0, U),
                                         ("M", items, ip_m, ix_m, va_m, U, M)):
        ipr = ip.cpu().numpy()
        sel = np.concatenate([np.arange(ipr[r], ipr[r + 1]) for r in rows])
        sel_t = torch.as_tensor(sel, device=dev)
        ids = ix[sel_t].cpu().numpy()
        vals = va[sel_t].cpu().numpy()
        ptr = np.zeros(len(rows) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum([ipr[r + 1] - ipr[r] for r in rows])
        cols, inv = np.unique(ids, return_inverse=True)
        A = synth.Csr(len(rows), len(cols), ptr, inv.astype(np.int32), vals.astype(np.float32))
        Ysub = Y[torch.as_tensor(cols, device=dev)][:, :n_f].cpu().numpy().astype(np.float64)
        ref = oracle.half_sweep(A, Ysub, lam)
        got = X[torch.as_tensor(rows, device=dev)][:, :n_f].cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
        for k, r in enumerate(rows):
            print(side, r, "len", ptr[k + 1] - ptr[k], "rel %.3e" % rel[k], flush=True)
        assert rel.max() <= tol, side


@pytest.fixture(scope="module")
def c1():
    print("generating the 20M-rating problem", flush=True)
    return synth.c1_ml20m()


@pytest.fixture(scope="module")
def c1_dev(ctx, c1):
    """Default plans with the benchmark's usual choices: users with 20..78
    ratings (67,275 rows) in the dual form (no item has fewer than 79), the
    user half-sweep over the split copy of M, the M-block gradient over the
    plan of R^T cut at 8 user slices."""
    from paper_1508_03110_amd.solver import DeviceProblem
    DP = DeviceProblem(ctx, c1.R, c1.Rt, c1.n_f, c1.lam, torch.float32)
    DP.R.set_dual(78)
    DP.R.set_split_copy(1)
    DP.Rt.set_grad_slices(8)
    assert DP.R.info()["dual_rows"] == 67275
    return DP


@pytest.mark.timeout(300)
def test_ml20m_shape_half_sweeps_sampled(ctx, c1, c1_dev):
    """The 20M-rating shape in the benchmark's launch configuration (default
    plans), including the most-rated item (137,241 ratings, split)."""
    P, DP = c1, c1_dev
    dev = ctx.torch_device
    M0 = torch.as_tensor(P.M0.astype(np.float32)).to(dev)
    U = torch.empty((P.n_u, P.n_f), dtype=torch.float32, device=dev)
    M = torch.empty((P.n_m, P.n_f), dtype=torch.float32, device=dev)
    DP.sweep("U", M0, U)
    DP.sweep("M", U, M)
    torch.cuda.synchronize()
    check_sampled(ctx, DP.R.indptr, DP.R.indices, DP.R.values, DP.Rt.indptr, DP.Rt.indices,
                  DP.Rt.values, M0, U, M, P.n_u, P.n_m, P.n_f, P.lam, seed=8, n_users=24,
                  n_items=12)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("mode", ["host", "device"])
def test_ml20m_shape_als_ncg_trajectory(ctx, c1, c1_dev, mode):
    """Ten FP32 ALS-NCG iterations at the 20M-rating shape (default plans,
    the benchmark's launch configuration) from the shared x0 (seeded U0, M0
    rounded to FP32): f(x_k) within 1e-5 relative of the FP64 oracle's
    trajectory from the same x0, stored by tests/golden/make_fstar.py from
    the oracle alone.  The oracle restarts once (iteration 2: the first
    direction is an ascent direction, g^T p = +6.4e9), so the restart path
    runs at full size.  Its accepted Armijo tests over these iterations are
    at least 2e-3 |g^T p| from the boundary, so no trial count flips in FP32."""
    from paper_1508_03110_amd.solver import AlsNcg
    ref = json.load(open(os.path.join(GOLDEN, "fstar_ml20m_shape.json")))
    assert ref["problem"]["csr_digest"] == c1.R.digest()
    traj = ref["f_trajectory"]
    s = AlsNcg(c1_dev).init(c1.U0.astype(np.float32), c1.M0.astype(np.float32))
    for k in range(1, 11):
        if mode == "host":
            s.step()
        else:
            s.step_device()
            s.read_state()
        print("iteration %d f %.10g oracle %.10g rel %.2e restarts %d" %
              (k, s.f, traj[k], abs(s.f - traj[k]) / traj[k], s.restarts), flush=True)
        assert s.f == pytest.approx(traj[k], rel=1e-5), k
    assert s.restarts == 1 and s.safeguards == 0


@pytest.mark.timeout(300)
def test_ml20m_shape_full_passes(ctx, c1, c1_dev):
    """One coefficient pass and one gradient (both blocks, f and ||g||^2) over
    all 20,000,263 ratings in the default plans (8192-rating chunks, 315
    split item rows; the M block over the plan cut at 8 user slices, then
    again over the ordinary plan) against the FP64 oracle on the same FP32
    inputs:
    coefficients within 1e-6 of the largest, gradient within 1e-5 relative
    (Frobenius, per block), f and ||g||^2 within 1e-6 and 1e-5."""
    P, DP = c1, c1_dev
    dev = ctx.torch_device
    rng = np.random.default_rng(77)
    U0, M0 = P.U0.astype(np.float32), P.M0.astype(np.float32)
    PU = rng.normal(0.0, 0.1, U0.shape).astype(np.float32)
    PM = rng.normal(0.0, 0.1, M0.shape).astype(np.float32)
    x, p = DP.pack(U0, M0), DP.pack(PU, PM)
    C = torch.zeros(5, dtype=torch.float64, device=dev)
    DP.coeffs(DP.U(x), DP.M(x), DP.U(p), DP.M(p), C)
    g = DP.zeros()
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    DP.gradient(DP.U(x), DP.M(x), DP.U(g), DP.M(g), out)
    torch.cuda.synchronize()
    print("oracle passes", flush=True)
    f64 = lambda a: a.astype(np.float64)  # noqa: E731
    ref = oracle.quartic(P.R, f64(U0), f64(M0), f64(PU), f64(PM), P.lam)
    Cg = C.cpu().numpy()
    print("coefficients", Cg, ref, flush=True)
    assert np.max(np.abs(Cg - ref)) <= 1e-6 * np.max(np.abs(ref))
    gU, gM = oracle.gradient(P.R, P.Rt, f64(U0), f64(M0), P.lam)
    f = oracle.loss(P.R, f64(U0), f64(M0), P.lam)
    for got, want in ((DP.U(g), gU), (DP.M(g), gM)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)
    fg, gg = out.cpu().tolist()
    assert fg == pytest.approx(f, rel=1e-6)
    assert gg == pytest.approx(float(np.sum(gU ** 2) + np.sum(gM ** 2)), rel=1e-5)
    # the same gradient over the ordinary plans of both orientations
    try:
        DP.Rt.set_grad_slices(0)
        g8 = DP.zeros()
        out8 = torch.zeros(2, dtype=torch.float64, device=dev)
        DP.gradient(DP.U(x), DP.M(x), DP.U(g8), DP.M(g8), out8)
        torch.cuda.synchronize()
    finally:
        DP.Rt.set_grad_slices(8)
    for got, want in ((DP.U(g8), gU), (DP.M(g8), gM)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want)
    fg8, gg8 = out8.cpu().tolist()
    assert fg8 == pytest.approx(f, rel=1e-6)
    assert gg8 == pytest.approx(float(np.sum(gU ** 2) + np.sum(gM ** 2)), rel=1e-5)


def test_ml20m_shape_split_copy_is_bitwise(ctx, c1, c1_dev):
    """Both half-sweeps over all 20,000,263 ratings (8192-rating chunks, split
    rows on both sides, the fused gradient on the user side) with and without
    the split copy of the fixed side: every output bit equal."""
    P, DP = c1, c1_dev
    dev = ctx.torch_device
    x = DP.pack(P.U0.astype(np.float32), P.M0.astype(np.float32))
    for side, A, Y, n in (("U", DP.R, DP.M(x), P.n_u), ("M", DP.Rt, DP.U(x), P.n_m)):
        outs = []
        try:
            for mode in (0, 1):
                A.set_split_copy(mode)
                X = torch.empty((n, DP.ld), dtype=torch.float32, device=dev)
                G = torch.empty((n, DP.ld), dtype=torch.float32, device=dev) if side == "U" else None
                DP.sweep(side, Y, X, X_at=DP.U(x) if side == "U" else None, grad_out=G)
                outs.append((X, G))
            torch.cuda.synchronize()
        finally:
            A.set_split_copy(1 if side == "U" else -1)
        print("split copy", side, flush=True)
        assert torch.equal(outs[0][0], outs[1][0])
        if side == "U":
            assert torch.equal(outs[0][1], outs[1][1])
