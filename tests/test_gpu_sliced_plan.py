"""GPU parity of the gradient pass over column-sliced plans (every row cut at
column-slice boundaries, one slice per accelerator die at a time) against
the FP64 oracle's gradient and loss of Eq. (1): both gradient blocks, f and
||g||^2 at the tolerances of the ordinary plans (FP64 1e-12, FP32 1e-5 of
the gradient's scale), bitwise repeatability for a fixed plan, the layout
(a multiple of 8 pieces, every rating in exactly one piece), and the calls
that refuse such a plan.
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


def fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def host(t, n_f):
    return t.detach().cpu().numpy().astype(np.float64)[:, :n_f]


def problem(seed, n_f, n_u=90, n_m=70):
    return synth.random_problem(n_u, n_m, n_f=n_f, lam=0.07, seed=seed, density=0.15,
                                long_rows=2, empty_rows=3, x0_sigma=0.5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n_slices,chunk", [(1, 0), (3, 0), (8, 0), (8, 8), (16, 0), (40, 4)])
@pytest.mark.parametrize("n_f", [20, 50, 100, 140])
def test_sliced_gradient_matches_oracle(ctx, dtype, n_slices, chunk, n_f):
    """Both blocks through sliced plans of R and R^T: slices with no ratings
    of a row, rows in one slice only, empty rows, pieces cut further by a
    small chunk, more slices than some rows have ratings."""
    from paper_1508_03110_amd.solver import DeviceProblem
    P = problem(40 + n_f, n_f)
    cast = (lambda a: a) if dtype == torch.float64 else r32
    U0, M0 = cast(P.U0), cast(P.M0)
    DP = DeviceProblem(ctx, P.R, P.Rt, n_f, P.lam, dtype)
    DP.R.set_grad_slices(n_slices, chunk)
    DP.Rt.set_grad_slices(n_slices, chunk)
    x = DP.pack(U0, M0)
    g = DP.zeros()
    out = torch.zeros(2, dtype=torch.float64, device=ctx.torch_device)
    DP.gradient(DP.U(x), DP.M(x), DP.U(g), DP.M(g), out)
    gU, gM = oracle.gradient(P.R, P.Rt, U0, M0, P.lam)
    f = oracle.loss(P.R, U0, M0, P.lam)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert fro(host(DP.U(g), n_f), gU) <= tol
    assert fro(host(DP.M(g), n_f), gM) <= tol
    # empty rows: a zero gradient row
    empty = np.flatnonzero(P.R.counts() == 0)
    assert empty.size and np.all(host(DP.U(g), n_f)[empty] == 0.0)
    fg, gg = out.cpu().tolist()
    assert fg == pytest.approx(f, rel=1e-12 if dtype == torch.float64 else 1e-6)
    assert gg == pytest.approx(float(np.sum(gU ** 2) + np.sum(gM ** 2)),
                               rel=1e-11 if dtype == torch.float64 else 1e-5)
    # a fixed plan gives the same bits again
    g2 = DP.zeros()
    out2 = torch.zeros(2, dtype=torch.float64, device=ctx.torch_device)
    DP.gradient(DP.U(x), DP.M(x), DP.U(g2), DP.M(g2), out2)
    assert torch.equal(g, g2) and torch.equal(out, out2)


@pytest.mark.parametrize("n_slices,chunk", [(1, 0), (5, 0), (8, 4), (16, 0)])
def test_sliced_plan_layout(ctx, n_slices, chunk):
    """Pieces come in whole groups of 8 (one per die); the split stage holds
    every row with more than one piece; a slice's spare positions are empty
    pieces (counted by the extra slot)."""
    from paper_1508_03110_amd import _lib as L
    from paper_1508_03110_amd.solver import DeviceCsr
    P = problem(7, 16)
    A = DeviceCsr.from_host(ctx, P.Rt)
    A.set_grad_slices(n_slices, chunk)
    info = L.als_plan_info(A.grad_plan)
    assert info["n_chunks"] % 8 == 0
    assert info["nnz"] == P.Rt.nnz and info["n_rows"] == P.Rt.n_rows
    # rows that touch more than one slice (or exceed the chunk) are split rows
    counts = P.Rt.counts()
    if n_slices == 1 and chunk == 0:
        assert info["split_rows"] == 0
    else:
        assert info["split_rows"] >= 1
    assert info["n_chunks"] >= P.Rt.n_rows
    assert int(np.sum(counts)) == P.Rt.nnz
    A.close()


def test_sliced_plan_refused_outside_the_gradient(ctx):
    from paper_1508_03110_amd import _lib as L
    from paper_1508_03110_amd.solver import DeviceProblem
    P = problem(9, 16)
    DP = DeviceProblem(ctx, P.R, P.Rt, 16, P.lam, torch.float32)
    DP.R.set_grad_slices(8)
    sp = DP.R.grad_plan
    x = DP.pack(r32(P.U0), r32(P.M0))
    X = torch.zeros((DP.n_u, DP.ld), dtype=torch.float32, device=ctx.torch_device)
    C = torch.zeros(5, dtype=torch.float64, device=ctx.torch_device)
    with pytest.raises(L.AlsError) as e:
        L.als_sweep(ctx.handle, sp, DP.R.csr, DP.M(x), X, 16, DP.ld, P.lam, DP.dt)
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.AlsError) as e:
        L.linesearch_coeffs(ctx.handle, sp, DP.R.csr, DP.Rt.csr, DP.U(x), DP.M(x), DP.U(x),
                            DP.M(x), 16, DP.ld, P.lam, DP.dt, C)
    assert e.value.status == L.E_INVAL
    with pytest.raises(L.AlsError) as e:
        L.als_plan_set_dual(sp, 14)
    assert e.value.status == L.E_INVAL
    for bad in (0, 4097):
        with pytest.raises(L.AlsError) as e:
            L.als_plan_create_sliced(ctx.handle, DP.R.csr, 0, bad)
        assert e.value.status == L.E_INVAL


def test_sliced_plan_needs_ascending_columns(ctx):
    """A row whose column ids are not ascending is refused (a slice would not
    be one segment of it)."""
    from paper_1508_03110_amd import _lib as L
    dev = ctx.torch_device
    indptr = torch.tensor([0, 3, 5], dtype=torch.int64, device=dev)
    indices = torch.tensor([0, 4, 2, 1, 3], dtype=torch.int32, device=dev)
    values = torch.ones(5, dtype=torch.float32, device=dev)
    csr = L.Csr(2, 5, 5, indptr.data_ptr(), indices.data_ptr(), values.data_ptr())
    with pytest.raises(L.AlsError) as e:
        L.als_plan_create_sliced(ctx.handle, csr, 0, 2)
    assert e.value.status == L.E_INVAL
    indices_ok = torch.tensor([0, 2, 4, 1, 3], dtype=torch.int32, device=dev)
    csr_ok = L.Csr(2, 5, 5, indptr.data_ptr(), indices_ok.data_ptr(), values.data_ptr())
    plan = L.als_plan_create_sliced(ctx.handle, csr_ok, 0, 2)
    L.als_plan_destroy(plan)
