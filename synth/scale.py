"""Billion-rating synthetic ratings matrix, generated on the device.

Shape of the paper's large synthetic experiments (MovieLens-resampled to
millions of users, Section VI), at 10,000,000 users x 1,000,000 items with
exactly 1,000,000,000 ratings:

* user activity: a discrete power law P(L = l) ~ l^-a on [1, 50000], the
  exponent a solved so that the mean is nnz / n_u (= 100); the total is made
  exact by +-1 on randomly chosen users;
* items: Zipf(s = 1.1) over a seeded random permutation of the item ids,
  distinct within a user (duplicates are redrawn from the same law until
  every user has its count);
* values: planted rank-20 model (U*, M* ~ N(0, 1/sqrt(20))) plus Gaussian
  noise of the signal's standard deviation, standardised, shifted by mu0 and
  rounded to half-stars in [0.5, 5]; mu0 is bisected on a sample so the mean
  is 3.5.

Everything runs in torch on `device` with one seeded torch.Generator, so the
matrix is reproducible on the same software and device type; the same code
runs on the CPU at small sizes for the tests.  This module holds no step of
the method: it only produces inputs.

Returns device tensors: CSR of R (indptr int64, indices int32, values float32)
and of R^T, plus x0 = (U0, M0) ~ N(0, 0.1).
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class DeviceRatings:
    n_u: int
    n_m: int
    nnz: int
    indptr: object       # torch int64 [n_u + 1]
    indices: object      # torch int32 [nnz]
    values: object       # torch float32 [nnz]
    indptr_t: object     # CSR of R^T
    indices_t: object
    values_t: object
    meta: dict


def power_law_exponent(mean: float, lo: int, hi: int) -> float:
    """a with sum l^(1-a) / sum l^-a = mean over l in [lo, hi] (bisection)."""
    l = np.arange(lo, hi + 1, dtype=np.float64)

    def m(a):
        w = l ** -a
        return float((l * w).sum() / w.sum())

    a0, a1 = 0.0, 4.0  # m is decreasing in a
    for _ in range(100):
        a = 0.5 * (a0 + a1)
        if m(a) > mean:
            a0 = a
        else:
            a1 = a
    return 0.5 * (a0 + a1)


def _rank_in_segment(sorted_rows):
    """Position of each element inside its run of equal values (sorted input)."""
    import torch
    n = sorted_rows.numel()
    first = torch.searchsorted(sorted_rows, sorted_rows, right=False)
    return torch.arange(n, device=sorted_rows.device) - first


def generate(n_u=10_000_000, n_m=1_000_000, nnz=1_000_000_000, *, max_len=50_000, zipf_s=1.1,
             rank=20, n_f=50, seed=2, device="cuda", block=1 << 27, target_mean=3.5,
             log=None) -> tuple:
    import torch
    if n_m > (1 << 20) or n_u > (1 << 24):
        raise ValueError("id packing needs n_m <= 2^20 and n_u <= 2^24")
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    t0 = time.perf_counter()
    say = log or (lambda *a: None)
    f64 = torch.float64

    # ---- row lengths
    a = power_law_exponent(nnz / n_u, 1, max_len)
    l = torch.arange(1, max_len + 1, dtype=f64, device=dev)
    cdf = torch.cumsum(l ** -a, 0)
    cdf = cdf / cdf[-1]
    L = torch.searchsorted(cdf, torch.rand(n_u, dtype=f64, device=dev, generator=gen)) + 1
    L = L.clamp_(1, max_len)
    for _ in range(1000):  # +-1 on random users (at most once per user per pass)
        d = int(nnz - int(L.sum()))
        if d == 0:
            break
        perm = torch.randperm(n_u, device=dev, generator=gen)
        ok = (L[perm] < max_len) if d > 0 else (L[perm] > 1)
        pick = perm[ok][: abs(d)]
        if pick.numel() == 0:
            raise RuntimeError("cannot reach the requested total")
        L[pick] += 1 if d > 0 else -1
    assert int(L.sum()) == nnz
    say("lengths: a=%.4f, max %d (%.1f s)" % (a, int(L.max()), time.perf_counter() - t0))

    # ---- item law
    ranks = torch.arange(1, n_m + 1, dtype=f64, device=dev)
    icdf = torch.cumsum(ranks ** -zipf_s, 0)
    icdf = icdf / icdf[-1]
    iperm = torch.randperm(n_m, device=dev, generator=gen)

    def draw_items(k):
        u = torch.rand(k, dtype=f64, device=dev, generator=gen)
        return iperm[torch.searchsorted(icdf, u).clamp_(max=n_m - 1)]

    # ---- distinct items per user, one block of whole users at a time
    indptr = torch.zeros(n_u + 1, dtype=torch.int64, device=dev)
    indptr[1:] = torch.cumsum(L, 0)
    keys_all = torch.empty(nnz, dtype=torch.int64, device=dev)
    u0 = 0
    rounds_max = 0
    while u0 < n_u:
        # users [u0, u1) with at most `block` ratings (at least one user)
        lim = int(indptr[u0]) + block
        u1 = int(torch.searchsorted(indptr, torch.tensor([lim], device=dev), right=True)) - 1
        u1 = max(u1, u0 + 1)
        u1 = min(u1, n_u)
        b0, b1 = int(indptr[u0]), int(indptr[u1])
        rows = torch.repeat_interleave(torch.arange(u0, u1, device=dev), L[u0:u1])
        keys = (rows << 20) | draw_items(b1 - b0)
        keys, _ = torch.sort(keys)
        dup = torch.zeros_like(keys, dtype=torch.bool)
        dup[1:] = keys[1:] == keys[:-1]
        acc = keys[~dup]
        need = torch.bincount((keys[dup] >> 20) - u0, minlength=u1 - u0)
        rounds = 0
        while int(need.sum()) > 0:
            rounds += 1
            if rounds > 400:
                raise RuntimeError("item redraws did not converge")
            over = 4 if rounds > 1 else 2
            cr = torch.repeat_interleave(torch.arange(u0, u1, device=dev), need * over)
            ck = (cr << 20) | draw_items(cr.numel())
            ck, _ = torch.sort(ck)
            fresh = torch.ones_like(ck, dtype=torch.bool)
            fresh[1:] = ck[1:] != ck[:-1]
            pos = torch.searchsorted(acc, ck).clamp_(max=acc.numel() - 1)
            fresh &= acc[pos] != ck
            ck = ck[fresh]
            r = ck >> 20
            keep = _rank_in_segment(r) < need[r - u0]
            ck = ck[keep]
            need -= torch.bincount((ck >> 20) - u0, minlength=u1 - u0)
            acc, _ = torch.sort(torch.cat([acc, ck]))
        rounds_max = max(rounds_max, rounds)
        assert acc.numel() == b1 - b0
        keys_all[b0:b1] = acc
        u0 = u1
    say("items: distinct per user, up to %d redraw rounds (%.1f s)" % (rounds_max, time.perf_counter() - t0))
    indices = (keys_all & ((1 << 20) - 1)).to(torch.int32)
    del keys_all

    # ---- values from the planted model
    Us = torch.randn(n_u, rank, device=dev, generator=gen) / math.sqrt(rank)
    Ms = torch.randn(n_m, rank, device=dev, generator=gen) / math.sqrt(rank)
    y = torch.empty(nnz, dtype=torch.float32, device=dev)
    step = 1 << 24
    rows_of = None
    for b0 in range(0, nnz, step):
        b1 = min(b0 + step, nnz)
        pos = torch.arange(b0, b1, device=dev)
        rows_of = torch.searchsorted(indptr, pos, right=True) - 1
        y[b0:b1] = (Us[rows_of] * Ms[indices[b0:b1].long()]).sum(1)
    del rows_of, Us
    sd = float(y.std())
    y += torch.randn(nnz, device=dev, generator=gen) * sd
    z = (y - float(y.mean())) / float(y.std())
    del y
    samp = z[torch.randint(0, nnz, (1 << 22,), device=dev, generator=gen)]

    def half_stars(v):
        return torch.clamp(torch.round(2.0 * v) / 2.0, 0.5, 5.0)

    lo, hi = target_mean - 2.0, target_mean + 2.0
    for _ in range(30):
        mu0 = 0.5 * (lo + hi)
        if float(half_stars(mu0 + samp).mean()) > target_mean:
            hi = mu0
        else:
            lo = mu0
    mu0 = 0.5 * (lo + hi)
    values = half_stars(mu0 + z).to(torch.float32)
    del z
    say("values: mean %.3f (%.1f s)" % (float(values.mean()), time.perf_counter() - t0))

    # ---- R^T: item-major order, by item ranges so that each sort stays small
    cnt_t = torch.bincount(indices.long(), minlength=n_m)
    indptr_t = torch.zeros(n_m + 1, dtype=torch.int64, device=dev)
    indptr_t[1:] = torch.cumsum(cnt_t, 0)
    indices_t = torch.empty(nnz, dtype=torch.int32, device=dev)
    values_t = torch.empty(nnz, dtype=torch.float32, device=dev)
    n_parts = max(1, (nnz + block - 1) // block)
    edges = np.linspace(0, n_m, n_parts + 1).astype(np.int64)
    for k in range(n_parts):
        i0, i1 = int(edges[k]), int(edges[k + 1])
        if i1 <= i0:
            continue
        sel = torch.nonzero((indices >= i0) & (indices < i1)).squeeze(1)
        r = torch.searchsorted(indptr, sel, right=True) - 1
        key = (indices[sel].long() << 24) | r
        key, order = torch.sort(key)
        t0k, t1k = int(indptr_t[i0]), int(indptr_t[i1])
        assert t1k - t0k == key.numel()
        indices_t[t0k:t1k] = (key & ((1 << 24) - 1)).to(torch.int32)
        values_t[t0k:t1k] = values[sel[order]]
    say("R^T built (%.1f s)" % (time.perf_counter() - t0))

    # ---- x0
    U0 = torch.randn(n_u, n_f, device=dev, generator=gen) * 0.1
    M0 = torch.randn(n_m, n_f, device=dev, generator=gen) * 0.1
    meta = {"power_law_a": a, "zipf_s": zipf_s, "rank": rank, "mu0": mu0, "seed": seed,
            "max_user_len": int(L.max()), "max_item_len": int(cnt_t.max()),
            "mean_rating": float(values.mean()), "redraw_rounds": rounds_max,
            "gen_seconds": time.perf_counter() - t0}
    R = DeviceRatings(n_u, n_m, nnz, indptr, indices, values, indptr_t, indices_t, values_t, meta)
    return R, U0, M0
