"""Seeded synthetic ratings problems for the ALS / ALS-NCG hot path.

This module builds inputs only: sparse rating matrices (CSR by users and
CSC = CSR of the transpose by items), initial factors and fold-in request
streams.  It holds none of the method's arithmetic (no normal equations, no
loss, no gradient, no line search), so both the FP64 oracle and the GPU path
may use it.

The workloads stand in for the paper's MovieLens-20M experiments (Section IV,
Section VI) and the ML-20M-resampled synthetics of Section VI, whose data is
not available: every generator here is parametric and seeded.

Layout conventions shared by every consumer:
  * ``indptr``  int64 [n_rows + 1], ``indices`` int32 [nnz], ``values``
    float32 [nnz]; column ids strictly increasing inside a row, no duplicate
    (row, col) pair.
  * Factors are row-major ``[n_entities, n_f]`` (one latent vector per row),
    the same memory image as the paper's column-per-entity n_f x n matrices.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Optional

import numpy as np

__all__ = [
    "Csr", "Problem", "csr_from_pairs", "transpose", "c0_tiny", "c1_ml20m",
    "zipf_lognormal", "random_problem", "dense_problem", "fold_in_requests",
    "initial_factors", "holdout_split",
]


@dataclasses.dataclass
class Csr:
    """One orientation of the ratings matrix (rows = users for R, items for R^T)."""

    n_rows: int
    n_cols: int
    indptr: np.ndarray   # int64 [n_rows + 1]
    indices: np.ndarray  # int32 [nnz]
    values: np.ndarray   # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.indptr)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.indptr, self.indices, self.values):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


@dataclasses.dataclass
class Problem:
    """A ratings matrix in both orientations plus the run parameters."""

    name: str
    R: Csr    # users x items
    Rt: Csr   # items x users
    n_f: int
    lam: float
    U0: np.ndarray  # float64 [n_u, n_f]
    M0: np.ndarray  # float64 [n_m, n_f]
    seed: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_u(self) -> int:
        return self.R.n_rows

    @property
    def n_m(self) -> int:
        return self.R.n_cols

    @property
    def nnz(self) -> int:
        return self.R.nnz


# ----------------------------------------------------------------------------
# sparse plumbing
# ----------------------------------------------------------------------------

def csr_from_pairs(rows: np.ndarray, cols: np.ndarray, values: np.ndarray,
                   n_rows: int, n_cols: int) -> Csr:
    """Sort (row, col) pairs row-major and build a CSR; duplicates are an error."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * n_cols + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) pair")
    r = rows[order]
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n_rows), out=indptr[1:])
    return Csr(n_rows, n_cols, indptr, cols[order].astype(np.int32),
               np.asarray(values, dtype=np.float32)[order])


def transpose(A: Csr) -> Csr:
    """CSR of A^T (equivalently the CSC of A), rows sorted by column id."""
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), A.counts())
    cols = A.indices.astype(np.int64)
    order = np.argsort(cols, kind="stable")  # stable keeps row ids ascending
    indptr = np.zeros(A.n_cols + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=A.n_cols), out=indptr[1:])
    return Csr(A.n_cols, A.n_rows, indptr, rows[order].astype(np.int32),
               A.values[order].copy())


def _half_stars(x: np.ndarray) -> np.ndarray:
    return np.clip(np.round(2.0 * x) / 2.0, 0.5, 5.0)


def initial_factors(rng: np.random.Generator, n_u: int, n_m: int, n_f: int,
                    sigma: float = 0.1):
    """x0: U0 and M0 i.i.d. N(0, sigma) (sigma is the standard deviation)."""
    U0 = rng.normal(0.0, sigma, size=(n_u, n_f))
    M0 = rng.normal(0.0, sigma, size=(n_m, n_f))
    return U0, M0


# ----------------------------------------------------------------------------
# tiny planted problem (the FP64 parity instance)
# ----------------------------------------------------------------------------

def c0_tiny(seed: int = 0, n_u: int = 600, n_m: int = 400, nnz: int = 20000,
            rank: int = 10, n_f: int = 10, lam: float = 0.05) -> Problem:
    """Planted rank-10 model, 600 x 400 with 20,000 distinct observed pairs.

    Recipe: U*, M* ~ N(0, 1/sqrt(rank)); every user first rates 5 distinct
    random items; every item with fewer than 3 raters then gets random new
    raters until it has 3; the rest is a uniform fill of new pairs.  Ratings are
    u*.m* + N(0, 0.5), min-max mapped to [0.5, 5] and rounded to half-stars
    (round half to even).  x0 ~ N(0, 0.1).
    """
    ss = np.random.SeedSequence(seed)
    g_model, g_pairs, g_noise, g_x0 = [np.random.default_rng(s) for s in ss.spawn(4)]
    Us = g_model.normal(0.0, 1.0 / math.sqrt(rank), size=(n_u, rank))
    Ms = g_model.normal(0.0, 1.0 / math.sqrt(rank), size=(n_m, rank))

    seen = set()
    pairs = []

    def add(u, m):
        k = (int(u), int(m))
        if k in seen:
            return False
        seen.add(k)
        pairs.append(k)
        return True

    for u in range(n_u):
        for m in g_pairs.choice(n_m, size=5, replace=False):
            add(u, m)
    item_count = np.zeros(n_m, dtype=np.int64)
    for _, m in pairs:
        item_count[m] += 1
    for m in range(n_m):
        while item_count[m] < 3:
            if add(g_pairs.integers(n_u), m):
                item_count[m] += 1
    while len(pairs) < nnz:
        need = nnz - len(pairs)
        us = g_pairs.integers(0, n_u, size=need)
        ms = g_pairs.integers(0, n_m, size=need)
        for u, m in zip(us, ms):
            if len(pairs) >= nnz:
                break
            add(u, m)
    P = np.array(sorted(pairs), dtype=np.int64)
    rows, cols = P[:, 0], P[:, 1]
    y = np.einsum("ij,ij->i", Us[rows], Ms[cols]) + g_noise.normal(0.0, 0.5, size=rows.size)
    r = 0.5 + 4.5 * (y - y.min()) / (y.max() - y.min())
    r = np.round(2.0 * r) / 2.0
    R = csr_from_pairs(rows, cols, r, n_u, n_m)
    U0, M0 = initial_factors(g_x0, n_u, n_m, n_f)
    return Problem("c0_tiny", R, transpose(R), n_f, lam, U0, M0, seed,
                   {"rank": rank, "noise_sd": 0.5})


# ----------------------------------------------------------------------------
# Zipf-popularity / log-normal-activity generator (ML-20M shape and friends)
# ----------------------------------------------------------------------------

def _lognormal_counts(rng, n_u, n_m, nnz, min_count, sigma):
    """Row lengths min_count + floor(LogNormal(mu, sigma)), mu solved so that
    the lengths sum to exactly nnz (remainder spread +1 on random rows)."""
    z = rng.standard_normal(n_u)
    cap = n_m

    def total(mu):
        c = min_count + np.floor(np.exp(mu + sigma * z))
        return np.minimum(c, cap).sum()

    if min_count * n_u > nnz or cap * n_u < nnz:
        raise ValueError("nnz incompatible with min_count / n_m")
    lo, hi = -20.0, math.log(cap) + 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) > nnz:
            hi = mid
        else:
            lo = mid
    counts = np.minimum(min_count + np.floor(np.exp(lo + sigma * z)), cap).astype(np.int64)
    rem = nnz - int(counts.sum())
    while rem > 0:
        room = np.flatnonzero(counts < cap)
        pick = rng.choice(room, size=min(rem, room.size), replace=False)
        counts[pick] += 1
        rem = nnz - int(counts.sum())
    return counts, lo


def _distinct_popular_items(rng, counts, n_m, s, perm):
    """For row u, counts[u] distinct items drawn successively with
    p(rank) proportional to rank^-s (first-distinct of an i.i.d. stream),
    item id = perm[rank]."""
    w = np.arange(1, n_m + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(k):
        rk = np.searchsorted(cdf, rng.random(k), side="right")
        return np.minimum(rk, n_m - 1)

    n_u = counts.size
    rows = np.repeat(np.arange(n_u, dtype=np.int64), counts)
    starts = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(counts, out=starts[1:])
    ranks = draw(rows.size)
    active = np.arange(rows.size)  # slots whose row may still hold duplicates
    while active.size:
        key = rows[active] * n_m + ranks[active]
        order = np.argsort(key)
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        bad = active[order[dup]]
        if bad.size == 0:
            break
        ranks[bad] = draw(bad.size)
        # re-check only the rows that received new draws (their slots are contiguous)
        br = np.unique(rows[bad])
        ln = counts[br]
        first = np.repeat(starts[br] - np.concatenate(([0], np.cumsum(ln)[:-1])), ln)
        active = first + np.arange(int(ln.sum()))
    return rows, perm[ranks]


def zipf_lognormal(n_u: int, n_m: int, nnz: int, *, n_f: int, lam: float,
                   seed: int, rank: int = 50, zipf_s: float = 1.0,
                   min_count: int = 20, sigma: float = 1.2,
                   target_mean: float = 3.5, name: str = "zipf_lognormal") -> Problem:
    """MovieLens-20M-shaped synthetic ratings.

    * user activity: min_count + floor(LogNormal(mu, sigma)), mu solved so the
      total is exactly nnz; capped at n_m;
    * item popularity: Zipf(zipf_s) over a seeded random permutation of item ids
      (so popularity is not correlated with the id);
    * values: planted rank-``rank`` model (U*, M* ~ N(0, 1/sqrt(rank))) plus
      Gaussian noise of the same standard deviation as the signal, standardised,
      shifted by mu0 and rounded to half-stars in [0.5, 5]; mu0 is bisected so
      the realised mean is ``target_mean``.
    """
    ss = np.random.SeedSequence(seed)
    g_cnt, g_perm, g_items, g_model, g_noise, g_x0 = [np.random.default_rng(s) for s in ss.spawn(6)]
    counts, mu = _lognormal_counts(g_cnt, n_u, n_m, nnz, min_count, sigma)
    perm = g_perm.permutation(n_m)
    rows, cols = _distinct_popular_items(g_items, counts, n_m, zipf_s, perm)
    Us = g_model.normal(0.0, 1.0 / math.sqrt(rank), size=(n_u, rank)).astype(np.float32)
    Ms = g_model.normal(0.0, 1.0 / math.sqrt(rank), size=(n_m, rank)).astype(np.float32)
    sig = np.empty(rows.size, dtype=np.float64)
    step = 1 << 21
    for a in range(0, rows.size, step):
        b = min(a + step, rows.size)
        sig[a:b] = np.einsum("ij,ij->i", Us[rows[a:b]], Ms[cols[a:b]])
    sd = float(sig.std()) or 1.0
    y = sig + g_noise.normal(0.0, sd, size=rows.size)
    z = (y - y.mean()) / y.std()
    z = z.astype(np.float32)
    lo, hi = target_mean - 2.0, target_mean + 2.0
    for _ in range(24):
        mu0 = 0.5 * (lo + hi)
        if _half_stars(mu0 + z).mean() > target_mean:
            hi = mu0
        else:
            lo = mu0
    mu0 = 0.5 * (lo + hi)
    vals = _half_stars(mu0 + z)
    R = csr_from_pairs(rows, cols, vals, n_u, n_m)
    U0, M0 = initial_factors(g_x0, n_u, n_m, n_f)
    meta = {"rank": rank, "zipf_s": zipf_s, "min_count": min_count,
            "lognormal_sigma": sigma, "lognormal_mu": mu, "mu0": mu0,
            "mean_rating": float(vals.mean()), "item_perm": perm,
            "M_star": Ms, "max_user_count": int(counts.max())}
    return Problem(name, R, transpose(R), n_f, lam, U0, M0, seed, meta)


def c1_ml20m(seed: int = 1, n_f: int = 100, lam: float = 0.05) -> Problem:
    """138,493 users x 26,744 items, exactly 20,000,263 ratings, n_f=100, lambda=0.05."""
    return zipf_lognormal(138_493, 26_744, 20_000_263, n_f=n_f, lam=lam, seed=seed,
                          name="ml20m_shape")


# ----------------------------------------------------------------------------
# small structured cases for tests
# ----------------------------------------------------------------------------

def random_problem(n_u: int, n_m: int, *, n_f: int, lam: float, seed: int,
                   density: float = 0.1, min_row: int = 0, long_rows: int = 0,
                   long_len: Optional[int] = None, empty_rows: int = 0,
                   x0_sigma: float = 0.1, name: str = "random") -> Problem:
    """Uniform random pattern with optional very long rows and empty rows.

    Each user row gets Binomial(n_m, density) distinct items (at least
    ``min_row``); ``long_rows`` rows get ``long_len`` items; ``empty_rows``
    rows get none.  Values are uniform half-stars.
    """
    ss = np.random.SeedSequence(seed)
    g_pat, g_val, g_x0 = [np.random.default_rng(s) for s in ss.spawn(3)]
    lens = np.maximum(g_pat.binomial(n_m, density, size=n_u), min(min_row, n_m))
    lens = np.minimum(lens, n_m)
    order = g_pat.permutation(n_u)
    if long_rows:
        lens[order[:long_rows]] = n_m if long_len is None else min(long_len, n_m)
    if empty_rows:
        lens[order[long_rows:long_rows + empty_rows]] = 0
    rows, cols = [], []
    for u in range(n_u):
        if lens[u]:
            c = g_pat.choice(n_m, size=int(lens[u]), replace=False)
            rows.append(np.full(c.size, u, dtype=np.int64))
            cols.append(c.astype(np.int64))
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = g_val.integers(1, 11, size=rows.size) / 2.0
    R = csr_from_pairs(rows, cols, vals, n_u, n_m)
    U0, M0 = initial_factors(g_x0, n_u, n_m, n_f, x0_sigma)
    return Problem(name, R, transpose(R), n_f, lam, U0, M0, seed, {})


def dense_problem(n_u: int, n_m: int, *, n_f: int, lam: float, seed: int,
                  rank: int = 3, noise: float = 0.1) -> Problem:
    """Every (user, item) observed; low-rank-plus-noise real values."""
    ss = np.random.SeedSequence(seed)
    g_m, g_n, g_x0 = [np.random.default_rng(s) for s in ss.spawn(3)]
    A = g_m.normal(size=(n_u, rank)) @ g_m.normal(size=(rank, n_m))
    A = A + noise * g_n.normal(size=A.shape)
    rows = np.repeat(np.arange(n_u), n_m)
    cols = np.tile(np.arange(n_m), n_u)
    R = csr_from_pairs(rows, cols, A.reshape(-1).astype(np.float32), n_u, n_m)
    U0, M0 = initial_factors(g_x0, n_u, n_m, n_f)
    return Problem("dense", R, transpose(R), n_f, lam, U0, M0, seed, {})


def holdout_split(P: Problem, frac: float, seed: int):
    """Remove a seeded fraction of ratings; returns (train Problem, held-out
    (rows, cols, values))."""
    rng = np.random.default_rng(seed)
    R = P.R
    rows = np.repeat(np.arange(R.n_rows, dtype=np.int64), R.counts())
    k = int(round(frac * R.nnz))
    held = np.zeros(R.nnz, dtype=bool)
    held[rng.choice(R.nnz, size=k, replace=False)] = True
    Rtr = csr_from_pairs(rows[~held], R.indices[~held], R.values[~held], R.n_rows, R.n_cols)
    P2 = dataclasses.replace(P, name=P.name + "_train", R=Rtr, Rt=transpose(Rtr))
    return P2, (rows[held], R.indices[held].astype(np.int64), R.values[held])


# ----------------------------------------------------------------------------
# fold-in request streams
# ----------------------------------------------------------------------------

def fold_in_requests(n_req: int, n_m: int, *, seed: int, max_len: int = 2000,
                     zipf_s_len: float = 1.0, zipf_s_item: float = 1.0,
                     item_perm: Optional[np.ndarray] = None,
                     M_star: Optional[np.ndarray] = None, min_len: int = 1):
    """Ragged batch of new-user requests (CSR with one row per request).

    Lengths ~ Zipf(zipf_s_len) on [min_len, max_len]; items distinct per
    request, drawn by the Zipf(zipf_s_item) popularity law over ``item_perm``;
    values from a fresh planted user vector against ``M_star`` plus noise,
    standardised and rounded to half-stars (uniform half-stars when no planted
    model is given).
    """
    ss = np.random.SeedSequence(seed)
    g_len, g_items, g_val = [np.random.default_rng(s) for s in ss.spawn(3)]
    L = np.arange(min_len, max_len + 1, dtype=np.float64)
    wl = L ** (-zipf_s_len)
    cl = np.cumsum(wl) / wl.sum()
    lens = L[np.minimum(np.searchsorted(cl, g_len.random(n_req), side="right"), L.size - 1)].astype(np.int64)
    lens = np.minimum(lens, n_m)
    perm = np.arange(n_m) if item_perm is None else item_perm
    rows, cols = _distinct_popular_items(g_items, lens, n_m, zipf_s_item, perm)
    if M_star is not None:
        rank = M_star.shape[1]
        u = g_val.normal(0.0, 1.0 / math.sqrt(rank), size=(n_req, rank))
        s = np.einsum("ij,ij->i", u[rows], M_star[cols].astype(np.float64))
        sd = float(s.std()) or 1.0
        y = s + g_val.normal(0.0, sd, size=s.size)
        vals = _half_stars(3.5 + (y - y.mean()) / (y.std() or 1.0))
    else:
        vals = g_val.integers(1, 11, size=rows.size) / 2.0
    return csr_from_pairs(rows, cols, vals, n_req, n_m)
