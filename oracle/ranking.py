"""Top-t ranking accuracy of Section IV (a modified Kendall tau distance).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product library.  Plain numpy in
float64; the swap count follows the procedure of Section IV step by step.

Readings where the paper is silent:
* the ranking of a user orders items by the predicted rating u_i . m_j,
  largest first, computed in float64 (FP32 factors are widened first);
* items with equal predicted ratings are ordered by increasing item id;
* the top-t items of the reference ranking are moved, in their reference
  order, to the front of the current ranking, each by adjacent swaps.
"""
from __future__ import annotations

import numpy as np


def ranking(U, M, rows=None) -> np.ndarray:
    """Full ranking of every user (Section IV): row r lists all item ids in
    decreasing order of predicted rating U[i] . M[j] (float64), equal ratings
    by increasing id, for i = rows[r] (all users when rows is None)."""
    U = np.asarray(U, np.float64)
    M = np.asarray(M, np.float64)
    if rows is not None:
        U = U[np.asarray(rows)]
    scores = U @ M.T
    ids = np.broadcast_to(np.arange(M.shape[0]), scores.shape)
    # lexsort: last key is the primary one
    return np.lexsort((ids, -scores), axis=-1)


def top_t(U, M, t: int, rows=None) -> np.ndarray:
    """The first t entries of each user's ranking, int32 [rows, t]."""
    return ranking(U, M, rows)[:, :t].astype(np.int32)


def s_max(n_m: int, t: int) -> int:
    """Largest swap count, reached when the two rankings are in opposite
    order: (n_m - 1) + (n_m - 2) + ... + (n_m - t) (Section IV)."""
    return t * (2 * n_m - t - 1) // 2


def swaps_to_match(top1, p2, return_moved: bool = False):
    """s_i of Section IV: for k = 1..t, find the k-th top item of the
    reference ranking in the current ranking (already rearranged by the
    earlier steps) and move it to position k by adjacent swaps; s_i counts
    the swaps.  top1: the reference top-t item ids in order; p2: the full
    current ranking.  With return_moved, also returns the rearranged ranking."""
    p = [int(v) for v in p2]
    s = 0
    for k, item in enumerate(int(v) for v in top1):
        pos = p.index(item)
        s += pos - k          # one swap per place it moves forward
        p.insert(k, p.pop(pos))
    return (s, p) if return_moved else s


def swaps(ref_top, U, M, rows=None) -> np.ndarray:
    """s_i for every user (or for rows): reference top-t lists ref_top
    [n_u, t] against the ranking of the current factors (U, M)."""
    R2 = ranking(U, M, rows)
    ref = np.asarray(ref_top)
    if rows is not None:
        ref = ref[np.asarray(rows)]
    return np.array([swaps_to_match(ref[r], R2[r]) for r in range(R2.shape[0])], np.int64)


def accuracy(ref_top, U, M, rows=None) -> float:
    """Ranking accuracy of Section IV: the mean over users of
    q_i = 1 - s_i / s_max."""
    t = np.asarray(ref_top).shape[1]
    s = swaps(ref_top, U, M, rows)
    return float(np.mean(1.0 - s / s_max(np.asarray(M).shape[0], t)))
