"""Pins of the ranking-accuracy oracle (Section IV) against facts the paper and
the mathematics fix: the paper's worked example, the extreme cases it states,
Kendall's tau of the full rankings (a library routine), a pair-count form of
the swap count, and brute-force sorting of exact integer ratings."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import ranking as rk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "kendall_top_t_example.json")))
    p1, p2, t = g["p1"], g["p2"], g["t"]
    s, moved = rk.swaps_to_match(p1[:t], p2, return_moved=True)
    assert s == g["swaps"]
    # after the first move the current ranking reads as the paper prints it
    s1, first = rk.swaps_to_match(p1[:1], p2, return_moved=True)
    assert first == g["after_first_move"] and s1 == g["swaps"]
    assert moved == g["after_first_move"]
    assert rk.s_max(g["n_m"], t) == g["s_max"]
    assert 1.0 - s / rk.s_max(g["n_m"], t) == pytest.approx(g["q"], abs=1e-15)


@pytest.mark.parametrize("n", [2, 3, 6, 17])
def test_identical_and_opposite_order(n):
    """Equal rankings need no swap; rankings in opposite order need the
    maximum (n-1) + ... + (n-t), the normalisation of Section IV."""
    rng = np.random.default_rng(n)
    p = rng.permutation(n)
    for t in range(1, n + 1):
        assert rk.swaps_to_match(p[:t], p) == 0
        assert rk.swaps_to_match(p[:t], p[::-1]) == rk.s_max(n, t)
        assert rk.s_max(n, t) == sum(n - k for k in range(1, t + 1))


@pytest.mark.parametrize("n,seed", [(5, 0), (12, 1), (40, 2)])
def test_full_ranking_is_kendall_tau(n, seed):
    """With t = n (and t = n - 1, the last place being forced) the swap count is
    the number of discordant pairs, so q = (1 + tau) / 2 with Kendall's tau."""
    rng = np.random.default_rng(seed)
    for _ in range(5):
        p1, p2 = rng.permutation(n), rng.permutation(n)
        pos1, pos2 = np.empty(n, int), np.empty(n, int)
        pos1[p1], pos2[p2] = np.arange(n), np.arange(n)
        tau = stats.kendalltau(pos1, pos2).statistic
        for t in (n, n - 1):
            q = 1.0 - rk.swaps_to_match(p1[:t], p2) / rk.s_max(n, t)
            assert q == pytest.approx((1.0 + tau) / 2.0, abs=1e-12)


def test_pair_count_form():
    """s counts the pairs (a_k, x) with x ranked ahead of a_k by the current
    ranking and x not one of a_1..a_{k-1}: discordant pairs inside the top-t
    set plus, for each a_k, the items outside the set ranked ahead of it."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(2, 60))
        t = int(rng.integers(1, n + 1))
        p1, p2 = rng.permutation(n), rng.permutation(n)
        pos2 = np.empty(n, int)
        pos2[p2] = np.arange(n)
        top = p1[:t]
        inside = sum(1 for i in range(t) for j in range(i + 1, t) if pos2[top[j]] < pos2[top[i]])
        outside_mask = np.ones(n, bool)
        outside_mask[top] = False
        outside_pos = np.sort(pos2[outside_mask])
        outside = int(np.searchsorted(outside_pos, pos2[top]).sum())
        assert rk.swaps_to_match(top, p2) == inside + outside


def test_ranking_brute_force_with_ties():
    """Integer factors make every predicted rating exact, with many ties
    (including zero rows, the factors of unrated items): the ranking equals a
    plain sort by (-rating, item id)."""
    rng = np.random.default_rng(11)
    U = rng.integers(-2, 3, size=(9, 3)).astype(np.float64)
    M = rng.integers(-2, 3, size=(23, 3)).astype(np.float64)
    M[[4, 9]] = 0.0
    M[15] = M[3]
    R = rk.ranking(U, M)
    for i in range(U.shape[0]):
        score = [sum(U[i, k] * M[j, k] for k in range(3)) for j in range(M.shape[0])]
        want = sorted(range(M.shape[0]), key=lambda j: (-score[j], j))
        assert list(R[i]) == want
    assert np.array_equal(rk.top_t(U, M, 5), R[:, :5])
    assert np.array_equal(rk.top_t(U, M, 5, rows=[2, 7]), R[[2, 7], :5])


def test_accuracy_extremes():
    """Against its own top-t the accuracy is 1; with every predicted rating
    negated (no ties) each ranking is reversed and the accuracy is 0."""
    rng = np.random.default_rng(5)
    U, M = rng.standard_normal((30, 4)), rng.standard_normal((50, 4))
    for t in (1, 7, 20, 50):
        ref = rk.top_t(U, M, t)
        assert rk.accuracy(ref, U, M) == 1.0
        assert rk.accuracy(ref, -U, M) == 0.0
        s = rk.swaps(ref, 2.0 * U + 0.3 * rng.standard_normal(U.shape), M)
        assert np.all((s >= 0) & (s <= rk.s_max(50, t)))
