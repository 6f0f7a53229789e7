"""Pins of the adaptive per-subband selection oracle (Supp. A) against independent facts: a library
median, the normal distribution's MAD, hand-worked examples, the literal tie rule, the budget
arithmetic (including the case where the per-band minimum breaks the total bound), reductions to
plain top-K and to the threshold set, and invariants on random coefficient sets."""
import numpy as np
import pytest

from oracle import adaptive as A
from oracle import select as S


@pytest.mark.parametrize("n", [1, 2, 7, 8, 1001, 1000])
def test_median_matches_numpy(n):
    x = np.random.default_rng(n).normal(size=n).astype(np.float32)
    assert A.median_f32(x) == np.median(x)


def test_mad_estimates_the_normal_scale():
    # for N(mu, s^2) samples the MAD tends to s * Phi^-1(3/4) = 0.6745 s
    x = np.random.default_rng(0).normal(10.0, 2.0, size=1_000_000).astype(np.float32)
    r = A.band_filter(x, 10, 1.0)
    assert abs(r["median"] - 10.0) < 0.01
    assert abs(r["sigma"] - 2.0) < 0.01
    assert r["T"] == r["sigma"]


def test_worked_examples():
    v = np.array([1, 2, 3, 4, 100], np.float32)
    # median 3, |v - 3| = [2, 1, 0, 1, 97] -> MAD 1, sigma = 1/0.6745 = 1.48258
    r = A.band_filter(v, 10, 3.0)
    assert r["median"] == 3.0 and r["mad"] == 1.0 and abs(r["sigma"] - 1.482580) < 1e-5
    assert r["C"] == 1 and r["K"] == 1 and r["vK"] == 100.0          # T = 4.4477: only 100 passes
    assert r["keep"].tolist() == [False, False, False, False, True]
    r = A.band_filter(v, 2, 0.5)                                      # T = 0.7413: all pass, budget 2
    assert r["C"] == 5 and r["K"] == 2 and r["vK"] == 4.0
    assert r["keep"].tolist() == [False, False, False, True, True]
    r = A.band_filter(v, 0, 0.5)                                      # no budget: nothing kept
    assert r["K"] == 0 and not r["keep"].any()


def test_ties_at_the_kth_value_are_all_kept():
    v = np.array([5, 5, 5, 1, 1], np.float32)
    r = A.band_filter(v, 2, 0.0)                                      # MAD 0 -> T 0
    assert r["T"] == 0.0 and r["K"] == 2 and r["vK"] == 5.0
    assert r["keep"].tolist() == [True, True, True, False, False]    # three kept for K = 2


def test_budget_allocation():
    E, N = np.array([1.0, 3.0]), np.array([8, 8])
    assert A.budgets(E, N, 100, 1.0, 0.0, 10).tolist() == [25, 75]
    # beta weighs the subband sizes: S = N when alpha = 0
    assert A.budgets(np.array([5.0, 5.0]), np.array([1, 3]), 100, 0.0, 1.0, 10).tolist() == [25, 75]
    # the per-band minimum fires and the total exceeds K_tot (the supplement's bound fails)
    k = A.budgets(np.array([1.0, 1000.0]), N, 100, 1.0, 0.0, 10)
    assert k.tolist() == [10, 99] and k.sum() == 109
    assert A.budgets(np.zeros(3), np.array([8, 8, 8]), 100, 1.0, 0.0, 10).tolist() == [10, 10, 10]


def test_single_band_without_floor_is_plain_topk():
    # lambda = 0 gives T = 0, so with one subband the filter is the global top-K (no ties here)
    rng = np.random.default_rng(3)
    G, J = 8, 1
    c = rng.normal(size=(4, G ** 3)).astype(np.float32)
    v = S.joint_norm_f32(c)
    r = A.band_filter(v, 37, 0.0)
    assert np.array_equal(np.nonzero(r["keep"])[0], S.topk(c, 37))


def test_unbounded_budget_keeps_the_threshold_set():
    v = np.random.default_rng(4).exponential(size=5000).astype(np.float32)
    r = A.band_filter(v, 10 ** 9, 2.0)
    assert np.array_equal(r["keep"], v >= r["T"]) and r["K"] == r["C"]


@pytest.mark.parametrize("G,J,K_tot,lam", [(16, 2, 300, 3.0), (16, 1, 2000, 1.0), (32, 3, 5000, 2.5)])
def test_invariants_on_random_coefficients(G, J, K_tot, lam):
    rng = np.random.default_rng(G + J)
    c = (rng.standard_t(3, size=(4, G ** 3)) * rng.uniform(0.1, 2.0, size=(4, 1))).astype(np.float32)
    kept, stats = A.select(c, G, J, K_tot, lam=lam)
    v = S.joint_norm_f32(c)
    assert np.all(np.diff(kept) > 0)
    assert len(stats) == 7 * J + 1 and sum(s["N"] for s in stats) == G ** 3
    for s in stats:
        vb = v[s["offset"]:s["offset"] + s["N"]]
        kb = kept[(kept >= s["offset"]) & (kept < s["offset"] + s["N"])] - s["offset"]
        assert s["kept"] == kb.size
        assert s["C"] == np.count_nonzero(vb >= s["T"])
        assert s["K"] == min(s["K_band"], s["C"])
        if s["K"] == 0:
            assert kb.size == 0
            continue
        thr = max(s["T"], s["vK"])
        assert np.all(vb[kb] >= thr)                                  # kept: at or above both floors
        drop = np.setdiff1d(np.arange(s["N"]), kb)
        assert np.all(vb[drop] < thr)                                 # dropped: below one of them
        assert kb.size >= s["K"]                                      # at least K (more only on ties)
        assert kb.size == s["K"] or np.count_nonzero(vb == s["vK"]) > 1
        # v_(K) is the K-th largest value (counted from the top)
        assert np.count_nonzero(vb > s["vK"]) < s["K"] <= np.count_nonzero(vb >= s["vK"])
    # energies are the reference channel's sums of squares
    E = A.energies(c, G, J)
    assert np.allclose(E, [np.sum(c[3][s["offset"]:s["offset"] + s["N"]].astype(np.float64) ** 2) for s in stats])
