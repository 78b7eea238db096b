"""Pins of the oracle's cut chain, compaction and adaptive ordering.

Cut predicates: hand-derived outcomes of golden/cut_cases.json.  Counters:
reached/passed per position of the current order (sections 3 and 5.2).
Compaction: the ascending list of survivors (numpy.flatnonzero).  Ordering:
for independent cuts the greedy rank order minimises the expected cost
sum_k c_k prod_{m<k} p_m, checked by brute force over all orders.
"""

import itertools

import numpy as np
import pytest

import hfgen

from . import cutcases


def test_cut_predicates_match_hand_derivation(orc):
    ev, cuts, expect, names = cutcases.load()
    for k, cut in enumerate(cuts):
        surv, reached, passed = orc.select(ev, [cut], [0])
        assert list(surv) == list(expect[:, k]), (cut["name"], [n for n, a, b in zip(names, surv, expect[:, k]) if a != b])
        assert reached[0] == ev["n"] and passed[0] == expect[:, k].sum()


def test_counters_follow_the_order(orc):
    ev, cuts, expect, names = cutcases.load()
    rng = np.random.default_rng(3)
    for _ in range(20):
        order = rng.permutation(len(cuts))
        surv, reached, passed = orc.select(ev, cuts, order)
        # the final mask is the AND of every cut, whatever the order
        assert list(surv) == list(expect.all(axis=1).astype(np.uint8))
        alive = np.ones(ev["n"], dtype=bool)
        for c in order:
            assert reached[c] == alive.sum()
            alive &= expect[:, c].astype(bool)
            assert passed[c] == alive.sum()


def test_counters_accumulate_and_skip_reco(orc):
    cfg = hfgen.config("ttbar10k")
    ev = hfgen.generate(cfg, n_events=500)
    order = hfgen.default_order(cfg["cuts"])
    s1, r1, p1 = orc.select(ev, cfg["cuts"], order)
    reco = [k for k, c in enumerate(cfg["cuts"]) if c["kind"] == "RECO"][0]
    assert r1[reco] == 0 and p1[reco] == 0
    assert r1[order[0]] == 500
    for a, b in zip(order[:-2], order[1:-1]):
        assert r1[b] == p1[a]
    assert p1[order[-2]] == s1.sum()


def test_compaction_is_flatnonzero(orc):
    rng = np.random.default_rng(0)
    for n in (0, 1, 63, 64, 65, 1000, 4097):
        for p in (0.0, 0.3, 1.0):
            m = (rng.uniform(size=n) < p).astype(np.uint8)
            got = orc.compact(m, index_base=1000)
            np.testing.assert_array_equal(got, np.flatnonzero(m) + 1000)
    m = (rng.uniform(size=500) < 0.5).astype(np.uint8)
    mp_ = rng.integers(0, 1 << 30, 500).astype(np.int32)
    np.testing.assert_array_equal(orc.compact(m, mapping=mp_), mp_[np.flatnonzero(m)])


def _expected_cost(order, c, p):
    tot, surv = 0.0, 1.0
    for k in order:
        tot += surv * c[k]
        surv *= p[k]
    return tot


@pytest.mark.parametrize("seed", range(12))
def test_reorder_minimises_expected_cost_independent_cuts(orc, seed):
    rng = np.random.default_rng(seed)
    n = 4 + seed % 5  # 4..8 cuts
    reached = rng.integers(1000, 100000, n).astype(np.uint64)
    passed = (reached * rng.uniform(0.05, 0.99, n)).astype(np.uint64)
    cost = (reached * rng.uniform(1, 500, n)).astype(np.uint64)
    order = orc.reorder(reached, passed, cost, np.zeros(n, dtype=np.uint64))
    p = passed / reached
    c = cost / reached
    best = min(_expected_cost(o, c, p) for o in itertools.permutations(range(n)))
    assert _expected_cost(order, c, p) == pytest.approx(best, rel=1e-12)


def test_reorder_respects_dependencies_and_ties(orc):
    cfg = hfgen.config("tth4M_v256")
    deps = np.array(hfgen.dep_masks(cfg["cuts"]), dtype=np.uint64)
    n = len(cfg["cuts"])
    rng = np.random.default_rng(1)
    for _ in range(50):
        reached = rng.integers(1, 1000, n).astype(np.uint64)
        passed = (reached * rng.uniform(0, 1, n)).astype(np.uint64)
        cost = (reached * rng.uniform(1, 100, n)).astype(np.uint64)
        order = orc.reorder(reached, passed, cost, deps)
        assert sorted(order) == list(range(n))
        placed = 0
        for c in order:
            assert int(deps[c]) & ~placed == 0
            placed |= 1 << int(c)
        assert cfg["cuts"][order[-1]]["kind"] == "RECO"
    # equal ranks keep the lower id first; never-reached cuts rank first
    z = np.zeros(4, dtype=np.uint64)
    same = np.array([10, 10, 10, 10], dtype=np.uint64)
    half = np.array([5, 5, 5, 5], dtype=np.uint64)
    assert list(orc.reorder(same, half, same, z)) == [0, 1, 2, 3]
    r = np.array([10, 0, 10, 10], dtype=np.uint64)
    assert list(orc.reorder(r, half, same, z))[0] == 1
    with pytest.raises(ValueError):
        orc.reorder(same, half, same, np.array([2, 1, 0, 0], dtype=np.uint64))
