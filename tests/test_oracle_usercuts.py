"""Pins of the oracle's user predicates (section 3: a cut is the user's own
boolean function of one event).  User bodies that restate built-in cuts must
give the built-in cuts' masks (the built-in cuts are pinned by the
hand-derived golden cases); the forward-jet predicate is the complement of
the built-in forward-jet veto; out-of-range accessors read 0; counters follow
the order with user cuts mixed in."""

import numpy as np
import pytest

import hfgen
from hfgen.configs import USER_CUTS, _cut, _user

from . import cutcases


def _sample():
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 7, n=20000)
    return ev


@pytest.mark.parametrize("user,builtin", [
    ("U_MET30", _cut("MET30", "MET_MIN", [30.0])),
    ("U_JETS2", _cut("JETS2", "JET_N_MIN", [25.0, 2.5], [2])),
    ("U_LEP2OS", _cut("LEP2OS", "LEP_N_OS", [20.0, 2.5], [2, 1])),
])
def test_user_restatements_equal_builtins(orc, user, builtin):
    for ev in (cutcases.load()[0], _sample()):
        su, _, _ = orc.select(ev, [_user(user, USER_CUTS[user])], [0])
        sb, _, _ = orc.select(ev, [builtin], [0])
        assert np.array_equal(su, sb), user
        assert 0 < sb.sum() < ev["n"]


def test_forward_jet_is_the_veto_complement(orc):
    ev = _sample()
    su, _, _ = orc.select(ev, [_user("U_FWDJET", USER_CUTS["U_FWDJET"])], [0])
    sv, _, _ = orc.select(ev, [_cut("FWDVETO", "FWD_JET_VETO", [25.0, 2.5, 4.5])], [0])
    assert np.array_equal(su, 1 - sv) and 0 < su.sum() < ev["n"]


def test_ht_by_hand(orc):
    ev = _sample()
    su, _, _ = orc.select(ev, [_user("U_HT150", USER_CUTS["U_HT150"])], [0])
    off = ev["jet_off"].astype(np.int64)
    want = np.zeros(ev["n"], dtype=np.uint8)
    for e in range(ev["n"]):
        ht = np.float32(0.0)
        for k in range(off[e], off[e + 1]):
            if ev["jet_pt"][k] > np.float32(25.0) and abs(ev["jet_eta"][k]) < np.float32(2.5):
                ht = np.float32(ht + ev["jet_pt"][k])
        want[e] = ht > np.float32(150.0)
    assert np.array_equal(su, want)


def test_out_of_range_accessors_read_zero(orc):
    ev = _sample()
    su, _, _ = orc.select(ev, [_user("U_LEAD40", USER_CUTS["U_LEAD40"])], [0])
    off = ev["lep_off"].astype(np.int64)
    lead = np.array([ev["lep_pt"][off[e]] if off[e + 1] > off[e] else 0.0 for e in range(ev["n"])])
    assert np.array_equal(su, (lead > np.float32(40.0)).astype(np.uint8))


def test_mixed_chain_counters_follow_order(orc):
    ev = _sample()
    cuts = hfgen.configs.chain_user_mix()
    singles = [orc.select(ev, [dict(c, deps=[])], [0])[0].astype(bool) for c in cuts]
    rng = np.random.default_rng(5)
    for _ in range(4):
        order = rng.permutation(len(cuts))
        surv, reached, passed = orc.select(ev, cuts, order)
        alive = np.ones(ev["n"], dtype=bool)
        for c in order:
            assert reached[c] == alive.sum()
            alive &= singles[c]
            assert passed[c] == alive.sum()
        assert np.array_equal(surv.astype(bool), alive)


# Loop budgets (a predicate is a function of one event, so it must end):
# each (body, units it spends on every event).  A for loop spends a unit as
# an iteration starts, a while or do-while loop when its condition lets
# another iteration run; nested loops add up.
LOOPS = [
    ("for", "int s = 0; for (int k = 0; k < 1000; ++k) s += k & 1; return s > 0;", 1000),
    ("while", "int k = 0; while (k < 10) ++k; return 1;", 10),
    ("do", "int k = 0; do { ++k; } while (k < 10); return 1;", 9),
    ("nested", "int s = 0; for (int a = 0; a < 30; ++a) for (int b = 0; b < 20; ++b) s += 1; return s == 600;",
     630),
    ("continue", "int s = 0; for (int k = 0; k < 50; ++k) { if (k & 1) continue; s += 1; } return s == 25;", 50),
]


@pytest.mark.parametrize("name,src,units", LOOPS)
def test_loop_budget_boundary(orc, name, src, units):
    ev = _sample()
    n = ev["n"]
    for budget, want in ((units, n), (units - 1, 0), (units + 7, n), (0, n)):
        s, r, p = orc.select(ev, [_user("U", src, budget=budget)], [0])
        assert int(s.sum()) == want and r[0] == n and p[0] == want, (name, budget)


def test_loop_budget_per_event(orc):
    """A loop over the event's jets with a budget of 3 units passes exactly
    the events with at most three jets (counted here from the offsets)."""
    ev = _sample()
    src = "int n = 0; for (int k = 0; k < n_jet(); ++k) n += jet_pt(k) > 25.0f; return n >= 0;"
    s, _, _ = orc.select(ev, [_user("U", src, budget=3)], [0])
    njet = np.diff(np.asarray(ev["jet_off"]))
    assert np.array_equal(s.astype(bool), njet <= 3)
    assert 0 < s.sum() < ev["n"]
