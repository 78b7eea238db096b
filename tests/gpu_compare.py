"""Comparison of reconstruction outputs: product (GPU) vs oracle.

Readings of the agreement targets:
  * the RECO pass/fail decision and the chosen (variation, jet pair) must agree
    in >= 99.9 % of events (a floating-point decision, not bit-exact);
  * the choice is the variation, the jet pair and the root of that pairing's
    quartic (two nearly coincident roots score almost alike, so rounding may
    swap them: a swap is a choice difference);
  * where the chosen solution is the same, every reconstructed quantity agrees
    within 1e-4 relative: momenta as |dp| / max(|p_ref|, 1 GeV), masses and the
    score as |d| / max(|ref|, 1).
"""

import numpy as np

FLOAT_KEYS = ("m_t", "m_tbar", "m_wp", "m_wm", "logw")
W_MASS = 80.4


def compare(g, w, n=None):
    """g, w: dicts of arrays over the same compacted positions.  Returns stats."""
    S = len(w["has_sol"]) if n is None else n
    hs_g, hs_w = g["has_sol"][:S].astype(bool), w["has_sol"][:S].astype(bool)
    both = hs_g & hs_w
    # same choice = same variation, same jet pair and the same root of that
    # pairing's quartic (identified by (px, py) of the neutrino within 1e-3)
    same_root = np.all(np.abs(g["nu"][:S, :2] - w["nu"][:S, :2]) <= 1e-3 * np.maximum(np.abs(w["nu"][:S, :2]), 1.0),
                       axis=1)
    same = both & (g["best_v"][:S] == w["best_v"][:S]) & (g["best_i"][:S] == w["best_i"][:S]) & \
        (g["best_j"][:S] == w["best_j"][:S]) & same_root
    st = {"S": int(S), "decision_agree": float(np.mean(hs_g == hs_w)) if S else 1.0,
          "n_both": int(both.sum()), "n_same": int(same.sum()),
          "choice_agree": float(same.sum() / both.sum()) if both.sum() else 1.0,
          "nsol_agree": float(np.mean(g["n_sol"][:S] == w["n_sol"][:S])) if S else 1.0}
    rels = []
    for k in ("nu", "nubar"):
        d = np.linalg.norm(g[k][:S][same] - w[k][:S][same], axis=1)
        r = d / np.maximum(np.linalg.norm(w[k][:S][same], axis=1), 1.0)
        st["max_rel_" + k] = float(r.max()) if r.size else 0.0
        rels.append(r)
    for k in FLOAT_KEYS:
        r = np.abs(g[k][:S][same] - w[k][:S][same]) / np.maximum(np.abs(w[k][:S][same]), 1.0)
        st["max_rel_" + k] = float(r.max()) if r.size else 0.0
        rels.append(r)
    allr = np.max(np.stack(rels), axis=0) if same.sum() else np.zeros(0)
    st["frac_within_1e-4"] = float(np.mean(allr <= 1e-4)) if allr.size else 1.0
    st["max_rel_any"] = float(allr.max()) if allr.size else 0.0
    # sentinel outputs where there is no solution
    nos = ~hs_g
    st["sentinel_ok"] = bool(np.all(g["m_t"][:S][nos] == -9999.0) and np.all(g["nu"][:S][nos] == -9999.0)
                             and np.all(g["best_v"][:S][nos] == -1))
    if "m_bb" in g and "m_bb" in w and g["m_bb"] is not None:
        r = np.abs(g["m_bb"][:S][same] - w["m_bb"][:S][same]) / np.maximum(np.abs(w["m_bb"][:S][same]), 1.0)
        st["max_rel_m_bb"] = float(r.max()) if r.size else 0.0
    return st


def assert_agree(st, min_agree=0.999, tol=1e-4, min_within=1.0):
    assert st["sentinel_ok"], st
    assert st["decision_agree"] >= min_agree, st
    assert st["choice_agree"] >= min_agree, st
    assert st["frac_within_1e-4"] >= min_within, st
    if min_within >= 1.0:
        assert st["max_rel_any"] <= tol, st


SEMILEP_FLOATS = ("m_tl", "m_wl", "m_th", "m_wh", "chi2")


def compare_semilep(g, w):
    """Single-neutrino reconstruction: the decision (a lepton and enough jets)
    is integer logic and must be identical; the choice (root, j, h, p, q) must
    agree in >= 99.9 % of events; where it agrees, the neutrino momentum is
    compared as |dp| / max(|p_ref|, 1 GeV) and masses and chi^2 as
    |d| / max(|ref|, 1)."""
    S = len(w["has_sol"])
    hs_g, hs_w = g["has_sol"][:S].astype(bool), w["has_sol"][:S].astype(bool)
    both = hs_g & hs_w
    same = both.copy()
    for k in ("root", "best_j", "best_h", "best_p", "best_q"):
        same &= g[k][:S] == w[k][:S]
    st = {"S": int(S), "decision_equal": bool(np.array_equal(hs_g, hs_w)), "n_both": int(both.sum()),
          "choice_agree": float(same.sum() / both.sum()) if both.sum() else 1.0}
    d = np.linalg.norm(g["nu"][:S][same] - w["nu"][:S][same], axis=1)
    rels = [d / np.maximum(np.linalg.norm(w["nu"][:S][same], axis=1), 1.0)]
    st["max_rel_nu"] = float(rels[0].max()) if rels[0].size else 0.0
    for k in SEMILEP_FLOATS:
        r = np.abs(g[k][:S][same] - w[k][:S][same]) / np.maximum(np.abs(w[k][:S][same]), 1.0)
        st["max_rel_" + k] = float(r.max()) if r.size else 0.0
        rels.append(r)
    st["max_rel_any"] = float(np.max([r.max() for r in rels if r.size])) if same.any() else 0.0
    nos = ~hs_g
    st["sentinel_ok"] = bool(np.all(g["chi2"][:S][nos] == -9999.0) and np.all(g["nu"][:S][nos] == -9999.0)
                             and np.all(g["best_j"][:S][nos] == -1) and np.all(g["root"][:S][nos] == -1))
    return st


def assert_agree_semilep(st, min_agree=0.999, tol=1e-4):
    assert st["sentinel_ok"], st
    assert st["decision_equal"], st
    assert st["choice_agree"] >= min_agree, st
    assert st["max_rel_any"] <= tol, st


CHI2_FLOATS = ("m_t", "m_tbar", "m_wp", "m_wm", "chi2")


def compare_chi2(g, w):
    """Dileptonic chi^2 fit: the decision (two opposite-sign leptons, two
    candidates) is integer logic and must be identical; the choice (split
    point, pairing, roots) must agree in >= 99.9 % of events; where it agrees,
    momenta as |dp| / max(|p_ref|, 1 GeV), masses and chi^2 as
    |d| / max(|ref|, 1)."""
    S = len(w["has_sol"])
    hs_g, hs_w = g["has_sol"][:S].astype(bool), w["has_sol"][:S].astype(bool)
    both = hs_g & hs_w
    core = both.copy()
    for k in ("best_i", "best_j"):
        core &= g[k][:S] == w[k][:S]
    core &= np.all(g["split"][:S] == w["split"][:S], axis=1)
    # With one top, the lepton side without it has only its W term; when both
    # of its p_z roots are real roots of the W mass condition the term is zero
    # for both, an exact tie that only rounding breaks: either root is the
    # same choice, provided both forms put that W on its mass shell.
    def free(side_best, root, mw):
        real = (g[root][:S] != 2) & (w[root][:S] != 2)
        shell = (np.abs(g[mw][:S] - W_MASS) <= 1e-9 * W_MASS) & (np.abs(w[mw][:S] - W_MASS) <= 1e-9 * W_MASS)
        return (g[side_best][:S] < 0) & (w[side_best][:S] < 0) & real & shell
    eq_p = g["root_nu"][:S] == w["root_nu"][:S]
    eq_m = g["root_nubar"][:S] == w["root_nubar"][:S]
    same = core & (eq_p | free("best_i", "root_nu", "m_wp")) & (eq_m | free("best_j", "root_nubar", "m_wm"))
    exact = same & eq_p & eq_m  # the same solution: its momenta are compared too
    st = {"S": int(S), "decision_equal": bool(np.array_equal(hs_g, hs_w)), "n_both": int(both.sum()),
          "choice_agree": float(same.sum() / both.sum()) if both.sum() else 1.0,
          "w_root_ties": int((same & ~exact).sum())}
    rels = []
    for k in ("nu", "nubar"):
        d = np.linalg.norm(g[k][:S][exact] - w[k][:S][exact], axis=1)
        r = d / np.maximum(np.linalg.norm(w[k][:S][exact], axis=1), 1.0)
        st["max_rel_" + k] = float(r.max()) if r.size else 0.0
        rels.append(r)
    for k in CHI2_FLOATS:
        r = np.abs(g[k][:S][same] - w[k][:S][same]) / np.maximum(np.abs(w[k][:S][same]), 1.0)
        st["max_rel_" + k] = float(r.max()) if r.size else 0.0
        rels.append(r)
    st["max_rel_any"] = float(np.max([r.max() for r in rels if r.size])) if same.any() else 0.0
    nos = ~hs_g
    st["sentinel_ok"] = bool(np.all(g["chi2"][:S][nos] == -9999.0) and np.all(g["nu"][:S][nos] == -9999.0)
                             and np.all(g["best_i"][:S][nos] == -1))
    return st


def choice_mismatches(g, w):
    """Positions where the decision or the chosen (variation, jet pair, root) differ."""
    hs_g, hs_w = g["has_sol"].astype(bool), w["has_sol"].astype(bool)
    same_root = np.all(np.abs(g["nu"][:, :2] - w["nu"][:, :2]) <= 1e-3 * np.maximum(np.abs(w["nu"][:, :2]), 1.0),
                       axis=1)
    same = (g["best_v"] == w["best_v"]) & (g["best_i"] == w["best_i"]) & (g["best_j"] == w["best_j"]) & same_root
    return np.flatnonzero((hs_g != hs_w) | (hs_g & hs_w & ~same))


def adjudicate(ev, ids, g, w, reco, positions):
    """Settle disagreements of the FP64 path with the oracle by the 50-digit
    brute force (brute_mp), which solves the pairing's constraints from the
    smeared four-vectors without the expanded eliminant.  At each position the
    product's chosen solution must be a genuine solution of its variation and
    jet pair and score above the oracle's choice (or the oracle found none):
    the oracle then missed a better solution, which its FP64 eliminant does
    for the close root pairs of a nearly degenerate conic.  Returns one record
    per position; raises AssertionError when the product is the one in error."""
    import oracle as orc
    from . import brute_mp
    out = []
    for p in positions:
        e, v, i, j = int(ids[p]), int(g["best_v"][p]), int(g["best_i"][p]), int(g["best_j"][p])
        assert g["has_sol"][p], ("product found no solution where the oracle did", p, e)
        if w["has_sol"][p]:
            assert g["logw"][p] > w["logw"][p], ("oracle's choice scores higher", p, e, g["logw"][p], w["logw"][p])
        st = orc.stage_vary(ev, e, v, reco)
        sols, _ = brute_mp.solve(st["lp"], st["cands"][i], st["lm"], st["cands"][j], st["met"][0], st["met"][1],
                                 mt=reco.get("m_t", 172.5), mw=reco.get("m_w", W_MASS))
        x, y = g["nu"][p, 0], g["nu"][p, 1]
        hit = [s for s in sols if abs(float(s[0]) - x) <= 1e-6 * max(abs(x), 1.0) and
               abs(float(s[1]) - y) <= 1e-6 * max(abs(y), 1.0)]
        assert hit, ("product's solution is not a solution of its pairing", p, e, v, i, j, x, y,
                     [(float(s[0]), float(s[1])) for s in sols])
        out.append((p, e, v, i, j, float(g["logw"][p]), float(w["logw"][p]), len(sols)))
    return out
