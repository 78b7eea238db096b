"""Pins of the oracle's two-neutrino reconstruction (section 4 of the paper:
W and top mass constraints per lepton / b-jet pairing, most probable solution
kept, events without a solution discarded).

  closure     generated (FP64 truth) neutrinos are among the solutions of the
              true pairing;
  invariants  every accepted solution satisfies the constraints;
  brute force a 50-digit solution by a different computational route;
  symmetries  rotation about the beam, boost along it, exchange of the two
              top legs;
  score       the p_T term of the score equals the generated top p_T.
"""

import numpy as np
import pytest

import hfgen

from . import brute_mp

M_T, M_W = 172.5, 80.4


@pytest.fixture(scope="module")
def truth_sample():
    return hfgen.generate("ttbar10k", n_events=4000, keep_fp64=True, seed=4242)


def _mass(p):
    m2 = p[0] ** 2 - p[1] ** 2 - p[2] ** 2 - p[3] ** 2
    return np.sqrt(max(m2, 0.0))


def _nu(s):
    return np.array([s[3], s[0], s[1], s[2]]), np.array([s[7], s[4], s[5], s[6]])


def test_closure_on_generated_truth(orc, truth_sample):
    tr = truth_sample["truth"]
    errs = []
    n_degenerate = 0
    for e in range(truth_sample["n"]):
        lp, lm, b, bb, nu, nub = (tr[k][e] for k in ("lp", "lm", "b", "bbar", "nu", "nubar"))
        sol = orc.solve_pairing(lp, b, lm, bb, nu[1] + nub[1], nu[2] + nub[2])
        # reading: a side whose linear maps are degenerate (|det| <= 1e-5 El Eb)
        # gives the pairing no solution
        degenerate = any(abs(l[3] * q[0] - l[0] * q[3]) <= 1e-5 * l[0] * q[0] for l, q in ((lp, b), (lm, bb)))
        if degenerate:
            assert len(sol) == 0
            n_degenerate += 1
            continue
        assert 1 <= len(sol) <= 4
        d1 = np.abs(sol[:, 0:3] - nu[1:4]).max(axis=1) / np.linalg.norm(nu[1:4])
        d2 = np.abs(sol[:, 4:7] - nub[1:4]).max(axis=1) / np.linalg.norm(nub[1:4])
        errs.append(np.maximum(d1, d2).min())
    errs = np.array(errs)
    # every event recovers its neutrinos; the tail is near-tangent conics whose
    # intersection is ill-conditioned in the inputs themselves
    assert errs.max() < 1e-4
    assert np.quantile(errs, 0.99) < 1e-9
    assert np.median(errs) < 1e-12
    assert n_degenerate <= 2


def test_closure_float32_inputs(orc):
    """With the stored float32 columns the true solution moves by the input
    rounding; at least 99 % of events stay within 1e-3."""
    ev = hfgen.generate("ttbar10k", n_events=3000, seed=99)
    tr = ev["truth"]
    errs = []
    for e in range(ev["n"]):
        lo, jo = int(ev["lep_off"][e]), int(ev["jet_off"][e])

        def p4(pre, k):
            pt, eta, phi, en = (float(ev[pre + c][k]) for c in ("pt", "eta", "phi", "e"))
            return np.array([en, pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)])

        lp = p4("lep_", lo + tr["lp_idx"][e])
        lm = p4("lep_", lo + tr["lm_idx"][e])
        b = p4("jet_", jo + tr["b_idx"][e])
        bb = p4("jet_", jo + tr["bbar_idx"][e])
        sol = orc.solve_pairing(lp, b, lm, bb, float(ev["met_x"][e]), float(ev["met_y"][e]))
        nu, nub = tr["nu"][e], tr["nubar"][e]
        if len(sol) == 0:
            errs.append(np.inf)
            continue
        d1 = np.abs(sol[:, 0:3] - nu[1:4]).max(axis=1) / np.linalg.norm(nu[1:4])
        d2 = np.abs(sol[:, 4:7] - nub[1:4]).max(axis=1) / np.linalg.norm(nub[1:4])
        errs.append(np.maximum(d1, d2).min())
    errs = np.array(errs)
    assert np.mean(errs < 1e-3) >= 0.99


def _smeared_cases(tr, n, seed):
    rng = np.random.default_rng(seed)
    for e in range(n):
        s = 1 + 0.1 * rng.standard_normal(4)
        lp, lm, b, bb = tr["lp"][e] * s[0], tr["lm"][e] * s[1], tr["b"][e] * s[2], tr["bbar"][e] * s[3]
        mx = tr["nu"][e][1] + tr["nubar"][e][1] + 10 * rng.standard_normal()
        my = tr["nu"][e][2] + tr["nubar"][e][2] + 10 * rng.standard_normal()
        yield lp, b, lm, bb, mx, my


def test_invariants_of_accepted_solutions(orc, truth_sample):
    tr = truth_sample["truth"]
    n_roots = 0
    for lp, b, lm, bb, mx, my in _smeared_cases(tr, 2500, 5):
        sol = orc.solve_pairing(lp, b, lm, bb, mx, my)
        assert len(sol) <= 4
        assert np.all(np.diff(sol[:, 0]) > 0)  # ascending in x
        for s in sol:
            nu, nub = _nu(s)
            n_roots += 1
            assert abs(_mass(lp + nu) - M_W) <= 1e-6
            assert abs(_mass(b + lp + nu) - M_T) <= 1e-6
            assert abs(_mass(lm + nub) - M_W) <= 1e-6
            assert abs(_mass(bb + lm + nub) - M_T) <= 1e-6
            assert abs(s[0] + s[4] - mx) <= 1e-9 and abs(s[1] + s[5] - my) <= 1e-9
            assert s[3] >= 0 and s[7] >= 0
            assert abs(s[3] - np.linalg.norm(s[0:3])) <= 1e-8 * s[3]
            assert abs(s[7] - np.linalg.norm(s[4:7])) <= 1e-8 * s[7]
    assert n_roots > 2500


def test_brute_force_50_digits(orc, truth_sample):
    tr = truth_sample["truth"]
    checked = 0
    for k, (lp, b, lm, bb, mx, my) in enumerate(_smeared_cases(tr, 120, 11)):
        # also wrong pairings (swapped b jets), which are often solution-free
        if k % 3 == 2:
            b, bb = bb, b
        want, sep = brute_mp.solve(lp, b, lm, bb, mx, my)
        got = orc.solve_pairing(lp, b, lm, bb, mx, my)
        if float(sep) < 1e-6:
            continue  # numerically a double root; counts may legitimately differ
        assert len(got) == len(want), (k, got, want)
        for g, w in zip(got, want):
            wv = np.array([float(v) for v in w])
            scale = np.linalg.norm(wv[0:3]) + np.linalg.norm(wv[4:7])
            tol = 1e-10 * max(1.0, 1e-3 / float(sep) * 100.0)
            assert np.abs(g - wv).max() <= tol * scale, (k, g, wv)
        checked += 1
    assert checked > 100


def _align(lep, b, d):
    """b made massless with its direction cosine along the beam equal to the
    (massless) lepton's shifted by d, azimuth and momentum kept: then
    |lz Eb - El bz| = d El Eb, the determinant of the linear maps."""
    pl = np.linalg.norm(lep[1:])
    ct = lep[3] / pl
    ctb = ct - d * np.sign(ct)
    stb = np.sqrt(1.0 - ctb * ctb)
    pb, phb = np.linalg.norm(b[1:]), np.arctan2(b[2], b[1])
    return np.array([pb, pb * stb * np.cos(phb), pb * stb * np.sin(phb), pb * ctb])


def test_near_degenerate_pairings(orc, truth_sample):
    """A lepton and b jet of nearly equal rapidity make the two linear mass
    conditions nearly dependent.  Readings pinned: below |det| = 1e-5 El Eb
    the pairing has no solution; above it every accepted solution satisfies
    the mass constraints to the acceptance bound (2e-6 mW^2 on m_nu^2, i.e.
    1e-6 relative on the masses, plus rounding) and matches the 50-digit
    brute force."""
    tr = truth_sample["truth"]
    n_sol = n_brute = 0
    for e in range(24):
        lp, lm, b, bb, nu, nub = (tr[k][e] for k in ("lp", "lm", "b", "bbar", "nu", "nubar"))
        lp0 = np.array([np.linalg.norm(lp[1:]), *lp[1:]])
        mx, my = nu[1] + nub[1], nu[2] + nub[2]
        assert len(orc.solve_pairing(lp0, _align(lp0, b, 3e-6), lm, bb, mx, my)) == 0
        assert len(orc.solve_pairing(lp0, _align(lp0, b, 0.0), lm, bb, mx, my)) == 0
        for d in (1e-3, 1e-4, 2e-5):
            b2 = _align(lp0, b, d)
            got = orc.solve_pairing(lp0, b2, lm, bb, mx, my)
            for sol in got:
                nv, nbv = _nu(sol)
                for m, want in ((_mass(lp0 + nv), M_W), (_mass(b2 + lp0 + nv), M_T),
                                (_mass(lm + nbv), M_W), (_mass(bb + lm + nbv), M_T)):
                    assert abs(m - want) <= 2e-6 * want, (e, d, m)
            n_sol += len(got)
            if d != 1e-3:
                want, sep = brute_mp.solve(lp0, b2, lm, bb, mx, my)
                if float(sep) < 1e-6:
                    continue
                assert len(got) == len(want), (e, d)
                for g, w in zip(got, want):
                    wv = np.array([float(v) for v in w])
                    scale = np.linalg.norm(wv[0:3]) + np.linalg.norm(wv[4:7])
                    assert np.abs(g - wv).max() <= 1e-6 * scale, (e, d, g, wv)
                n_brute += len(want)
    assert n_sol > 20 and n_brute > 8


def _rot(v, th):
    c, s = np.cos(th), np.sin(th)
    return np.array([v[0], c * v[1] - s * v[2], s * v[1] + c * v[2], v[3]])


def _boost_z(v, beta):
    g = 1.0 / np.sqrt(1 - beta * beta)
    return np.array([g * (v[0] + beta * v[3]), v[1], v[2], g * (v[3] + beta * v[0])])


def _match(a, b, tol):
    assert len(a) == len(b)
    used = set()
    for x in a:
        d = [np.abs(x - y).max() if i not in used else np.inf for i, y in enumerate(b)]
        i = int(np.argmin(d))
        assert d[i] <= tol, (x, b[i])
        used.add(i)


def test_symmetries(orc, truth_sample):
    tr = truth_sample["truth"]
    for k, (lp, b, lm, bb, mx, my) in enumerate(_smeared_cases(tr, 200, 21)):
        base = orc.solve_pairing(lp, b, lm, bb, mx, my)
        if len(base) == 0:
            continue
        if len(base) > 1 and np.min(np.diff(base[:, 0])) < 1e-2:
            continue  # near-tangent: the symmetry holds only to conditioning
        sc = 1e-7 * (1 + np.abs(base).max())
        # rotation about the beam axis
        th = 0.1 + k * 0.37
        rot = orc.solve_pairing(_rot(lp, th), _rot(b, th), _rot(lm, th), _rot(bb, th),
                                np.cos(th) * mx - np.sin(th) * my, np.sin(th) * mx + np.cos(th) * my)
        want = []
        for s in base:
            nu, nub = _nu(s)
            r1, r2 = _rot(nu, th), _rot(nub, th)
            want.append(np.array([r1[1], r1[2], r1[3], r1[0], r2[1], r2[2], r2[3], r2[0]]))
        _match(rot, want, sc)
        # boost along the beam axis (MET is transverse and unchanged)
        beta = -0.6 + 0.006 * k
        bo = orc.solve_pairing(_boost_z(lp, beta), _boost_z(b, beta), _boost_z(lm, beta), _boost_z(bb, beta), mx, my)
        want = []
        for s in base:
            nu, nub = _nu(s)
            r1, r2 = _boost_z(nu, beta), _boost_z(nub, beta)
            want.append(np.array([r1[1], r1[2], r1[3], r1[0], r2[1], r2[2], r2[3], r2[0]]))
        _match(bo, want, sc * 10)
        # exchanging the two legs exchanges neutrino and antineutrino
        sw = orc.solve_pairing(lm, bb, lp, b, mx, my)
        _match(sw, [np.concatenate([s[4:8], s[0:4]]) for s in base], sc)


def test_reco_score_pt_term_matches_generated_tops(orc, truth_sample):
    """Unsmeared, one variation: log w = -(pT(t) + pT(tbar)) / 100 GeV.  When the
    chosen solution is the generated one, pT(t) must be the generated top pT."""
    ev = truth_sample
    cfg = hfgen.config("ttbar10k")
    reco = dict(cfg["reco"])
    idx = np.arange(ev["n"], dtype=np.int32)
    out = orc.ttbar_reco(ev, idx, reco, fp64=True)
    tr = ev["truth"]
    hit = 0
    for s in range(ev["n"]):
        if not out["has_sol"][s]:
            continue
        if out["best_i"][s] != tr["b_idx"][s] or out["best_j"][s] != tr["bbar_idx"][s]:
            continue
        if np.abs(out["nu"][s] - tr["nu"][s][1:4]).max() > 1e-6 * np.linalg.norm(tr["nu"][s][1:4]):
            continue
        want = -(tr["top_pt"][s] + tr["tbar_pt"][s]) / 100.0
        assert out["logw"][s] == pytest.approx(want, rel=1e-9)
        assert out["m_t"][s] == pytest.approx(M_T, abs=1e-6)
        assert out["m_wm"][s] == pytest.approx(M_W, abs=1e-6)
        hit += 1
    assert hit > 500


def test_reco_no_solution_sentinel(orc):
    ev = hfgen.generate("ttbar10k", n_events=300, seed=7)
    cfg = hfgen.config("ttbar10k")
    out = orc.ttbar_reco(ev, np.arange(300, dtype=np.int32), cfg["reco"])
    none = out["has_sol"] == 0
    assert none.any() and (~none).any()
    for k in ("m_t", "m_tbar", "m_wp", "m_wm", "logw", "m_bb"):
        assert np.all(out[k][none] == -9999.0)
    assert np.all(out["nu"][none] == -9999.0) and np.all(out["nubar"][none] == -9999.0)
    assert np.all(out["best_v"][none] == -1)
    assert np.all(out["n_sol"][none] == 0)


def test_mbb_closure_on_tth_truth(orc):
    """m_bb of the two remaining b jets is the Higgs mass when the chosen top
    jets are the true ones (FP64 truth inputs)."""
    ev = hfgen.generate("tth4M_v256", n_events=4000, keep_fp64=True, seed=31)
    reco = dict(hfgen.config("tth4M_v256")["reco"])
    reco.update(smear=0, n_var=1, want_mbb=1)
    out = orc.ttbar_reco(ev, np.arange(ev["n"], dtype=np.int32), reco, fp64=True)
    tr = ev["truth"]
    hits = 0
    for s in range(ev["n"]):
        if not out["has_sol"][s]:
            continue
        if out["best_i"][s] != tr["b_idx"][s] or out["best_j"][s] != tr["bbar_idx"][s]:
            continue
        lo, hi = int(ev["jet_off"][s]), int(ev["jet_off"][s + 1])
        # remaining selected tagged jets must be exactly the two Higgs b jets
        rest = [k for k in range(hi - lo) if k not in (tr["b_idx"][s], tr["bbar_idx"][s])
                and ev["fp64"]["jet_pt"][lo + k] > 25 and abs(ev["fp64"]["jet_eta"][lo + k]) < 2.5
                and ev["jet_btag"][lo + k] > 0.5]
        if sorted(rest) != sorted([tr["hb1_idx"][s], tr["hb2_idx"][s]]):
            continue
        assert out["m_bb"][s] == pytest.approx(125.0, abs=1e-9)
        hits += 1
    assert hits > 100
