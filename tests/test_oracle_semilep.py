"""Pins of the oracle's single-neutrino chi^2 reconstruction (section 6.2,
Eq. (chi2): E_T^miss is the neutrino's transverse momentum, p_z follows from
the W mass, and the jet assignment with the smallest chi^2 is kept).

  roots       the p_z candidates satisfy m(l + nu) = m_W, and every root of
              the unsquared mass condition, found by bracketing, is among
              them;
  real part   with no real root, the candidate is the real part of the
              complex pair of the squared condition, built here from samples
              of the mass function and solved with numpy.roots;
  brute force a plain itertools / numpy minimisation of chi^2 over every
              jet assignment and root, per topology;
  closure     on generated signal, the true jets and the true neutrino p_z
              give chi^2 ~ 0 and are the ones chosen.
"""

import itertools

import numpy as np
import pytest

import hfgen

M_T, M_W, S_T, S_W = 172.5, 80.4, 11.5, 7.5


def _m2(p):
    return p[0] ** 2 - p[1] ** 2 - p[2] ** 2 - p[3] ** 2


def _mass(p):
    return np.sqrt(max(_m2(p), 0.0))


def _nu(mx, my, pz):
    return np.array([np.sqrt(mx * mx + my * my + pz * pz), mx, my, pz])


def _random_lep_met(rng):
    pt = rng.exponential(50.0) + 20.0
    eta = rng.uniform(-2.5, 2.5)
    phi = rng.uniform(-np.pi, np.pi)
    m = rng.choice([0.0, 0.000511, 0.1057])
    p = np.array([pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)])
    lep = np.array([np.sqrt(m * m + p @ p), *p])
    met = rng.normal(0.0, 60.0, 2)
    return lep, met


def _f(lep, mx, my, pz):
    """m^2(l + nu) - m_W^2 straight from the 4-vectors (no squaring)."""
    return _m2(lep + _nu(mx, my, pz)) - M_W * M_W


def _bracket_roots(lep, mx, my):
    """Roots of the unsquared condition: sign changes on a fine grid, then
    bisection to full precision."""
    grid = np.sinh(np.linspace(-9.0, 9.0, 20001)) * 10.0  # dense near 0, out to +-40 TeV
    fv = np.array([_f(lep, mx, my, z) for z in grid])
    roots = []
    for k in np.nonzero(np.sign(fv[:-1]) * np.sign(fv[1:]) < 0)[0]:
        lo, hi = grid[k], grid[k + 1]
        flo = fv[k]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = _f(lep, mx, my, mid)
            if (fm < 0) == (flo < 0):
                lo, flo = mid, fm
            else:
                hi = mid
            if hi - lo <= 1e-13 * max(1.0, abs(mid)):
                break
        roots.append(0.5 * (lo + hi))
    return roots


def test_nu_pz_roots_are_the_w_mass_roots(orc):
    rng = np.random.default_rng(11)
    n_two = n_found = 0
    for _ in range(300):
        lep, (mx, my) = _random_lep_met(rng)
        pz, kind = orc.nu_pz(lep, mx, my, M_W)
        br = _bracket_roots(lep, mx, my)
        if kind[0] == 2:
            assert len(pz) == 1 and len(br) == 0
            continue
        n_two += 1
        assert len(pz) == 2 and list(kind) == [0, 1] and pz[0] <= pz[1]
        for z in pz:
            nu = _nu(mx, my, z)
            # a root of the squared condition that is not one of the unsquared
            # one needs E_l E_nu = -(mu + pz_l pz) < 0: impossible unless mu < 0
            assert abs(_mass(lep + nu) - M_W) < 1e-9 * M_W or lep[0] * nu[0] - lep[1:] @ nu[1:] < 0
        for z in br:
            assert np.min(np.abs(pz - z)) <= 1e-7 * max(1.0, abs(z))
            n_found += 1
    assert n_two > 150 and n_found >= 2 * n_two - 2


def test_nu_pz_real_part_when_no_root(orc):
    rng = np.random.default_rng(12)
    n_cplx = 0
    for _ in range(400):
        lep, (mx, my) = _random_lep_met(rng)
        pz, kind = orc.nu_pz(lep, mx, my, M_W)
        if kind[0] != 2:
            continue
        n_cplx += 1
        # g(pz) = (E_l E_nu)^2 - (E_l E_nu - f/2)^2, an exact quadratic in pz;
        # recover its coefficients from three samples
        xs = np.array([-100.0, 0.0, 100.0])
        g = []
        for z in xs:
            a = lep[0] * _nu(mx, my, z)[0]
            b = a - 0.5 * _f(lep, mx, my, z)
            g.append(a * a - b * b)
        r = np.roots(np.polyfit(xs, g, 2))
        assert np.all(np.abs(r.imag) > 0)
        assert abs(pz[0] - r.real[0]) <= 1e-6 * max(1.0, abs(r.real[0]))
        # no real root: the W mass exceeds m_W for every pz
        assert _f(lep, mx, my, pz[0]) > 0
    assert n_cplx > 20


def _brute(ev, e, sl, topology):
    """min chi^2 over assignments by itertools, p_z by bracketing (or the
    real part from numpy.roots of the sampled squared condition)."""
    l0, l1 = int(ev["lep_off"][e]), int(ev["lep_off"][e + 1])
    j0, j1 = int(ev["jet_off"][e]), int(ev["jet_off"][e + 1])
    f64 = lambda k, i: float(ev[k][i])
    lep = None
    for k in range(l0, l1):
        if f64("lep_pt", k) > np.float32(sl["lep_pt_min"]) and abs(f64("lep_eta", k)) < np.float32(sl["lep_eta_max"]):
            pt, eta, phi = f64("lep_pt", k), f64("lep_eta", k), f64("lep_phi", k)
            lep = np.array([f64("lep_e", k), pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)])
            break
    jets, loc = [], []
    for k in range(j0, j1):
        if len(jets) == sl["max_cands"]:
            break
        if f64("jet_pt", k) > np.float32(sl["jet_pt_min"]) and abs(f64("jet_eta", k)) < np.float32(sl["jet_eta_max"]):
            pt, eta, phi = f64("jet_pt", k), f64("jet_eta", k), f64("jet_phi", k)
            jets.append(np.array([f64("jet_e", k), pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)]))
            loc.append(k - j0)
    need = {"TCHAN": 1, "WT": 3, "TTSEMI": 4}[topology]
    if lep is None or len(jets) < need:
        return None
    mx, my = float(ev["met_x"][e]), float(ev["met_y"][e])
    pzs = _bracket_roots(lep, mx, my)
    if not pzs:
        xs = np.array([-100.0, 0.0, 100.0])
        g = []
        for z in xs:
            a = lep[0] * _nu(mx, my, z)[0]
            b = a - 0.5 * _f(lep, mx, my, z)
            g.append(a * a - b * b)
        pzs = [float(np.roots(np.polyfit(xs, g, 2)).real[0])]
    best = None
    nj = len(jets)
    for pz in pzs:
        w = lep + _nu(mx, my, pz)
        for j in range(nj):
            if topology == "TCHAN":
                assigns = [(j, -1, -1, -1)]
            else:
                rest = [x for x in range(nj) if x != j]
                hs = rest if topology == "TTSEMI" else [-1]
                assigns = [(j, h, p, q) for h in hs for p, q in itertools.combinations([x for x in rest if x != h], 2)]
            for (j_, h, p, q) in assigns:
                chi2 = (_mass(w + jets[j_]) - M_T) ** 2 / S_T ** 2 + (_mass(w) - M_W) ** 2 / S_W ** 2
                if p >= 0:
                    chi2 += (_mass(jets[p] + jets[q]) - M_W) ** 2 / S_W ** 2
                if h >= 0:
                    chi2 += (_mass(jets[h] + jets[p] + jets[q]) - M_T) ** 2 / S_T ** 2
                key = (loc[j_], loc[h] if h >= 0 else -1, loc[p] if p >= 0 else -1, loc[q] if q >= 0 else -1)
                if best is None or chi2 < best[0]:
                    best = (chi2, key, pz)
    return best


@pytest.mark.parametrize("topology,kind", [("TCHAN", "tchan"), ("WT", "wt"), ("TTSEMI", "ttsemi")])
def test_brute_force_choice(orc, topology, kind):
    cfg = hfgen.configs.config("tchan1M")
    cfg["kind"] = kind
    cfg["n_extra_max"] = 3
    ev = hfgen.generate(cfg, n_events=200, seed=77)
    sl = cfg["semilep"]
    idx = np.arange(ev["n"], dtype=np.int32)
    r = orc.semilep_reco(ev, idx, sl, topology)
    n_cmp = 0
    for e in range(ev["n"]):
        b = _brute(ev, e, sl, topology)
        if b is None:
            assert r["has_sol"][e] == 0 and r["best_j"][e] == -1 and r["chi2"][e] == -9999.0
            continue
        assert r["has_sol"][e] == 1
        chi2, key, pz = b
        assert abs(r["chi2"][e] - chi2) <= 1e-7 * max(1.0, chi2)
        got = (r["best_j"][e], r["best_h"][e], r["best_p"][e], r["best_q"][e])
        assert tuple(int(x) for x in got) == key
        assert abs(r["nu"][e, 2] - pz) <= 1e-6 * max(1.0, abs(pz))
        n_cmp += 1
    assert n_cmp > 40


@pytest.mark.parametrize("topology,kind", [("TCHAN", "tchan"), ("WT", "wt"), ("TTSEMI", "ttsemi")])
def test_closure_on_generated_truth(orc, topology, kind):
    cfg = hfgen.configs.config("tchan1M")
    cfg["kind"] = kind
    cfg["bkg_frac"] = 0.0
    ev = hfgen.generate(cfg, n_events=3000, seed=78)
    sl = cfg["semilep"]
    tr = ev["truth"]
    names = {"TCHAN": ["b_idx"], "WT": ["b_idx", "q1_idx", "q2_idx"],
             "TTSEMI": ["b_idx", "bh_idx", "q1_idx", "q2_idx"]}[topology]
    # events whose lepton and truth jets are all selected and within the cap
    jsel = (ev["jet_pt"] > np.float32(25.0)) & (np.abs(ev["jet_eta"]) < np.float32(2.5))
    off = ev["jet_off"].astype(np.int64)
    keep = []
    for e in range(ev["n"]):
        lk = off[e] + tr["lep_idx"][e]
        l_ok = tr["lep_idx"][e] == 0 and ev["lep_pt"][ev["lep_off"][e]] > 20 and \
            abs(ev["lep_eta"][ev["lep_off"][e]]) < 2.5
        sel = np.nonzero(jsel[off[e]:off[e + 1]])[0]
        if l_ok and all(tr[k][e] in sel[:12] for k in names) and lk >= 0:
            keep.append(e)
    keep = np.array(keep, dtype=np.int32)
    assert keep.size > 400
    r = orc.semilep_reco(ev, keep, sl, topology)
    assert r["has_sol"].all()
    # float32 inputs put the true assignment at chi^2 ~ 1e-8 or below
    assert np.quantile(r["chi2"], 0.99) < 1e-6
    got_b = r["best_j"] == tr["b_idx"][keep]
    agree = got_b.copy()
    if topology != "TCHAN":
        q = np.sort(np.stack([tr["q1_idx"][keep], tr["q2_idx"][keep]], 1), 1)
        agree &= (r["best_p"] == q[:, 0]) & (r["best_q"] == q[:, 1])
    if topology == "TTSEMI":
        agree &= r["best_h"] == tr["bh_idx"][keep]
    assert agree.mean() >= 0.99
    nu_pz = tr["nu"][keep, 3]
    rel = np.abs(r["nu"][:, 2] - nu_pz) / np.maximum(1.0, np.abs(nu_pz))
    assert np.quantile(rel[agree], 0.99) < 1e-3
    # the leptonic W is on shell (real roots), the top masses at m_t
    assert np.all(np.abs(r["m_wl"][r["root"] != 2] - M_W) < 1e-6 * M_W)
    assert np.median(np.abs(r["m_tl"] - M_T)) < 1e-3


def test_degenerate_inputs(orc):
    sl = hfgen.configs.config("tchan1M")["semilep"]
    z = np.zeros
    # event 0: no lepton; event 1: lepton but no selected jet; event 2: one jet
    ev = {"n": 3, "lep_off": np.array([0, 0, 1, 2], np.uint32), "jet_off": np.array([0, 1, 2, 3], np.uint32),
          "lep_pt": np.array([40, 40], np.float32), "lep_eta": z(2, np.float32), "lep_phi": z(2, np.float32),
          "lep_e": np.array([40, 40], np.float32), "lep_q": np.ones(2, np.float32),
          "jet_pt": np.array([50, 10, 60], np.float32), "jet_eta": z(3, np.float32),
          "jet_phi": np.array([1, 1, 2], np.float32), "jet_e": np.array([50, 10, 60], np.float32),
          "jet_btag": z(3, np.float32), "met_x": np.array([30, 30, 30], np.float32),
          "met_y": z(3, np.float32), "n_var": None}
    idx = np.arange(3, dtype=np.int32)
    r = orc.semilep_reco(ev, idx, sl, "TCHAN")
    assert list(r["has_sol"]) == [0, 0, 1]
    assert r["best_j"][2] == 0 and r["best_h"][2] == -1 and r["m_th"][2] == -9999.0
    for topo in ("WT", "TTSEMI"):
        assert not orc.semilep_reco(ev, idx, sl, topo)["has_sol"].any()
    assert orc.semilep_reco(ev, idx[:0], sl, "TCHAN")["n_pass"] == 0
