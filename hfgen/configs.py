"""Workload definitions: event-sample recipes, cut chains and reconstruction
parameters, as plain data.

Nothing here computes anything of the method; both the product path (through
its binding) and the oracle (through its own wrapper) translate these
descriptions into their own structures.

Cut chains follow the dileptonic selections of the paper (section 4, the
18-cut ttH pipeline ending in the kinematic reconstruction; section 6.1, the
HL-LHC selection: isolated opposite-sign leptons, missing transverse energy
above 30 GeV, jet pseudorapidity regions, M_ll above 40 GeV).  Energies are in
GeV throughout (the paper's example code uses MeV).
"""

import copy

# Cut kinds understood by both implementations.  Parameters:
#   LEP_N_OS      f=[pt_min, abs_eta_max]               i=[n_exact, need_opposite_sign]
#   JET_N_MIN     f=[pt_min, abs_eta_max]               i=[n_min]
#   BTAG_N_MIN    f=[pt_min, abs_eta_max, btag_min]     i=[n_min]
#   BTAG_N_EQ     f=[pt_min, abs_eta_max, btag_min]     i=[n_exact]
#   MET_MIN       f=[met_min]
#   MLL_MIN       f=[lep_pt_min, lep_abs_eta_max, mll_min]
#   FWD_JET_VETO  f=[pt_min, abs_eta_lo, abs_eta_hi]    (fails on any jet in [lo, hi))
#   LEP_ISO       f=[lep_pt_min, lep_abs_eta_max, jet_pt_min, jet_abs_eta_max, dr_min]
#   RECO          marker for the kinematic reconstruction (last cut)
#   MTW_MIN       f=[lep_pt_min, lep_abs_eta_max, mtw_min]  (W transverse mass of the leading lepton)
#   USER          a user predicate: "src" holds the body of a C function of one event
#   JET_N_RANGE   f=[pt_min, abs_eta_lo, abs_eta_hi]    i=[n_min, n_max]  (jets in [lo, hi) counted)
CUT_KINDS = ("LEP_N_OS", "JET_N_MIN", "BTAG_N_MIN", "BTAG_N_EQ", "MET_MIN",
             "MLL_MIN", "FWD_JET_VETO", "LEP_ISO", "RECO", "MTW_MIN", "USER", "JET_N_RANGE")


def _cut(name, kind, f=(), i=(), deps=()):
    return {"name": name, "kind": kind, "f": list(f), "i": list(i), "deps": list(deps)}


def chain_dilepton():
    """Four-cut dileptonic chain plus the reconstruction."""
    return [
        _cut("LEP2OS", "LEP_N_OS", [20.0, 2.5], [2, 1]),
        _cut("JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
        _cut("BTAG1", "BTAG_N_MIN", [25.0, 2.5, 0.5], [1]),
        _cut("MET30", "MET_MIN", [30.0]),
        _cut("RECO", "RECO", deps=["LEP2OS", "JETS2", "BTAG1", "MET30"]),
    ]


def chain_tth8():
    """Eight-cut ttH-like chain (user order as written)."""
    return [
        _cut("LEP2OS", "LEP_N_OS", [20.0, 2.5], [2, 1]),
        _cut("JETS4", "JET_N_MIN", [25.0, 2.5], [4]),
        _cut("BTAG3", "BTAG_N_MIN", [25.0, 2.5, 0.5], [3]),
        _cut("MET30", "MET_MIN", [30.0]),
        _cut("MLL40", "MLL_MIN", [20.0, 2.5, 40.0], deps=["LEP2OS"]),
        _cut("FWDVETO", "FWD_JET_VETO", [25.0, 2.5, 3.5]),
        _cut("LEPISO", "LEP_ISO", [20.0, 2.5, 25.0, 2.5, 0.4], deps=["LEP2OS"]),
        _cut("RECO", "RECO", deps=["LEP2OS", "JETS4", "BTAG3", "MET30",
                                   "MLL40", "FWDVETO", "LEPISO"]),
    ]


# Single-neutrino reconstruction (section 6.2): chi^2 of the top and W
# masses with the widths the paper uses.
SEMILEP_DEFAULTS = {
    "m_t": 172.5, "m_w": 80.4, "sigma_t": 11.5, "sigma_w": 7.5,
    "lep_pt_min": 20.0, "lep_eta_max": 2.5, "jet_pt_min": 25.0, "jet_eta_max": 2.5, "max_cands": 12,
}

# Dileptonic chi^2 fit with a MET split (section 6.2): the masses and widths
# of Eq. (chi2); the split grid (offsets from the even split within
# +-half_range GeV, n_grid points per axis, n_refine 5x5 refinements at a
# quarter of the previous step) is a reading.
CHI2_DEFAULTS = {
    "m_t": 172.5, "m_w": 80.4, "sigma_t": 11.5, "sigma_w": 7.5,
    "half_range": 200.0, "n_grid": 17, "n_refine": 2, "n_top": 2,
    "lep_pt_min": 20.0, "lep_eta_max": 2.5, "jet_pt_min": 25.0, "jet_eta_max": 2.5, "btag_min": 0.5,
    "pair_mode": "BTAG_FILL", "max_cands": 12,
}

RECO_DEFAULTS = {
    "m_t": 172.5, "m_w": 80.4, "lambda_pt": 100.0,
    "jet_a": 1.0, "jet_c": 0.05, "lep_sigma": 0.02, "met_sigma": 10.0,
    "lep_pt_min": 20.0, "lep_eta_max": 2.5,
    "jet_pt_min": 25.0, "jet_eta_max": 2.5, "btag_min": 0.5,
    "seed": 0, "smear": 0, "n_var": 1,
    "pair_mode": "BTAG_FILL", "max_cands": 12, "want_mbb": 0,
}

# Sample recipes.  kind: "ttbar" (dileptonic ttbar, optional background
# fraction) or "tth" (ttbar + H->bb).  n_extra_max: extra light jets drawn
# uniformly from 0..n_extra_max.  var_mode: "uniform" or "loguniform1024".
CONFIGS = {
    "ttbar10k": {
        "index": 0, "n_events": 10_000, "kind": "ttbar", "n_extra_max": 4,
        "bkg_frac": 0.0, "bkg_jet_max": 6, "chain": "dilepton",
        "reco": {"smear": 0, "n_var": 1},
        "desc": "10k dileptonic ttbar, 2-6 jets, no smearing, V=1",
    },
    "ttbar1M_v64": {
        "index": 1, "n_events": 1_000_000, "kind": "ttbar", "n_extra_max": 8,
        "bkg_frac": 0.2, "bkg_jet_max": 10, "chain": "dilepton",
        "reco": {"smear": 1, "n_var": 64},
        "desc": "1M events, 2-10 jets, 20% background, 64 smeared variations",
    },
    "tth4M_v256": {
        "index": 2, "n_events": 4_000_000, "kind": "tth", "n_extra_max": 6,
        "bkg_frac": 0.0, "bkg_jet_max": 10, "chain": "tth8",
        "reco": {"smear": 1, "n_var": 256, "want_mbb": 1},
        "desc": "4M ttH-like events, 4-10 jets, >=3 b-tags, 256 variations, 8 cuts",
    },
    "tchan1M": {
        "index": 5, "n_events": 1_000_000, "kind": "tchan", "n_extra_max": 4,
        "bkg_frac": 0.3, "bkg_jet_max": 6, "chain": "semilep",
        "reco": {"smear": 0, "n_var": 1},
        "desc": "1M single-top t-channel-like events (one lepton), 2-6 jets, 30% W+jets-like background",
    },
    "hlhc50M": {
        "index": 4, "n_events": 50_000_000, "chunk": 1_000_000, "kind": "hlhc", "n_extra_max": 4,
        "bkg_jet_max": 8, "chain": "hlhc",
        "fractions": {"ttbar": 0.20, "ttsemi": 0.20, "tchan": 0.15, "wt": 0.10, "wtdilep": 0.05, "bkg": 0.30},
        "reco": {"smear": 1, "n_var": 64},
        "desc": "50M mixed events in 1M chunks (20% dileptonic and 20% semileptonic ttbar, 15% t-channel, 10% "
                "semileptonic and 5% dileptonic Wt, 30% background) through the five signal bins of the HL-LHC "
                "selection, each with its reconstruction",
    },
    "stress2M_heavytail": {
        "index": 3, "n_events": 2_000_000, "kind": "ttbar", "n_extra_max": 10,
        "bkg_frac": 0.2, "bkg_jet_max": 12, "chain": "dilepton",
        "var_mode": "loguniform1024",
        "reco": {"smear": 1, "n_var": 0},
        "desc": "2M events, 2-12 jets, variations log-uniform in 1..1024",
    },
}


def chain_hlhc_dilepton():
    """HL-LHC dileptonic channel (section 6.1): two isolated opposite-sign
    leptons, jets, a b tag, E_T^miss > 30, M_ll > 40, then the two-neutrino
    reconstruction."""
    return [
        _cut("D_LEP2OS", "LEP_N_OS", [20.0, 2.5], [2, 1]),
        _cut("D_JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
        _cut("D_BTAG1", "BTAG_N_MIN", [25.0, 2.5, 0.5], [1]),
        _cut("D_MET30", "MET_MIN", [30.0]),
        _cut("D_MLL40", "MLL_MIN", [20.0, 2.5, 40.0], deps=["D_LEP2OS"]),
        _cut("D_RECO", "RECO", deps=["D_LEP2OS", "D_JETS2", "D_BTAG1", "D_MET30", "D_MLL40"]),
    ]


def chain_hlhc_single():
    """HL-LHC one-lepton single-top channel (section 6.1): exactly one
    lepton, jets, exactly one b tag, E_T^miss > 30, M_T^W > 50, then the
    single-neutrino chi^2 reconstruction."""
    return [
        _cut("S_LEP1", "LEP_N_OS", [20.0, 2.5], [1, 0]),
        _cut("S_JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
        _cut("S_BTAG1", "BTAG_N_EQ", [25.0, 2.5, 0.5], [1]),
        _cut("S_MET30", "MET_MIN", [30.0]),
        _cut("S_MTW50", "MTW_MIN", [20.0, 2.5, 50.0], deps=["S_LEP1"]),
        _cut("S_RECO", "RECO", deps=["S_LEP1", "S_JETS2", "S_BTAG1", "S_MET30", "S_MTW50"]),
    ]


# The HL-LHC signal bins (section 6.1).  Jet pseudorapidity regions: I
# |eta| < 2.5, II 2.5 <= |eta| < 2.75, III 2.75 <= |eta| < 3.5 (the paper's
# strict inequalities leave the boundaries unassigned; reading: each lower
# edge belongs to its region).  Jets count with pT > 25 GeV, b jets are
# tagged Region I jets, leptons have pT > 20 GeV and |eta| < 2.5, isolated
# when no Region I jet lies within Delta R < 0.4 (reading of "isolated").
# Every bin requires E_T^miss > 30 GeV.
REGION_I = [0.0, 2.5]
REGIONS_II_III = [2.5, 3.5]
_MANY = 99


def _lep(name, n):
    return _cut(name, "LEP_N_OS", [20.0, 2.5], [n, 1 if n == 2 else 0])


def _iso(name, lep):
    return _cut(name, "LEP_ISO", [20.0, 2.5, 25.0, 2.5, 0.4], deps=[lep])


def _jets(name, region, lo, hi):
    return _cut(name, "JET_N_RANGE", [25.0] + list(region), [lo, hi])


def chains_hlhc_bins():
    """The five signal bins of section 6.1, each a chain ending in its
    reconstruction (section 6.2):
      ttsemi   1 lepton, >= 4 Region I jets, 2 b, no Region II/III jet;
      ttdilep  2 opposite-sign leptons, >= 2 Region I jets, 2 b, no Region
               II/III jet, M_ll > 40;
      tchan    1 lepton, exactly 1 Region I jet and 1 Region II/III jet, 1 b;
      wtsemi   1 lepton, 3 Region I jets, 1 b, no Region II/III jet,
               M_T^W > 50;
      wtdilep  2 opposite-sign leptons, 1 or 2 Region I jets, 1 b, no Region
               II/III jet."""
    fwd = lambda n: _cut(n, "FWD_JET_VETO", [25.0] + REGIONS_II_III)
    btag = lambda n, k: _cut(n, "BTAG_N_EQ", [25.0, 2.5, 0.5], [k])
    met = lambda n: _cut(n, "MET_MIN", [30.0])
    bins = {
        "ttsemi": [_lep("L1", 1), _iso("ISO", "L1"), _jets("JI4", REGION_I, 4, _MANY), btag("B2", 2), fwd("VETO"),
                   met("MET30")],
        "ttdilep": [_lep("L2", 2), _iso("ISO", "L2"), _jets("JI2", REGION_I, 2, _MANY), btag("B2", 2), fwd("VETO"),
                    met("MET30"), _cut("MLL40", "MLL_MIN", [20.0, 2.5, 40.0], deps=["L2"])],
        "tchan": [_lep("L1", 1), _iso("ISO", "L1"), _jets("JI1", REGION_I, 1, 1), _jets("JF1", REGIONS_II_III, 1, 1),
                  btag("B1", 1), met("MET30")],
        "wtsemi": [_lep("L1", 1), _iso("ISO", "L1"), _jets("JI3", REGION_I, 3, 3), btag("B1", 1), fwd("VETO"),
                   met("MET30"), _cut("MTW50", "MTW_MIN", [20.0, 2.5, 50.0], deps=["L1"])],
        "wtdilep": [_lep("L2", 2), _iso("ISO", "L2"), _jets("JI12", REGION_I, 1, 2), btag("B1", 1), fwd("VETO"),
                    met("MET30")],
    }
    for name, cuts in bins.items():
        cuts.append(_cut("RECO", "RECO", deps=[c["name"] for c in cuts]))
    return bins


# Reconstruction of each bin: the single-neutrino chi^2 in its topology, the
# two-neutrino solve ("quartic": up to four solutions per pairing) at the
# configuration's variations, or the dileptonic
# chi^2 fit with a MET split with one top (Wt: one top and two W bosons).
HLHC_BIN_RECO = {
    "ttsemi": ("semilep", "TTSEMI"),
    "ttdilep": ("quartic", None),
    "tchan": ("semilep", "TCHAN"),
    "wtsemi": ("semilep", "WT"),
    "wtdilep": ("chi2", 1),
}


def _user(name, src, deps=(), budget=0):
    """A user predicate (section 3: the user's own cut, a boolean function of
    one event): the body of a C function over the accessors n_lep(),
    n_jet(), lep_pt(i) ... jet_btag(i), met_x(), met_y().  budget: loop
    iterations it may run per event (0: the library default)."""
    return {"name": name, "kind": "USER", "f": [], "i": [0, int(budget)], "deps": list(deps), "src": src}


# User predicates, some restating built-in cuts (so that the two paths can be
# checked against each other), some new: a forward jet in the paper's
# Regions II/III (section 6.1), a scalar pT sum, a leading-lepton cut.
USER_CUTS = {
    "U_MET30": "double mx = met_x(), my = met_y(); return mx * mx + my * my > 30.0 * 30.0;",
    "U_JETS2": ("int n = 0;\nfor (int k = 0; k < n_jet(); ++k)\n"
                "    if (jet_pt(k) > 25.0f && fabsf(jet_eta(k)) < 2.5f) ++n;\nreturn n >= 2;"),
    "U_LEP2OS": ("int n = 0; float q = 1.0f;\nfor (int k = 0; k < n_lep(); ++k)\n"
                 "    if (lep_pt(k) > 20.0f && fabsf(lep_eta(k)) < 2.5f) { ++n; q *= lep_q(k); }\n"
                 "return n == 2 && q < 0.0f;"),
    "U_FWDJET": ("for (int k = 0; k < n_jet(); ++k) {\n    float a = fabsf(jet_eta(k));\n"
                 "    if (jet_pt(k) > 25.0f && a >= 2.5f && a < 4.5f) return 1;\n}\nreturn 0;"),
    "U_HT150": ("float ht = 0.0f;\nfor (int k = 0; k < n_jet(); ++k)\n"
                "    if (jet_pt(k) > 25.0f && fabsf(jet_eta(k)) < 2.5f) ht += jet_pt(k);\nreturn ht > 150.0f;"),
    "U_LEAD40": "return n_lep() > 0 && lep_pt(0) > 40.0f && lep_pt(n_lep()) == 0.0f && jet_eta(-1) == 0.0f;",
}


def chain_user_mix():
    """Built-in and user cuts mixed (eight cuts, no reconstruction)."""
    return [
        _user("U_LEP2OS", USER_CUTS["U_LEP2OS"]),
        _cut("JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
        _user("U_HT150", USER_CUTS["U_HT150"]),
        _cut("MET30", "MET_MIN", [30.0]),
        _user("U_FWDJET", USER_CUTS["U_FWDJET"]),
        _user("U_LEAD40", USER_CUTS["U_LEAD40"], deps=["U_LEP2OS"]),
        _cut("MLL40", "MLL_MIN", [20.0, 2.5, 40.0], deps=["U_LEP2OS"]),
        _user("U_MET30", USER_CUTS["U_MET30"]),
    ]


def chain_semilep():
    """Single-lepton chain plus the single-neutrino reconstruction."""
    return [
        _cut("LEP1", "LEP_N_OS", [20.0, 2.5], [1, 0]),
        _cut("JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
        _cut("BTAG1", "BTAG_N_MIN", [25.0, 2.5, 0.5], [1]),
        _cut("MET30", "MET_MIN", [30.0]),
        _cut("RECO", "RECO", deps=["LEP1", "JETS2", "BTAG1", "MET30"]),
    ]


def config(name):
    c = copy.deepcopy(CONFIGS[name])
    c["name"] = name
    c["seed"] = 1000 + c["index"]
    reco = dict(RECO_DEFAULTS)
    reco.update(c["reco"])
    reco["seed"] = c["seed"]
    c["reco"] = reco
    c["semilep"] = dict(SEMILEP_DEFAULTS)
    c["chi2"] = dict(CHI2_DEFAULTS)
    if c["chain"] == "hlhc":
        c["chains"] = chains_hlhc_bins()
        c["cuts"] = [cut for cuts in c["chains"].values() for cut in cuts]
    else:
        c["cuts"] = {"dilepton": chain_dilepton, "tth8": chain_tth8, "semilep": chain_semilep}[c["chain"]]()
    return c


def default_order(cuts):
    return list(range(len(cuts)))


def dep_masks(cuts):
    """Dependency bit masks: bit j set in entry k means cut j must precede cut k."""
    idx = {c["name"]: k for k, c in enumerate(cuts)}
    out = []
    for c in cuts:
        m = 0
        for d in c["deps"]:
            m |= 1 << idx[d]
        out.append(m)
    return out
