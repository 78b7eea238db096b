"""Builds an SoA sample from the hand-written cut cases in golden/cut_cases.json."""

import json
import os

import numpy as np

import hfgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cut_cases.json")

CUT_DEFS = {c["name"]: c for c in hfgen.configs.chain_dilepton() + hfgen.configs.chain_tth8()}
CUT_DEFS["JETS4"] = [c for c in hfgen.configs.chain_tth8() if c["name"] == "JETS4"][0]
CUT_DEFS["BTAG3"] = [c for c in hfgen.configs.chain_tth8() if c["name"] == "BTAG3"][0]
CUT_DEFS["JETS_I_1TO2"] = {"name": "JETS_I_1TO2", "kind": "JET_N_RANGE", "f": [25.0, 0.0, 2.5], "i": [1, 2],
                            "deps": []}
CUT_DEFS["JETS_FWD1"] = {"name": "JETS_FWD1", "kind": "JET_N_RANGE", "f": [25.0, 2.5, 3.5], "i": [1, 1], "deps": []}
CUT_DEFS["JETS_II1"] = {"name": "JETS_II1", "kind": "JET_N_RANGE", "f": [25.0, 2.5, 2.75], "i": [1, 99], "deps": []}
CUT_DEFS["MTW50"] = dict([c for c in hfgen.configs.chain_hlhc_single() if c["name"] == "S_MTW50"][0],
                         name="MTW50")


def load():
    d = json.load(open(GOLD))
    n = len(d["cases"])
    ev = {"n": n}
    cols = {k: [] for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q",
                            "jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag")}
    loff, joff = [0], [0]
    metx, mety = [], []
    for c in d["cases"]:
        for pt, eta, phi, q in c["leps"]:
            cols["lep_pt"].append(pt); cols["lep_eta"].append(eta); cols["lep_phi"].append(phi)
            cols["lep_e"].append(pt * np.cosh(eta)); cols["lep_q"].append(q)
        for pt, eta, phi, tag in c["jets"]:
            cols["jet_pt"].append(pt); cols["jet_eta"].append(eta); cols["jet_phi"].append(phi)
            cols["jet_e"].append(pt * np.cosh(eta)); cols["jet_btag"].append(tag)
        loff.append(loff[-1] + len(c["leps"]))
        joff.append(joff[-1] + len(c["jets"]))
        metx.append(c["met"][0]); mety.append(c["met"][1])
    for k, v in cols.items():
        ev[k] = np.asarray(v, dtype=np.float32)
    ev["lep_off"] = np.asarray(loff, dtype=np.uint32)
    ev["jet_off"] = np.asarray(joff, dtype=np.uint32)
    ev["met_x"] = np.asarray(metx, dtype=np.float32)
    ev["met_y"] = np.asarray(mety, dtype=np.float32)
    ev["n_var"] = None
    cuts = [dict(CUT_DEFS[name], deps=[]) for name in d["cuts"]]
    expect = np.array([[c["expect"][name] for name in d["cuts"]] for c in d["cases"]], dtype=np.uint8)
    return ev, cuts, expect, [c["name"] for c in d["cases"]]
