"""The five signal bins of the HL-LHC selection (section 6.1) on hand-built
events whose bin membership is derived by hand (golden/bin_cases.json), and
their disjointness on a generated mixed sample."""

import json
import os

import numpy as np
import pytest

import hfgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "bin_cases.json")


def load_bin_cases():
    d = json.load(open(GOLD))
    cols = {k: [] for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q",
                            "jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag")}
    loff, joff, mx, my = [0], [0], [], []
    for c in d["cases"]:
        for pt, eta, phi, q in c["leps"]:
            cols["lep_pt"].append(pt); cols["lep_eta"].append(eta); cols["lep_phi"].append(phi)
            cols["lep_e"].append(pt * np.cosh(eta)); cols["lep_q"].append(q)
        for pt, eta, phi, tag in c["jets"]:
            cols["jet_pt"].append(pt); cols["jet_eta"].append(eta); cols["jet_phi"].append(phi)
            cols["jet_e"].append(pt * np.cosh(eta)); cols["jet_btag"].append(tag)
        loff.append(loff[-1] + len(c["leps"]))
        joff.append(joff[-1] + len(c["jets"]))
        mx.append(c["met"][0]); my.append(c["met"][1])
    ev = {k: np.asarray(v, np.float32) for k, v in cols.items()}
    ev.update(n=len(d["cases"]), lep_off=np.asarray(loff, np.uint32), jet_off=np.asarray(joff, np.uint32),
              met_x=np.asarray(mx, np.float32), met_y=np.asarray(my, np.float32), n_var=None)
    return ev, d["cases"]


@pytest.mark.parametrize("name", list(hfgen.configs.chains_hlhc_bins()))
def test_bins_hand_derived(orc, name):
    ev, cases = load_bin_cases()
    cuts = hfgen.configs.chains_hlhc_bins()[name]
    surv, _, _ = orc.select(ev, cuts, list(range(len(cuts))))
    want = np.array([c["expect"][name] for c in cases], dtype=np.uint8)
    bad = [(c["name"], c["why"]) for c, g, w in zip(cases, surv, want) if g != w]
    assert not bad, bad


def test_bins_are_disjoint_and_populated(orc):
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 0, n=100_000)
    masks = {}
    for name, cuts in cfg["chains"].items():
        masks[name], _, _ = orc.select(ev, cuts, list(range(len(cuts))))
    total = sum(m.astype(int) for m in masks.values())
    assert total.max() <= 1
    proc = ev["truth"]["process"]
    code = {p: i for i, p in enumerate(hfgen.events.HLHC_PROCESSES)}
    # each bin is dominated by, or at least well populated with, its own process
    for name, p in (("ttsemi", "ttsemi"), ("ttdilep", "ttbar"), ("tchan", "tchan"), ("wtsemi", "wt"),
                    ("wtdilep", "wtdilep")):
        assert (masks[name] & (proc == code[p])).sum() > 100, name
