"""GPU parity of the single-neutrino chi^2 reconstruction (section 6.2,
Eq. (chi2)) through the C ABI against the FP64 oracle: the selection and
compaction in front of it bit-exact, the decision identical, the chosen
assignment in >= 99.9 % of events and every output within 1e-4 relative
(gpu_compare.compare_semilep)."""

import sys

import numpy as np
import pytest

import hfgen

from .gpu_compare import assert_agree_semilep, compare_semilep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOPOLOGIES = [("TCHAN", "tchan"), ("WT", "wt"), ("TTSEMI", "ttsemi")]


def _say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14346_amd import binding
    binding.lib()
    return binding


def _cfg(kind, **over):
    cfg = hfgen.config("tchan1M")
    cfg["kind"] = kind
    cfg.update(over)
    return cfg


def _run_chain(ev, cfg, topology):
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cfg["cuts"], None, semilep=cfg["semilep"], topology=topology)
    ch.step()
    return ch, ch.results()


@pytest.mark.parametrize("topology,kind", TOPOLOGIES)
def test_semilep_chain_matches_oracle(B, orc, topology, kind):
    cfg = _cfg(kind)
    ev = hfgen.generate(cfg, n_events=6000, seed=301)
    _say("semilep chain", topology, ev["n"])
    ch, got = _run_chain(ev, cfg, topology)
    cuts = cfg["cuts"]
    s_w, r_w, p_w = orc.select(ev, cuts, list(range(len(cuts))))
    assert np.array_equal(got["survive"], s_w)
    assert np.array_equal(got["idx"], np.flatnonzero(s_w))
    n_sel = len(cuts) - 1
    assert np.array_equal(got["counters"][:n_sel, 0], r_w[:n_sel])
    assert np.array_equal(got["counters"][:n_sel, 1], p_w[:n_sel])
    want = orc.semilep_reco(ev, got["idx"], cfg["semilep"], topology)
    st = compare_semilep(got["reco"], want)
    _say(st)
    assert_agree_semilep(st)
    assert np.array_equal(got["final"], got["idx"][got["reco"]["has_sol"].astype(bool)])
    assert got["counters"][n_sel, 0] == got["count"]
    assert got["counters"][n_sel, 1] == len(got["final"])


def _reco_direct(B, ev, ids, sl, topology, index_base=0, count=None):
    dev = B.DeviceEvents(ev, index_base=index_base)
    cap = max(1, len(ids))
    idx = torch.zeros(cap, dtype=torch.int32, device="cuda")
    idx[:len(ids)] = torch.as_tensor(np.asarray(ids, dtype=np.int32))
    n = len(ids) if count is None else count
    cnt = torch.tensor([n], dtype=torch.int64, device="cuda")
    outs = B.SemilepOutputs(cap)
    counters = torch.zeros(1, 3, dtype=torch.int64, device="cuda")
    B.semilep_reco(dev, idx, cnt, cap, B.semilep_params(sl, topology, reco_cut=0), outs, counters)
    torch.cuda.synchronize()
    return outs.host(cap), counters.cpu().numpy()[0]


def _edge_events():
    """Hand-built ragged events: no lepton; lepton but no jet; one jet; a
    lepton failing eta then a good one; 15 selected jets (the cap of 12
    applies); jets failing pT / eta between selected ones; a complex-root
    case (large MET along the lepton); MET of zero."""
    rng = np.random.default_rng(5)
    evs = []

    def add(leps, jets, met):
        evs.append((leps, jets, met))

    def lep(pt, eta, phi):
        return (pt, eta, phi, pt * np.cosh(eta), 1.0)

    def jet(pt, eta, phi, m=5.0):
        return (pt, eta, phi, np.sqrt(m * m + (pt * np.cosh(eta)) ** 2), 0.0)

    add([], [jet(60, 0.1, 1.0)], (30, 5))
    add([lep(40, 0.2, 0.3)], [], (30, 5))
    add([lep(40, 0.2, 0.3)], [jet(60, 0.1, 1.0)], (30, 5))
    add([lep(50, 2.7, 0.3), lep(30, 1.0, -2.0)], [jet(60, 0.1, 1.0), jet(45, -1.0, 2.5), jet(35, 0.5, -1.0),
                                                  jet(28, 1.5, 0.0)], (-20, 40))
    add([lep(45, -0.4, 1.2)], [jet(300 - 15 * k, rng.uniform(-2.4, 2.4), rng.uniform(-3, 3)) for k in range(15)],
        (25, -30))
    add([lep(35, 1.1, -0.7)], [jet(90, 0.3, 0.2), jet(80, 3.0, 1.0), jet(70, -0.5, 2.0), jet(60, 2.6, -2.0),
                               jet(50, 1.0, -1.0), jet(20, 0.0, 0.5), jet(40, -2.0, 3.1)], (40, 10))
    add([lep(30, 0.0, 0.0)], [jet(100, 0.5, 2.0), jet(70, -0.3, -2.5), jet(55, 1.2, 1.0), jet(30, 0.0, 3.0)],
        (-200, 0))
    add([lep(60, 0.8, -1.5)], [jet(80, -0.2, 1.6), jet(75, 0.9, -0.1), jet(66, -1.8, 2.2), jet(41, 0.4, 0.9),
                               jet(33, -0.9, -2.9)], (0, 0))
    ev = {"n": len(evs)}
    lo, jo = [0], [0]
    cols = {k: [] for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                            "jet_e", "jet_btag")}
    mx, my = [], []
    for leps, jets, met in evs:
        for l in leps:
            for k, v in zip(("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q"), l):
                cols[k].append(v)
        for j in sorted(jets, key=lambda x: -x[0]):
            for k, v in zip(("jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag"), j):
                cols[k].append(v)
        lo.append(lo[-1] + len(leps))
        jo.append(jo[-1] + len(jets))
        mx.append(met[0])
        my.append(met[1])
    for k, v in cols.items():
        ev[k] = np.array(v, dtype=np.float32)
    ev["lep_off"] = np.array(lo, dtype=np.uint32)
    ev["jet_off"] = np.array(jo, dtype=np.uint32)
    ev["met_x"] = np.array(mx, dtype=np.float32)
    ev["met_y"] = np.array(my, dtype=np.float32)
    ev["n_var"] = None
    return ev


@pytest.mark.parametrize("topology", ["TCHAN", "WT", "TTSEMI"])
@pytest.mark.parametrize("max_cands", [1, 4, 12])
def test_semilep_edge_cases(B, orc, topology, max_cands):
    ev = _edge_events()
    sl = dict(hfgen.config("tchan1M")["semilep"])
    sl["max_cands"] = max_cands
    base = 1000
    # every event, in a shuffled order, plus two ids outside the chunk
    ids = list(np.random.default_rng(2).permutation(ev["n"]) + base) + [base - 1, base + ev["n"]]
    _say("edge", topology, max_cands)
    got, cnt = _reco_direct(B, ev, ids, sl, topology, index_base=base)
    want = orc.semilep_reco(ev, np.array(ids[:-2]) - base, sl, topology)
    st = compare_semilep({k: v[:len(ids) - 2] for k, v in got.items()}, want)
    _say(st)
    assert_agree_semilep(st, min_agree=1.0)
    assert np.all(got["has_sol"][-2:] == 0) and np.all(got["chi2"][-2:] == -9999.0)
    assert cnt[0] == len(ids) and cnt[1] == got["has_sol"].sum()
    if topology == "TCHAN" and max_cands >= 4:
        assert (got["root"][:len(ids) - 2] == 2).any()  # the complex-root event is in the set


def test_semilep_zero_count_leaves_outputs(B):
    ev = _edge_events()
    sl = hfgen.config("tchan1M")["semilep"]
    got, cnt = _reco_direct(B, ev, [0, 1, 2], sl, "TCHAN", count=0)
    assert np.all(got["has_sol"] == 0) and np.all(got["chi2"] == 0.0)  # untouched zeros
    assert cnt[0] == 0 and cnt[1] == 0


def test_semilep_full_size_sampled(B, orc):
    """tchan1M in the launch configuration the benchmark times: selection
    bit-exact in full, the reconstruction against the oracle on a sample and
    by properties everywhere."""
    cfg = hfgen.config("tchan1M")
    ev = hfgen.generate(cfg)
    _say("semilep full size", ev["n"])
    ch, got = _run_chain(ev, cfg, "TCHAN")
    cuts = cfg["cuts"]
    s_w, r_w, p_w = orc.select(ev, cuts, list(range(len(cuts))))
    assert np.array_equal(got["survive"], s_w)
    assert np.array_equal(got["idx"], np.flatnonzero(s_w))
    S = got["count"]
    rng = np.random.default_rng(4)
    pos = np.sort(rng.choice(S, size=4000, replace=False))
    want = orc.semilep_reco(ev, got["idx"][pos], cfg["semilep"], "TCHAN")
    st = compare_semilep({k: v[pos] for k, v in got["reco"].items()}, want)
    _say(st)
    assert_agree_semilep(st)
    r = got["reco"]
    hs = r["has_sol"].astype(bool)
    # the chain requires a lepton and two selected jets: every survivor has a solution
    assert hs.all()
    real = r["root"] != 2
    assert np.all(np.abs(r["m_wl"][real] - 80.4) <= 1e-9 * 80.4)
    assert np.all(r["chi2"] >= 0.0) and np.all(r["best_h"] == -1) and np.all(r["best_p"] == -1)
    assert np.array_equal(got["final"], got["idx"][hs])


def test_semilep_graph_replay(B):
    cfg = hfgen.config("tchan1M")
    ev = hfgen.generate(cfg, n_events=20000, seed=91)
    _say("semilep graph replay")
    ch, ref = _run_chain(ev, cfg, "TCHAN")
    ch.capture()
    for rep in range(3):
        ch.reset_counters()
        ch.out.t["chi2"].fill_(7.0)
        ch.replay()
        torch.cuda.synchronize()
        r = ch.results()
        assert np.array_equal(r["final"], ref["final"])
        for k in ("chi2", "best_j", "root", "nu", "m_tl"):
            assert np.array_equal(r["reco"][k], ref["reco"][k]), k
        assert np.array_equal(r["counters"][:, :2], ref["counters"][:, :2])
