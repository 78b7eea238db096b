"""GPU parity of the dileptonic chi^2 fit with a MET split (section 6.2)
through the C ABI against the FP64 oracle: decisions identical, the chosen
split point, pairing and roots in >= 99.9 % of events, every output within
1e-4 relative (gpu_compare.compare_chi2)."""

import sys

import numpy as np
import pytest

import hfgen

from .gpu_compare import assert_agree_semilep, compare_chi2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _direct(B, ev, ids, cp, index_base=0):
    dev = B.DeviceEvents(ev, index_base=index_base)
    cap = max(1, len(ids))
    idx = torch.zeros(cap, dtype=torch.int32, device="cuda")
    idx[:len(ids)] = torch.as_tensor(np.asarray(ids, dtype=np.int32))
    cnt = torch.tensor([len(ids)], dtype=torch.int64, device="cuda")
    outs = B.Chi2Outputs(cap)
    counters = torch.zeros(1, 3, dtype=torch.int64, device="cuda")
    B.dilep_chi2_reco(dev, idx, cnt, cap, B.chi2_params(cp, reco_cut=0), outs, counters)
    torch.cuda.synchronize()
    return outs.host(len(ids)), counters.cpu().numpy()[0]


@pytest.mark.parametrize("name,n,over", [
    ("ttbar10k", 8000, {}),
    ("ttbar1M_v64", 4000, {"pair_mode": "ALL_JETS", "max_cands": 6, "n_grid": 9, "n_refine": 3}),
])
def test_chi2_chain_matches_oracle(B, orc, name, n, over):
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config(name)
    ev = hfgen.generate(cfg, n_events=n, seed=401)
    cp = dict(cfg["chi2"], **over)
    _say("chi2 chain", name, n, over)
    ch = Chain(ev, cfg["cuts"], None, chi2=cp)
    ch.step()
    got = ch.results()
    s_w, _, _ = orc.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
    assert np.array_equal(got["survive"], s_w)
    want = orc.dilep_chi2_reco(ev, got["idx"], cp)
    st = compare_chi2(got["reco"], want)
    _say(st)
    assert_agree_semilep(st)
    assert np.array_equal(got["final"], got["idx"][got["reco"]["has_sol"].astype(bool)])


@pytest.mark.parametrize("refine", [2, 0])
def test_chi2_one_top_matches_oracle(B, orc, refine):
    """Wt events (one top, two W): every candidate forms the top with either
    lepton; one and two b candidates, with and without refinement."""
    cfg = {"kind": "wtdilep", "n_extra_max": 3, "bkg_frac": 0.0, "seed": 41}
    ev = hfgen.generate(cfg, n_events=6000, seed=41)
    cuts = hfgen.configs.chain_dilepton()[:2]
    s_w, _, _ = orc.select(ev, cuts, [0, 1])
    ids = np.flatnonzero(s_w)
    cp = dict(hfgen.configs.CHI2_DEFAULTS, n_top=1, n_refine=refine)
    _say("chi2 one top", ids.size, refine)
    got, cnt = _direct(B, ev, ids, cp)
    want = orc.dilep_chi2_reco(ev, ids, cp)
    st = compare_chi2(got, want)
    _say(st)
    diff = np.flatnonzero((got["best_i"] != want["best_i"]) | (got["best_j"] != want["best_j"]) |
                          np.any(got["split"] != want["split"], axis=1) | (got["root_nu"] != want["root_nu"]) |
                          (got["root_nubar"] != want["root_nubar"]))
    for q in diff[:6]:
        _say("differs", int(q), "chi2", float(got["chi2"][q]), float(want["chi2"][q]), "ij", int(got["best_i"][q]),
             int(got["best_j"][q]), int(want["best_i"][q]), int(want["best_j"][q]), "split", got["split"][q],
             want["split"][q], "roots", int(got["root_nu"][q]), int(got["root_nubar"][q]), int(want["root_nu"][q]),
             int(want["root_nubar"][q]))
    assert_agree_semilep(st, min_agree=0.999)
    assert st["n_both"] > 0.9 * ids.size
    # one side carries the top: exactly one of best_i / best_j is set
    hs = got["has_sol"].astype(bool)
    assert np.all((got["best_i"][hs] >= 0) != (got["best_j"][hs] >= 0))
    assert cnt[0] == ids.size and cnt[1] == hs.sum()


def _staging_events():
    """Events aimed at the staging's object chunks (sixteen objects per event
    and pass) and its candidate fill: selected objects in a later chunk only."""
    rng = np.random.default_rng(17)

    def obj(pt, eta, phi, aux):
        return [pt, eta, phi, pt * np.cosh(eta), aux]

    L = [obj(60, 0.3, 0.1, 1), obj(40, -0.7, 2.5, -1)]
    fwd = [obj(100 - k, 2.7 + 0.01 * k, rng.uniform(-3, 3), 1) for k in range(18)]  # never selected
    late = [obj(70, 0.2, -1.0, 1), obj(55, -0.4, 2.0, 0), obj(45, 1.1, 0.5, 0), obj(35, -1.5, -2.2, 0)]
    soft_leps = [obj(5 + 0.5 * k, 0.1 * k, 0.2 * k, 1) for k in range(17)]  # below the lepton pT cut
    return [
        # the only tagged jet and the fillers after 18 unselected jets: a second chunk
        {"leps": L, "jets": fwd + late, "met": [30, -20]},
        # no tagged jet at all, the untagged fillers in the second chunk
        {"leps": L, "jets": fwd + [obj(65, 0.5, 1.0, 0), obj(50, -0.9, -2.0, 0)], "met": [-25, 15]},
        # the second selected lepton is object 17 (after sixteen soft ones)
        {"leps": [L[0]] + soft_leps + [L[1]], "jets": late, "met": [10, 40]},
        # l+ listed second
        {"leps": [L[1], L[0]], "jets": late, "met": [20, 20]},
        # a zero charge: not an opposite-sign pair
        {"leps": [L[0], obj(40, -0.7, 2.5, 0)], "jets": late, "met": [20, 20]},
    ]


@pytest.mark.parametrize("mode", ["ALL_JETS", "BTAG_FILL"])
def test_chi2_edge_cases(B, orc, mode):
    from .test_gpu_parity import _edge_sample
    ev = _edge_sample(_staging_events())
    cp = dict(hfgen.config("ttbar10k")["chi2"], pair_mode=mode)
    base = 500
    ids = list(np.random.default_rng(3).permutation(ev["n"]) + base) + [base - 1, base + ev["n"]]
    _say("chi2 edge cases", mode)
    got, cnt = _direct(B, ev, ids, cp, index_base=base)
    want = orc.dilep_chi2_reco(ev, np.array(ids[:-2]) - base, cp)
    st = compare_chi2({k: v[:len(ids) - 2] for k, v in got.items()}, want)
    _say(st)
    assert_agree_semilep(st, min_agree=0.999)
    assert np.all(got["has_sol"][-2:] == 0)
    assert cnt[0] == len(ids) and cnt[1] == got["has_sol"].sum()


def test_chi2_zero_and_clamped_count(B, orc):
    """A zero count leaves the outputs and counters untouched (every block
    leaves at once); a count above the capacity is clamped to it, with the
    last block of four events only partly filled."""
    cfg = hfgen.config("ttbar10k")
    ev = hfgen.generate(cfg, n_events=300, seed=5)
    cap = 37
    ids = np.arange(cap, dtype=np.int32)
    dev = B.DeviceEvents(ev)
    idx = torch.as_tensor(ids).cuda()
    outs = B.Chi2Outputs(cap)
    outs.t["chi2"].fill_(7.0)
    counters = torch.zeros(1, 3, dtype=torch.int64, device="cuda")
    params = B.chi2_params(cfg["chi2"], reco_cut=0)
    _say("chi2 zero count")
    B.dilep_chi2_reco(dev, idx, torch.zeros(1, dtype=torch.int64, device="cuda"), cap, params, outs, counters)
    torch.cuda.synchronize()
    assert bool(torch.all(outs.t["chi2"] == 7.0))
    assert counters.cpu().numpy()[0, :2].tolist() == [0, 0]
    _say("chi2 count above the capacity")
    B.dilep_chi2_reco(dev, idx, torch.tensor([10 * cap], dtype=torch.int64, device="cuda"), cap, params, outs,
                      counters)
    torch.cuda.synchronize()
    got = outs.host(cap)
    want = orc.dilep_chi2_reco(ev, ids, cfg["chi2"])
    st = compare_chi2(got, want)
    _say(st)
    assert_agree_semilep(st, min_agree=0.999)
    c = counters.cpu().numpy()[0]
    assert c[0] == cap and c[1] == got["has_sol"].sum()


def test_chi2_full_size_sampled(B, orc):
    """1M events of the benchmark sample: the reconstruction against the
    oracle on a sample of the compacted events, properties on all."""
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("ttbar1M_v64")
    ev = hfgen.generate(cfg)
    _say("chi2 full size", ev["n"])
    ch = Chain(ev, cfg["cuts"], None, chi2=cfg["chi2"])
    ch.step()
    got = ch.results()
    S = got["count"]
    pos = np.sort(np.random.default_rng(6).choice(S, size=1500, replace=False))
    want = orc.dilep_chi2_reco(ev, got["idx"][pos], cfg["chi2"], n_threads=16)
    st = compare_chi2({k: v[pos] for k, v in got["reco"].items()}, want)
    _say(st)
    assert_agree_semilep(st)
    r = got["reco"]
    hs = r["has_sol"].astype(bool)
    e = got["idx"][hs]
    assert np.allclose(r["nu"][hs, 0] + r["nubar"][hs, 0], ev["met_x"][e].astype(float), atol=1e-9)
    assert np.allclose(r["nu"][hs, 1] + r["nubar"][hs, 1], ev["met_y"][e].astype(float), atol=1e-9)
    real = hs & (r["root_nu"] != 2)
    assert np.all(np.abs(r["m_wp"][real] - 80.4) < 1e-9 * 80.4)
    assert np.all(r["chi2"][hs] >= 0)


def test_chi2_graph_replay(B):
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("ttbar10k")
    ev = hfgen.generate(cfg, n_events=5000, seed=93)
    ch = Chain(ev, cfg["cuts"], None, chi2=cfg["chi2"])
    ch.step()
    ref = ch.results()
    ch.capture()
    for rep in range(3):
        ch.reset_counters()
        ch.out.t["chi2"].fill_(7.0)
        ch.replay()
        torch.cuda.synchronize()
        r = ch.results()
        for k in ("chi2", "best_i", "best_j", "split", "nu"):
            assert np.array_equal(r["reco"][k], ref["reco"][k]), k
        assert np.array_equal(r["counters"][:, :2], ref["counters"][:, :2])
