"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Integer work (survive masks, per-cut counters, compaction indices, raw
random words) must be bit-exact; reconstruction outputs follow the
agreement targets in gpu_compare.py.  Every expected value comes from the
oracle on the same seeded inputs.
"""

import sys

import numpy as np
import pytest

import hfgen

from . import cutcases
from .gpu_compare import adjudicate, choice_mismatches, assert_agree, compare

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


def _chain(ev, cuts, reco, precision, order=None, schedule="auto"):
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cuts, reco, precision=precision, order=order, schedule=schedule)
    ch.step()
    return ch, ch.results()


def _check_selection(got, want, cuts):
    assert np.array_equal(got["survive"], want["survive"])
    assert np.array_equal(got["idx"], want["idx"])
    assert np.array_equal(got["counters"][:, 0], want["reached"])
    assert np.array_equal(got["counters"][:, 1], want["passed"])


# --------------------------------------------------------------------- RNG

def test_philox_raw_words_bit_exact(B, orc):
    import json
    import os
    _say("philox raw words")
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")))
    rng = np.random.default_rng(1)
    for v in kat["vectors"]:
        ctr = np.array([[int(x, 16) for x in v["ctr"]]], dtype=np.uint32)
        key = [int(x, 16) for x in v["key"]]
        seed = key[0] | (key[1] << 32)
        out = torch.zeros(1, 4, dtype=torch.int32, device="cuda")
        B.philox_blocks(torch.from_numpy(ctr.view(np.int32)).cuda(), seed, out)
        got = out.cpu().numpy().view(np.uint32)[0]
        assert [int(x) for x in got] == [int(x, 16) for x in v["out"]]
    n = 5000
    ctr = rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0xDEADBEEF12345678
    out = torch.zeros(n, 4, dtype=torch.int32, device="cuda")
    B.philox_blocks(torch.from_numpy(ctr.view(np.int32)).cuda(), seed, out)
    got = out.cpu().numpy().view(np.uint32)
    for k in range(0, n, 7):
        want = orc.philox(ctr[k], [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(got[k], want), k


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 5e-5)])
def test_gauss_draws_match_oracle(B, orc, precision, tol):
    _say("gauss draws", precision)
    rng = np.random.default_rng(2)
    n = 4000
    g = rng.integers(0, 2 ** 31, n).astype(np.int64)
    v = rng.integers(0, 1024, n).astype(np.int32)
    s = rng.integers(0, 20, n).astype(np.int32)
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    seed = 1001
    B.gauss_draws(seed, torch.from_numpy(g).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(s).cuda(), z,
                  precision)
    got = z.cpu().numpy()
    want = np.array([orc.gauss(seed, int(a), int(b), int(c)) for a, b, c in zip(g, v, s)])
    _say("gauss max abs diff", precision, np.abs(got - want).max())
    assert np.abs(got - want).max() <= tol


# --------------------------------------------------------------- selection

def test_select_hand_derived_cases(B):
    _say("select: hand-derived cut cases")
    ev, cuts, expect, names = cutcases.load()
    from paper_2211_14346_amd.binding import DeviceEvents
    dev = DeviceEvents(ev)
    for k, cut in enumerate(cuts):
        arr = B.cut_table([cut])
        order = torch.zeros(1, dtype=torch.int32, device="cuda")
        surv = torch.zeros(ev["n"], dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, 3, dtype=torch.int64, device="cuda")
        ws = B.workspace(B.lib().hf_select_workspace_size(ev["n"], 1))
        B.select(dev, arr, 1, order, surv, cnt, ws)
        got = surv.cpu().numpy()
        assert list(got) == list(expect[:, k]), (cut["name"], names)
        c = cnt.cpu().numpy()[0]
        assert c[0] == ev["n"] and c[1] == expect[:, k].sum()


def test_select_counters_follow_order(B, orc):
    _say("select: counters under random orders")
    ev, cuts, expect, names = cutcases.load()
    big = hfgen.generate("tth4M_v256", n_events=30000, seed=5)
    cfg = hfgen.config("tth4M_v256")
    from paper_2211_14346_amd.binding import DeviceEvents
    rng = np.random.default_rng(4)
    for sample, cl in ((ev, cuts), (big, cfg["cuts"])):
        dev = DeviceEvents(sample)
        arr = B.cut_table(cl)
        nc = len(cl)
        for _ in range(4):
            order = rng.permutation(nc).astype(np.int32)
            surv = torch.zeros(max(sample["n"], 1), dtype=torch.uint8, device="cuda")
            cnt = torch.zeros(nc, 3, dtype=torch.int64, device="cuda")
            ws = B.workspace(B.lib().hf_select_workspace_size(sample["n"], nc))
            B.select(dev, arr, nc, torch.from_numpy(order).cuda(), surv, cnt, ws)
            s_w, r_w, p_w = orc.select(sample, cl, order)
            assert np.array_equal(surv.cpu().numpy()[:sample["n"]], s_w)
            c = cnt.cpu().numpy()
            assert np.array_equal(c[:, 0].astype(np.uint64), r_w)
            assert np.array_equal(c[:, 1].astype(np.uint64), p_w)


@pytest.mark.parametrize("name,n", [("ttbar10k", 10000), ("ttbar1M_v64", 100003), ("stress2M_heavytail", 70001)])
def test_select_and_compact_samples(B, orc, name, n):
    _say("select+compact", name, n)
    cfg = hfgen.config(name)
    ev = hfgen.generate(cfg, n_events=n)
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cfg["cuts"], cfg["reco"], precision="mixed")
    ch.run_select()
    ch.run_compact()
    torch.cuda.synchronize()
    s_w, r_w, p_w = orc.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
    assert np.array_equal(ch.survive.cpu().numpy()[:n], s_w)
    S = int(ch.count.item())
    assert np.array_equal(ch.idx.cpu().numpy()[:S], np.flatnonzero(s_w))
    c = ch.counters_host()
    assert np.array_equal(c[:, 0], r_w) and np.array_equal(c[:, 1], p_w)


# -------------------------------------------------------------- compaction

@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 99991, (1 << 20) + 3, 64 * 8192 + 5])
def test_compact_adversarial(B, n):
    _say("compact n =", n)
    rng = np.random.default_rng(n)
    cap = max(n, 1)
    pats = {
        "zeros": np.zeros(n, np.uint8), "ones": np.ones(n, np.uint8),
        "alternate": (np.arange(n) % 2).astype(np.uint8),
        "every64": (np.arange(n) % 64 == 63).astype(np.uint8),
        "tile_edges": (np.isin(np.arange(n) % 8192, [0, 8191])).astype(np.uint8),
        "random": (rng.uniform(size=n) < 0.37).astype(np.uint8),
        "bytes": rng.integers(0, 256, n).astype(np.uint8),
    }
    ws = B.workspace(B.lib().hf_compact_workspace_size(cap + 1))
    for pname, m in pats.items():
        # a one-byte offset into the buffer exercises the unaligned load path
        for off in (0, 1):
            buf = torch.zeros(cap + 1, dtype=torch.uint8, device="cuda")
            buf[off:off + n] = torch.from_numpy(m).cuda()
            mask = buf[off:off + cap]
            idx = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            B.compact(mask, n, idx, cnt, ws, index_base=1000)
            torch.cuda.synchronize()
            want = np.flatnonzero(m) + 1000
            c = int(cnt.item())
            assert c == want.size, (pname, off)
            got = idx.cpu().numpy()
            assert np.array_equal(got[:c], want), (pname, off)
            assert np.all(got[c:] == -7), (pname, off)  # nothing written past the count
    # device-side length and an index map
    if n > 2:
        m = pats["random"]
        dn = torch.tensor([n // 2], dtype=torch.int64, device="cuda")
        mp = rng.integers(0, 2 ** 31 - 1, n).astype(np.int32)
        idx = torch.zeros(cap, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        B.compact(torch.from_numpy(m).cuda(), n, idx, cnt, ws, d_n=dn, mapping=torch.from_numpy(mp).cuda())
        torch.cuda.synchronize()
        want = mp[np.flatnonzero(m[: n // 2])]
        assert int(cnt.item()) == want.size
        assert np.array_equal(idx.cpu().numpy()[:want.size], want)


# ---------------------------------------------------------- reconstruction

def _full_chain_check(B, orc, name, n, precision, reco_over=None, min_within=1.0, seed=None, schedule="auto"):
    cfg = hfgen.config(name)
    ev = hfgen.generate(cfg, n_events=n, seed=seed)
    reco = dict(cfg["reco"])
    if reco_over:
        reco.update(reco_over)
    _say("chain", name, n, precision, reco_over, schedule)
    ch, got = _chain(ev, cfg["cuts"], reco, precision, schedule=schedule)
    want = orc.run_chain(ev, cfg["cuts"], reco)
    _check_selection(got, want, cfg["cuts"])
    st = compare(got["reco"], want["reco"])
    _say(st)
    assert_agree(st, min_within=min_within)
    # final compaction = compacted ids with a solution
    assert np.array_equal(got["final"], got["idx"][got["reco"]["has_sol"].astype(bool)])
    rid = [k for k, c in enumerate(cfg["cuts"]) if c["kind"] == "RECO"][0]
    assert got["counters"][rid, 0] == got["count"]
    assert got["counters"][rid, 1] == len(got["final"])
    return got, want, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reco_unsmeared_10k(B, orc, precision):
    _full_chain_check(B, orc, "ttbar10k", 10000, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reco_smeared_v64(B, orc, precision):
    _full_chain_check(B, orc, "ttbar1M_v64", 3000, precision, seed=77)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reco_tth_v256_mbb(B, orc, precision):
    got, want, st = _full_chain_check(B, orc, "tth4M_v256", 800, precision, seed=78)
    assert st.get("max_rel_m_bb", 0.0) <= 1e-9


@pytest.mark.parametrize("precision,schedule", [("fp64", "event"), ("mixed", "event"), ("mixed", "event_wg64")])
def test_reco_heavy_tailed_variations(B, orc, precision, schedule):
    _full_chain_check(B, orc, "stress2M_heavytail", 1500, precision, seed=79, schedule=schedule)


@pytest.mark.parametrize("precision,schedule", [("fp64", "event"), ("mixed", "event"), ("mixed", "event_wg128")])
def test_reco_uneven_variation_counts(B, orc, precision, schedule):
    """Per-event variation counts at the edges of the 64-lane passes: 1, a
    few, 63, 64, 65, 128 and large counts (up to 1024, sixteen passes of one
    wavefront), mixed with small random counts."""
    _say("uneven variation counts", precision, schedule)
    cfg = hfgen.config("ttbar1M_v64")
    ev = hfgen.generate(cfg, n_events=400, seed=93)
    rng = np.random.default_rng(93)
    fixed = [1024, 1, 2, 3, 700, 17, 64, 65, 128, 5, 16, 15, 33, 1000, 1, 1, 1, 1, 1, 1, 63, 900]
    nv = np.concatenate([fixed, rng.integers(1, 40, ev["n"] - len(fixed))]).astype(np.uint16)
    ev["n_var"] = nv
    reco = dict(cfg["reco"])
    ch, got = _chain(ev, cfg["cuts"], reco, precision, schedule=schedule)
    want = orc.run_chain(ev, cfg["cuts"], reco)
    _check_selection(got, want, cfg["cuts"])
    st = compare(got["reco"], want["reco"])
    _say(schedule, st)
    assert_agree(st, min_agree=0.999)
    stats = got["reco"]["stats"]
    assert stats[0] == got["count"] and stats[4] == got["reco"]["n_sol"].sum()


def _reco_direct(B, ev, ids, reco, precision, schedule, index_base=0):
    from paper_2211_14346_amd.binding import DeviceEvents, RecoOutputs
    dev = DeviceEvents(ev, index_base=index_base)
    S = len(ids)
    outs = RecoOutputs(S)
    p = B.reco_params(reco, precision=precision, reco_cut=0, schedule=schedule)
    ws = B.workspace(B.lib().hf_ttbar_reco_workspace_size(S))
    idx = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int32)).cuda()
    cnt = torch.tensor([S], dtype=torch.int64, device="cuda")
    B.ttbar_reco(dev, idx, cnt, S, p, outs, torch.zeros(1, 3, dtype=torch.int64, device="cuda"), ws)
    return outs.host(S), (dev, idx, cnt, S, p, outs, ws)


def test_event_counters_cover_every_position(B, orc):
    """The one-wavefront-per-event search takes its events from counters in
    the workspace header (one per class of blocks, cleared at every launch).
    With device counts far below the capacity, fewer blocks than classes,
    and launches repeated on one workspace, every position below the count
    must get the same result as in a run over all events, the statistics
    must count exactly those events, and positions past the count stay
    untouched."""
    _say("event counters")
    from paper_2211_14346_amd.binding import DeviceEvents, RecoOutputs
    cfg = hfgen.config("ttbar1M_v64")
    ev = hfgen.generate(cfg, n_events=3000, seed=97)
    s_w, _, _ = orc.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
    ids = np.flatnonzero(s_w)
    ref, _ = _reco_direct(B, ev, ids, cfg["reco"], "mixed", "event")
    keys = ("has_sol", "n_sol", "best_v", "best_i", "best_j", "nu", "nubar", "m_t", "m_tbar", "m_wp", "m_wm", "logw")
    dev = DeviceEvents(ev)
    cap = len(ids)
    idx = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int32)).cuda()
    p = B.reco_params(cfg["reco"], precision="mixed", reco_cut=0, schedule="event")
    ws = B.workspace(B.lib().hf_ttbar_reco_workspace_size(cap))
    # (device count, capacity); a count above the capacity is clamped to it
    for n, capacity in ((1, cap), (2, 5), (7, 7), (8, cap), (9, 9), (65, cap), (cap - 1, cap), (cap, cap),
                        (cap + 5, cap), (40, 31), (3, cap)):
        S = min(n, capacity)
        outs = RecoOutputs(cap)
        outs.t["has_sol"].fill_(7)
        cnt = torch.tensor([n], dtype=torch.int64, device="cuda")
        for rep in range(2):
            outs.t["stats"].zero_()
            B.ttbar_reco(dev, idx, cnt, capacity, p, outs, torch.zeros(1, 3, dtype=torch.int64, device="cuda"), ws)
            got = outs.host(cap)
            for k in keys:
                assert np.array_equal(got[k][:S], ref[k][:S]), (S, capacity, rep, k)
            assert np.all(got["has_sol"][S:] == 7), (S, capacity, "wrote past the count")
            assert got["stats"][0] == S, (S, capacity, got["stats"])
            assert got["stats"][4] == ref["n_sol"][:S].sum(), (S, capacity, got["stats"])


@pytest.mark.parametrize("name,n", [("stress2M_heavytail", 2000), ("ttbar1M_v64", 2000)])
def test_schedules_give_identical_results(B, orc, name, n):
    """The launch choices (workgroups of four, two or one wavefronts) run the
    same arithmetic per event; every output must be bit-identical."""
    _say("schedules", name)
    cfg = hfgen.config(name)
    ev = hfgen.generate(cfg, n_events=n, seed=94)
    s_w, _, _ = orc.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
    ids = np.flatnonzero(s_w)
    a, _ = _reco_direct(B, ev, ids, cfg["reco"], "mixed", "event")
    for sched in ("event_wg128", "event_wg64"):
        b, _ = _reco_direct(B, ev, ids, cfg["reco"], "mixed", sched)
        for k in ("has_sol", "n_sol", "best_v", "best_i", "best_j", "nu", "nubar", "m_t", "m_tbar", "m_wp", "m_wm",
                  "logw"):
            assert np.array_equal(a[k], b[k]), (sched, k)
        assert np.array_equal(a["stats"], b["stats"]), sched


def test_autotune_picks_a_schedule_and_caches_it(B, tmp_path, monkeypatch):
    _say("autotune")
    cache = tmp_path / "hf_tune.txt"
    monkeypatch.setenv("HF_AUTOTUNE_CACHE", str(cache))
    cfg = hfgen.config("stress2M_heavytail")
    ev = hfgen.generate(cfg, n_events=3000, seed=95)
    ids = np.arange(ev["n"], dtype=np.int32)
    ref, args = _reco_direct(B, ev, ids, cfg["reco"], "mixed", "event")
    dev, idx, cnt, S, p, outs, ws = args
    outs.t["has_sol"].fill_(7)
    ms = B.ttbar_reco_autotune(dev, idx, cnt, S, p, outs, ws)
    _say("autotune ms", ms, "->", p.schedule)
    assert all(m > 0 for m in ms)
    assert p.schedule == (1, 4, 3)[int(np.argmin(ms))]
    got = outs.host(S)
    for k in ("has_sol", "best_v", "nu", "logw"):
        assert np.array_equal(got[k], ref[k]), k
    line = cache.read_text().strip().splitlines()[-1].split()
    assert int(line[1]) == p.schedule and "per_event" in line[0]


def test_reco_all_jets_mode(B, orc):
    _full_chain_check(B, orc, "ttbar1M_v64", 1500, "mixed", reco_over={"pair_mode": "ALL_JETS", "n_var": 16},
                      seed=80)


def test_reco_ties_pick_first_variation(B, orc):
    # no smearing with several variations: all variations tie, the first wins
    got, want, st = _full_chain_check(B, orc, "ttbar10k", 3000, "mixed", reco_over={"n_var": 5}, seed=81)
    hs = got["reco"]["has_sol"].astype(bool)
    assert np.all(got["reco"]["best_v"][hs] == 0)
    assert np.all(got["reco"]["n_sol"] % 5 == 0)


def _edge_sample(extra=()):
    """Hand-built events covering the degenerate cases of the reconstruction
    (`extra`: more events, each {"leps": [[pt, eta, phi, e, q]...],
    "jets": [[pt, eta, phi, e, btag]...], "met": [x, y]}, appended)."""
    rng = np.random.default_rng(11)
    base = hfgen.generate("ttbar10k", n_events=64, keep_fp64=False, seed=12)
    evs = []
    for e in range(base["n"]):
        lo, hi = base["lep_off"][e], base["lep_off"][e + 1]
        jo, jh = base["jet_off"][e], base["jet_off"][e + 1]
        evs.append({"leps": [[base[k][i] for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q")]
                             for i in range(lo, hi)],
                    "jets": [[base[k][i] for k in ("jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag")]
                             for i in range(jo, jh)],
                    "met": [base["met_x"][e], base["met_y"][e]]})
    L = [[60, 0.3, 0.1, 60 * np.cosh(0.3), 1], [40, -0.7, 2.5, 40 * np.cosh(0.7), -1]]
    J = [[80, 0.5, -2.0, 80 * np.cosh(0.5), 1], [50, -1.0, 1.0, 50 * np.cosh(1.0), 1]]
    evs.append({"leps": [], "jets": J, "met": [40, 10]})                          # no leptons
    evs.append({"leps": L + [[30, 0, 0, 30, 1]], "jets": J, "met": [40, 10]})     # three leptons
    evs.append({"leps": [L[0], [40, -0.7, 2.5, 40 * np.cosh(0.7), 1]], "jets": J, "met": [40, 10]})  # same sign
    evs.append({"leps": L, "jets": [], "met": [40, 10]})                           # no jets
    evs.append({"leps": L, "jets": J[:1], "met": [40, 10]})                        # one jet
    many = [[300 - 4 * k, rng.uniform(-2.4, 2.4), rng.uniform(-3, 3), 0, float(k % 3 == 0)] for k in range(70)]
    for j in many:
        j[3] = j[0] * np.cosh(j[1])
    evs.append({"leps": L, "jets": many, "met": [40, 10]})                         # 70 jets (> one wave)
    evs.append({"leps": L, "jets": J, "met": [0, 0]})                              # zero MET
    # last: b exactly collinear with l+ and massless, so that side's 2x2 system is
    # singular (both forms stage the 4-vectors in FP64 and see the degeneracy)
    evs.append({"leps": L, "jets": [[90, 0.3, 0.1, 90 * np.cosh(0.3), 1], J[1]], "met": [40, 10]})
    evs.extend(extra)
    cols = {k: [] for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                            "jet_e", "jet_btag")}
    loff, joff, mx, my = [0], [0], [], []
    for d in evs:
        for o in d["leps"]:
            for k, v in zip(("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q"), o):
                cols[k].append(v)
        for o in d["jets"]:
            for k, v in zip(("jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag"), o):
                cols[k].append(v)
        loff.append(loff[-1] + len(d["leps"]))
        joff.append(joff[-1] + len(d["jets"]))
        mx.append(d["met"][0])
        my.append(d["met"][1])
    ev = {k: np.asarray(v, np.float32) for k, v in cols.items()}
    ev.update(n=len(evs), lep_off=np.asarray(loff, np.uint32), jet_off=np.asarray(joff, np.uint32),
              met_x=np.asarray(mx, np.float32), met_y=np.asarray(my, np.float32), n_var=None)
    return ev


@pytest.mark.parametrize("mode,precision", [("BTAG_FILL", "mixed"), ("ALL_JETS", "mixed"), ("ALL_JETS", "fp64")])
def test_reco_edge_cases(B, orc, mode, precision):
    _say("reco edge cases", mode, precision)
    ev = _edge_sample()
    reco = dict(hfgen.config("ttbar1M_v64")["reco"])
    reco.update(pair_mode=mode, n_var=8)
    from paper_2211_14346_amd.binding import DeviceEvents, RecoOutputs
    dev = DeviceEvents(ev, index_base=500)
    n = ev["n"]
    # every event, plus two ids outside the chunk (no solution expected)
    ids = np.concatenate([np.arange(n) + 500, [10, 500 + n]]).astype(np.int32)
    S = ids.size
    idx = torch.from_numpy(ids).cuda()
    cnt = torch.tensor([S], dtype=torch.int64, device="cuda")
    outs = RecoOutputs(S)
    counters = torch.zeros(1, 3, dtype=torch.int64, device="cuda")
    p = B.reco_params(reco, precision=precision, reco_cut=0)
    ws = B.workspace(B.lib().hf_ttbar_reco_workspace_size(S))
    B.ttbar_reco(dev, idx, cnt, S, p, outs, counters, ws)
    got = outs.host(S)
    want = orc.ttbar_reco(ev, ids[:n], reco, index_base=500)
    st = compare({k: v[:n] for k, v in got.items() if k != "stats"}, {k: v[:n] for k, v in want.items()
                                                                      if k != "n_pass"})
    _say(st)
    assert_agree(st, min_agree=1.0)
    assert np.all(got["has_sol"][n:] == 0)
    c = counters.cpu().numpy()[0]
    assert c[0] == S and c[1] == got["has_sol"].sum()


def test_reco_empty_and_zero_count(B):
    _say("empty chunk")
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("ttbar10k")
    ev = hfgen.generate(cfg, n_events=0)
    ch = Chain(ev, cfg["cuts"], cfg["reco"])
    ch.step()
    r = ch.results()
    assert r["count"] == 0 and len(r["final"]) == 0
    assert np.all(r["counters"][:, :2] == 0)


def test_full_size_bench_config_sampled(B, orc):
    """1M events, 64 variations, the launch configuration the benchmark times:
    selection bit-exact in full, properties of the reconstruction on every
    compacted event, and its most off-shell solutions against the oracle
    (the sampled agreement statistics are in test_gpu_fullsize.py)."""
    cfg = hfgen.config("ttbar1M_v64")
    ev = hfgen.generate(cfg)
    _say("full size", cfg["name"], ev["n"])
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cfg["cuts"], cfg["reco"], precision="mixed")
    ch.step()
    got = ch.results()
    s_w, r_w, p_w = orc.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
    assert np.array_equal(got["survive"], s_w)
    assert np.array_equal(got["idx"], np.flatnonzero(s_w))
    assert np.array_equal(got["counters"][:4, 0], r_w[:4]) and np.array_equal(got["counters"][:4, 1], p_w[:4])
    S = got["count"]
    r = got["reco"]
    hs = r["has_sol"].astype(bool)
    # Every accepted solution satisfies the mass constraints: a point is
    # accepted when both neutrinos' squared masses are within 2e-6 mW^2 of
    # zero, which bounds each mass's offset by 1e-6 relative; 2e-6 leaves room
    # for the rounding of the output masses.
    dev = np.zeros(S)
    for k, m in (("m_wp", 80.4), ("m_wm", 80.4), ("m_t", 172.5), ("m_tbar", 172.5)):
        d = np.abs(r[k] - m) / m
        dev = np.maximum(dev, np.where(hs, d, 0.0))
    assert dev.max() <= 2e-6, dev.max()
    # The most off-shell accepted solutions are the worst-conditioned ones:
    # close pairs of common points, mostly from a nearly degenerate l- conic
    # (lepton and b jet almost parallel along the beam), where the oracle's
    # expanded FP64 eliminant can lose a close root pair that the product's
    # pencil keeps.  The FP64 form sees the oracle's inputs: wherever its
    # choice differs, the 50-digit brute force must confirm that the product
    # chose a genuine solution scoring above the oracle's (a solution the
    # oracle missed).  The mixed form's FP32 draws differ from the oracle's at
    # the 1e-7 level, enough to make or remove a near-tangent intersection
    # here; it must take the same decision in every one of these events.
    worst = np.sort(np.argsort(-dev)[:32])
    sub = {k: v[worst] for k, v in r.items() if k != "stats"}
    want_w = orc.ttbar_reco(ev, got["idx"][worst], cfg["reco"])
    st_w = compare(sub, want_w)
    _say("most off-shell, mixed", float(dev.max()), st_w)
    assert st_w["decision_agree"] == 1.0, st_w
    ids = torch.from_numpy(np.ascontiguousarray(got["idx"][worst])).cuda()
    from paper_2211_14346_amd.binding import RecoOutputs
    outs = RecoOutputs(len(worst), want_mbb=False)
    ws = B.workspace(B.lib().hf_ttbar_reco_workspace_size(len(worst)))
    B.ttbar_reco(ch.dev, ids, torch.tensor([len(worst)], dtype=torch.int64, device="cuda"), len(worst),
                 B.reco_params(cfg["reco"], precision="fp64", reco_cut=0), outs,
                 torch.zeros(1, 3, dtype=torch.int64, device="cuda"), ws)
    g64 = {k: v for k, v in outs.host(len(worst)).items() if k != "stats"}
    st64 = compare(g64, want_w)
    _say("most off-shell, fp64", st64)
    mis = choice_mismatches(g64, want_w)
    settled = adjudicate(ev, got["idx"][worst], g64, want_w, cfg["reco"], mis)
    _say("fp64 choices differing from the oracle, settled by the brute force "
         "(pos, event, v, i, j, logw product, logw oracle, solutions):", settled)
    assert st64["decision_agree"] == 1.0 and len(mis) <= 8, st64
    assert st64["frac_within_1e-4"] == 1.0, st64
    assert np.array_equal(got["final"], got["idx"][hs])
    stats = r["stats"]
    assert stats[0] == S and stats[4] == r["n_sol"].sum() and stats[3] >= stats[4]


def test_graph_replay_matches_eager(B):
    _say("graph replay")
    cfg = hfgen.config("ttbar1M_v64")
    ev = hfgen.generate(cfg, n_events=20000, seed=90)
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cfg["cuts"], cfg["reco"], precision="mixed")
    ch.step()
    ref = ch.results()
    ch.capture()
    for rep in range(3):
        ch.reset_counters()
        ch.out.t["has_sol"].fill_(7)
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        ch.replay()
        torch.cuda.synchronize()
        r = ch.results()
        assert np.array_equal(r["survive"], ref["survive"]), rep
        assert np.array_equal(r["idx"], ref["idx"]), rep
        assert np.array_equal(r["final"], ref["final"]), rep
        for k in ("has_sol", "best_v", "best_i", "best_j", "n_sol", "nu", "nubar", "logw"):
            assert np.array_equal(r["reco"][k], ref["reco"][k]), (rep, k)
        assert np.array_equal(r["counters"][:, :2], ref["counters"][:, :2]), rep


def test_reorder_device_matches_host(B, orc):
    _say("device reorder")
    rng = np.random.default_rng(12)
    for name in ("ttbar10k", "tth4M_v256"):
        cuts = hfgen.config(name)["cuts"]
        n = len(cuts)
        deps = np.array(hfgen.dep_masks(cuts), dtype=np.uint64)
        arr = B.cut_table(cuts)
        order = torch.zeros(n, dtype=torch.int32, device="cuda")
        for _ in range(100):
            reached = rng.integers(0, 10 ** 6, n).astype(np.uint64)
            reached[rng.uniform(size=n) < 0.1] = 0
            passed = (reached * rng.uniform(0, 1, n)).astype(np.uint64)
            passed[rng.uniform(size=n) < 0.1] = 0  # some cuts reject everything they see
            cost = (reached * rng.uniform(0, 1000, n)).astype(np.uint64)
            cnt = np.stack([reached, passed, cost], axis=1)
            B.reorder_device(torch.from_numpy(cnt.view(np.int64)).cuda(), arr, n, order)
            got = order.cpu().numpy().tolist()
            assert got == B.reorder_stats(cnt, arr, n)
            assert got == list(orc.reorder(reached, passed, cost, deps))


def test_graph_with_device_reorder(B):
    """A recorded step that reorders its own cuts gives, replay after replay,
    the order the host rule gives for the same accumulated counters."""
    _say("graph with device reorder")
    cfg = hfgen.config("tth4M_v256")
    ev = hfgen.generate(cfg, n_events=20000, seed=92)
    from paper_2211_14346_amd.chain import Chain
    ch = Chain(ev, cfg["cuts"], cfg["reco"], precision="mixed")
    ch.capture(reorder=True)
    ch.reset_counters()
    ref = None
    for rep in range(4):
        before = ch.order.cpu().numpy().tolist()
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        ch.replay()
        torch.cuda.synchronize()
        r = ch.results()
        if ref is None:
            ref = r
        # the selection outcome does not depend on the order; the counters' reached column does
        assert np.array_equal(r["survive"], ref["survive"]) and np.array_equal(r["final"], ref["final"]), rep
        want = B.reorder_stats(ch.counters_host(), ch.cut_arr, ch.n_cuts)
        assert ch.order.cpu().numpy().tolist() == want, (rep, before, want)
    _say("device reorder: order after four steps", want)


def test_deterministic_repeat(B):
    _say("determinism")
    cfg = hfgen.config("stress2M_heavytail")
    ev = hfgen.generate(cfg, n_events=5000, seed=91)
    a = _chain(ev, cfg["cuts"], cfg["reco"], "mixed")[1]
    b = _chain(ev, cfg["cuts"], cfg["reco"], "mixed")[1]
    for k in ("has_sol", "best_v", "nu", "nubar", "logw", "n_sol"):
        assert np.array_equal(a["reco"][k], b["reco"][k]), k
