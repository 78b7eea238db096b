"""GPU parity of the chunked stream (two device slots filled from pinned
host memory on a copy stream while the compute stream runs the channels):
every chunk of a mixed HL-LHC-like sample through the five signal bins of
section 6.1, each with its reconstruction (section 6.2: the single-neutrino
chi^2 in the semileptonic ttbar, t-channel and Wt topologies, the
two-neutrino quartic at 64 variations for dileptonic ttbar, the chi^2 fit
with a MET split and one top for dileptonic Wt), against the FP64 oracle
under the cut order the GPU ran it with; counters accumulated over the
stream against the oracle's sums; hand-built events of known bin."""

import sys

import numpy as np
import pytest

import hfgen

from .gpu_compare import (assert_agree, assert_agree_semilep, compare, compare_chi2, compare_semilep)
from .test_oracle_bins import load_bin_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BIN_RECO = hfgen.configs.HLHC_BIN_RECO


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


def _channels(cfg, cap):
    from paper_2211_14346_amd.stream import Channel
    chans = []
    for name, cuts in cfg["chains"].items():
        kind, arg = BIN_RECO[name]
        if kind == "semilep":
            chans.append(Channel(name, cuts, cap, semilep=cfg["semilep"], topology=arg))
        elif kind == "chi2":
            chans.append(Channel(name, cuts, cap, chi2=dict(cfg["chi2"], n_top=arg)))
        else:
            chans.append(Channel(name, cuts, cap, reco=cfg["reco"]))
    return chans


def _oracle_reco(orc, cfg, name, ev, idx, base):
    kind, arg = BIN_RECO[name]
    if kind == "semilep":
        return orc.semilep_reco(ev, idx, cfg["semilep"], arg, index_base=base)
    if kind == "chi2":
        return orc.dilep_chi2_reco(ev, idx, dict(cfg["chi2"], n_top=arg), index_base=base)
    return orc.ttbar_reco(ev, idx, cfg["reco"], index_base=base)


def _check_reco(name, got, want):
    kind = BIN_RECO[name][0]
    if kind == "semilep":
        st = compare_semilep(got, want)
        _say(name, st)
        assert_agree_semilep(st)
    elif kind == "chi2":
        st = compare_chi2(got, want)
        _say(name, st)
        assert_agree_semilep(st)
    else:
        st = compare(got, want)
        _say(name, st)
        assert_agree(st)
    return st


def _setup(n_chunk, n_chunks, packed=False):
    from paper_2211_14346_amd.stream import EventStream, HostChunk
    cfg = hfgen.config("hlhc50M")
    samples = [hfgen.stream_chunk(cfg, i, n=n_chunk) for i in range(n_chunks)]
    chunks = [HostChunk(ev, base, packed=packed) for ev, base in samples]
    assert all(c.packed == bool(packed) for c in chunks)
    lep_cap = max(c.n_lep for c in chunks)
    jet_cap = max(c.n_jet for c in chunks) + 3  # ragged: slots larger than any chunk
    chans = _channels(cfg, n_chunk)
    es = EventStream(chans, n_chunk, lep_cap, jet_cap)
    return cfg, samples, chunks, chans, es


@pytest.mark.parametrize("packed", [False, True])
def test_stream_chunks_match_oracle(B, orc, packed):
    cfg, samples, chunks, chans, es = _setup(20011, 3, packed)
    sums = [np.zeros((ch.n_cuts, 2), dtype=np.uint64) for ch in chans]
    seen = []

    def check(i, hc, orders):
        ev, base = samples[i]
        _say("stream chunk", i, "orders", [list(o) for o in orders])
        for c, (ch, order) in enumerate(zip(chans, orders)):
            got = ch.results(hc.n)
            surv, reached, passed = orc.select(ev, ch.cuts, list(order), index_base=base)
            assert np.array_equal(got["survive"], surv), (ch.name, i)
            idx = orc.compact(surv, base)
            assert np.array_equal(got["idx"], idx), (ch.name, i)
            assert idx.size > 0, (ch.name, i)
            want = _oracle_reco(orc, cfg, ch.name, ev, idx, base)
            _check_reco(ch.name, got["reco"], want)
            # the final compaction keeps the GPU's own decisions (agreement checked above)
            assert np.array_equal(got["final"], idx[got["reco"]["has_sol"].astype(bool)]), (ch.name, i)
            r = ch.reco_id
            reached[r] += np.uint64(idx.size)
            passed[r] += np.uint64(got["reco"]["has_sol"].sum())
            sums[c][:, 0] += reached
            sums[c][:, 1] += passed
        seen.append(i)

    es.run(chunks, on_chunk=check)
    assert seen == [0, 1, 2]
    for c, ch in enumerate(chans):
        cnt = ch.counters.cpu().numpy().astype(np.uint64)
        assert np.array_equal(cnt[:, :2], sums[c]), ch.name


def test_stream_overlapped_matches_oracle(B, orc):
    """The same chunks with no host synchronisation between them (copies of
    one slot overlapping compute on the other).  The measured costs, and so
    the cut orders, vary from run to run; the orders each chunk ran under are
    logged on the device, and the counters accumulated over the stream must
    equal the oracle's under those orders.  The last chunk's results must
    equal the oracle's."""
    cfg, samples, chunks, chans, es = _setup(20000, 4)
    log = []
    es.run(chunks, order_log=log)
    torch.cuda.synchronize()
    assert len(log) == len(chunks)
    for c, ch in enumerate(chans):
        want = np.zeros((ch.n_cuts, 2), dtype=np.uint64)
        for i, (ev, base) in enumerate(samples):
            order = log[i][c].cpu().numpy()
            surv, reached, passed = orc.select(ev, ch.cuts, list(order), index_base=base)
            idx = orc.compact(surv, base)
            rec = _oracle_reco(orc, cfg, ch.name, ev, idx, base)
            reached[ch.reco_id] += np.uint64(idx.size)
            passed[ch.reco_id] += np.uint64(rec["has_sol"].sum())
            want[:, 0] += reached
            want[:, 1] += passed
        got = ch.counters.cpu().numpy().astype(np.uint64)[:, :2]
        _say(ch.name, "orders", [list(o[c].cpu().numpy()) for o in log])
        if ch.kind != "quartic":
            assert np.array_equal(got, want), ch.name
        else:
            # the dileptonic RECO decision is floating point (>= 99.9 % agreement)
            assert np.array_equal(np.delete(got, ch.reco_id, 0), np.delete(want, ch.reco_id, 0)), ch.name
            assert got[ch.reco_id, 0] == want[ch.reco_id, 0]
            assert abs(int(got[ch.reco_id, 1]) - int(want[ch.reco_id, 1])) <= 1e-3 * want[ch.reco_id, 0]
        last = ch.results(chunks[-1].n)
        ev, base = samples[-1]
        surv, _, _ = orc.select(ev, ch.cuts, list(range(ch.n_cuts)), index_base=base)
        assert np.array_equal(last["survive"], surv), ch.name


def test_bins_hand_derived_on_the_gpu(B, orc):
    """The hand-built events of known bin (golden/bin_cases.json) through the
    five channels: every bin's survive mask as derived by hand, and each
    bin's reconstruction against the oracle."""
    from paper_2211_14346_amd.stream import EventStream, HostChunk
    cfg = hfgen.config("hlhc50M")
    ev, cases = load_bin_cases()
    hc = HostChunk(ev, 300)
    chans = _channels(cfg, ev["n"])
    es = EventStream(chans, ev["n"], hc.n_lep, hc.n_jet)
    es.run([hc])
    torch.cuda.synchronize()
    for ch in chans:
        got = ch.results(ev["n"])
        want = np.array([c["expect"][ch.name] for c in cases], dtype=np.uint8)
        bad = [c["name"] for c, g, w in zip(cases, got["survive"], want) if g != w]
        assert not bad, (ch.name, bad)
        idx = np.flatnonzero(want).astype(np.int32) + 300
        assert np.array_equal(got["idx"], idx), ch.name
        _check_reco(ch.name, got["reco"], _oracle_reco(orc, cfg, ch.name, ev, idx, 300))


@pytest.mark.parametrize("n", [0, 1, 17, 20011, 70000])
def test_unpack_events_bit_exact(B, n):
    """hf_unpack_events rebuilds offsets, charges and b-tags exactly."""
    from paper_2211_14346_amd.stream import pack_plan
    cfg = hfgen.config("hlhc50M")
    ev = hfgen.generate(cfg, n_events=n, seed=600 + n)
    assert pack_plan(ev)
    lc = np.diff(ev["lep_off"].astype(np.int64)).astype(np.uint8)
    jc = np.diff(ev["jet_off"].astype(np.int64)).astype(np.uint8)
    n_lep, n_jet = int(ev["lep_off"][-1]), int(ev["jet_off"][-1])
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dt).cuda() if a.size else \
        torch.zeros(16, dtype=dt, device="cuda")
    d_lc = torch.zeros(max(16, n + 16), dtype=torch.uint8, device="cuda")
    d_jc = torch.zeros(max(16, n + 16), dtype=torch.uint8, device="cuda")
    if n:
        d_lc[:n] = torch.as_tensor(lc).cuda()
        d_jc[:n] = torch.as_tensor(jc).cuda()
    q8 = dev(ev["lep_q"].astype(np.int8), torch.int8)
    b8 = dev(ev["jet_btag"].astype(np.uint8), torch.uint8)
    loff = torch.full((n + 1,), -1, dtype=torch.int32, device="cuda")
    joff = torch.full((n + 1,), -1, dtype=torch.int32, device="cuda")
    q = torch.full((max(1, n_lep),), 9.0, dtype=torch.float32, device="cuda")
    b = torch.full((max(1, n_jet),), 9.0, dtype=torch.float32, device="cuda")
    ws = B.workspace(B.lib().hf_unpack_workspace_size(n))
    B.unpack_events(n, d_lc, d_jc, n_lep, n_jet, q8, b8, loff, joff, q, b, ws)
    torch.cuda.synchronize()
    assert np.array_equal(loff.cpu().numpy().astype(np.int64), ev["lep_off"].astype(np.int64))
    assert np.array_equal(joff.cpu().numpy().astype(np.int64), ev["jet_off"].astype(np.int64))
    assert np.array_equal(q.cpu().numpy()[:n_lep], ev["lep_q"].astype(np.float32))
    assert np.array_equal(b.cpu().numpy()[:n_jet], ev["jet_btag"].astype(np.float32))
