"""GPU parity of segmented cut chains (hf_select_segment,
hf_chain_select_segment): the cuts at the first s positions of the order run
over all events, the rest over the compacted survivors; survivors and
per-cut counters must equal one unsegmented pass and the oracle, for every
split point, built-in and user-compiled chains, and graph replay."""

import sys

import numpy as np
import pytest

import hfgen

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


def _select_only(ch):
    ch.run_select()
    ch.run_compact()
    torch.cuda.synchronize()
    S = int(ch.count.item())
    return ch.idx[:S].cpu().numpy(), ch.counters.cpu().numpy()


@pytest.mark.parametrize("seg", [0, 2, 4, 7, 8])
def test_segmented_tth8_chain(B, orc, seg):
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("tth4M_v256")
    ev = hfgen.generate(cfg, n_events=60000, seed=501)
    _say("segmented tth8", seg)
    rng = np.random.default_rng(seg)
    for rep in range(2):
        order = list(range(len(cfg["cuts"]))) if rep == 0 else list(rng.permutation(len(cfg["cuts"])))
        ref = Chain(ev, cfg["cuts"], cfg["reco"], order=order)
        ch = Chain(ev, cfg["cuts"], cfg["reco"], order=order, segment_at=seg)
        i_ref, c_ref = _select_only(ref)
        i_seg, c_seg = _select_only(ch)
        assert np.array_equal(i_seg, i_ref), (seg, order)
        assert np.array_equal(c_seg[:, :2], c_ref[:, :2]), (seg, order)
        s_w, r_w, p_w = orc.select(ev, cfg["cuts"], order)
        assert np.array_equal(i_seg, np.flatnonzero(s_w))
        assert np.array_equal(c_seg[:, 0], r_w) and np.array_equal(c_seg[:, 1], p_w)


def test_segmented_full_step_and_graph(B):
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("tth4M_v256")
    ev = hfgen.generate(cfg, n_events=30000, seed=502)
    reco = dict(cfg["reco"], n_var=16)
    ref = Chain(ev, cfg["cuts"], reco)
    ref.step()
    want = ref.results()
    ch = Chain(ev, cfg["cuts"], reco, segment_at=3)
    ch.step()
    got = ch.results()
    assert np.array_equal(got["final"], want["final"])
    for k in ("best_v", "best_i", "best_j", "nu", "logw"):
        assert np.array_equal(got["reco"][k], want["reco"][k]), k
    ch.capture()
    for rep in range(3):
        ch.reset_counters()
        ch.out.t["has_sol"].fill_(5)
        ch.replay()
        torch.cuda.synchronize()
        r = ch.results()
        assert np.array_equal(r["final"], want["final"])
        assert np.array_equal(r["counters"][:, :2], want["counters"][:, :2])


def test_segmented_user_chain(B, orc):
    from paper_2211_14346_amd.chain import Chain
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 21, n=50000)
    cuts = hfgen.configs.chain_user_mix()
    reco = dict(hfgen.config("ttbar10k")["reco"])
    ch = Chain(ev, cuts, reco, segment_at=3)
    i_seg, c_seg = _select_only(ch)
    s_w, r_w, p_w = orc.select(ev, cuts, list(range(len(cuts))))
    assert np.array_equal(i_seg, np.flatnonzero(s_w))
    assert np.array_equal(c_seg[:, 0], r_w) and np.array_equal(c_seg[:, 1], p_w)
