"""GPU parity of cut chains with user predicates compiled at run time
(hf_chain_compile / hf_chain_select): survive masks and per-cut counters
bit-exact against the oracle (which compiles the same predicate bodies with
gcc) for several orders; user restatements of built-in cuts equal to the
library's own chain kernel; graph replay; an empty chunk."""

import sys

import numpy as np
import pytest

import hfgen
from hfgen.configs import USER_CUTS, _cut, _user

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


def _buffers(B, ev, n_cuts):
    dev = B.DeviceEvents(ev)
    n = max(1, dev.n)
    surv = torch.zeros(n, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(n_cuts, 3, dtype=torch.int64, device="cuda")
    ws = B.workspace(B.lib().hf_select_workspace_size(dev.n, n_cuts))
    return dev, surv, cnt, ws


@pytest.mark.parametrize("seed", [0, 1])
def test_user_chain_matches_oracle(B, orc, seed):
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 11 + seed, n=60000)
    cuts = hfgen.configs.chain_user_mix()
    _say("user chain", seed, [c["name"] for c in cuts])
    ch = B.CompiledChain(cuts)
    dev, surv, cnt, ws = _buffers(B, ev, len(cuts))
    rng = np.random.default_rng(seed)
    for rep in range(3):
        order = list(rng.permutation(len(cuts))) if rep else list(range(len(cuts)))
        # the dependencies of U_LEAD40 and MLL40 on U_LEP2OS do not bind a
        # given order here: both implementations take the order as given
        cnt.zero_()
        B.chain_select(ch, dev, torch.tensor(order, dtype=torch.int32, device="cuda"), surv, cnt, ws)
        torch.cuda.synchronize()
        s_w, r_w, p_w = orc.select(ev, cuts, order)
        assert np.array_equal(surv[:ev["n"]].cpu().numpy(), s_w), order
        c = cnt.cpu().numpy()
        assert np.array_equal(c[:, 0], r_w) and np.array_equal(c[:, 1], p_w), order
        assert np.all(c[:, 2][r_w > 0] > 0)  # costs measured for every reached cut


def test_user_restatements_equal_library_kernel(B):
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 3, n=50000)
    user = [_user(k, USER_CUTS[k]) for k in ("U_LEP2OS", "U_JETS2", "U_MET30")]
    builtin = [_cut("LEP2OS", "LEP_N_OS", [20.0, 2.5], [2, 1]), _cut("JETS2", "JET_N_MIN", [25.0, 2.5], [2]),
               _cut("MET30", "MET_MIN", [30.0])]
    ch = B.CompiledChain(user)
    dev, s_u, c_u, ws = _buffers(B, ev, 3)
    order = torch.arange(3, dtype=torch.int32, device="cuda")
    B.chain_select(ch, dev, order, s_u, c_u, ws)
    s_b = torch.zeros_like(s_u)
    c_b = torch.zeros_like(c_u)
    B.select(dev, B.cut_table(builtin), 3, order, s_b, c_b, ws)
    torch.cuda.synchronize()
    assert torch.equal(s_u, s_b)
    assert torch.equal(c_u[:, :2], c_b[:, :2])
    # a chain of built-in cuts only, compiled at run time, is the library's kernel too
    ch0 = B.CompiledChain(builtin)
    s_0 = torch.zeros_like(s_u)
    c_0 = torch.zeros_like(c_u)
    B.chain_select(ch0, dev, order, s_0, c_0, ws)
    torch.cuda.synchronize()
    assert torch.equal(s_0, s_b) and torch.equal(c_0[:, :2], c_b[:, :2])


def test_user_chain_graph_replay(B):
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 5, n=30000)
    cuts = hfgen.configs.chain_user_mix()
    ch = B.CompiledChain(cuts)
    dev, surv, cnt, ws = _buffers(B, ev, len(cuts))
    order = torch.arange(len(cuts), dtype=torch.int32, device="cuda")
    B.chain_select(ch, dev, order, surv, cnt, ws)
    torch.cuda.synchronize()
    ref_s, ref_c = surv.clone(), cnt.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.chain_select(ch, dev, order, surv, cnt, ws, s)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.chain_select(ch, dev, order, surv, cnt, ws)
    for rep in range(3):
        surv.fill_(9)
        cnt.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(surv, ref_s), rep
        assert torch.equal(cnt[:, :2], ref_c[:, :2]), rep


def test_user_chain_empty_chunk(B):
    ev = hfgen.generate("hlhc50M", n_events=0)
    cuts = hfgen.configs.chain_user_mix()
    ch = B.CompiledChain(cuts)
    dev, surv, cnt, ws = _buffers(B, ev, len(cuts))
    B.chain_select(ch, dev, torch.arange(len(cuts), dtype=torch.int32, device="cuda"), surv, cnt, ws)
    torch.cuda.synchronize()
    assert np.all(cnt.cpu().numpy()[:, :2] == 0)


def test_loop_budgets_match_oracle(B, orc):
    """Budgeted loops (every loop here ends after at most 1000 iterations, so
    a run cannot hang whatever the budget does): at the budget each predicate
    passes, one unit below it fails, and a loop over the event's jets with a
    budget of 3 fails exactly the events with more than three jets; masks and
    counters equal the oracle's."""
    from .test_oracle_usercuts import LOOPS
    cfg = hfgen.config("hlhc50M")
    ev, _ = hfgen.stream_chunk(cfg, 13, n=20000)
    jets = "int n = 0; for (int k = 0; k < n_jet(); ++k) n += jet_pt(k) > 25.0f; return n >= 0;"
    cuts = []
    for name, src, units in LOOPS:
        cuts.append(_user(f"U_{name}_at", src, budget=units))
        cuts.append(_user(f"U_{name}_below", src, budget=units - 1))
    cuts.append(_user("U_jets3", jets, budget=3))
    _say("loop budgets", [c["name"] for c in cuts])
    ch = B.CompiledChain(cuts)
    dev, surv, cnt, ws = _buffers(B, ev, len(cuts))
    n = ev["n"]
    for k, c in enumerate(cuts):
        # cut k first: its own counters give its pass count over every event
        order = [k] + [j for j in range(len(cuts)) if j != k]
        cnt.zero_()
        B.chain_select(ch, dev, torch.tensor(order, dtype=torch.int32, device="cuda"), surv, cnt, ws)
        torch.cuda.synchronize()
        s_w, r_w, p_w = orc.select(ev, cuts, order)
        c_g = cnt.cpu().numpy()
        assert np.array_equal(surv[:n].cpu().numpy(), s_w), c["name"]
        assert np.array_equal(c_g[:, 0], r_w) and np.array_equal(c_g[:, 1], p_w), c["name"]
        assert c_g[k, 0] == n
        if c["name"] == "U_jets3":
            assert c_g[k, 1] == int((np.diff(np.asarray(ev["jet_off"])) <= 3).sum())
        else:
            assert c_g[k, 1] == (n if c["name"].endswith("_at") else 0), c["name"]
