"""C-ABI checks that need no GPU: libhf loads, exports every entry point
include/hf.h declares, its structures have the documented layout, host-side
validation rejects malformed calls before touching the device, and the host
reorder entry point agrees with the oracle."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import hfgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hf.h")


@pytest.fixture(scope="module")
def B():
    from paper_2211_14346_amd import binding
    binding.lib()
    return binding


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hf_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(B):
    names = _declared()
    assert "hf_select" in names and "hf_ttbar_reco" in names and "hf_reorder_stats" in names
    L = B.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in hf.h but not exported"


def test_struct_layouts(B):
    assert C.sizeof(B.Cut) == 64
    assert C.sizeof(B.Counters) == 24
    assert C.sizeof(B.RecoParams) == 120
    assert C.sizeof(B.Events) == 16 + 8 * 15
    assert C.sizeof(B.RecoOut) == 8 * 14


def test_workspace_queries(B):
    L = B.lib()
    assert L.hf_select_workspace_size(1000, 5) > 0
    assert L.hf_select_workspace_size(-1, 5) == 0
    assert L.hf_select_workspace_size(10, 0) == 0
    assert L.hf_compact_workspace_size(0) >= 8
    assert L.hf_compact_workspace_size(10 ** 6) > L.hf_compact_workspace_size(10)
    assert L.hf_ttbar_reco_workspace_size(10 ** 6) > 0


def test_validation_errors_are_reported(B):
    L = B.lib()
    cuts = B.cut_table(hfgen.config("ttbar10k")["cuts"])
    ev = B.Events(n=10, index_base=0)
    dummy = C.c_void_p(16)  # never dereferenced: validation fails first
    # NULL event columns
    rc = L.hf_select(C.byref(ev), C.cast(cuts, C.c_void_p), 5, dummy, dummy, dummy, dummy, 1 << 20, None)
    assert rc == -1 and b"NULL" in L.hf_last_error()
    # bad cut count
    rc = L.hf_select(C.byref(ev), C.cast(cuts, C.c_void_p), 0, dummy, dummy, dummy, dummy, 1 << 20, None)
    assert rc == -1
    # unknown cut kind
    bad = B.cut_table(hfgen.config("ttbar10k")["cuts"])
    bad[0].kind = 99
    rc = L.hf_select(C.byref(ev), C.cast(bad, C.c_void_p), 5, dummy, dummy, dummy, dummy, 1 << 20, None)
    assert rc == -1 and b"kind" in L.hf_last_error()
    # compaction: short workspace, negative capacity
    rc = L.hf_compact(dummy, 1000, None, 0, None, dummy, dummy, dummy, 1, None)
    assert rc == -2
    rc = L.hf_compact(dummy, -1, None, 0, None, dummy, dummy, dummy, 1 << 20, None)
    assert rc == -1
    # reconstruction: bad precision / pair mode / candidate cap
    full = B.Events(n=10, index_base=0, **{k: 16 for k in ("lep_off", "jet_off", "lep_pt", "lep_eta", "lep_phi",
                                                            "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                                                            "jet_e", "jet_btag", "met_x", "met_y")})
    out = B.RecoOut(**{k: 16 for k in ("has_sol", "n_sol", "best_v", "best_i", "best_j", "nu", "nubar", "m_t",
                                       "m_tbar", "m_wp", "m_wm", "logw", "m_bb", "stats")})
    reco = hfgen.config("ttbar10k")["reco"]
    for field, val in (("precision", 7), ("pair_mode", 5), ("max_cands", 40), ("n_var_uniform", 0), ("smear", 3)):
        p = B.reco_params(reco)
        setattr(p, field, val)
        rc = L.hf_ttbar_reco(C.byref(full), dummy, dummy, 10, C.byref(p), C.byref(out), None, dummy, 1 << 20, None)
        assert rc == -1, field
    p = B.reco_params(reco)
    rc = L.hf_ttbar_reco(C.byref(full), dummy, dummy, 10, C.byref(p), C.byref(out), None, dummy, 0, None)
    assert rc == -2
    # RNG entry points
    assert L.hf_philox_blocks(None, 0, None, 5, None) == -1
    assert L.hf_gauss_draws(0, dummy, dummy, dummy, 5, 9, dummy, None) == -1


def test_reorder_matches_oracle(B, orc):
    rng = np.random.default_rng(8)
    for name in ("ttbar10k", "tth4M_v256"):
        cuts = hfgen.config(name)["cuts"]
        n = len(cuts)
        deps = np.array(hfgen.dep_masks(cuts), dtype=np.uint64)
        arr = B.cut_table(cuts)
        for _ in range(200):
            reached = rng.integers(0, 10 ** 6, n).astype(np.uint64)
            reached[rng.uniform(size=n) < 0.1] = 0
            passed = (reached * rng.uniform(0, 1, n)).astype(np.uint64)
            cost = (reached * rng.uniform(0, 1000, n)).astype(np.uint64)
            cnt = np.stack([reached, passed, cost], axis=1)
            got = B.reorder_stats(cnt, arr, n)
            want = orc.reorder(reached, passed, cost, deps)
            assert list(got) == list(want)


def test_reorder_rejects_cycles(B):
    cuts = [{"name": "a", "kind": "MET_MIN", "f": [1], "deps": ["b"]},
            {"name": "b", "kind": "MET_MIN", "f": [1], "deps": ["a"]}]
    arr = B.cut_table(cuts)
    with pytest.raises(B.HFError):
        B.reorder_stats(np.zeros((2, 3), dtype=np.uint64), arr, 2)


def test_reorder_device_validates_on_the_host(B):
    """Errors are reported before anything is launched (no GPU needed)."""
    import ctypes as C
    L = B.lib()
    cuts = [{"name": "a", "kind": "MET_MIN", "f": [1], "deps": ["b"]},
            {"name": "b", "kind": "MET_MIN", "f": [1], "deps": ["a"]}]
    arr = B.cut_table(cuts)
    dummy = C.c_void_p(16)
    cyc = C.cast(arr, C.c_void_p)
    assert L.hf_reorder_device(dummy, cyc, 2, dummy, None) == -1  # cyclic
    assert L.hf_reorder_device(None, cyc, 2, dummy, None) == -1
    assert L.hf_reorder_device(dummy, None, 2, dummy, None) == -1
    assert L.hf_reorder_device(dummy, cyc, 0, dummy, None) == -1
    assert L.hf_reorder_device(dummy, cyc, 33, dummy, None) == -1
    # a dependency on a cut beyond n_cuts: b depends on a, only b is passed
    two = B.cut_table([{"name": "b", "kind": "MET_MIN", "f": [1], "deps": ["a"]},
                       {"name": "a", "kind": "MET_MIN", "f": [1], "deps": []}])
    assert L.hf_reorder_device(dummy, C.cast(two, C.c_void_p), 1, dummy, None) == -1


def test_semilep_validation(B):
    L = B.lib()
    full = B.Events(n=10, index_base=0, **{k: 16 for k in ("lep_off", "jet_off", "lep_pt", "lep_eta", "lep_phi",
                                                           "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                                                           "jet_e", "jet_btag", "met_x", "met_y")})
    dummy = C.c_void_p(16)
    sl = hfgen.config("tchan1M")["semilep"]
    out = B.SemilepOut(**{k: 16 for k, _ in B.SemilepOut._fields_})

    def call(p, o=out, ev=full, count=dummy):
        return L.hf_semilep_reco(C.byref(ev), dummy, count, 10, C.byref(p), C.byref(o), None, None)

    assert C.sizeof(B.SemilepParams) == 64 and C.sizeof(B.SemilepOut) == 8 * 12
    for field, val, word in (("topology", 3, b"topology"), ("max_cands", 0, b"max_cands"),
                             ("max_cands", 13, b"max_cands"), ("sigma_t", 0.0, b"widths"),
                             ("sigma_w", float("nan"), b"widths"), ("m_w", 200.0, b"masses"),
                             ("reserved", 1, b"reserved")):
        p = B.semilep_params(sl)
        setattr(p, field, val)
        assert call(p) == -1 and word in L.hf_last_error(), field
    p = B.semilep_params(sl)
    assert call(p, count=None) == -1
    bad = B.SemilepOut(**{k: 16 for k, _ in B.SemilepOut._fields_})
    bad.chi2 = None
    assert call(p, o=bad) == -1 and b"NULL" in L.hf_last_error()
    assert call(p, ev=B.Events(n=10, index_base=0)) == -1


def test_user_chain_validation(B):
    L = B.lib()
    user = [{"name": "U", "kind": "USER", "f": [], "i": [], "deps": [], "src": "return n_jet() >= 2;"}]
    arr = B.cut_table(user)
    srcs = (C.c_char_p * 1)(b"return n_jet() >= 2;")
    h = C.c_void_p()
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(srcs, C.c_void_p), 1, None) == -1
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, None, 1, C.byref(h)) == -1
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(srcs, C.c_void_p), 0, C.byref(h)) == -1
    assert b"user source" in L.hf_last_error() and not h.value
    bad = (C.c_char_p * 1)(b"return n_jet( > 2;")
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(bad, C.c_void_p), 1, C.byref(h)) == -1
    assert b"do not compile" in L.hf_last_error() and b"error" in L.hf_last_error() and not h.value
    noret = (C.c_char_p * 1)(b"int x = n_jet(); (void)x;")
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(noret, C.c_void_p), 1, C.byref(h)) == -1
    # a valid source compiles here; loading it needs a device (HF_ERR_DEVICE without one)
    rc = L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(srcs, C.c_void_p), 1, C.byref(h))
    assert rc in (0, -3), L.hf_last_error()
    if rc == 0:
        L.hf_chain_destroy(h)
    else:
        assert not h.value
    L.hf_chain_destroy(None)
    # a negative loop budget is refused before compiling; goto does not compile
    neg = B.cut_table([dict(user[0], i=[0, -1])])
    assert L.hf_chain_compile(C.cast(neg, C.c_void_p), 1, C.cast(srcs, C.c_void_p), 1, C.byref(h)) == -1
    assert b"loop budget" in L.hf_last_error() and not h.value
    jump = (C.c_char_p * 1)(b"again: goto again; return 1;")
    assert L.hf_chain_compile(C.cast(arr, C.c_void_p), 1, C.cast(jump, C.c_void_p), 1, C.byref(h)) == -1
    assert b"goto" in L.hf_last_error() and not h.value
    # the library's own chain kernel refuses user cuts
    dummy = C.c_void_p(16)
    ev = B.Events(n=10, index_base=0)
    assert L.hf_select(C.byref(ev), C.cast(arr, C.c_void_p), 1, dummy, dummy, dummy, dummy, 1 << 20, None) == -1
    assert b"hf_chain_compile" in L.hf_last_error()
    assert L.hf_chain_select(None, C.byref(ev), dummy, dummy, dummy, dummy, 1 << 20, None) == -1


def test_segment_validation(B):
    L = B.lib()
    full = B.Events(n=10, index_base=0, **{k: 16 for k in ("lep_off", "jet_off", "lep_pt", "lep_eta", "lep_phi",
                                                           "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                                                           "jet_e", "jet_btag", "met_x", "met_y")})
    cuts = B.cut_table(hfgen.config("ttbar10k")["cuts"])
    d = C.c_void_p(16)

    def call(pb, pe, idx=None, cnt=None, cap=10, ws=1 << 20):
        return L.hf_select_segment(C.byref(full), C.cast(cuts, C.c_void_p), 5, d, pb, pe, idx, cnt, cap, d, d, d, ws,
                                   None)

    assert call(-1, 2) == -1 and call(3, 2) == -1 and call(0, 6) == -1
    assert call(0, 2, idx=d) == -1 and b"d_count" in L.hf_last_error()
    assert call(0, 2, idx=d, cnt=d, cap=-1) == -1
    assert call(0, 2, ws=0) == -2
    assert L.hf_chain_select_segment(None, C.byref(full), d, 0, 1, None, None, 0, d, d, d, 1 << 20, None) == -1
