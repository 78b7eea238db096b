"""hf_compact_noalloc (workspace held by the library) against hf_compact.

Two calls in a row on one device, the second with a smaller input, so the
second call runs on the status words the first one left behind; each output
must equal what hf_compact gives for the same mask with a workspace passed
in (integer work: bit-exact).
"""

import sys

import numpy as np
import pytest

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


def _both(B, m, index_base=0, d_n=None, mapping=None):
    n = m.size
    cap = max(n, 1)
    mask = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    mask[:n] = torch.from_numpy(m).cuda()
    out = {}
    for which in ("ws", "noalloc"):
        idx = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        if which == "ws":
            ws = B.workspace(B.lib().hf_compact_workspace_size(cap))
            B.compact(mask, n, idx, cnt, ws, d_n=d_n, index_base=index_base, mapping=mapping)
        else:
            B.compact_noalloc(mask, n, idx, cnt, d_n=d_n, index_base=index_base, mapping=mapping)
        torch.cuda.synchronize()
        out[which] = (int(cnt.item()), idx.cpu().numpy())
    return out


def test_noalloc_matches_workspace_entry_two_calls(B):
    rng = np.random.default_rng(7)
    # first call: many tiles and a ragged tail; second call: smaller, so the
    # library's status words still hold the first call's values for later tiles
    for n, p in ((3_000_017, 0.41), (70_001, 0.63)):
        _say("compact_noalloc n =", n)
        m = (rng.uniform(size=n) < p).astype(np.uint8)
        out = _both(B, m, index_base=11)
        c_ws, i_ws = out["ws"]
        c_na, i_na = out["noalloc"]
        assert c_na == c_ws == int(m.sum())
        assert np.array_equal(i_na, i_ws)
        assert np.array_equal(i_na[:c_na], np.flatnonzero(m) + 11)


def test_noalloc_device_length_and_map(B):
    rng = np.random.default_rng(8)
    n = 200_003
    m = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    dn = torch.tensor([n // 3], dtype=torch.int64, device="cuda")
    mp = torch.from_numpy(rng.integers(0, 2 ** 31 - 1, n).astype(np.int32)).cuda()
    _say("compact_noalloc with device length and map, n =", n)
    out = _both(B, m, d_n=dn, mapping=mp)
    assert out["noalloc"][0] == out["ws"][0]
    assert np.array_equal(out["noalloc"][1], out["ws"][1])
    # an empty mask after a non-empty one
    out = _both(B, np.zeros(0, np.uint8))
    assert out["noalloc"][0] == out["ws"][0] == 0
    assert np.array_equal(out["noalloc"][1], out["ws"][1])


def test_noalloc_rejects_capacity_above_maximum(B):
    import ctypes
    L = B.lib()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    dummy = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = L.hf_compact_noalloc(ctypes.c_void_p(dummy.data_ptr()), (1 << 28) + 1, None, 0, None,
                              ctypes.c_void_p(dummy.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), None)
    assert B.HF_ERR.get(rc) == "HF_ERR_CAPACITY"
    assert b"maximum" in L.hf_last_error()
