"""ctypes binding of libhf (include/hf.h).  Argument marshalling only: every
step of the path runs in the HIP kernels behind the C ABI; PyTorch supplies
device memory and the stream.  Importing fails loudly if libhf.so is absent.
"""

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhf.so")

HF_OK = 0
HF_ERR = {-1: "HF_ERR_INVAL", -2: "HF_ERR_CAPACITY", -3: "HF_ERR_DEVICE", -4: "HF_ERR_UNSUPPORTED"}
HF_MAX_CUTS = 32
HF_MAX_CANDS = 12
HF_NO_SOLUTION = -9999.0
CUT_KIND = {"LEP_N_OS": 0, "JET_N_MIN": 1, "BTAG_N_MIN": 2, "BTAG_N_EQ": 3, "MET_MIN": 4, "MLL_MIN": 5,
            "FWD_JET_VETO": 6, "LEP_ISO": 7, "RECO": 8, "MTW_MIN": 9, "USER": 10, "JET_N_RANGE": 11}
PREC = {"fp64": 0, "mixed": 1}
PAIR = {"BTAG_FILL": 0, "ALL_JETS": 1}


class HFError(RuntimeError):
    pass


class Events(C.Structure):
    _fields_ = [("n", C.c_int64), ("index_base", C.c_int64), ("lep_off", C.c_void_p), ("jet_off", C.c_void_p)] + \
               [(k, C.c_void_p) for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q", "jet_pt", "jet_eta",
                                          "jet_phi", "jet_e", "jet_btag", "met_x", "met_y", "n_var")]


class Cut(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("dep_mask", C.c_uint64), ("f", C.c_float * 8),
                ("i", C.c_int32 * 4)]


class Counters(C.Structure):
    _fields_ = [("reached", C.c_uint64), ("passed", C.c_uint64), ("cost", C.c_uint64)]


class RecoParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "lambda_pt", "jet_a", "jet_c", "lep_sigma",
                                          "met_sigma")] + \
               [(k, C.c_float) for k in ("lep_pt_min", "lep_eta_max", "jet_pt_min", "jet_eta_max", "btag_min")] + \
               [("reco_cut", C.c_int32), ("seed", C.c_uint64)] + \
               [(k, C.c_int32) for k in ("smear", "n_var_uniform", "precision", "pair_mode", "max_cands",
                                         "want_mbb", "schedule", "reserved")]


class RecoOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "n_sol", "best_v", "best_i", "best_j", "nu", "nubar", "m_t",
                                          "m_tbar", "m_wp", "m_wm", "logw", "m_bb", "stats")]


TOPO = {"TCHAN": 0, "WT": 1, "TTSEMI": 2}


class SemilepParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "sigma_t", "sigma_w")] + \
               [(k, C.c_float) for k in ("lep_pt_min", "lep_eta_max", "jet_pt_min", "jet_eta_max")] + \
               [(k, C.c_int32) for k in ("topology", "max_cands", "reco_cut", "reserved")]


class SemilepOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "root", "best_j", "best_h", "best_p", "best_q", "nu", "m_tl",
                                          "m_wl", "m_th", "m_wh", "chi2")]


class Chi2Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "sigma_t", "sigma_w", "half_range")] + \
               [(k, C.c_float) for k in ("lep_pt_min", "lep_eta_max", "jet_pt_min", "jet_eta_max", "btag_min")] + \
               [(k, C.c_int32) for k in ("pair_mode", "max_cands", "n_grid", "n_refine", "reco_cut", "n_top")]


class Chi2Out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "root_nu", "root_nubar", "best_i", "best_j", "nu", "nubar",
                                          "m_t", "m_tbar", "m_wp", "m_wm", "chi2", "split")]


assert C.sizeof(Cut) == 64 and C.sizeof(RecoParams) == 120 and C.sizeof(Counters) == 24
assert C.sizeof(Chi2Params) == 88
assert C.sizeof(SemilepParams) == 64

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HFError(f"libhf.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.hf_last_error.restype = C.c_char_p
        L.hf_version.restype = C.c_char_p
        L.hf_select_workspace_size.argtypes = [C.c_int64, C.c_int]
        L.hf_select_workspace_size.restype = C.c_size_t
        L.hf_select.argtypes = [C.POINTER(Events), P, C.c_int, P, P, P, P, C.c_size_t, P]
        L.hf_compact_workspace_size.argtypes = [C.c_int64]
        L.hf_compact_workspace_size.restype = C.c_size_t
        L.hf_compact.argtypes = [P, C.c_int64, P, C.c_int64, P, P, P, P, C.c_size_t, P]
        L.hf_compact_noalloc.argtypes = [P, C.c_int64, P, C.c_int64, P, P, P, P]
        L.hf_ttbar_reco_workspace_size.argtypes = [C.c_int64]
        L.hf_ttbar_reco_workspace_size.restype = C.c_size_t
        L.hf_ttbar_reco.argtypes = [C.POINTER(Events), P, P, C.c_int64, C.POINTER(RecoParams), C.POINTER(RecoOut), P,
                                    P, C.c_size_t, P]
        L.hf_reorder_stats.argtypes = [P, P, C.c_int, P]
        L.hf_reorder_device.argtypes = [P, P, C.c_int, P, P]
        L.hf_ttbar_reco_autotune.argtypes = [C.POINTER(Events), P, P, C.c_int64, C.POINTER(RecoParams),
                                             C.POINTER(RecoOut), P, C.c_size_t, P, P]
        L.hf_reco_timing_events.argtypes = [P, P]
        L.hf_reco_timing_events.restype = C.c_int
        L.hf_philox_blocks.argtypes = [P, C.c_uint64, P, C.c_int64, P]
        L.hf_gauss_draws.argtypes = [C.c_uint64, P, P, P, C.c_int64, C.c_int, P, P]
        L.hf_chain_compile.argtypes = [P, C.c_int, P, C.c_int, C.POINTER(C.c_void_p)]
        L.hf_chain_select.argtypes = [P, C.POINTER(Events), P, P, P, P, C.c_size_t, P]
        L.hf_select_segment.argtypes = [C.POINTER(Events), P, C.c_int, P, C.c_int, C.c_int, P, P, C.c_int64, P, P,
                                        P, C.c_size_t, P]
        L.hf_chain_select_segment.argtypes = [P, C.POINTER(Events), P, C.c_int, C.c_int, P, P, C.c_int64, P, P, P,
                                              C.c_size_t, P]
        L.hf_unpack_workspace_size.argtypes = [C.c_int64]
        L.hf_unpack_workspace_size.restype = C.c_size_t
        L.hf_unpack_events.argtypes = [C.c_int64, P, P, C.c_int64, C.c_int64, P, P, P, P, P, P, P, C.c_size_t, P]
        L.hf_chain_log.argtypes = [P]
        L.hf_chain_log.restype = C.c_char_p
        L.hf_chain_destroy.argtypes = [P]
        L.hf_chain_destroy.restype = None
        L.hf_dilep_chi2_reco.argtypes = [C.POINTER(Events), P, P, C.c_int64, C.POINTER(Chi2Params),
                                         C.POINTER(Chi2Out), P, P]
        L.hf_semilep_reco.argtypes = [C.POINTER(Events), P, P, C.c_int64, C.POINTER(SemilepParams),
                                      C.POINTER(SemilepOut), P, P]
        for f in ("hf_select", "hf_compact", "hf_compact_noalloc", "hf_ttbar_reco", "hf_ttbar_reco_autotune", "hf_reorder_stats",
                  "hf_reorder_device", "hf_philox_blocks", "hf_gauss_draws", "hf_semilep_reco", "hf_chain_compile",
                  "hf_chain_select", "hf_dilep_chi2_reco", "hf_select_segment", "hf_chain_select_segment",
                  "hf_unpack_events"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, what):
    if rc != HF_OK:
        msg = lib().hf_last_error().decode()
        raise HFError(f"{what} failed with {HF_ERR.get(rc, rc)}: {msg}")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------- structures

def cut_table(cuts):
    """hfgen-style cut descriptions -> ctypes array of Cut.  A USER cut
    carries its predicate body in "src"; its i[0] becomes the index of that
    source in user_sources(cuts)."""
    names = {c["name"]: k for k, c in enumerate(cuts)}
    arr = (Cut * len(cuts))()
    u = 0
    for k, c in enumerate(cuts):
        arr[k].kind = CUT_KIND[c["kind"]]
        arr[k].reserved = 0
        m = 0
        for d in c.get("deps", []):
            m |= 1 << names[d]
        arr[k].dep_mask = m
        for j, v in enumerate(c.get("f", [])):
            arr[k].f[j] = float(v)
        for j, v in enumerate(c.get("i", [])):
            arr[k].i[j] = int(v)
        if c["kind"] == "USER":
            arr[k].i[0] = u
            u += 1
    return arr


def user_sources(cuts):
    """Predicate bodies of the USER cuts, in cut-table order."""
    return [c["src"] for c in cuts if c["kind"] == "USER"]


class CompiledChain:
    """A cut chain with user predicates compiled for the device
    (hf_chain_compile); released with the object."""

    def __init__(self, cuts):
        self.cut_arr = cut_table(cuts)
        self.n_cuts = len(cuts)
        srcs = [s.encode() for s in user_sources(cuts)]
        self._srcs = (C.c_char_p * max(1, len(srcs)))(*srcs)
        self.h = C.c_void_p()
        _check(lib().hf_chain_compile(C.cast(self.cut_arr, C.c_void_p), self.n_cuts, C.cast(self._srcs, C.c_void_p),
                                      len(srcs), C.byref(self.h)), "hf_chain_compile")

    @property
    def log(self):
        return lib().hf_chain_log(self.h).decode()

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.hf_chain_destroy(self.h)
            self.h = C.c_void_p()


def _check_order(order, n_cuts, counters, survive, n):
    """The kernels read n_cuts order entries, n_cuts counter rows and n mask
    bytes from device pointers: refuse shorter tensors before the call."""
    if order.numel() < n_cuts or counters.numel() < 3 * n_cuts or survive.numel() < n:
        raise ValueError(f"order needs {n_cuts} entries, counters {n_cuts} rows and survive {n} bytes")


def chain_select(chain, dev, order, survive, counters, ws, stream=None):
    _check_order(order, chain.n_cuts, counters, survive, dev.n)
    rc = lib().hf_chain_select(chain.h, dev.ptr, _p(order), _p(survive), _p(counters), _p(ws),
                               ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, "hf_chain_select")


SCHED = {"auto": 0, "event": 1, "event_wg64": 3, "event_wg128": 4}
SCHED_NAME = {v: k for k, v in SCHED.items()}


def reco_params(reco, precision="mixed", reco_cut=-1, schedule="auto"):
    return RecoParams(
        m_t=reco["m_t"], m_w=reco["m_w"], lambda_pt=reco["lambda_pt"], jet_a=reco["jet_a"], jet_c=reco["jet_c"],
        lep_sigma=reco["lep_sigma"], met_sigma=reco["met_sigma"], lep_pt_min=reco["lep_pt_min"],
        lep_eta_max=reco["lep_eta_max"], jet_pt_min=reco["jet_pt_min"], jet_eta_max=reco["jet_eta_max"],
        btag_min=reco["btag_min"], reco_cut=int(reco_cut), seed=int(reco["seed"]), smear=int(reco["smear"]),
        n_var_uniform=int(reco["n_var"]) if reco["n_var"] else 1, precision=PREC[precision],
        pair_mode=PAIR[reco["pair_mode"]], max_cands=int(reco["max_cands"]), want_mbb=int(reco["want_mbb"]),
        schedule=SCHED[schedule] if isinstance(schedule, str) else int(schedule))


class DeviceEvents:
    """A chunk of events resident in device memory (torch tensors) and the
    hf_events_t that points at them."""

    COLS = ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag",
            "met_x", "met_y")

    def __init__(self, ev, device="cuda", index_base=0):
        self.n = int(ev["n"])
        self.index_base = int(index_base)
        self.t = {}
        for k in self.COLS:
            self.t[k] = torch.as_tensor(ev[k], dtype=torch.float32).to(device)
        self.t["lep_off"] = torch.as_tensor(ev["lep_off"].astype("int64")).to(torch.int32).to(device)
        self.t["jet_off"] = torch.as_tensor(ev["jet_off"].astype("int64")).to(torch.int32).to(device)
        nv = ev.get("n_var")
        self.t["n_var"] = None if nv is None else torch.as_tensor(nv.astype("int32")).to(torch.int16).to(device)
        self.s = Events(n=self.n, index_base=self.index_base,
                        **{k: (None if v is None else v.data_ptr()) for k, v in self.t.items()})

    @property
    def ptr(self):
        return C.byref(self.s)


def select(dev, cuts_arr, n_cuts, order, survive, counters, ws, stream=None):
    _check_order(order, n_cuts, counters, survive, dev.n)
    rc = lib().hf_select(dev.ptr, C.cast(cuts_arr, C.c_void_p), n_cuts, _p(order), _p(survive), _p(counters),
                         _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, "hf_select")


def select_segment(dev, cuts_arr, n_cuts, order, pos_begin, pos_end, survive, counters, ws, idx=None, count=None,
                   capacity=0, chain=None, stream=None):
    """Cuts at order positions [pos_begin, pos_end) over all events (idx None)
    or over compacted ids idx[0:*count] (survive then indexed by position).
    With `chain` (a CompiledChain) its compiled kernel runs."""
    _check_order(order, chain.n_cuts if chain is not None else n_cuts, counters, survive,
                 dev.n if idx is None else min(int(capacity), dev.n) if capacity else 0)
    args = (int(pos_begin), int(pos_end), _p(idx), _p(count), int(capacity), _p(survive), _p(counters), _p(ws),
            ws.numel() * ws.element_size(), _stream(stream))
    if chain is not None:
        rc = lib().hf_chain_select_segment(chain.h, dev.ptr, _p(order), *args)
    else:
        rc = lib().hf_select_segment(dev.ptr, C.cast(cuts_arr, C.c_void_p), n_cuts, _p(order), *args)
    _check(rc, "hf_select_segment")


def unpack_events(n, lep_cnt, jet_cnt, n_lep, n_jet, lep_q8, jet_btag8, lep_off, jet_off, lep_q, jet_btag, ws,
                  stream=None):
    rc = lib().hf_unpack_events(int(n), _p(lep_cnt), _p(jet_cnt), int(n_lep), int(n_jet), _p(lep_q8), _p(jet_btag8),
                                _p(lep_off), _p(jet_off), _p(lep_q), _p(jet_btag), _p(ws),
                                ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, "hf_unpack_events")


def compact(mask, capacity, idx, count, ws, d_n=None, index_base=0, mapping=None, stream=None):
    rc = lib().hf_compact(_p(mask), int(capacity), _p(d_n), int(index_base), _p(mapping), _p(idx), _p(count),
                          _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, "hf_compact")


def compact_noalloc(mask, capacity, idx, count, d_n=None, index_base=0, mapping=None, stream=None):
    rc = lib().hf_compact_noalloc(_p(mask), int(capacity), _p(d_n), int(index_base), _p(mapping), _p(idx),
                                  _p(count), _stream(stream))
    _check(rc, "hf_compact_noalloc")


class RecoOutputs:
    """Device output arrays of hf_ttbar_reco for `capacity` positions."""

    def __init__(self, capacity, device="cuda", want_mbb=True):
        cap = max(1, int(capacity))
        f64 = dict(dtype=torch.float64, device=device)
        self.t = {
            "has_sol": torch.zeros(cap, dtype=torch.uint8, device=device),
            "n_sol": torch.zeros(cap, dtype=torch.int32, device=device),
            "best_v": torch.zeros(cap, dtype=torch.int32, device=device),
            "best_i": torch.zeros(cap, dtype=torch.int16, device=device),
            "best_j": torch.zeros(cap, dtype=torch.int16, device=device),
            "nu": torch.zeros(cap, 3, **f64), "nubar": torch.zeros(cap, 3, **f64),
            "m_t": torch.zeros(cap, **f64), "m_tbar": torch.zeros(cap, **f64), "m_wp": torch.zeros(cap, **f64),
            "m_wm": torch.zeros(cap, **f64), "logw": torch.zeros(cap, **f64),
            "m_bb": torch.zeros(cap, **f64) if want_mbb else None,
            "stats": torch.zeros(5, dtype=torch.int64, device=device),
        }
        self.s = RecoOut(**{k: (None if v is None else v.data_ptr()) for k, v in self.t.items()})

    def host(self, n):
        return {k: (v[:n].cpu().numpy() if k != "stats" else v.cpu().numpy()) for k, v in self.t.items()
                if v is not None}


def ttbar_reco(dev, idx, count, capacity, params, outs, counters, ws, stream=None):
    rc = lib().hf_ttbar_reco(dev.ptr, _p(idx), _p(count), int(capacity), C.byref(params), C.byref(outs.s),
                             _p(counters), _p(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, "hf_ttbar_reco")


def semilep_params(sl, topology="TCHAN", reco_cut=-1):
    return SemilepParams(m_t=sl["m_t"], m_w=sl["m_w"], sigma_t=sl["sigma_t"], sigma_w=sl["sigma_w"],
                         lep_pt_min=sl["lep_pt_min"], lep_eta_max=sl["lep_eta_max"], jet_pt_min=sl["jet_pt_min"],
                         jet_eta_max=sl["jet_eta_max"], topology=TOPO[topology], max_cands=int(sl["max_cands"]),
                         reco_cut=int(reco_cut), reserved=0)


class SemilepOutputs:
    """Device output arrays of hf_semilep_reco for `capacity` positions."""

    def __init__(self, capacity, device="cuda"):
        cap = max(1, int(capacity))
        f64 = dict(dtype=torch.float64, device=device)
        i16 = dict(dtype=torch.int16, device=device)
        self.t = {
            "has_sol": torch.zeros(cap, dtype=torch.uint8, device=device),
            "root": torch.zeros(cap, dtype=torch.int8, device=device),
            "best_j": torch.zeros(cap, **i16), "best_h": torch.zeros(cap, **i16),
            "best_p": torch.zeros(cap, **i16), "best_q": torch.zeros(cap, **i16),
            "nu": torch.zeros(cap, 3, **f64), "m_tl": torch.zeros(cap, **f64), "m_wl": torch.zeros(cap, **f64),
            "m_th": torch.zeros(cap, **f64), "m_wh": torch.zeros(cap, **f64), "chi2": torch.zeros(cap, **f64),
        }
        self.s = SemilepOut(**{k: v.data_ptr() for k, v in self.t.items()})

    def host(self, n):
        return {k: v[:n].cpu().numpy() for k, v in self.t.items()}


def semilep_reco(dev, idx, count, capacity, params, outs, counters=None, stream=None):
    rc = lib().hf_semilep_reco(dev.ptr, _p(idx), _p(count), int(capacity), C.byref(params), C.byref(outs.s),
                               _p(counters), _stream(stream))
    _check(rc, "hf_semilep_reco")


def chi2_params(cp, reco_cut=-1):
    return Chi2Params(m_t=cp["m_t"], m_w=cp["m_w"], sigma_t=cp["sigma_t"], sigma_w=cp["sigma_w"],
                      half_range=cp["half_range"], lep_pt_min=cp["lep_pt_min"], lep_eta_max=cp["lep_eta_max"],
                      jet_pt_min=cp["jet_pt_min"], jet_eta_max=cp["jet_eta_max"], btag_min=cp["btag_min"],
                      pair_mode=PAIR[cp["pair_mode"]], max_cands=int(cp["max_cands"]), n_grid=int(cp["n_grid"]),
                      n_refine=int(cp["n_refine"]), reco_cut=int(reco_cut), n_top=int(cp.get("n_top", 2)))


class Chi2Outputs:
    """Device output arrays of hf_dilep_chi2_reco for `capacity` positions."""

    def __init__(self, capacity, device="cuda"):
        cap = max(1, int(capacity))
        f64 = dict(dtype=torch.float64, device=device)
        self.t = {
            "has_sol": torch.zeros(cap, dtype=torch.uint8, device=device),
            "root_nu": torch.zeros(cap, dtype=torch.int8, device=device),
            "root_nubar": torch.zeros(cap, dtype=torch.int8, device=device),
            "best_i": torch.zeros(cap, dtype=torch.int16, device=device),
            "best_j": torch.zeros(cap, dtype=torch.int16, device=device),
            "nu": torch.zeros(cap, 3, **f64), "nubar": torch.zeros(cap, 3, **f64),
            "m_t": torch.zeros(cap, **f64), "m_tbar": torch.zeros(cap, **f64), "m_wp": torch.zeros(cap, **f64),
            "m_wm": torch.zeros(cap, **f64), "chi2": torch.zeros(cap, **f64), "split": torch.zeros(cap, 2, **f64),
        }
        self.s = Chi2Out(**{k: v.data_ptr() for k, v in self.t.items()})

    def host(self, n):
        return {k: v[:n].cpu().numpy() for k, v in self.t.items()}


def dilep_chi2_reco(dev, idx, count, capacity, params, outs, counters=None, stream=None):
    rc = lib().hf_dilep_chi2_reco(dev.ptr, _p(idx), _p(count), int(capacity), C.byref(params), C.byref(outs.s),
                                  _p(counters), _stream(stream))
    _check(rc, "hf_dilep_chi2_reco")


def reorder_stats(counters_host, cuts_arr, n_cuts):
    """counters_host: uint64 numpy array [n_cuts, 3]; returns the new order (list)."""
    import numpy as np
    cnt = np.ascontiguousarray(counters_host, dtype=np.uint64)
    order = (C.c_int32 * n_cuts)()
    rc = lib().hf_reorder_stats(C.c_void_p(cnt.ctypes.data), C.cast(cuts_arr, C.c_void_p), n_cuts,
                                C.cast(order, C.c_void_p))
    _check(rc, "hf_reorder_stats")
    return list(order)


def ttbar_reco_autotune(dev, idx, count, capacity, params, outs, ws, stream=None):
    """Times the candidate launches on this input, stores the fastest in params
    (and in the HF_AUTOTUNE_CACHE file if set); returns the milliseconds of
    (event, event_wg128, event_wg64)."""
    ms = (C.c_double * 3)()
    rc = lib().hf_ttbar_reco_autotune(dev.ptr, _p(idx), _p(count), int(capacity), C.byref(params), C.byref(outs.s),
                                      _p(ws), ws.numel() * ws.element_size(), _stream(stream), ms)
    _check(rc, "hf_ttbar_reco_autotune")
    return ms[0], ms[1], ms[2]


def reorder_device(counters, cuts_arr, n_cuts, order, stream=None):
    """New order from the device counters [n_cuts, 3] into the device order buffer, on the stream."""
    _check(lib().hf_reorder_device(_p(counters), C.cast(cuts_arr, C.c_void_p), n_cuts, _p(order), _stream(stream)),
           "hf_reorder_device")


def philox_blocks(ctr, seed, out, stream=None):
    _check(lib().hf_philox_blocks(_p(ctr), int(seed), _p(out), ctr.shape[0], _stream(stream)), "hf_philox_blocks")


def gauss_draws(seed, g, v, slot, z, precision="mixed", stream=None):
    _check(lib().hf_gauss_draws(int(seed), _p(g), _p(v), _p(slot), g.shape[0], PREC[precision], _p(z),
                                _stream(stream)), "hf_gauss_draws")


class KernelTimer:
    """HIP events that hf_ttbar_reco records around its search kernel."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.start, self.stop = C.c_void_p(), C.c_void_p()
        for ev in (self.start, self.stop):
            if self.hip.hipEventCreate(C.byref(ev)) != 0:
                raise HFError("hipEventCreate failed")

    def __enter__(self):
        _check(lib().hf_reco_timing_events(self.start, self.stop), "hf_reco_timing_events")
        return self

    def __exit__(self, *exc):
        lib().hf_reco_timing_events(None, None)

    def elapsed_ms(self):
        self.hip.hipEventSynchronize(self.stop)
        ms = C.c_float()
        if self.hip.hipEventElapsedTime(C.byref(ms), self.start, self.stop) != 0:
            raise HFError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        self.hip.hipEventDestroy(self.start)
        self.hip.hipEventDestroy(self.stop)


def workspace(nbytes, device="cuda"):
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device=device)
