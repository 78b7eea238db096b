"""ctypes wrapper around the FP64 CPU oracle (oracle/hf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; it translates the plain-data workload descriptions of
hfgen.configs into its own structures.
"""

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhf_oracle.so")
SRC_PATH = os.path.join(_HERE, "hf_oracle.c")

KIND = {"LEP_N_OS": 0, "JET_N_MIN": 1, "BTAG_N_MIN": 2, "BTAG_N_EQ": 3, "MET_MIN": 4,
        "MLL_MIN": 5, "FWD_JET_VETO": 6, "LEP_ISO": 7, "RECO": 8, "MTW_MIN": 9, "USER": 10, "JET_N_RANGE": 11}
PAIR_MODE = {"BTAG_FILL": 0, "ALL_JETS": 1}
NOSOL = -9999.0


def build(force=True):
    """Compile the oracle: plain C, IEEE double, no contraction, OpenMP."""
    hdr = os.path.join(_HERE, "orc_events.h")
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= max(os.path.getmtime(SRC_PATH), os.path.getmtime(hdr)):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-I", _HERE, "-o", tmp, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Events(C.Structure):
    _fields_ = [("n", C.c_int64), ("index_base", C.c_int64),
                ("lep_off", C.c_void_p), ("jet_off", C.c_void_p)] + \
               [(k, C.c_void_p) for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q",
                                          "jet_pt", "jet_eta", "jet_phi", "jet_e", "jet_btag",
                                          "met_x", "met_y", "n_var")]


class Cut(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("f", C.c_double * 8),
                ("i", C.c_int32 * 4), ("dep_mask", C.c_uint64)]


class RecoParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "lambda_pt", "jet_a", "jet_c", "lep_sigma",
                                          "met_sigma", "lep_pt_min", "lep_eta_max", "jet_pt_min",
                                          "jet_eta_max", "btag_min")] + \
               [("seed", C.c_uint64)] + \
               [(k, C.c_int32) for k in ("smear", "n_var_uniform", "pair_mode", "max_cands",
                                         "want_mbb", "pad")]


class RecoOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "n_sol", "best_v", "best_i", "best_j", "nu",
                                          "nubar", "m_t", "m_tbar", "m_wp", "m_wm", "logw", "m_bb")]


TOPOLOGY = {"TCHAN": 0, "WT": 1, "TTSEMI": 2}


class SemilepParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "sigma_t", "sigma_w", "lep_pt_min", "lep_eta_max",
                                          "jet_pt_min", "jet_eta_max")] + \
               [("topology", C.c_int32), ("max_cands", C.c_int32)]


class SemilepOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "root", "best_j", "best_h", "best_p", "best_q", "nu",
                                          "m_tl", "m_wl", "m_th", "m_wh", "chi2")]


class Chi2Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("m_t", "m_w", "sigma_t", "sigma_w", "half_range", "lep_pt_min",
                                          "lep_eta_max", "jet_pt_min", "jet_eta_max", "btag_min")] + \
               [(k, C.c_int32) for k in ("pair_mode", "max_cands", "n_grid", "n_refine", "n_top")]


class Chi2Out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("has_sol", "root_nu", "root_nubar", "best_i", "best_j", "nu", "nubar",
                                          "m_t", "m_tbar", "m_wp", "m_wm", "chi2", "split")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)  # rebuilt when older than its sources
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_gauss.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_gauss.restype = C.c_double
        L.orc_select.argtypes = [C.POINTER(Events), P, C.c_int, P, P, P, P]
        L.orc_select_user.argtypes = [C.POINTER(Events), P, C.c_int, P, P, P, P, P]
        L.orc_compact.argtypes = [P, C.c_int64, C.c_int64, P, P]
        L.orc_compact.restype = C.c_int64
        L.orc_reorder.argtypes = [P, P, P, P, C.c_int, P]
        L.orc_real_roots.argtypes = [P, P]
        L.orc_solve_pairing.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_pairing_quartic.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_ttbar_reco.argtypes = [C.POINTER(Events), P, C.c_int64, C.POINTER(RecoParams),
                                     C.POINTER(RecoOut), C.c_int]
        L.orc_ttbar_reco.restype = C.c_int64
        L.orc_nu_pz.argtypes = [P, C.c_double, C.c_double, C.c_double, P, P]
        L.orc_dilep_chi2_reco.argtypes = [C.POINTER(Events), P, C.c_int64, C.POINTER(Chi2Params),
                                          C.POINTER(Chi2Out), C.c_int]
        L.orc_dilep_chi2_reco.restype = C.c_int64
        L.orc_semilep_reco.argtypes = [C.POINTER(Events), P, C.c_int64, C.POINTER(SemilepParams),
                                       C.POINTER(SemilepOut), C.c_int]
        L.orc_semilep_reco.restype = C.c_int64
        L.orc_stage_vary.argtypes = [C.POINTER(Events), C.c_int64, C.c_int, C.POINTER(RecoParams), P, P, P, P]
        L.orc_stage_vary.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _EventsHolder:
    """Widens a float32 SoA sample to FP64 (exact) and keeps the arrays alive."""

    def __init__(self, ev, index_base=0, fp64=False):
        src = ev["fp64"] if fp64 else ev
        self.arrs = {}
        for k in ("lep_pt", "lep_eta", "lep_phi", "lep_e", "lep_q", "jet_pt", "jet_eta", "jet_phi",
                  "jet_e", "jet_btag", "met_x", "met_y"):
            self.arrs[k] = np.ascontiguousarray(src[k] if k in src else ev[k], dtype=np.float64)
        self.arrs["lep_off"] = np.ascontiguousarray(ev["lep_off"], dtype=np.uint32)
        self.arrs["jet_off"] = np.ascontiguousarray(ev["jet_off"], dtype=np.uint32)
        nv = ev.get("n_var")
        self.arrs["n_var"] = None if nv is None else np.ascontiguousarray(nv, dtype=np.int32)
        self.s = Events(n=int(ev["n"]), index_base=int(index_base),
                        **{k: _ptr(v) for k, v in self.arrs.items()})


def _cut_array(cuts):
    from hfgen.configs import dep_masks
    deps = dep_masks(cuts)
    arr = (Cut * len(cuts))()
    u = 0
    for k, c in enumerate(cuts):
        arr[k].kind = KIND[c["kind"]]
        for j, v in enumerate(c["f"]):
            # thresholds are float32 values on the product side; use the same values
            arr[k].f[j] = float(np.float32(v))
        for j, v in enumerate(c["i"]):
            arr[k].i[j] = int(v)
        if c["kind"] == "USER":
            arr[k].i[0] = u  # index of its predicate in the compiled user library
            u += 1
        arr[k].dep_mask = deps[k]
    return arr


# The accessors a user predicate is written against (section 3: a cut is a
# boolean function of one event): float values of the event's columns, 0
# for an index outside the event's list.
_USER_PRELUDE = """#include <math.h>
#include "orc_events.h"
static float orc_col(const double *col, uint32_t base, uint32_t n, int i)
{
    return (i >= 0 && (uint32_t)i < n) ? (float)col[base + (uint32_t)i] : 0.0f;
}
#define n_lep() ((int)nl_)
#define n_jet() ((int)nj_)
#define lep_pt(i) orc_col(ev_->lep_pt, l0_, nl_, (i))
#define lep_eta(i) orc_col(ev_->lep_eta, l0_, nl_, (i))
#define lep_phi(i) orc_col(ev_->lep_phi, l0_, nl_, (i))
#define lep_e(i) orc_col(ev_->lep_e, l0_, nl_, (i))
#define lep_q(i) orc_col(ev_->lep_q, l0_, nl_, (i))
#define jet_pt(i) orc_col(ev_->jet_pt, j0_, nj_, (i))
#define jet_eta(i) orc_col(ev_->jet_eta, j0_, nj_, (i))
#define jet_phi(i) orc_col(ev_->jet_phi, j0_, nj_, (i))
#define jet_e(i) orc_col(ev_->jet_e, j0_, nj_, (i))
#define jet_btag(i) orc_col(ev_->jet_btag, j0_, nj_, (i))
#define met_x() ((float)ev_->met_x[e_])
#define met_y() ((float)ev_->met_y[e_])
"""

# Reading (a predicate is a boolean function of one event, so it must end):
# every loop iteration of a predicate spends one unit of a budget per event
# (the cut's i[1], or USER_LOOP_BUDGET when that is 0); a for loop spends it
# as an iteration starts, a while or do-while loop when its condition lets
# another iteration run.  A predicate whose loops would run past the budget
# stops there and fails the event.  goto is not accepted.
USER_LOOP_BUDGET = 65536
_USER_LOOPS = """#define for(...) for (__VA_ARGS__) if (--*budget_ < 0) { *over_ = 1; break; } else
#define while(...) while ((__VA_ARGS__) && (--*budget_ >= 0 || (*over_ = 1, 0)))
#define goto orc_user_cuts_may_not_use_goto
"""
_USER_LOOPS_END = "#undef for\n#undef while\n#undef goto\n"

_user_libs = {}


def _user_fns(cuts):
    """Compiles the USER cuts' predicate bodies with gcc (IEEE single
    precision, no contraction) into a library of the oracle's own and returns
    (library, array of function pointers), cached by source."""
    import hashlib
    import tempfile
    srcs = [c["src"] for c in cuts if c["kind"] == "USER"]
    if not srcs:
        return None, None
    key = hashlib.sha256("\0".join(srcs).encode()).hexdigest()[:16]
    if key not in _user_libs:
        body = [_USER_PRELUDE]
        for u, src in enumerate(srcs):
            body.append(f"static int orc_user_body_{u}(const orc_events *ev_, int64_t e_, int64_t *budget_, int *over_)\n"
                        f"{{\n"
                        f"    const uint32_t l0_ = ev_->lep_off[e_], nl_ = ev_->lep_off[e_ + 1] - l0_;\n"
                        f"    const uint32_t j0_ = ev_->jet_off[e_], nj_ = ev_->jet_off[e_ + 1] - j0_;\n"
                        f"    (void)nl_;\n    (void)nj_;\n    (void)budget_;\n    (void)over_;\n"
                        f"{_USER_LOOPS}#line 1 \"user_cut_{u}\"\n{src}\n#line 1 \"orc_user_tail\"\n"
                        f"{_USER_LOOPS_END}}}\n"
                        f"int orc_user_cut_{u}(const orc_events *ev_, int64_t e_, int32_t budget)\n{{\n"
                        f"    int64_t b_ = budget > 0 ? budget : {USER_LOOP_BUDGET};\n    int over_ = 0;\n"
                        f"    const int r_ = orc_user_body_{u}(ev_, e_, &b_, &over_);\n"
                        f"    return r_ && !over_;\n}}\n")
        d = tempfile.mkdtemp(prefix="orc_user_")
        c_path, so_path = os.path.join(d, "user.c"), os.path.join(d, "user.so")
        with open(c_path, "w") as f:
            f.write("\n".join(body))
        subprocess.run(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                        "-Werror=return-type", "-I", _HERE, "-o", so_path, c_path, "-lm"], check=True)
        ul = C.CDLL(so_path)
        fns = (C.c_void_p * len(srcs))(*[C.cast(getattr(ul, f"orc_user_cut_{u}"), C.c_void_p).value
                                          for u in range(len(srcs))])
        _user_libs[key] = (ul, fns)
    return _user_libs[key]


def select(ev, cuts, order, index_base=0):
    """Returns (survive uint8[n], reached uint64[n_cuts], passed uint64[n_cuts])."""
    h = _EventsHolder(ev, index_base)
    n = int(ev["n"])
    surv = np.zeros(n, dtype=np.uint8)
    reached = np.zeros(len(cuts), dtype=np.uint64)
    passed = np.zeros(len(cuts), dtype=np.uint64)
    order = np.ascontiguousarray(order, dtype=np.int32)
    if order.size != len(cuts):
        raise ValueError(f"order has {order.size} entries for {len(cuts)} cuts")
    arr = _cut_array(cuts)
    _, fns = _user_fns(cuts)
    lib().orc_select_user(C.byref(h.s), C.cast(arr, C.c_void_p), len(cuts), _ptr(order),
                          None if fns is None else C.cast(fns, C.c_void_p), _ptr(surv), _ptr(reached), _ptr(passed))
    return surv, reached, passed


def compact(mask, index_base=0, mapping=None):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    idx = np.zeros(max(1, mask.size), dtype=np.int32)
    m = None if mapping is None else np.ascontiguousarray(mapping, dtype=np.int32)
    cnt = lib().orc_compact(_ptr(mask), mask.size, int(index_base), _ptr(m), _ptr(idx))
    return idx[:cnt].copy()


def reorder(reached, passed, cost, dep_mask):
    n = len(reached)
    r = np.ascontiguousarray(reached, dtype=np.uint64)
    p = np.ascontiguousarray(passed, dtype=np.uint64)
    c = np.ascontiguousarray(cost, dtype=np.uint64)
    d = np.ascontiguousarray(dep_mask, dtype=np.uint64)
    out = np.zeros(n, dtype=np.int32)
    rc = lib().orc_reorder(_ptr(r), _ptr(p), _ptr(c), _ptr(d), n, _ptr(out))
    if rc != 0:
        raise ValueError("cyclic cut dependencies")
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def gauss(seed, g, v, slot):
    return lib().orc_gauss(int(seed), int(g), int(v), int(slot))


def real_roots(c):
    """Sign-changing real roots of c0 + c1 t + ... + c4 t^4 (ascending)."""
    cc = np.zeros(5)
    cc[:len(c)] = c
    out = np.zeros(4)
    n = lib().orc_real_roots(_ptr(cc), _ptr(out))
    return out[:n].copy()


def _v4(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def solve_pairing(lp, b, lm, bb, metx, mety, mt=172.5, mw=80.4):
    """Accepted solutions for one pairing; 4-vectors as (E, px, py, pz).
    Returns array [k, 8]: nu (x, y, z, E), nubar (x, y, z, E)."""
    out = np.zeros(32)
    n = lib().orc_solve_pairing(_ptr(_v4(lp)), _ptr(_v4(b)), _ptr(_v4(lm)), _ptr(_v4(bb)),
                                float(metx), float(mety), float(mt), float(mw), _ptr(out))
    return out[:8 * n].reshape(n, 8).copy()


def pairing_quartic(lp, b, lm, bb, metx, mety, mt=172.5, mw=80.4):
    out = np.zeros(5)
    ok = lib().orc_pairing_quartic(_ptr(_v4(lp)), _ptr(_v4(b)), _ptr(_v4(lm)), _ptr(_v4(bb)),
                                   float(metx), float(mety), float(mt), float(mw), _ptr(out))
    return out if ok else None


def reco_params(reco):
    return RecoParams(
        m_t=reco["m_t"], m_w=reco["m_w"], lambda_pt=reco["lambda_pt"], jet_a=reco["jet_a"],
        jet_c=reco["jet_c"], lep_sigma=reco["lep_sigma"], met_sigma=reco["met_sigma"],
        lep_pt_min=float(np.float32(reco["lep_pt_min"])), lep_eta_max=float(np.float32(reco["lep_eta_max"])),
        jet_pt_min=float(np.float32(reco["jet_pt_min"])), jet_eta_max=float(np.float32(reco["jet_eta_max"])),
        btag_min=float(np.float32(reco["btag_min"])), seed=int(reco["seed"]), smear=int(reco["smear"]),
        n_var_uniform=int(reco["n_var"]), pair_mode=PAIR_MODE[reco["pair_mode"]],
        max_cands=int(reco["max_cands"]), want_mbb=int(reco["want_mbb"]), pad=0)


def ttbar_reco(ev, idx, reco, index_base=0, n_threads=0, fp64=False):
    """Reconstruct compacted events (global ids idx).  Returns a dict of arrays."""
    h = _EventsHolder(ev, index_base, fp64=fp64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    S = idx.size
    m = max(S, 1)
    o = {"has_sol": np.zeros(m, np.uint8), "n_sol": np.zeros(m, np.int32), "best_v": np.zeros(m, np.int32),
         "best_i": np.zeros(m, np.int16), "best_j": np.zeros(m, np.int16), "nu": np.zeros((m, 3)),
         "nubar": np.zeros((m, 3)), "m_t": np.zeros(m), "m_tbar": np.zeros(m), "m_wp": np.zeros(m),
         "m_wm": np.zeros(m), "logw": np.zeros(m), "m_bb": np.zeros(m)}
    ro = RecoOut(**{k: _ptr(v) for k, v in o.items()})
    prm = reco_params(reco)
    npass = lib().orc_ttbar_reco(C.byref(h.s), _ptr(idx), S, C.byref(prm), C.byref(ro), int(n_threads))
    res = {k: v[:S].copy() for k, v in o.items()}
    res["n_pass"] = int(npass)
    return res


def stage_vary(ev, e, v, reco, index_base=0):
    """Staged candidates and one resolution variation of event e (local index).

    Returns None when the event lacks two selected opposite-sign leptons, else
    a dict: cand (jet indices within the event), lp, lm (E, px, py, pz),
    cands [nc, 4], met (x, y) and the draws z_lp, z_lm, z_mx, z_my, z_cand."""
    h = _EventsHolder(ev, index_base)
    prm = reco_params(reco)
    cand = np.zeros(16, np.int32)
    vecs = np.zeros(4 * 16)
    met = np.zeros(2)
    z = np.zeros(16)
    nc = lib().orc_stage_vary(C.byref(h.s), int(e), int(v), C.byref(prm), _ptr(cand), _ptr(vecs), _ptr(met),
                              _ptr(z))
    if nc < 0:
        return None
    vecs = vecs.reshape(16, 4)
    return {"cand": cand[:nc].copy(), "lp": vecs[0].copy(), "lm": vecs[1].copy(), "cands": vecs[2:2 + nc].copy(),
            "met": met.copy(), "z_lp": z[0], "z_lm": z[1], "z_mx": z[2], "z_my": z[3], "z_cand": z[4:4 + nc].copy()}


def nu_pz(lep, metx, mety, mw=80.4):
    """Neutrino p_z candidates from the W mass; lep = (E, px, py, pz).
    Returns (pz array, kind array): kind 0/1 minus/plus root, 2 real part."""
    pz = np.zeros(2)
    kind = np.zeros(2, dtype=np.int32)
    n = lib().orc_nu_pz(_ptr(_v4(lep)), float(metx), float(mety), float(mw), _ptr(pz), _ptr(kind))
    return pz[:n].copy(), kind[:n].copy()


def semilep_params(sl, topology="TCHAN"):
    return SemilepParams(
        m_t=sl["m_t"], m_w=sl["m_w"], sigma_t=sl["sigma_t"], sigma_w=sl["sigma_w"],
        lep_pt_min=float(np.float32(sl["lep_pt_min"])), lep_eta_max=float(np.float32(sl["lep_eta_max"])),
        jet_pt_min=float(np.float32(sl["jet_pt_min"])), jet_eta_max=float(np.float32(sl["jet_eta_max"])),
        topology=TOPOLOGY[topology], max_cands=int(sl["max_cands"]))


def semilep_reco(ev, idx, sl, topology="TCHAN", index_base=0, n_threads=0, fp64=False):
    """Single-neutrino chi^2 reconstruction of events idx (global ids)."""
    h = _EventsHolder(ev, index_base, fp64=fp64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    S = idx.size
    m = max(S, 1)
    o = {"has_sol": np.zeros(m, np.uint8), "root": np.zeros(m, np.int8), "best_j": np.zeros(m, np.int16),
         "best_h": np.zeros(m, np.int16), "best_p": np.zeros(m, np.int16), "best_q": np.zeros(m, np.int16),
         "nu": np.zeros((m, 3)), "m_tl": np.zeros(m), "m_wl": np.zeros(m), "m_th": np.zeros(m),
         "m_wh": np.zeros(m), "chi2": np.zeros(m)}
    so = SemilepOut(**{k: _ptr(v) for k, v in o.items()})
    prm = semilep_params(sl, topology)
    npass = lib().orc_semilep_reco(C.byref(h.s), _ptr(idx), S, C.byref(prm), C.byref(so), int(n_threads))
    res = {k: v[:S].copy() for k, v in o.items()}
    res["n_pass"] = int(npass)
    return res


def chi2_params(cp):
    f32 = lambda k: float(np.float32(cp[k]))
    return Chi2Params(m_t=cp["m_t"], m_w=cp["m_w"], sigma_t=cp["sigma_t"], sigma_w=cp["sigma_w"],
                      half_range=cp["half_range"], lep_pt_min=f32("lep_pt_min"), lep_eta_max=f32("lep_eta_max"),
                      jet_pt_min=f32("jet_pt_min"), jet_eta_max=f32("jet_eta_max"), btag_min=f32("btag_min"),
                      pair_mode=PAIR_MODE[cp["pair_mode"]], max_cands=int(cp["max_cands"]),
                      n_grid=int(cp["n_grid"]), n_refine=int(cp["n_refine"]), n_top=int(cp.get("n_top", 2)))


def dilep_chi2_reco(ev, idx, cp, index_base=0, n_threads=0, fp64=False):
    """Dileptonic chi^2 fit with a MET split (section 6.2) of events idx."""
    h = _EventsHolder(ev, index_base, fp64=fp64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    S = idx.size
    m = max(S, 1)
    o = {"has_sol": np.zeros(m, np.uint8), "root_nu": np.zeros(m, np.int8), "root_nubar": np.zeros(m, np.int8),
         "best_i": np.zeros(m, np.int16), "best_j": np.zeros(m, np.int16), "nu": np.zeros((m, 3)),
         "nubar": np.zeros((m, 3)), "m_t": np.zeros(m), "m_tbar": np.zeros(m), "m_wp": np.zeros(m),
         "m_wm": np.zeros(m), "chi2": np.zeros(m), "split": np.zeros((m, 2))}
    co = Chi2Out(**{k: _ptr(v) for k, v in o.items()})
    prm = chi2_params(cp)
    npass = lib().orc_dilep_chi2_reco(C.byref(h.s), _ptr(idx), S, C.byref(prm), C.byref(co), int(n_threads))
    res = {k: v[:S].copy() for k, v in o.items()}
    res["n_pass"] = int(npass)
    return res


def run_chain(ev, cuts, reco, order=None, index_base=0, n_threads=0):
    """select -> compact -> reco -> compact for one chunk; returns a dict."""
    if order is None:
        order = list(range(len(cuts)))
    t0 = time.perf_counter()
    surv, reached, passed = select(ev, cuts, order, index_base)
    idx = compact(surv, index_base)
    rec = ttbar_reco(ev, idx, reco, index_base, n_threads)
    final = compact(rec["has_sol"], 0, idx)
    rid = [k for k, c in enumerate(cuts) if c["kind"] == "RECO"]
    if rid:
        reached[rid[0]] += np.uint64(idx.size)
        passed[rid[0]] += np.uint64(final.size)
    return {"survive": surv, "reached": reached, "passed": passed, "idx": idx, "reco": rec,
            "final": final, "seconds": time.perf_counter() - t0}
