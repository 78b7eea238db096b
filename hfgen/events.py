"""Seeded synthetic collision events in structure-of-arrays form.

The paper's inputs (Delphes-simulated ttH and HL-LHC ATLAS samples, section 4
and section 6) are not available, so these samples stand in for them.  Each
event is generated in FP64 and stored as float32 columns in a ragged CSR
layout; an FP64 truth sidecar keeps the generated partons and neutrinos.

Recipe (all energies in GeV):
  * top and antitop independently: pT ~ Exp(mean 100), rapidity ~ U(-2.5, 2.5),
    phi ~ U[-pi, pi), mass 172.5 (no width);
  * t -> b W+ and W+ -> l+ nu isotropic in the parent rest frame, m_W = 80.4,
    m_b = 4.8, massless leptons and neutrinos; antitop likewise;
  * missing transverse momentum = transverse sum of the two neutrinos;
  * extra jets: count ~ U{0..n_extra_max}, pT ~ Exp(40), eta ~ U(-3.5, 3.5),
    massless; b-tag probability 0.70 for true b jets, 0.01 for extra jets;
  * background events (fraction bkg_frac): lepton count ~ U{0..3} with
    pT ~ Exp(30), |eta| < 2.5 and random charge; jet count ~ U{2..bkg_jet_max}
    with pT ~ Exp(40), eta ~ U(-3.5, 3.5), b-tag probability 0.10; MET x, y ~
    N(0, 20^2);
  * ttH: ttbar plus H (pT ~ Exp(100), |y| < 2.5, m = 125) decaying to b bbar;
    the four true b jets are tagged at 0.70 and re-drawn until at least three
    are tagged; 0..n_extra_max extra jets;
  * per-event variation counts for the heavy-tailed stress sample:
    V = clamp(floor(2^(10u)), 1, 1024) with u ~ U(0, 1);
  * one-lepton samples (for the single-neutrino reconstruction): t or tbar
    (equal odds) with the top recipe above, t -> b W, W -> l nu, MET = the
    neutrino's pT, plus: one light jet pT ~ Exp(50), eta ~ U(-4, 4)
    (t-channel-like); or a W (pT ~ Exp(100), |y| < 2.5) decaying to two
    massless quarks (Wt-like); or a second top decaying hadronically
    (semileptonic ttbar); b jets tagged at 0.70, other jets at 0.01, extra
    jets as above; background (W+jets-like): 0..2 leptons pT ~ Exp(40), jets
    as above tagged at 0.10, MET x, y ~ N(0, 30^2);
  * HL-LHC mixture: per chunk, process counts drawn multinomially from the
    fractions (dileptonic ttbar, t-channel, Wt, background), each generated
    with its recipe above (the background with the dileptonic sample's
    background recipe), then shuffled.
Objects are sorted by descending pT within each event.

This module holds no arithmetic of the method under test (selection,
reconstruction, smearing); it only produces inputs.
"""

import numpy as np

from . import configs as _cfgs

M_TOP = 172.5
M_W = 80.4
M_B = 4.8
M_H = 125.0

CHUNK = 1 << 20


def _p4_pt_y_phi_m(pt, y, phi, m):
    mt = np.sqrt(m * m + pt * pt)
    return np.stack([mt * np.cosh(y), pt * np.cos(phi), pt * np.sin(phi), mt * np.sinh(y)], axis=-1)


def _boost(v, parent, mass):
    """Boost rest-frame 4-vectors v (E, px, py, pz) into the frame where the
    parent has 4-momentum `parent` and invariant mass `mass`."""
    e = parent[:, 0]
    beta = parent[:, 1:] / e[:, None]
    gamma = e / mass
    b2 = np.sum(beta * beta, axis=1)
    bp = np.sum(beta * v[:, 1:], axis=1)
    safe = np.where(b2 > 0, b2, 1.0)
    g2 = np.where(b2 > 0, (gamma - 1.0) / safe, 0.0)
    p = v[:, 1:] + (g2 * bp + gamma * v[:, 0])[:, None] * beta
    en = gamma * (v[:, 0] + bp)
    return np.concatenate([en[:, None], p], axis=1)


def _two_body(rng, parent, mass, m1, m2):
    n = parent.shape[0]
    mass = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    pstar = np.sqrt((mass ** 2 - (m1 + m2) ** 2) * (mass ** 2 - (m1 - m2) ** 2)) / (2.0 * mass)
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    d = np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=-1) * pstar[:, None]
    e1 = np.sqrt(m1 * m1 + pstar * pstar)
    e2 = np.sqrt(m2 * m2 + pstar * pstar)
    r1 = np.concatenate([e1[:, None], d], axis=1)
    r2 = np.concatenate([e2[:, None], -d], axis=1)
    return _boost(r1, parent, mass), _boost(r2, parent, mass)


def _polar(p4):
    pt = np.hypot(p4[..., 1], p4[..., 2])
    eta = np.arcsinh(p4[..., 3] / pt)
    phi = np.arctan2(p4[..., 2], p4[..., 1])
    return pt, eta, phi, p4[..., 0]


def _top_decay(rng, n):
    pt = rng.exponential(100.0, n)
    y = rng.uniform(-2.5, 2.5, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    top = _p4_pt_y_phi_m(pt, y, phi, M_TOP)
    b, w = _two_body(rng, top, M_TOP, M_B, M_W)
    lep, nu = _two_body(rng, w, M_W, 0.0, 0.0)
    return top, b, lep, nu


def _random_objects(rng, n, kmax_shape, pt_mean, eta_lo, eta_hi, mass=0.0):
    pt = rng.exponential(pt_mean, kmax_shape)
    eta = rng.uniform(eta_lo, eta_hi, kmax_shape)
    phi = rng.uniform(-np.pi, np.pi, kmax_shape)
    e = np.sqrt(mass * mass + (pt * np.cosh(eta)) ** 2)
    return pt, eta, phi, e


def _pack(cols, valid):
    """Sort each row by descending pt among valid entries and flatten to CSR."""
    key = np.where(valid, -cols["pt"], np.inf)
    order = np.argsort(key, axis=1, kind="stable")
    vs = np.take_along_axis(valid, order, axis=1)
    out = {k: np.take_along_axis(v, order, axis=1)[vs] for k, v in cols.items()}
    counts = valid.sum(axis=1)
    off = np.zeros(valid.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return out, off, order, vs


def _chunk(rng, cfg, n):
    kind = cfg["kind"]
    kx = cfg["n_extra_max"]
    is_sig = np.ones(n, dtype=bool)
    if cfg.get("bkg_frac", 0.0) > 0:
        is_sig = rng.uniform(0.0, 1.0, n) >= cfg["bkg_frac"]

    t, b, lp, nu = _top_decay(rng, n)
    if kind == "wtdilep":
        # Wt: the top's W and a second W from the hard process (pT ~ Exp(100),
        # |y| < 2.5), decaying isotropically to l- nubar; no second b
        tb = _p4_pt_y_phi_m(rng.exponential(100.0, n), rng.uniform(-2.5, 2.5, n), rng.uniform(-np.pi, np.pi, n),
                            M_W)
        lm, nub = _two_body(rng, tb, M_W, 0.0, 0.0)
        bb = None
    else:
        tb, bb, lm, nub = _top_decay(rng, n)
    truth = {"top": t, "tbar": tb, "b": b, "lp": lp, "lm": lm, "nu": nu, "nubar": nub}
    if bb is not None:
        truth["bbar"] = bb

    # ---- leptons -----------------------------------------------------------
    nl_max = 3
    lpt = np.zeros((n, nl_max)); leta = np.zeros((n, nl_max)); lphi = np.zeros((n, nl_max))
    le = np.zeros((n, nl_max)); lq = np.zeros((n, nl_max)); lorig = np.full((n, nl_max), -1)
    lval = np.zeros((n, nl_max), dtype=bool)
    for slot, (p4, q) in enumerate(((lp, 1.0), (lm, -1.0))):
        pt, eta, phi, e = _polar(p4)
        lpt[:, slot], leta[:, slot], lphi[:, slot], le[:, slot] = pt, eta, phi, e
        lq[:, slot] = q
        lorig[:, slot] = slot
        lval[:, slot] = True
    # background leptons overwrite the signal ones
    bk = ~is_sig
    nbk = int(bk.sum())
    if nbk:
        cnt = rng.integers(0, nl_max + 1, nbk)
        pt, eta, phi, e = _random_objects(rng, nbk, (nbk, nl_max), 30.0, -2.5, 2.5)
        q = np.where(rng.uniform(0, 1, (nbk, nl_max)) < 0.5, -1.0, 1.0)
        lpt[bk], leta[bk], lphi[bk], le[bk], lq[bk] = pt, eta, phi, e, q
        lorig[bk] = -1
        lval[bk] = np.arange(nl_max)[None, :] < cnt[:, None]

    # ---- jets --------------------------------------------------------------
    nh = 2 if kind == "tth" else 0
    nj_sig = (1 if kind == "wtdilep" else 2) + nh + kx
    nj_max = max(nj_sig, cfg.get("bkg_jet_max", 0))
    jpt = np.zeros((n, nj_max)); jeta = np.zeros((n, nj_max)); jphi = np.zeros((n, nj_max))
    je = np.zeros((n, nj_max)); jtag = np.zeros((n, nj_max)); jorig = np.full((n, nj_max), -1)
    jval = np.zeros((n, nj_max), dtype=bool)
    bq = [b] if bb is None else [b, bb]
    if kind == "tth":
        hpt = rng.exponential(100.0, n)
        hy = rng.uniform(-2.5, 2.5, n)
        hphi = rng.uniform(-np.pi, np.pi, n)
        h = _p4_pt_y_phi_m(hpt, hy, hphi, M_H)
        hb1, hb2 = _two_body(rng, h, M_H, M_B, M_B)
        truth.update({"higgs": h, "hb1": hb1, "hb2": hb2})
        bq += [hb1, hb2]
    for slot, p4 in enumerate(bq):
        pt, eta, phi, e = _polar(p4)
        jpt[:, slot], jeta[:, slot], jphi[:, slot], je[:, slot] = pt, eta, phi, e
        jorig[:, slot] = slot
        jval[:, slot] = True
    nb = len(bq)
    tags = rng.uniform(0, 1, (n, nb)) < 0.70
    if kind == "tth":
        need = tags.sum(axis=1) < 3
        while need.any():
            tags[need] = rng.uniform(0, 1, (int(need.sum()), nb)) < 0.70
            need = tags.sum(axis=1) < 3
    jtag[:, :nb] = tags
    nextra = rng.integers(0, kx + 1, n)
    pt, eta, phi, e = _random_objects(rng, n, (n, kx), 40.0, -3.5, 3.5)
    jpt[:, nb:nb + kx], jeta[:, nb:nb + kx], jphi[:, nb:nb + kx], je[:, nb:nb + kx] = pt, eta, phi, e
    jtag[:, nb:nb + kx] = rng.uniform(0, 1, (n, kx)) < 0.01
    jval[:, nb:nb + kx] = np.arange(kx)[None, :] < nextra[:, None]
    if nbk:
        jm = cfg["bkg_jet_max"]
        cnt = rng.integers(2, jm + 1, nbk)
        pt, eta, phi, e = _random_objects(rng, nbk, (nbk, nj_max), 40.0, -3.5, 3.5)
        jpt[bk], jeta[bk], jphi[bk], je[bk] = pt, eta, phi, e
        jtag[bk] = rng.uniform(0, 1, (nbk, nj_max)) < 0.10
        jorig[bk] = -1
        jval[bk] = np.arange(nj_max)[None, :] < cnt[:, None]

    # ---- missing transverse momentum -----------------------------------------
    metx = nu[:, 1] + nub[:, 1]
    mety = nu[:, 2] + nub[:, 2]
    if nbk:
        metx[bk] = rng.normal(0.0, 20.0, nbk)
        mety[bk] = rng.normal(0.0, 20.0, nbk)

    # ---- variation counts ------------------------------------------------------
    nvar = None
    if cfg.get("var_mode") == "loguniform1024":
        u = rng.uniform(0.0, 1.0, n)
        nvar = np.clip(np.floor(2.0 ** (10.0 * u)), 1, 1024).astype(np.uint16)

    lep, loff, lorder, lvs = _pack({"pt": lpt, "eta": leta, "phi": lphi, "e": le, "q": lq,
                                    "orig": lorig}, lval)
    jet, joff, jorder, jvs = _pack({"pt": jpt, "eta": jeta, "phi": jphi, "e": je, "btag": jtag,
                                    "orig": jorig}, jval)

    # position of each true object after sorting (index within the event)
    def _pos(orig_sorted_flat, off, code):
        out = np.full(n, -1, dtype=np.int32)
        ev = np.repeat(np.arange(n), np.diff(off))
        local = np.arange(orig_sorted_flat.size) - off[ev]
        hit = orig_sorted_flat == code
        out[ev[hit]] = local[hit]
        return out

    truth["is_signal"] = is_sig
    truth["lp_idx"] = _pos(lep["orig"], loff, 0)
    truth["lm_idx"] = _pos(lep["orig"], loff, 1)
    truth["b_idx"] = _pos(jet["orig"], joff, 0)
    truth["bbar_idx"] = _pos(jet["orig"], joff, 1) if bb is not None else np.full(n, -1, dtype=np.int32)
    if kind == "tth":
        truth["hb1_idx"] = _pos(jet["orig"], joff, 2)
        truth["hb2_idx"] = _pos(jet["orig"], joff, 3)
    truth["top_pt"] = np.hypot(t[:, 1], t[:, 2])
    truth["tbar_pt"] = np.hypot(tb[:, 1], tb[:, 2])
    for k in list(truth):
        if truth[k].dtype == np.float64 and truth[k].ndim == 2:
            truth[k][~is_sig] = np.nan

    ev64 = {
        "lep_pt": lep["pt"], "lep_eta": lep["eta"], "lep_phi": lep["phi"], "lep_e": lep["e"],
        "lep_q": lep["q"], "jet_pt": jet["pt"], "jet_eta": jet["eta"], "jet_phi": jet["phi"],
        "jet_e": jet["e"], "jet_btag": jet["btag"], "met_x": metx, "met_y": mety,
    }
    return ev64, loff, joff, nvar, truth


def _chunk_single(rng, cfg, n):
    """One-lepton samples.  Every kind has t -> b W+, W+ -> l+ nu (or the
    charge conjugate, equal odds); the other truth jets are
      tchan:  one light jet, pT ~ Exp(50), eta ~ U(-4, 4);
      wt:     the two quarks of a W (pT ~ Exp(100), |y| < 2.5) decaying
              isotropically to massless quarks;
      ttsemi: the b and the two quarks of a hadronically decaying top drawn
              with the top recipe.
    Background: 0..2 random leptons, random jets, Gaussian MET."""
    kind = cfg["kind"]
    kx = cfg["n_extra_max"]
    is_sig = rng.uniform(0.0, 1.0, n) >= cfg.get("bkg_frac", 0.0)
    top, b, lep, nu = _top_decay(rng, n)
    q = np.where(rng.uniform(0.0, 1.0, n) < 0.5, 1.0, -1.0)
    truth = {"top": top, "b": b, "lep": lep, "nu": nu}
    if kind == "tchan":
        pt, eta, phi, e = _random_objects(rng, n, (n,), 50.0, -4.0, 4.0)
        light = np.stack([e, pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)], axis=-1)
        others = [light]
    elif kind == "wt":
        w = _p4_pt_y_phi_m(rng.exponential(100.0, n), rng.uniform(-2.5, 2.5, n), rng.uniform(-np.pi, np.pi, n),
                           M_W)
        q1, q2 = _two_body(rng, w, M_W, 0.0, 0.0)
        truth["q1"], truth["q2"] = q1, q2
        others = [q1, q2]
    elif kind == "ttsemi":
        top2 = _p4_pt_y_phi_m(rng.exponential(100.0, n), rng.uniform(-2.5, 2.5, n),
                              rng.uniform(-np.pi, np.pi, n), M_TOP)
        bh, w2 = _two_body(rng, top2, M_TOP, M_B, M_W)
        q1, q2 = _two_body(rng, w2, M_W, 0.0, 0.0)
        truth["bh"], truth["q1"], truth["q2"] = bh, q1, q2
        others = [bh, q1, q2]
    else:
        raise ValueError(f"unknown one-lepton kind {kind!r}")
    nt = 1 + len(others)
    nl_max = 2
    lpt = np.zeros((n, nl_max)); leta = np.zeros((n, nl_max)); lphi = np.zeros((n, nl_max))
    le = np.zeros((n, nl_max)); lq = np.zeros((n, nl_max)); lorig = np.full((n, nl_max), -1)
    lval = np.zeros((n, nl_max), dtype=bool)
    pt, eta, phi, e = _polar(lep)
    lpt[:, 0], leta[:, 0], lphi[:, 0], le[:, 0], lq[:, 0] = pt, eta, phi, e, q
    lorig[:, 0] = 0
    lval[:, 0] = True
    bk = ~is_sig
    nbk = int(bk.sum())
    if nbk:
        cnt = rng.integers(0, nl_max + 1, nbk)
        pt, eta, phi, e = _random_objects(rng, nbk, (nbk, nl_max), 40.0, -2.5, 2.5)
        lpt[bk], leta[bk], lphi[bk], le[bk] = pt, eta, phi, e
        lq[bk] = np.where(rng.uniform(0, 1, (nbk, nl_max)) < 0.5, -1.0, 1.0)
        lorig[bk] = -1
        lval[bk] = np.arange(nl_max)[None, :] < cnt[:, None]
    nj_max = max(nt + kx, cfg.get("bkg_jet_max", 0))
    jpt = np.zeros((n, nj_max)); jeta = np.zeros((n, nj_max)); jphi = np.zeros((n, nj_max))
    je = np.zeros((n, nj_max)); jtag = np.zeros((n, nj_max)); jorig = np.full((n, nj_max), -1)
    jval = np.zeros((n, nj_max), dtype=bool)
    for c, p4 in enumerate([b] + others):
        pt, eta, phi, e = _polar(p4)
        jpt[:, c], jeta[:, c], jphi[:, c], je[:, c] = pt, eta, phi, e
        is_b = c == 0 or (kind == "ttsemi" and c == 1)
        jtag[:, c] = rng.uniform(0, 1, n) < (0.70 if is_b else 0.01)
        jorig[:, c] = c
        jval[:, c] = True
    nextra = rng.integers(0, kx + 1, n)
    pt, eta, phi, e = _random_objects(rng, n, (n, kx), 40.0, -3.5, 3.5)
    jpt[:, nt:nt + kx], jeta[:, nt:nt + kx], jphi[:, nt:nt + kx], je[:, nt:nt + kx] = pt, eta, phi, e
    jtag[:, nt:nt + kx] = rng.uniform(0, 1, (n, kx)) < 0.01
    jval[:, nt:nt + kx] = np.arange(kx)[None, :] < nextra[:, None]
    if nbk:
        jm = cfg["bkg_jet_max"]
        cnt = rng.integers(2, jm + 1, nbk)
        pt, eta, phi, e = _random_objects(rng, nbk, (nbk, nj_max), 40.0, -3.5, 3.5)
        jpt[bk], jeta[bk], jphi[bk], je[bk] = pt, eta, phi, e
        jtag[bk] = rng.uniform(0, 1, (nbk, nj_max)) < 0.10
        jorig[bk] = -1
        jval[bk] = np.arange(nj_max)[None, :] < cnt[:, None]
    metx = nu[:, 1].copy()
    mety = nu[:, 2].copy()
    if nbk:
        metx[bk] = rng.normal(0.0, 30.0, nbk)
        mety[bk] = rng.normal(0.0, 30.0, nbk)
    lp_, loff, _, _ = _pack({"pt": lpt, "eta": leta, "phi": lphi, "e": le, "q": lq, "orig": lorig}, lval)
    jt_, joff, _, _ = _pack({"pt": jpt, "eta": jeta, "phi": jphi, "e": je, "btag": jtag, "orig": jorig}, jval)

    def _pos(orig_sorted_flat, off, code):
        out = np.full(n, -1, dtype=np.int32)
        ev = np.repeat(np.arange(n), np.diff(off))
        local = np.arange(orig_sorted_flat.size) - off[ev]
        hit = orig_sorted_flat == code
        out[ev[hit]] = local[hit]
        return out

    truth["is_signal"] = is_sig
    truth["lep_idx"] = _pos(lp_["orig"], loff, 0)
    names = ["b_idx"] + {"tchan": ["light_idx"], "wt": ["q1_idx", "q2_idx"],
                         "ttsemi": ["bh_idx", "q1_idx", "q2_idx"]}[kind]
    for c, k in enumerate(names):
        truth[k] = _pos(jt_["orig"], joff, c)
    for k in list(truth):
        if truth[k].dtype == np.float64 and truth[k].ndim == 2:
            truth[k][~is_sig] = np.nan
    ev64 = {
        "lep_pt": lp_["pt"], "lep_eta": lp_["eta"], "lep_phi": lp_["phi"], "lep_e": lp_["e"],
        "lep_q": lp_["q"], "jet_pt": jt_["pt"], "jet_eta": jt_["eta"], "jet_phi": jt_["phi"],
        "jet_e": jt_["e"], "jet_btag": jt_["btag"], "met_x": metx, "met_y": mety,
    }
    return ev64, loff, joff, None, truth


HLHC_PROCESSES = ("ttbar", "ttsemi", "tchan", "wt", "wtdilep", "bkg")


def _chunk_hlhc(rng, cfg, n):
    """Mixed HL-LHC-like chunk: dileptonic and semileptonic ttbar, t-channel
    and semileptonic Wt single top (one lepton), dileptonic Wt and
    background in the fractions cfg["fractions"],
    generated per process and shuffled.  Truth keeps the process code
    (index into HLHC_PROCESSES) only."""
    fr = cfg["fractions"]
    counts = rng.multinomial(n, [fr.get(p, 0.0) for p in HLHC_PROCESSES])
    if n == 0:  # an empty chunk: the dileptonic generator's empty layout
        part = _chunk(rng, {"kind": "ttbar", "n_extra_max": cfg["n_extra_max"], "bkg_jet_max": cfg["bkg_jet_max"],
                            "bkg_frac": 0.0}, 0)
        return part[0], part[1], part[2], None, {"process": np.zeros(0, dtype=np.int8)}
    parts = []
    for code, (proc, m) in enumerate(zip(HLHC_PROCESSES, counts)):
        m = int(m)
        if m == 0:
            continue
        sub = {"n_extra_max": cfg["n_extra_max"], "bkg_jet_max": cfg["bkg_jet_max"]}
        if proc in ("ttbar", "wtdilep"):
            sub.update(kind=proc, bkg_frac=0.0)
            part = _chunk(rng, sub, m)
        elif proc == "bkg":
            sub.update(kind="ttbar", bkg_frac=1.0)
            part = _chunk(rng, sub, m)
        else:
            sub.update(kind=proc, bkg_frac=0.0)
            part = _chunk_single(rng, sub, m)
        parts.append((part[0], part[1], part[2], None, {"process": np.full(m, code, dtype=np.int8)}))
    ev64, loff, joff, _, truth = parts[0] if len(parts) == 1 else _concat(parts)
    tmp = dict(ev64, n=n, lep_off=loff, jet_off=joff, n_var=None, truth=truth)
    out = subset(tmp, rng.permutation(n))
    ev64 = {k: v for k, v in out.items() if k not in ("n", "lep_off", "jet_off", "n_var", "truth")}
    return ev64, out["lep_off"].astype(np.int64), out["jet_off"].astype(np.int64), None, out["truth"]


def _concat(parts):
    ev = {k: np.concatenate([p[0][k] for p in parts]) for k in parts[0][0]}
    offs = []
    for which in (1, 2):
        base = 0
        chunks = []
        for i, p in enumerate(parts):
            o = p[which]
            chunks.append((o if i == 0 else o[1:]) + base)
            base += o[-1]
        offs.append(np.concatenate(chunks))
    nvar = None if parts[0][3] is None else np.concatenate([p[3] for p in parts])
    truth = {k: np.concatenate([p[4][k] for p in parts]) for k in parts[0][4]}
    return ev, offs[0], offs[1], nvar, truth


def generate(cfg, n_events=None, seed=None, keep_fp64=False):
    """Generate a sample.

    cfg: a config name (see hfgen.configs.CONFIGS) or a config dict.
    Returns a dict with float32 SoA columns, uint32 CSR offsets, optional
    uint16 per-event variation counts and an FP64 truth sidecar.  With
    keep_fp64 the unrounded FP64 columns are kept under "fp64".
    """
    if isinstance(cfg, str):
        cfg = _cfgs.config(cfg)
    n = int(cfg["n_events"] if n_events is None else n_events)
    seed = int(cfg.get("seed", 0) if seed is None else seed)
    ss = np.random.SeedSequence(seed)
    nchunks = max(1, (n + CHUNK - 1) // CHUNK)
    children = ss.spawn(nchunks)
    parts = []
    for c in range(nchunks):
        m = min(CHUNK, n - c * CHUNK)
        gen = _chunk_single if cfg["kind"] in ("tchan", "wt", "ttsemi") else \
            _chunk_hlhc if cfg["kind"] == "hlhc" else _chunk
        parts.append(gen(np.random.Generator(np.random.PCG64(children[c])), cfg, m))
    ev64, loff, joff, nvar, truth = parts[0] if len(parts) == 1 else _concat(parts)
    if loff[-1] >= 2 ** 32 or joff[-1] >= 2 ** 32:
        raise ValueError("sample too large for 32-bit object offsets")
    out = {"n": n, "lep_off": loff.astype(np.uint32), "jet_off": joff.astype(np.uint32)}
    for k, v in ev64.items():
        out[k] = v.astype(np.float32)
    out["n_var"] = nvar
    out["truth"] = truth
    if keep_fp64:
        out["fp64"] = ev64
    return out


def subset(ev, sel):
    """Events `sel` (ascending int array) of a sample, re-packed; truth follows."""
    sel = np.asarray(sel, dtype=np.int64)
    out = {"n": int(sel.size)}
    for pre, offk in (("lep_", "lep_off"), ("jet_", "jet_off")):
        off = ev[offk].astype(np.int64)
        cnt = off[sel + 1] - off[sel]
        noff = np.zeros(sel.size + 1, dtype=np.int64)
        np.cumsum(cnt, out=noff[1:])
        idx = np.repeat(off[sel] - noff[:-1], cnt) + np.arange(noff[-1])
        for k in ev:
            if k.startswith(pre) and k != offk:
                out[k] = ev[k][idx]
        out[offk] = noff.astype(np.uint32)
    out["met_x"] = ev["met_x"][sel]
    out["met_y"] = ev["met_y"][sel]
    out["n_var"] = None if ev.get("n_var") is None else ev["n_var"][sel]
    out["truth"] = {k: v[sel] for k, v in ev["truth"].items()}
    if "fp64" in ev:
        f = {}
        for pre, offk in (("lep_", "lep_off"), ("jet_", "jet_off")):
            off = ev[offk].astype(np.int64)
            cnt = off[sel + 1] - off[sel]
            noff = out[offk].astype(np.int64)
            idx = np.repeat(off[sel] - noff[:-1], cnt) + np.arange(noff[-1])
            for k in ev["fp64"]:
                if k.startswith(pre):
                    f[k] = ev["fp64"][k][idx]
        f["met_x"] = ev["fp64"]["met_x"][sel]
        f["met_y"] = ev["fp64"]["met_y"][sel]
        out["fp64"] = f
    return out


def stream_chunk(cfg, i, n=None):
    """Chunk i of a streamed sample (a config with a "chunk" size): generated
    with its own seed; its events take the global ids i*n .. i*n + n - 1.
    Returns (sample, index_base)."""
    if isinstance(cfg, str):
        cfg = _cfgs.config(cfg)
    m = int(cfg["chunk"] if n is None else n)
    ev = generate(cfg, n_events=m, seed=int(cfg["seed"]) * 100003 + int(i))
    return ev, int(i) * m
