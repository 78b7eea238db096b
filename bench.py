"""Throughput of the hot path on one MI355X.

Workload: 1M synthetic events (80 % dileptonic ttbar, 20 % background, 2-10
jets), cut chain of four cuts plus the reconstruction at 64 smeared
variations per event.  One step = one pass of the whole path over the
batch: hf_select -> hf_compact -> hf_ttbar_reco -> hf_compact -> the cut
reordering from the accumulated counters (hf_reorder_device), recorded as one
HIP graph.  Inputs are resident in HBM before timing starts.

A second leg measures the single-neutrino chi^2 reconstruction the same way
(1M one-lepton t-channel-like events, four cuts plus hf_semilep_reco, one HIP
graph per step) and reports it under "semilep" in the same line.  A third
leg streams 50 chunks of 1M mixed events from pinned host memory through the
five HL-LHC signal bins (copies overlapped with compute) and reports the
end-to-end rate and the events per bin under "stream".  Further legs run the
10k, 4M ttH and 2M heavy-tailed batches under "workloads".

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "ttbar1M_v64"
SEMILEP_WORKLOAD = "tchan1M"
STREAM_WORKLOAD = "hlhc50M"
# further workloads, each reported under "workloads" with its own roofline and oracle baseline
EXTRA_WORKLOADS = ("ttbar10k", "tth4M_v256", "stress2M_heavytail")

# Algorithmic FP operations of the reconstruction search kernel per unit of
# work (one each for add, mul, div, sqrt, transcendental; two for FMA),
# measured by paper_2211_14346_amd/perf/opcount.py, which runs the kernel's
# own math header on the host with counting scalar types over a sample of
# this workload: per variation the Box-Muller draws, smear factors, MET shifts
# and lepton-side terms; per pairing the l- side terms, MET reflection, the
# balanced pencil, its cubic and isolated root, the line pair and the two
# line-conic quadratics; per intersection point the residual check (and the
# rare polish), the energies' signs and the score.
FLOP_PER_VARIATION = 78
FLOP_PER_PAIRING = 257
FLOP_PER_POINT = 63

# MI355X vector peaks (256 CUs at 2.4 GHz): FP64 78.6 TFLOP/s; FP32 157.3 with
# packed FP32, which this build does not use (non-packed FP32 issues at the
# FP64 rate).  The search kernel's arithmetic is FP64 apart from the draws and
# the cubic seeds, so the FP64 vector peak is its ceiling.
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200_000)
    ap.add_argument("--profile-only", action="store_true", help="few steps, no CPU baseline (for profilers)")
    ap.add_argument("--no-semilep", action="store_true", help="skip the single-neutrino reconstruction leg")
    ap.add_argument("--no-stream", action="store_true", help="skip the chunked-stream leg")
    ap.add_argument("--no-chi2", action="store_true", help="skip the dileptonic chi^2 fit leg")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the further workloads (10k unsmeared, 4M ttH at 256 variations, 2M heavy-tailed)")
    ap.add_argument("--workloads-only", action="store_true", help="run only the further workloads")
    ap.add_argument("--stream-only", action="store_true",
                    help="run only the chunked-stream leg and print its JSON object (for profilers)")
    ap.add_argument("--stream-chunks", type=int, default=50)
    ap.add_argument("--stream-pool", type=int, default=4,
                    help="distinct generated chunks the stream cycles through (each pass gets new event ids)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB a few times (to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters into bytes) and exit")
    return ap.parse_args()


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU in this build; the path shards by event ranges and "
              "needs no collective, but multi-GPU runs are not part of it.", file=sys.stderr)
        sys.exit(2)
    import torch

    import hfgen
    from paper_2211_14346_amd import binding as B
    from paper_2211_14346_amd.chain import Chain

    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}))
        return
    if args.stream_only:
        print(json.dumps({"stream": stream_leg(args, torch)}))
        return
    if args.workloads_only:
        print(json.dumps({"workloads": {name: workload_leg(args, torch, name) for name in EXTRA_WORKLOADS}}))
        return
    cfg = hfgen.config(WORKLOAD)
    t0 = time.time()
    ev = hfgen.generate(cfg)
    print(f"[bench] generated {ev['n']} events in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def run_form(precision, steps, warmup):
        ch = Chain(ev, cfg["cuts"], cfg["reco"], precision=precision)
        for _ in range(max(1, warmup)):
            ch.step()
        torch.cuda.synchronize()
        ch.capture(reorder=True)  # each step ends with the device-side reordering
        ch.reset_counters()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            ch.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t_start
        return ch, dt

    ch, dt = run_form(args.precision, args.steps, args.warmup)
    n = ev["n"]
    ms_per_step = 1e3 * dt / args.steps
    value = n * args.steps / dt
    print(f"[bench] {args.precision}: {ms_per_step:.3f} ms/step, {value:.4g} events/s", file=sys.stderr, flush=True)

    # ---- dominant kernel: the reconstruction search, timed alone with HIP events
    res = ch.results()
    kname = "k_search_ev<float>" if args.precision == "mixed" else "k_search_ev<double>"
    roofline = search_roofline(B, ch, args.steps, kname)
    roofline["traffic"] = measured_traffic(kname)
    roofline["issued_view"] = issued_view(kname, roofline["kernel_ms"])
    sel_roof = select_roofline(torch, ch, ev)

    out = {"metric": cfg_metric(), "value": round(value, 1), "unit": "events/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": WORKLOAD, "events": n, "variations": cfg["reco"]["n_var"],
                      "cuts": [c["name"] for c in cfg["cuts"]], "precision": args.precision,
                      "survivors": int(res["count"]), "reconstructed": int(len(res["final"])),
                      "parallelism": "1 GPU"},
           "roofline": roofline, "select_roofline": sel_roof}

    if not args.profile_only and not args.no_fp64_form and args.precision == "mixed":
        del ch
        torch.cuda.empty_cache()
        ch64, dt64 = run_form("fp64", max(3, args.steps // 2), 1)
        out["fp64_form"] = {"value": round(n * max(3, args.steps // 2) / dt64, 1), "unit": "events/s",
                            "ms_per_step": round(1e3 * dt64 / max(3, args.steps // 2), 4)}
        ch = ch64

    if not args.profile_only and not args.no_cpu_baseline:
        out["cpu_baseline"], acc = cpu_baseline(ev, cfg, args, torch)
        out["accuracy_vs_oracle"] = acc
    if not args.no_semilep:
        del ch
        torch.cuda.empty_cache()
        out["semilep"] = semilep_leg(args, torch)
    if not args.no_chi2:
        torch.cuda.empty_cache()
        out["chi2"] = chi2_leg(args, torch, ev, cfg)
    if not args.no_stream:
        torch.cuda.empty_cache()
        out["stream"] = stream_leg(args, torch)
    if not args.no_workloads:
        out["workloads"] = {}
        for name in EXTRA_WORKLOADS:
            torch.cuda.empty_cache()
            out["workloads"][name] = workload_leg(args, torch, name)
    print(json.dumps(out))


def search_roofline(B, ch, steps, kname):
    """The reconstruction search kernel of a chain timed alone (HIP events that
    hf_ttbar_reco records around it) over a few launches; its algorithmic
    FP64 work from the launch's unit counts (variations, pairings,
    intersection points) against the FP64 vector peak."""
    stats0 = ch.out.t["stats"].cpu().numpy().astype(np.int64).copy()
    timer = B.KernelTimer()
    kms = []
    with timer:
        for _ in range(max(3, min(10, steps))):
            ch.run_reco()
            kms.append(timer.elapsed_ms())
    timer.close()
    stats1 = ch.out.t["stats"].cpu().numpy().astype(np.int64)
    per = (stats1 - stats0) / len(kms)  # events, variations, pairings, points, solutions per launch
    kernel_ms = float(np.mean(kms))
    flops = FLOP_PER_VARIATION * per[1] + FLOP_PER_PAIRING * per[2] + FLOP_PER_POINT * per[3]
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": kname,
            "achieved": round(achieved, 3), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_ALU_TFLOPS, 4), "traffic": None,
            "kernel_ms": round(kernel_ms, 4), "flop_per_launch": float(flops),
            "units_per_launch": {"events": int(per[0]), "variations": int(per[1]), "pairings": int(per[2]),
                                 "points": int(per[3]), "solutions": int(per[4])},
            "flop_per_unit": {"variation": FLOP_PER_VARIATION, "pairing": FLOP_PER_PAIRING,
                              "point": FLOP_PER_POINT}}


# Algorithmic HBM bytes of the cut stage per event (hf_select): the two
# offsets of each object list (16), per lepton pT, eta and charge (12), per
# jet pT, eta and b-tag (12), MET (8) and the survive byte (1); cuts that
# read phi and E (M_ll, isolation) add 8 per object.  A cut after an event's
# first failure reads nothing, so this counts every column once per event:
# the bytes a chain of these cuts needs when no event is dropped early.
def select_bytes(ev, cuts):
    n = ev["n"]
    n_lep, n_jet = int(ev["lep_off"][-1]), int(ev["jet_off"][-1])
    kinds = {c["kind"] for c in cuts}
    per_obj = 12 + (8 if kinds & {"MLL_MIN", "LEP_ISO"} else 0)
    return n * (16 + 8 + 1) + (n_lep + n_jet) * per_obj


def select_roofline(torch, ch, ev):
    """hf_select of a chain timed alone with torch events on its stream, against
    the HBM peak with the cut stage's algorithmic bytes."""
    s = torch.cuda.current_stream()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    ch.run_select()
    for a, b in pairs:
        a.record(s)
        ch.run_select()
        b.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in pairs]))
    nbytes = select_bytes(ev, ch.cuts)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_select", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "kernel_ms": round(ms, 4), "bytes_per_launch": int(nbytes),
            "note": "bytes of every column the chain reads, once per event; waves whose events have all "
                    "failed skip the later cuts' columns, so the kernel may read less"}


def workload_leg(args, torch, name):
    """One further workload of the hot path: generated at its stated size,
    select -> compact -> reconstruction -> compact -> device reorder recorded
    as one HIP graph per step; the search kernel's roofline from its unit
    counts; the oracle on the first 2^16 events beside it (with the GPU's
    agreement on those events).  The 8-cut ttH chain also runs with the cut
    order fixed at the user's order (no reordering) for comparison; the
    heavy-tailed batch reports the autotuner's choice of launch."""
    import hfgen
    from paper_2211_14346_amd import binding as B
    from paper_2211_14346_amd.chain import Chain

    cfg = hfgen.config(name)
    t0 = time.time()
    ev = hfgen.generate(cfg)
    n = ev["n"]
    print(f"[bench] {name}: generated {n} events in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    steps = max(3, args.steps // 2) if n >= 2_000_000 else args.steps
    leg = {"metric": "events/s through cut chain + ttbar reco; % VALU roofline of the search kernel",
           "unit": "events/s", "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": name, "events": n, "cuts": [c["name"] for c in cfg["cuts"]],
                      "variations": "per event (1..1024 log-uniform)" if cfg.get("var_mode") else cfg["reco"]["n_var"],
                      "precision": "mixed"}}
    ch = Chain(ev, cfg["cuts"], cfg["reco"], precision="mixed")
    ch.step()
    torch.cuda.synchronize()
    if cfg.get("var_mode"):
        # the autotuner on this batch: both schedules timed, the faster one kept
        res0 = ch.results()
        p = ch.params
        ms = B.ttbar_reco_autotune(ch.dev, ch.idx, ch.count, ch.n, p, ch.out, ch.ws_reco)
        leg["autotune"] = {"choice": B.SCHED_NAME.get(int(p.schedule), int(p.schedule)),
                           "ms_per_call": {"event (4 waves/workgroup)": round(ms[0], 4),
                                           "event_wg128 (2 waves/workgroup)": round(ms[1], 4),
                                           "event_wg64 (1 wave/workgroup)": round(ms[2], 4)},
                           "survivors": int(res0["count"])}
        ch.params = p
    if name == "tth4M_v256":
        # the user's order, never reordered
        g_user = ch.capture(reorder=False)
        ch.reset_counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ch.replay()
        torch.cuda.synchronize()
        dt_user = time.perf_counter() - t0
        sel_user = select_roofline(torch, ch, ev)
        del g_user
        ch.graph = None
        # adaptive: reorder from the counters after each step until the order settles
        for _ in range(3):
            ch.step(reorder=True)
        torch.cuda.synchronize()
        order = [cfg["cuts"][k]["name"] for k in ch.order.cpu().numpy()]
        leg["orders"] = {"user": {"order": [c["name"] for c in cfg["cuts"]], "ms_per_step": round(1e3 * dt_user / steps, 4),
                                  "select_ms": sel_user["kernel_ms"]},
                         "adaptive": {"order": order}}
    for _ in range(max(1, args.warmup)):
        ch.step(reorder=True)
    torch.cuda.synchronize()
    ch.capture(reorder=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ch.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    leg["value"] = round(n * steps / dt, 1)
    leg["ms_per_step"] = round(1e3 * dt / steps, 4)
    leg["steps"] = steps
    res = ch.results()
    leg["config"]["survivors"] = int(res["count"])
    leg["config"]["reconstructed"] = int(len(res["final"]))
    leg["roofline"] = search_roofline(B, ch, steps, "k_search_ev<float>")
    leg["select_roofline"] = select_roofline(torch, ch, ev)
    if "orders" in leg:
        leg["orders"]["adaptive"]["ms_per_step"] = leg["ms_per_step"]
        leg["orders"]["adaptive"]["select_ms"] = leg["select_roofline"]["kernel_ms"]
    if name == "ttbar10k":
        leg["roofline"]["note"] = ("10k events at one variation: the launch is too small to fill the GPU, "
                                   "its time is launch latency, not arithmetic")
    print(f"[bench] {name}: {leg['ms_per_step']} ms/step, search {leg['roofline']['kernel_ms']} ms, "
          f"frac {leg['roofline']['frac']}", file=sys.stderr, flush=True)
    if not args.profile_only and not args.no_cpu_baseline:
        import oracle
        from tests.gpu_compare import compare
        m = min(n, 1 << 16)
        sub = hfgen.subset(ev, np.arange(m))
        threads = min(os.cpu_count() or 1, 16)
        oracle.lib()
        t0 = time.perf_counter()
        surv, _, _ = oracle.select(sub, cfg["cuts"], list(range(len(cfg["cuts"]))))
        idx = oracle.compact(surv)
        rec = oracle.ttbar_reco(sub, idx, cfg["reco"], n_threads=threads)
        oracle.compact(rec["has_sol"], 0, idx)
        dtc = time.perf_counter() - t0
        leg["cpu_baseline"] = {"value": round(m / dtc, 1), "unit": "events/s", "cores": threads, "kind": "oracle",
                               "sample": f"first {m} events of the {name} batch (a seeded subset: the generator "
                                         f"draws events independently), select+compact+reco+compact, "
                                         f"{dtc:.1f} s wall on {threads} threads"}
        k = int(np.searchsorted(res["idx"], m))  # compacted positions of the sample's survivors
        assert np.array_equal(res["idx"][:k], idx)
        st = compare({kk: v[:k] for kk, v in res["reco"].items() if kk != "stats"}, rec)
        leg["accuracy_vs_oracle"] = {kk: (round(v, 8) if isinstance(v, float) else v) for kk, v in st.items()}
    del ch
    return leg


# Algorithmic FP64 operations of the chi^2 fit (hf_dilep_chi2_reco), counted
# by hand from its formulas (add, mul, div, sqrt = 1, FMA = 2): per split
# point the two neutrinos' transverse momenta (8); per lepton side the p_z
# quadratic with both roots and their mass-shell tests (21) and per root the
# neutrino energy and l + nu (7); per candidate, side and root the top mass
# and its term (16); per candidate the sum of the two sides (1).  A root on
# the W mass shell has a zero W term, which is not computed (the real part of
# a complex pair and the squaring's extra root are rare and not counted).
# Per split point: 8 + 2 * (21 + 2 * 7) = 78, plus 65 per candidate.
CHI2_FLOP_POINT = 78
CHI2_FLOP_POINT_CAND = 65


def chi2_candidates(ev, idx, cp):
    """b candidates per compacted event, by the staging rule: tagged selected
    jets (at most max_cands), filled up to two with untagged selected ones."""
    e = np.asarray(idx, dtype=np.int64)
    jo = ev["jet_off"].astype(np.int64)
    sel = (ev["jet_pt"] > np.float32(cp["jet_pt_min"])) & (np.abs(ev["jet_eta"]) < np.float32(cp["jet_eta_max"]))
    tag = sel & (ev["jet_btag"] > np.float32(cp["btag_min"]))
    cs = np.concatenate([[0], np.cumsum(sel, dtype=np.int64)])
    ct = np.concatenate([[0], np.cumsum(tag, dtype=np.int64)])
    n_sel = cs[jo[e + 1]] - cs[jo[e]]
    n_tag = np.minimum(ct[jo[e + 1]] - ct[jo[e]], cp["max_cands"])
    return np.where(n_tag >= 2, n_tag, np.minimum(n_sel, 2))


def chi2_leg(args, torch, ev, cfg):
    """select -> compact -> hf_dilep_chi2_reco -> compact -> reorder over the
    benchmark batch (1M events), one HIP graph per step; the fit's kernel
    timed alone with HIP events on its stream; the oracle beside it."""
    from paper_2211_14346_amd.chain import Chain

    cp = cfg["chi2"]
    n = ev["n"]
    ch = Chain(ev, cfg["cuts"], None, chi2=cp)
    for _ in range(max(1, args.warmup)):
        ch.step()
    torch.cuda.synchronize()
    ch.capture(reorder=True)
    ch.reset_counters()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        ch.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = ch.results()
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    for a, b in evs:
        a.record(s)
        ch.run_reco()
        b.record(s)
    torch.cuda.synchronize()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    nc = chi2_candidates(ev, res["idx"], cp)
    ok = res["reco"]["has_sol"].astype(bool)
    points = cp["n_grid"] ** 2 + 25 * cp["n_refine"]
    flops = float(points * (CHI2_FLOP_POINT * ok.sum() + CHI2_FLOP_POINT_CAND * nc[ok].sum()))
    tf = flops / (kernel_ms * 1e-3) / 1e12
    leg = {"metric": "events/s through cut chain + dileptonic chi^2 fit with a MET split",
           "value": round(n * steps / dt, 1), "unit": "events/s", "ms_per_step": round(1e3 * dt / steps, 4),
           "dtype": "f64",
           "config": {"workload": WORKLOAD, "events": n, "grid": f"{cp['n_grid']}x{cp['n_grid']} + "
                      f"{cp['n_refine']} x 5x5", "survivors": int(res["count"]), "fitted": int(ok.sum())},
           "roofline": {"bound": "alu", "kernel": "k_chi2", "achieved": round(tf, 3), "peak": PEAK_ALU_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tf / PEAK_ALU_TFLOPS, 4),
                        "traffic": measured_traffic("k_chi2", "chi2"),
                        "kernel_ms": round(kernel_ms, 4), "flop_per_launch": flops,
                        "units_per_launch": {"events": int(ok.sum()), "split_points_per_event": points,
                                             "candidates": int(nc[ok].sum())},
                        "flop_per_unit": {"point": CHI2_FLOP_POINT, "point_candidate": CHI2_FLOP_POINT_CAND}}}
    print(f"[bench] chi2: {leg['ms_per_step']} ms/step, kernel {kernel_ms:.3f} ms, {tf:.2f} TFLOP/s",
          file=sys.stderr, flush=True)
    if not args.profile_only and not args.no_cpu_baseline:
        import hfgen
        import oracle
        from tests.gpu_compare import compare_chi2
        threads = min(os.cpu_count() or 1, 16)
        m = min(args.cpu_sample, n)
        sub = hfgen.subset(ev, np.arange(m))
        t0 = time.perf_counter()
        surv, _, _ = oracle.select(sub, cfg["cuts"], list(range(len(cfg["cuts"]))))
        idx = oracle.compact(surv)
        rec = oracle.dilep_chi2_reco(sub, idx, cp, n_threads=threads)
        oracle.compact(rec["has_sol"], 0, idx)
        dtc = time.perf_counter() - t0
        leg["cpu_baseline"] = {"value": round(m / dtc, 1), "unit": "events/s", "cores": threads, "kind": "oracle",
                               "sample": f"first {m} events of the {WORKLOAD} batch, select+compact+fit+compact, "
                                         f"{dtc:.1f} s wall on {threads} threads"}
        k = int(idx.size)
        st = compare_chi2({kk: v[:k] for kk, v in res["reco"].items()}, rec)
        leg["accuracy_vs_oracle"] = {kk: (round(v, 12) if isinstance(v, float) else v) for kk, v in st.items()}
    return leg


def stream_leg(args, torch):
    """50 chunks of 1M mixed events (dileptonic and semileptonic ttbar,
    t-channel, semileptonic and dileptonic Wt, background) streamed from
    pinned host memory through the five signal bins of section 6.1, each with
    its reconstruction: two device slots, copies on their own stream
    overlapped with compute.  Also the copy-only and compute-only rates of
    the same chunks, to show which one bounds the stream."""
    import hfgen
    from paper_2211_14346_amd.stream import Channel, EventStream, HostChunk

    cfg = hfgen.config(STREAM_WORKLOAD)
    m = cfg["chunk"]
    n_chunks = max(2, 10 if args.profile_only else args.stream_chunks)
    t0 = time.time()
    pool = [hfgen.stream_chunk(cfg, i)[0] for i in range(max(1, args.stream_pool))]
    print(f"[bench] stream: generated {len(pool)} chunks in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    # chunk i reuses pool[i % P]'s kinematics with its own event ids (and so its own variation draws);
    # chunks travel in the packed transfer format (bytes for counts, charges, b-tags) when lossless
    host = [HostChunk(ev, 0, packed="auto") for ev in pool]
    chunks = [host[i % len(host)].with_base(i * m) for i in range(n_chunks)]
    lep_cap = max(c.n_lep for c in host)
    jet_cap = max(c.n_jet for c in host)
    chans = []
    for name, cuts in cfg["chains"].items():  # the five signal bins, each with its reconstruction
        kind, arg = hfgen.configs.HLHC_BIN_RECO[name]
        if kind == "semilep":
            chans.append(Channel(name, cuts, m, semilep=cfg["semilep"], topology=arg))
        elif kind == "chi2":
            chans.append(Channel(name, cuts, m, chi2=dict(cfg["chi2"], n_top=arg)))
        else:
            chans.append(Channel(name, cuts, m, reco=cfg["reco"]))
    es = EventStream(chans, m, lep_cap, jet_cap)
    # warm-up: one untimed pass over the whole stream (the first pass pays
    # one-time host costs of the copies and launches, about 0.5 ms a chunk)
    es.run(chunks)
    torch.cuda.synchronize()
    es.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    es.run(chunks)
    t_issue = time.perf_counter() - t0
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cnt = {ch.name: ch.counters.cpu().numpy() for ch in chans}
    # copy only: the same H2D copies, alternating slots, no compute
    t1 = time.perf_counter()
    for i, hc in enumerate(chunks):
        es.slots[i % 2].load(hc, es.copy_stream)
    es.copy_stream.synchronize()
    dt_copy = time.perf_counter() - t1
    # compute only: the channels on a resident chunk
    es.slots[0].load(chunks[0], es.copy_stream)
    es.copy_stream.synchronize()
    reps = min(10, n_chunks)
    t2 = time.perf_counter()
    for _ in range(reps):
        for ch in chans:
            ch.run(es.slots[0], es.compute_stream)
    es.compute_stream.synchronize()
    dt_comp = (time.perf_counter() - t2) / reps
    nbytes = sum(c.nbytes for c in chunks)
    n = m * n_chunks
    # the same stream in the plain layout (32-bit offsets, float charges and b-tags), for comparison
    plain_host = [HostChunk(ev, 0, packed=False) for ev in pool]
    plain = [plain_host[i % len(plain_host)].with_base(i * m) for i in range(n_chunks)]
    es.run(plain)
    torch.cuda.synchronize()
    es.reset()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    es.run(plain)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t3
    leg = {"metric": "events/s end to end, pinned host chunks -> the five HL-LHC signal bins (37 cuts; "
                     "single-neutrino chi^2 x3, dileptonic two-neutrino solve @64 variations, chi^2 fit with a MET split)",
           "value": round(n / dt, 1), "unit": "events/s", "dtype": "f32+f64",
           "ms_per_chunk": round(1e3 * dt / n_chunks, 4),
           "config": {"workload": STREAM_WORKLOAD, "events": n, "chunk": m, "chunks": n_chunks,
                      "distinct_chunks": len(pool), "cuts": len(cfg["cuts"]),
                      "fractions": cfg["fractions"], "variations": cfg["reco"]["n_var"],
                      "bins": {ch.name: {"reconstruction": "/".join(str(x) for x in hfgen.configs.HLHC_BIN_RECO[ch.name]
                                                                   if x is not None),
                                         "selected": int(cnt[ch.name][ch.reco_id, 0]),
                                         "reconstructed": int(cnt[ch.name][ch.reco_id, 1])} for ch in chans},
                      "input_bytes": int(nbytes)},
           "h2d_only": {"GB_per_s": round(nbytes / dt_copy / 1e9, 2), "ms_per_chunk": round(1e3 * dt_copy / n_chunks, 4)},
           "compute_only": {"events_per_s": round(m / dt_comp, 1), "ms_per_chunk": round(1e3 * dt_comp, 4)},
           "overlap": round(max(dt_copy / n_chunks, dt_comp) / (dt / n_chunks), 3),
           "host_issue_ms_per_chunk": round(1e3 * t_issue / n_chunks, 4),
           "h2d_GB_per_s_in_stream": round(nbytes / dt / 1e9, 2),
           "transfer_format": "packed" if all(c.packed for c in chunks) else "plain",
           "plain_layout": {"events_per_s": round(n / dt_plain, 1), "ms_per_chunk": round(1e3 * dt_plain / n_chunks, 4),
                            "input_bytes": int(sum(c.nbytes for c in plain))}}
    print(f"[bench] stream: {leg['ms_per_chunk']} ms/chunk, copy {leg['h2d_only']['ms_per_chunk']} ms, "
          f"compute {leg['compute_only']['ms_per_chunk']} ms", file=sys.stderr, flush=True)
    return leg


# Algorithmic HBM bytes of hf_semilep_reco per unit: per compacted event the
# index (4), the two offsets of each object list (16), MET (8) and the outputs
# (has_sol 1, root 1, four jet indices 8, nu 24, five masses/chi^2 40); per
# lepton of the event pT and eta (8) and for the chosen one phi and E (8); per
# jet pT and eta (8) and for each candidate jet phi and E (8).
SL_BYTES_EVENT = 4 + 16 + 8 + (1 + 1 + 8 + 24 + 40)
SL_BYTES_OBJ = 8
SL_BYTES_PICKED = 8


def semilep_bytes(ev, idx, sl):
    """Algorithmic bytes of one hf_semilep_reco launch over the compacted ids."""
    e = np.asarray(idx, dtype=np.int64)
    lo, jo = ev["lep_off"].astype(np.int64), ev["jet_off"].astype(np.int64)
    n_lep = int((lo[e + 1] - lo[e]).sum())
    n_jet = int((jo[e + 1] - jo[e]).sum())
    sel = (ev["jet_pt"] > np.float32(sl["jet_pt_min"])) & (np.abs(ev["jet_eta"]) < np.float32(sl["jet_eta_max"]))
    csel = np.concatenate([[0], np.cumsum(sel, dtype=np.int64)])
    n_cand = int(np.minimum(csel[jo[e + 1]] - csel[jo[e]], sl["max_cands"]).sum())
    return e.size * (SL_BYTES_EVENT + SL_BYTES_PICKED) + (n_lep + n_jet) * SL_BYTES_OBJ + n_cand * SL_BYTES_PICKED


def semilep_leg(args, torch):
    """select -> compact -> hf_semilep_reco (t-channel) -> compact -> reorder,
    one HIP graph per step over 1M one-lepton events; the reconstruction
    kernel timed alone with HIP events on its stream; the oracle beside it."""
    import hfgen
    from paper_2211_14346_amd.chain import Chain

    cfg = hfgen.config(SEMILEP_WORKLOAD)
    ev = hfgen.generate(cfg)
    n = ev["n"]
    ch = Chain(ev, cfg["cuts"], None, semilep=cfg["semilep"], topology="TCHAN")
    for _ in range(max(1, args.warmup)):
        ch.step()
    torch.cuda.synchronize()
    ch.capture(reorder=True)
    ch.reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ch.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = ch.results()
    # the reconstruction kernel alone (one launch per call, on torch's current stream)
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(max(3, min(10, args.steps)))]
    for a, b in evs:
        a.record(s)
        ch.run_reco()
        b.record(s)
    torch.cuda.synchronize()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    nbytes = semilep_bytes(ev, res["idx"], cfg["semilep"])
    gbs = nbytes / (kernel_ms * 1e-3) / 1e9
    leg = {"metric": "events/s through cut chain + single-neutrino chi^2 reco (t-channel)",
           "value": round(n * args.steps / dt, 1), "unit": "events/s",
           "ms_per_step": round(1e3 * dt / args.steps, 4), "dtype": "f64",
           "config": {"workload": SEMILEP_WORKLOAD, "events": n, "topology": "TCHAN",
                      "cuts": [c["name"] for c in cfg["cuts"]], "survivors": int(res["count"]),
                      "reconstructed": int(len(res["final"]))},
           "roofline": {"bound": "hbm", "kernel": "k_semilep_tchan", "achieved": round(gbs, 1),
                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                        "traffic": measured_traffic("k_semilep_tchan", "semilep"), "kernel_ms": round(kernel_ms, 4),
                        "bytes_per_launch": int(nbytes)}}
    print(f"[bench] semilep: {leg['ms_per_step']} ms/step, kernel {kernel_ms:.4f} ms, {gbs:.0f} GB/s",
          file=sys.stderr, flush=True)
    if not args.profile_only and not args.no_cpu_baseline:
        import oracle
        from tests.gpu_compare import compare_semilep
        threads = min(os.cpu_count() or 1, 16)
        oracle.lib()
        t0 = time.perf_counter()
        surv, _, _ = oracle.select(ev, cfg["cuts"], list(range(len(cfg["cuts"]))))
        idx = oracle.compact(surv)
        rec = oracle.semilep_reco(ev, idx, cfg["semilep"], "TCHAN", n_threads=threads)
        oracle.compact(rec["has_sol"], 0, idx)
        dtc = time.perf_counter() - t0
        leg["cpu_baseline"] = {"value": round(n / dtc, 1), "unit": "events/s", "cores": threads, "kind": "oracle",
                               "sample": f"all {n} events of the {SEMILEP_WORKLOAD} batch, "
                                         f"select+compact+reco+compact, {dtc:.1f} s wall on {threads} threads"}
        st = compare_semilep(res["reco"], rec)
        leg["accuracy_vs_oracle"] = {k: (round(v, 12) if isinstance(v, float) else v) for k, v in st.items()}
    return leg


def measured_traffic(kernel, kind="search"):
    """HBM bytes per launch of a profiled kernel (the search kernel, or the
    single-neutrino kernel with kind="semilep") from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE scaled by a device-copy
    calibration), or None when the summary is for another kernel or for
    different kernel sources than the ones built here."""
    from paper_2211_14346_amd.perf import built_source_hash, source_hash
    built = built_source_hash(kind)
    if built is None or built != source_hash(kind):
        return None  # library and sources differ: the counters cannot be attributed
    name = {"search": "k_search_ttbar1M_v64_counters.txt", "semilep": "k_semilep_tchan1M.txt",
            "chi2": "k_chi2_ttbar1M_v64.txt"}[kind]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get(f"{kind}_kernel") != kernel or kv.get(f"{kind}_source_hash") != built:
        return None
    return int(kv[f"{kind}_traffic_bytes_per_launch"])


def issued_view(kernel, kernel_ms):
    """Second view of the search kernel's roofline: the floating-point VALU
    instructions it issues (rocprofv3 SQ_INSTS_VALU_* per launch, from the
    committed counter summary) priced at the issue rates, against its
    measured time.  Each FP64 or FP32 add, multiply or FMA wave instruction
    takes 64 lane slots of the 39.3e12 per second behind the 78.6 TFLOP/s
    FP64 peak (FP32 without packed instructions issues at the same rate);
    transcendental instructions take four slots per lane.  None when the
    summary does not match the built sources."""
    from paper_2211_14346_amd.perf import built_source_hash, source_hash
    built = built_source_hash("search")
    path = os.path.join(ROOT, "profiles", "k_search_ttbar1M_v64_counters.txt")
    if built is None or built != source_hash("search") or not os.path.exists(path):
        return None
    vals, cur = {}, None
    for line in open(path):
        line = line.rstrip()
        if line.startswith("[") and line.endswith("]"):
            cur = line[1:-1]
        elif cur == kernel and line.startswith("  ") and "(" in line:
            parts = line.split()
            vals[parts[0]] = float(parts[1])
        elif line.startswith("search_source_hash:") and line.split(":", 1)[1].strip() != built:
            return None
    need = [f"SQ_INSTS_VALU_{op}_{t}" for t in ("F64", "F32") for op in ("FMA", "MUL", "ADD", "TRANS")]
    if any(k not in vals for k in need):
        return None
    slots = sum(vals[f"SQ_INSTS_VALU_{op}_{t}"] * (4.0 if op == "TRANS" else 1.0)
                for t in ("F64", "F32") for op in ("FMA", "MUL", "ADD", "TRANS"))
    t_star = 64.0 * slots / (PEAK_ALU_TFLOPS * 1e12 / 2.0)
    return {"t_star_ms": round(1e3 * t_star, 4), "frac": round(1e3 * t_star / kernel_ms, 4),
            "fp_wave_instructions": {k.replace("SQ_INSTS_VALU_", ""): vals[k] for k in need},
            "source": "profiles/k_search_ttbar1M_v64_counters.txt"}


def cfg_metric():
    return "events/s through cut chain + ttbar reco @64 variations; % HBM/VALU roofline"


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ev, cfg, args, torch):
    """The FP64 oracle on the first `cpu_sample` events of the same batch, on
    the host's cores; and the GPU forms' agreement with it on that sample."""
    import hfgen
    import oracle
    from paper_2211_14346_amd.chain import Chain
    from tests.gpu_compare import compare

    m = min(args.cpu_sample, ev["n"])
    sub = hfgen.subset(ev, np.arange(m))
    threads = min(os.cpu_count() or 1, 16)
    oracle.lib()
    t0 = time.perf_counter()
    surv, reached, passed = oracle.select(sub, cfg["cuts"], list(range(len(cfg["cuts"]))))
    idx = oracle.compact(surv)
    rec = oracle.ttbar_reco(sub, idx, cfg["reco"], n_threads=threads)
    oracle.compact(rec["has_sol"], 0, idx)
    dt = time.perf_counter() - t0
    base = {"value": round(m / dt, 1), "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} events of the {WORKLOAD} batch, select+compact+reco+compact, "
                      f"{dt:.1f} s wall on {threads} threads",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    # one core, on the first tenth of the sample
    m1 = max(1, m // 10)
    sub1 = hfgen.subset(ev, np.arange(m1))
    t0 = time.perf_counter()
    surv1, _, _ = oracle.select(sub1, cfg["cuts"], list(range(len(cfg["cuts"]))))
    idx1 = oracle.compact(surv1)
    rec1 = oracle.ttbar_reco(sub1, idx1, cfg["reco"], n_threads=1)
    oracle.compact(rec1["has_sol"], 0, idx1)
    dt1 = time.perf_counter() - t0
    base["single_core"] = {"value": round(m1 / dt1, 1), "unit": "events/s",
                           "sample": f"first {m1} events, {dt1:.1f} s on 1 thread"}
    acc = {}
    for prec in ("mixed", "fp64"):
        ch = Chain(sub, cfg["cuts"], cfg["reco"], precision=prec)
        ch.step()
        r = ch.results()
        st = compare(r["reco"], rec)
        acc[prec] = {k: (round(v, 8) if isinstance(v, float) else v) for k, v in st.items()}
        del ch
    return base, acc


if __name__ == "__main__":
    main()
