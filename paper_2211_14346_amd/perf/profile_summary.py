"""Short text summaries of rocprofv3 runs of bench.py, for profiles/.

    python -m paper_2211_14346_amd.perf.profile_summary \\
        --trace DIR --pmc DIR [DIR ...] --cal-fetch DIR --cal-write DIR \\
        --cal-bytes N --hash H --out profiles/

DIR arguments are rocprofv3 output directories written with
`-o run --output-format csv` (run_kernel_stats.csv / run_counter_collection.csv).

Writes
  k_search_ttbar1M_v64_kernel_stats.txt   per-kernel calls and durations
  k_search_ttbar1M_v64_counters.txt       per-dispatch counters of each kernel,
                                          HBM traffic of the search kernel
  k_semilep_tchan1M.txt                   duration, counters and HBM traffic of
                                          the single-neutrino kernel (bench's
                                          second leg), with --semilep-hash
  stream_hlhc50M_kernel_stats.txt         per-kernel durations of the chunked
                                          stream, with --stream-trace
  k_chi2_ttbar1M_v64.txt                  duration (and traffic) of the
                                          dileptonic chi^2 fit's kernel
FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled into bytes by what
each reads for a plain device copy of known size (--cal-bytes read and
written once per copy): factor = copy bytes / (counter KiB * 1024).
"""

import argparse
import collections
import csv
import os

SEARCH = "k_search_ev<float>"
SEMILEP = "k_semilep_tchan"
TRACE_CMD = ("rocprofv3 --kernel-trace --stats -d <dir> -o run --output-format csv -- "
             "python3 bench.py --profile-only --steps 5 --warmup 1 --no-stream --no-workloads")
PMC_CMD = ("rocprofv3 --pmc <counters> -d <dir> -o run --output-format csv -- "
           "python3 bench.py --profile-only --steps 2 --warmup 1 --no-stream --no-workloads")
STREAM_TRACE_CMD = ("rocprofv3 --kernel-trace --stats -d <dir> -o run --output-format csv -- "
                    "python3 bench.py --stream-only --profile-only")
CAL_CMD = ("rocprofv3 --pmc <FETCH_SIZE|WRITE_SIZE> -d <dir> -o run --output-format csv -- "
           "python3 bench.py --copy-calibration 256")


def _short(name):
    n = name.replace("hf::(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0]


def kernel_stats(d):
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_stats.csv"))))
    return [(_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
             float(r["Percentage"])) for r in rows]


def counters(d):
    """{(kernel, counter): mean value per dispatch}, plus dispatch counts."""
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        vals[(_short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def copy_factor(d, counter, nbytes):
    c = counters(d)
    kib = [v for (k, name), (v, n) in c.items() if name == counter and "copyBuffer" in k]
    if not kib:
        raise SystemExit(f"no copy kernel with {counter} in {d}")
    return nbytes / (kib[0] * 1024.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--stream-trace", default=None, help="trace of the chunked-stream leg alone")
    ap.add_argument("--pmc", nargs="+", required=True)
    ap.add_argument("--cal-fetch", required=True)
    ap.add_argument("--cal-write", required=True)
    ap.add_argument("--cal-bytes", type=int, default=256 << 20)
    ap.add_argument("--hash", required=True, help="search kernel source hash of the profiled tree")
    ap.add_argument("--semilep-hash", default=None, help="single-neutrino kernel source hash of the profiled tree")
    ap.add_argument("--chi2-hash", default=None, help="chi^2 fit kernel source hash of the profiled tree")
    ap.add_argument("--out", default="profiles")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)

    ks = kernel_stats(a.trace)
    lines = ["# Kernel durations, bench workload ttbar1M_v64 (1M events, 64 variations, mixed precision)",
             f"# command: {TRACE_CMD}", f"# search kernel source hash: {a.hash}", "",
             f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>7s}"]
    for name, calls, avg, mn, mx, pct in ks:
        lines.append(f"{name[:40]:40s} {calls:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} {pct:7.2f}")
    with open(os.path.join(a.out, "k_search_ttbar1M_v64_kernel_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    fetch_f = copy_factor(a.cal_fetch, "FETCH_SIZE", a.cal_bytes)
    write_f = copy_factor(a.cal_write, "WRITE_SIZE", a.cal_bytes)
    merged = {}
    for d in a.pmc:
        merged.update(counters(d))
    # the search kernel is instantiated per workgroup size ("k_search_ev<float, 4>"):
    # its counters go under the family name, the instance that ran is recorded
    inst = sorted({k for k, _ in merged if k.startswith(SEARCH[:-1])})
    if inst:
        merged.update({(SEARCH, c): v for (k, c), v in list(merged.items()) if k == inst[0]})
        for k in [k for k in merged if k[0] == inst[0]]:
            del merged[k]
    kernels = sorted({k for k, _ in merged if k.startswith("k_")}, key=lambda k: (k != SEARCH, k))
    names = sorted({c for _, c in merged})
    lines = ["# Per-dispatch counters, bench workload ttbar1M_v64 (mixed precision)",
             f"# command (one run per counter group): {PMC_CMD}",
             f"# calibration: {CAL_CMD}",
             f"# calibration on a {a.cal_bytes} B device copy: bytes = FETCH_SIZE * 1024 * {fetch_f:.4f}, "
             f"bytes = WRITE_SIZE * 1024 * {write_f:.4f}",
             f"# search kernel source hash: {a.hash}", ""]
    for k in kernels:
        lines.append(f"[{k}]")
        for c in names:
            if (k, c) in merged:
                v, n = merged[(k, c)]
                lines.append(f"  {c:28s} {v:18.1f}   ({n} dispatches)")
    sf = merged.get((SEARCH, "FETCH_SIZE"))
    sw = merged.get((SEARCH, "WRITE_SIZE"))
    if sf and sw:
        fb, wb = sf[0] * 1024.0 * fetch_f, sw[0] * 1024.0 * write_f
        lines += ["", f"search_kernel: {SEARCH}", f"search_instance: {inst[0] if inst else SEARCH}",
                  f"search_fetch_bytes_per_launch: {fb:.0f}",
                  f"search_write_bytes_per_launch: {wb:.0f}", f"search_traffic_bytes_per_launch: {fb + wb:.0f}",
                  f"search_source_hash: {a.hash}"]
    with open(os.path.join(a.out, "k_search_ttbar1M_v64_counters.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    if a.stream_trace:
        lines = ["# Kernel durations of the chunked stream, workload hlhc50M (1M-event chunks of mixed events "
                 "from pinned host memory through the five signal bins of section 6.1 -- semileptonic and "
                 "dileptonic ttbar, t-channel, semileptonic and dileptonic Wt -- each a cut chain ending in its "
                 "reconstruction: single-neutrino chi^2 (ttbar, t-channel, Wt topologies), the two-neutrino solve "
                 "at 64 variations, the MET-split chi^2 with one top; 10 chunks after a full warm-up pass)",
                 f"# command: {STREAM_TRACE_CMD}", "",
                 f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>7s}"]
        for name, calls, avg, mn, mx, pct in kernel_stats(a.stream_trace):
            lines.append(f"{name[:40]:40s} {calls:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} {pct:7.2f}")
        with open(os.path.join(a.out, "stream_hlhc50M_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")

    row = [r for r in ks if r[0] == "k_chi2"]
    if row:
        name, calls, avg, mn, mx, pct = row[0]
        cf, cw = merged.get(("k_chi2", "FETCH_SIZE")), merged.get(("k_chi2", "WRITE_SIZE"))
        lines = ["# Dileptonic chi^2 fit with a MET split (hf_dilep_chi2_reco), bench workload ttbar1M_v64 "
                 "(311868 events after the 4 cuts, 17x17 + 2 x 5x5 split points)",
                 f"# trace command: {TRACE_CMD}", "",
                 f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}",
                 f"{name[:40]:40s} {calls:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f}"]
        if cf and cw:
            lines += ["", f"# counter command (one run per counter): {PMC_CMD}",
                      f"FETCH_SIZE KiB per dispatch  {cf[0]:12.1f}   ({cf[1]} dispatches)",
                      f"WRITE_SIZE KiB per dispatch  {cw[0]:12.1f}   ({cw[1]} dispatches)",
                      f"calibration on a {a.cal_bytes} B device copy: bytes = FETCH_SIZE * 1024 * {fetch_f:.4f}, "
                      f"bytes = WRITE_SIZE * 1024 * {write_f:.4f}", "",
                      "chi2_kernel: k_chi2", f"chi2_avg_us: {avg / 1e3:.2f}",
                      f"chi2_traffic_bytes_per_launch: {cf[0] * 1024.0 * fetch_f + cw[0] * 1024.0 * write_f:.0f}"]
            if a.chi2_hash:
                lines.append(f"chi2_source_hash: {a.chi2_hash}")
        with open(os.path.join(a.out, "k_chi2_ttbar1M_v64.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")

    lf, lw = merged.get((SEMILEP, "FETCH_SIZE")), merged.get((SEMILEP, "WRITE_SIZE"))
    row = [r for r in ks if r[0] == SEMILEP]
    if a.semilep_hash and lf and lw and row:
        name, calls, avg, mn, mx, pct = row[0]
        fb, wb = lf[0] * 1024.0 * fetch_f, lw[0] * 1024.0 * write_f
        lines = ["# Single-neutrino chi^2 reconstruction (t-channel), bench workload tchan1M "
                 "(1M one-lepton events, 4 cuts + hf_semilep_reco)",
                 f"# trace command: {TRACE_CMD}",
                 f"# counter command (one run per counter): {PMC_CMD}",
                 f"# calibration: {CAL_CMD}",
                 f"# calibration on a {a.cal_bytes} B device copy: bytes = FETCH_SIZE * 1024 * {fetch_f:.4f}, "
                 f"bytes = WRITE_SIZE * 1024 * {write_f:.4f}", "",
                 f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}",
                 f"{name[:40]:40s} {calls:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f}", "",
                 f"FETCH_SIZE KiB per dispatch  {lf[0]:12.1f}   ({lf[1]} dispatches)",
                 f"WRITE_SIZE KiB per dispatch  {lw[0]:12.1f}   ({lw[1]} dispatches)", "",
                 f"semilep_kernel: {SEMILEP}", f"semilep_avg_us: {avg / 1e3:.2f}",
                 f"semilep_fetch_bytes_per_launch: {fb:.0f}", f"semilep_write_bytes_per_launch: {wb:.0f}",
                 f"semilep_traffic_bytes_per_launch: {fb + wb:.0f}", f"semilep_source_hash: {a.semilep_hash}"]
        with open(os.path.join(a.out, "k_semilep_tchan1M.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
