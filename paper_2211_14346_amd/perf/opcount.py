"""Per-unit algorithmic FLOP counts of the reconstruction search kernel.

Builds opcount.cpp (host) and runs it over a sample of smeared pairings of
the benchmark workload (1M-event ttbar sample, 64 variations): events from
hfgen, the same lepton and b-candidate rules as the kernel, Gaussian
resolution variations drawn with numpy (the counts depend on the
distribution of the inputs, not on the exact draws).  Prints the counts as
JSON; the benchmark multiplies them by the unit counts the kernel reports.

Per variation (not in the harness, counted from the kernel's formulas):
Box-Muller in FP32 for two Philox blocks (per pair: scale, log, sqrt,
cosine, sine, two products = 7), lepton smear factors, MET shifts and the
two W terms in FP64 (2 x 2 + 2 x 2 + 2 x 5 = 18), the per-candidate smear
factors and the l+ side terms (2 candidates x 16 = 32).
"""

import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

PER_VARIATION_FP32 = 4 * 7
PER_VARIATION_FP64 = 18 + 32


def _p4(ev, pre, k):
    pt, eta, phi, e = (float(ev[pre + c][k]) for c in ("pt", "eta", "phi", "e"))
    return np.array([e, pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)])


def sample_pairings(n_events=3000, n_var=64, seed=7):
    import hfgen
    cfg = hfgen.config("ttbar1M_v64")
    reco = cfg["reco"]
    ev = hfgen.generate(cfg, n_events=n_events, seed=seed)
    rng = np.random.default_rng(seed)
    rows = []
    for e in range(ev["n"]):
        lo, hi = ev["lep_off"][e], ev["lep_off"][e + 1]
        jo, jh = ev["jet_off"][e], ev["jet_off"][e + 1]
        sel = [k for k in range(lo, hi) if ev["lep_pt"][k] > 20 and abs(ev["lep_eta"][k]) < 2.5]
        if len(sel) != 2 or ev["lep_q"][sel[0]] * ev["lep_q"][sel[1]] >= 0:
            continue
        kp = sel[0] if ev["lep_q"][sel[0]] > 0 else sel[1]
        km = sel[1] if kp == sel[0] else sel[0]
        jets = [k for k in range(jo, jh) if ev["jet_pt"][k] > 25 and abs(ev["jet_eta"][k]) < 2.5]
        cand = [k for k in jets if ev["jet_btag"][k] > 0.5][:12]
        cand += [k for k in jets if not ev["jet_btag"][k] > 0.5][:max(0, 2 - len(cand))]
        if len(cand) < 2 or ev["met_x"][e] ** 2 + ev["met_y"][e] ** 2 <= 900:
            continue
        lp0, lm0 = _p4(ev, "lep_", kp), _p4(ev, "lep_", km)
        cv = [_p4(ev, "jet_", k) for k in cand]
        sig = [np.sqrt(reco["jet_a"] ** 2 / c[0] + reco["jet_c"] ** 2) for c in cv]
        for v in range(n_var):
            z = rng.standard_normal(4 + len(cand))
            lp = lp0 * max(1 + reco["lep_sigma"] * z[0], 0.01)
            lm = lm0 * max(1 + reco["lep_sigma"] * z[1], 0.01)
            mx = ev["met_x"][e] + reco["met_sigma"] * z[2]
            my = ev["met_y"][e] + reco["met_sigma"] * z[3]
            for i in range(len(cand)):
                for j in range(len(cand)):
                    if i == j:
                        continue
                    b = cv[i] * max(1 + sig[i] * z[4 + i], 0.01)
                    bb = cv[j] * max(1 + sig[j] * z[4 + j], 0.01)
                    rows.append(np.concatenate([lp, b, lm, bb, [mx, my]]))
    return np.asarray(rows, dtype=np.float64)


def build(out="/tmp/hf_opcount"):
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", os.path.join(HERE, "opcount.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def main():
    exe = build()
    rows = sample_pairings()
    path = "/tmp/hf_opcount_pairs.bin"
    rows.tofile(path)
    txt = subprocess.run([exe, path], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in txt.splitlines():
        parts = line.split()
        if parts[0] == "pairings":
            res.update(pairings=int(parts[1]), points=int(parts[3]), accepted=int(parts[5]))
        else:
            res[parts[0]] = {parts[k]: float(parts[k + 1]) for k in range(1, len(parts), 2)}
    res["per_variation"] = {"fp32_flops": PER_VARIATION_FP32, "fp64_flops": PER_VARIATION_FP64}
    res["flop_per_variation"] = PER_VARIATION_FP32 + PER_VARIATION_FP64
    res["flop_per_pairing"] = res["pairing_fp64_per_pairing"]["flops"] + res["pairing_fp32_per_pairing"]["flops"]
    res["flop_per_point"] = res["point_fp64_per_point"]["flops"] + res["point_fp32_per_point"]["flops"]
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
