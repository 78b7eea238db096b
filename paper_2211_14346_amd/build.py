"""Builds libhf.so (gfx950) in-tree with hipcc.

Every HIP unit is compiled with packed-FP32 instruction selection disabled
(-packed-fp32-ops); the selection unit also with -ffp-contract=off so that
its FP64 comparisons round exactly as written.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhf.so")
ARCH = os.environ.get("HF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]

UNITS = {
    "hf_select.hip": ["-ffp-contract=off"],
    "hf_compact.hip": [],
    "hf_reco.hip": [],
    "hf_rng.hip": [],
    "hf_semilep.hip": [],
    "hf_api.cpp": [],
}


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(UNITS))) as ex:
        futs = [ex.submit(_compile, s, e) for s, e in UNITS.items()]
        objs = []
        for f in futs:
            obj, err = f.result()
            objs.append(obj)
            if verbose and err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # identity of the search kernel's sources this library was built from
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2211_14346_amd.perf import SOURCES, source_hash
    with open(LIB + ".srchash", "w") as f:
        for kind in SOURCES:
            f.write(f"{kind} {source_hash(kind)}\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
