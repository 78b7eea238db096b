"""Measurement helpers: per-unit FLOP counts of the reconstruction search
(opcount.py), rocprofv3 summaries (profile_summary.py) and the identity of
the kernel sources a summary was measured on."""

import hashlib
import os

_CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "csrc")

# Sources that determine each profiled kernel's code: the dileptonic
# reconstruction search, the single-neutrino reconstruction and the
# dileptonic chi^2 fit.
SOURCES = {
    "search": ("hf_reco.hip", "hf_reco_math.hpp", "hf_device.hpp", "hf_internal.hpp"),
    "semilep": ("hf_semilep.hip", "hf_device.hpp", "hf_internal.hpp"),
    "chi2": ("hf_chi2.hip", "hf_chi2.hpp", "hf_device.hpp", "hf_internal.hpp", "hf_reco_math.hpp"),
}
SEARCH_SOURCES = SOURCES["search"]


def source_hash(kind="search"):
    """sha256 (first 16 hex digits) over one kernel's sources."""
    h = hashlib.sha256()
    for name in SOURCES[kind]:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def search_source_hash():
    return source_hash("search")


def built_source_hash(kind="search"):
    """The source_hash(kind) of the sources libhf.so was built from, or None
    when the build recorded none."""
    path = os.path.join(os.path.dirname(_CSRC), "libhf.so.srchash")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 2 and parts[0] == kind:
                return parts[1]
    return None
