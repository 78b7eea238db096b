"""Measurement helpers: per-unit FLOP counts of the reconstruction search
(opcount.py), rocprofv3 summaries (profile_summary.py) and the identity of
the kernel sources a summary was measured on."""

import hashlib
import os

_CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "csrc")

# Sources that determine the reconstruction search kernel's code.
SEARCH_SOURCES = ("hf_reco.hip", "hf_reco_math.hpp", "hf_device.hpp", "hf_internal.hpp")


def search_source_hash():
    """sha256 (first 16 hex digits) over the search kernel's sources."""
    h = hashlib.sha256()
    for name in SEARCH_SOURCES:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def built_source_hash():
    """The search_source_hash() of the sources libhf.so was built from, or
    None when the build recorded none."""
    path = os.path.join(os.path.dirname(_CSRC), "libhf.so.srchash")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return f.read().strip()
