"""Content hash of the search kernel's sources.

A stored HBM-traffic measurement (rocprofv3 FETCH_SIZE / WRITE_SIZE) is only
reported while the kernel it was taken on is unchanged; this hash names it.
"""
import hashlib
import os

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
SEARCH_SOURCES = ("henn_search.hip", "henn_device.h", "henn_internal.h")


def search_kernel_hash() -> str:
    h = hashlib.sha256()
    for name in SEARCH_SOURCES:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]
