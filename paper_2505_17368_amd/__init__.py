"""HENN (arXiv 2505.17368) on MI355X: C-ABI HIP library + thin Python binding."""
from .henn import (GRAPH, SAMPLER, HennError, HennIndex, default_build_params,  # noqa: F401
                   henn_autotune, henn_build, henn_delete, henn_free, henn_import, henn_insert,
                   henn_nsw_insert, henn_search_batch, load_library, search_params, SearchGraph, Server,
                   workspace_size)
