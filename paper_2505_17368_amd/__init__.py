"""HENN (arXiv 2505.17368) on MI355X: C-ABI HIP library + thin Python binding."""
from .henn import (HennError, HennIndex, default_build_params, henn_build, henn_free,  # noqa: F401
                   henn_import, henn_search_batch, load_library, search_params)
