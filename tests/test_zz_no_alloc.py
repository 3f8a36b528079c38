"""henn_search_batch_noalloc: the search with the library's fixed scratch
array instead of any allocation, against henn_search_batch on the same
inputs (bit for bit), on two calls in a row, the second smaller."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2505_17368_amd as hn
    X, Q = wl.make("uniform_10k_d32")
    # complete root: the search needs root-scan keys in its scratch
    idx = hn.henn_build(to_dev(X), degree=16, graph=1, max_degree=32, root_complete_max=1000,
                        storage=2)
    yield hn, X, Q, idx
    idx.free()


@pytest.mark.parametrize("persistent", [False, True])
def test_noalloc_equals_search_batch_twice(setup, persistent):
    import torch
    hn, X, Q, idx = setup
    for nq in (1000, 300):           # the second call is smaller
        Qd = to_dev(Q[:nq])
        ref_i, ref_d = hn.henn_search_batch(idx, Qd, k=10, ef=64, persistent=persistent)
        out_i = torch.full((nq, 10), -7, dtype=torch.int32, device="cuda:0")
        out_d = torch.zeros((nq, 10), dtype=torch.float32, device="cuda:0")
        gi, gd = hn.henn_search_batch(idx, Qd, k=10, ef=64, persistent=persistent,
                                      noalloc=True, out_ids=out_i, out_dist=out_d)
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), ref_i.cpu().numpy()), nq
        assert np.array_equal(gd.cpu().numpy().view(np.uint32),
                              ref_d.cpu().numpy().view(np.uint32)), nq


def test_noalloc_rejects_a_search_beyond_its_scratch(setup):
    import torch
    hn, X, Q, idx = setup
    nq = 400_000                      # root keys and shortlists above 32 MiB
    Qd = torch.from_numpy(np.tile(Q[:1000], (nq // 1000, 1))).to("cuda:0")
    out_i = torch.empty((nq, 10), dtype=torch.int32, device="cuda:0")
    out_d = torch.empty((nq, 10), dtype=torch.float32, device="cuda:0")
    with pytest.raises(hn.HennError) as e:
        hn.henn_search_batch(idx, Qd, k=10, ef=64, noalloc=True, out_ids=out_i,
                             out_dist=out_d)
    assert e.value.status == 1 and "scratch" in str(e.value)      # HENN_E_INVAL
    torch.cuda.synchronize()
