"""Error paths of the library on the GPU, driven by the test-only allocation
injector (include/henn_testing.h): every device allocation that a build, a
search or a server needs can fail; the call then returns HENN_E_NOMEM, frees
what it had allocated, and the next calls work as if nothing had happened."""
import numpy as np
import pytest

import workloads as wl
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture
def hn():
    import paper_2505_17368_amd as hn
    from paper_2505_17368_amd import henn
    yield henn
    henn.fail_alloc_after(-1)


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _first_success(hn, call, limit=400):
    """Runs call() with the injector at n = 0, 1, 2, ... until it succeeds;
    every failure must be HENN_E_NOMEM.  Returns (n, result)."""
    for n in range(limit):
        hn.fail_alloc_after(n)
        try:
            out = call()
        except hn.HennError as e:
            assert e.status == hn.HENN_E_NOMEM, (n, str(e))
            continue
        finally:
            hn.fail_alloc_after(-1)
        return n, out
    raise AssertionError("never succeeded")


def test_build_search_and_server_fail_cleanly_at_every_allocation(hn):
    import torch
    X, Q = wl.make("uniform_10k_d32")
    X, Q = X[:3000], Q[:200]
    kw = dict(degree=12, graph=1, max_degree=24, root_complete_max=400, storage=2)
    Xd, Qd = to_dev(X), to_dev(Q)
    ref = hn.henn_build(Xd, **kw)
    ref_i, ref_d = hn.henn_search_batch(ref, Qd, k=10, ef=32, persistent=True)
    ref_i, ref_d = ref_i.cpu().numpy(), ref_d.cpu().numpy()
    # a first server makes the runtime set up the hardware queues behind its two
    # streams; HIP keeps those for later streams, so they are not counted below
    hn.Server(ref, max_slots=64, pool_bytes=4 << 20, k_max=10, ef_max=32).close()
    ref.free()
    before = _free_bytes()

    n_build, idx = _first_success(hn, lambda: hn.henn_build(Xd, **kw))
    print(f"build: {n_build} device allocations; every earlier failure returned NOMEM")
    assert n_build >= 10

    # a persistent search allocates its work counter and root-scan scratch
    n_search, (gi, gd) = _first_success(
        hn, lambda: hn.henn_search_batch(idx, Qd, k=10, ef=32, persistent=True))
    torch.cuda.synchronize()
    assert n_search >= 1
    assert np.array_equal(gi.cpu().numpy(), ref_i)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), ref_d.view(np.uint32))

    n_srv, srv = _first_success(
        hn, lambda: hn.Server(idx, max_slots=64, pool_bytes=4 << 20, k_max=10, ef_max=32))
    assert n_srv >= 5
    srv.submit_batch(Q[:20], np.full(20, 10, np.int32), np.full(20, 32, np.int32),
                     np.arange(20, dtype=np.int64))
    got = {}
    for _ in range(10000):
        srv.tick()
        tags, ids, dist = srv.poll()
        for t, i in zip(tags, ids):
            got[int(t)] = i.copy()
        if len(got) == 20:
            break
    for t in range(20):
        assert np.array_equal(got[t], ref_i[t]), t
    srv.close()
    idx.free()
    del gi, gd
    torch.cuda.empty_cache()
    after = _free_bytes()
    # what the failed calls allocated was released (slack for the runtime's pools)
    print(f"device memory not returned: {(before - after) / 2**20:.2f} MiB")
    assert before - after < (4 << 20), (before, after)
