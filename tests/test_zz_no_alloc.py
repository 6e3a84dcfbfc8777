"""GPU tests of dd_project_noalloc (the projection without device allocation,
its buffers in the library's scratch array), through the C ABI: two calls in a
row, the second with a smaller batch, give dd_project's indices and distances
bit for bit, and the oracle's; the fallback scans (driven by candidate-list
overflow on duplicated points) run from the scratch array too."""
import sys

import numpy as np
import pytest

import ddsynth
import oracle
from gpu_util import compare_to_oracle, to_dev

pytestmark = pytest.mark.gpu

FP64, ANN, KMEANS = 0x1, 0x10, 0x20


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_00357_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def data(L, C0):
    N = 200_000
    e, s = ddsynth.data_points(N, 1040)
    qe, qs, base = ddsynth.queries(e, s, 5000, 1041)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | ANN | KMEANS)
    return dict(N=N, ds=ds, states=to_dev(ddsynth.states(qe, qs)), warm=to_dev(base),
                oi=oi, od=od, o2=o2)


@pytest.mark.parametrize("mode,kw", [("fp64", {}), ("ann", {}), ("kmeans", {}),
                                     ("ann", dict(ann_budget=4)), ("kmeans", dict(ann_fd=0.5))])
def test_noalloc_equals_dd_project_twice(L, data, mode, kw):
    import torch
    ds, states, warm = data["ds"], data["states"], data["warm"]
    exact = not kw
    for m in (5000, 300):
        _say(f"noalloc {mode} {kw} m={m}")
        q = states[:m].contiguous()
        w = warm[:m].contiguous()
        want_i, want_d = L.dd_project(ds, q, warm_start_idx=w, mode=mode, **kw)
        got_i, got_d = L.dd_project_noalloc(ds, q, warm_start_idx=w, mode=mode, **kw)
        torch.cuda.synchronize()
        assert torch.equal(got_i, want_i) and torch.equal(got_d, want_d)
        if exact:
            compare_to_oracle(got_i.cpu().numpy(), got_d.cpu().numpy(), data["oi"][:m],
                              data["od"][:m], data["o2"][:m])


@pytest.mark.parametrize("mode", ["fp64", "ann", "kmeans"])
def test_noalloc_fallbacks_on_duplicates(L, C0, mode):
    """70 copies of one point overflow every candidate list: the queries at that
    point go through the FP64 scan (walk modes) and the direct scan, all from
    the scratch array, and still get the lowest index; a second, smaller call
    after it gives the oracle's answers."""
    n = 6000
    e, s = ddsynth.data_points(n, 77)
    dup_at = np.arange(2000, 2070)
    e[dup_at], s[dup_at] = e[1234], s[1234]
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | ANN | KMEANS)
    picks = np.array([1234, 2005, 0, n - 1, 3333])
    idx, dist = L.dd_project_noalloc(ds, to_dev(ddsynth.states(e[picks], s[picks])), mode=mode)
    assert idx.cpu().tolist() == [1234, 1234, 0, n - 1, 3333]
    assert np.all(dist.cpu().numpy() == 0.0)
    qe, qs, _ = ddsynth.queries(e, s, 3, 78)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    idx, dist = L.dd_project_noalloc(ds, to_dev(ddsynth.states(qe, qs)), mode=mode)
    compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), oi, od, o2)
    ds.close()


def test_noalloc_limits(L, data):
    import torch
    ds = data["ds"]
    big = torch.zeros((L.DD_NOALLOC_MAX_QUERIES + 1, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(L.DDError) as ex:
        L.dd_project_noalloc(ds, big, mode="fp64")
    assert ex.value.status == 6
    with pytest.raises(L.DDError) as ex:
        L.dd_project_noalloc(ds, data["states"][:4].contiguous(), mode="bf16")
    assert ex.value.status == 8
    empty = torch.empty((0, 12), dtype=torch.float64, device="cuda")
    i0, _ = L.dd_project_noalloc(ds, empty, mode="ann")
    assert i0.numel() == 0
