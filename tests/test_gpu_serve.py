"""GPU tests of the serving loop (dd_server_*): concurrent DD solves of
different meshes against one resident dataset, projections batched across
solves, admission by device footprint, through the C ABI."""
import sys
import time

import numpy as np
import pytest

import ddsynth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

FP64, BF16 = 0x1, 0x4


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
    N = 1 << 18
    e, s = ddsynth.data_points(N, 1004)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | BF16)
    return dict(N=N, ds=ds)


def _requests(N, sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate(sizes):
        t = float(rng.uniform(50.0, 200.0))
        mask, force = ddsynth.box_bc(n, t)
        init = ddsynth.indices(8 * n ** 3, N, seed * 100 + k)
        out.append(((n, n, n), mask, force, init))
    return out


def _same(a, b):
    assert a["iterations"] == b["iterations"]
    assert np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["u"], b["u"])
    assert np.array_equal(a["d_half"], b["d_half"]) and np.array_equal(a["d_full"], b["d_full"])
    assert np.array_equal(a["changed"], b["changed"])
    assert np.array_equal(a["eps"], b["eps"]) and np.array_equal(a["sig"], b["sig"])


def test_results_alone_equal_results_in_the_mix(L, data):
    """Each solve gives bitwise the result of dd_solve alone, whether it runs in
    a mix of concurrent solves with staggered arrivals or alone on the server."""
    N, ds = data["N"], data["ds"]
    reqs = _requests(N, [2, 3, 4, 6, 2, 5, 3, 4], 1)
    alone = [L.dd_solve(ds, *r, mode="bf16") for r in reqs]
    srv = L.DDServer(ds, mode="bf16")
    try:
        tickets = []
        for k, r in enumerate(reqs):
            tickets.append(srv.submit(*r))
            if k % 3 == 2:
                time.sleep(0.002)   # staggered arrivals: some join while others run
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
        _say("mix stats", {k: st[k] for k in ("completed", "batches", "queries", "peak_active",
                                               "proj_p50_ms", "proj_p99_ms", "solve_p50_ms",
                                               "solve_p99_ms")})
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["peak_active"] > 1                     # the solves overlapped
        assert st["batches"] < sum(r["iterations"] for r in alone)   # batched across solves
        for a, b in zip(alone, mixed):
            assert b["status"] == 0 and b["converged"]
            _same(a, b)
        # alone on the server too
        t = srv.submit(*reqs[3])
        _same(alone[3], srv.wait(t))
    finally:
        srv.close()


def test_large_mesh_spans_batches(L, data):
    """A solve with more material points than a batch holds is projected in
    several batches and still gives the dd_solve result."""
    N, ds = data["N"], data["ds"]
    reqs = _requests(N, [6, 2], 2)                      # 1728 and 64 material points
    alone = [L.dd_solve(ds, *r, mode="bf16") for r in reqs]
    srv = L.DDServer(ds, mode="bf16", max_batch=1000)
    try:
        tickets = [srv.submit(*r) for r in reqs]
        for a, t in zip(alone, tickets):
            _same(a, srv.wait(t))
        assert srv.stats()["batches"] >= 2 * alone[0]["iterations"]
    finally:
        srv.close()


def test_admission_by_footprint(L, data):
    """A budget that holds one solve at a time admits them one by one (all
    finish); a solve larger than the whole budget is rejected at submit."""
    N, ds = data["N"], data["ds"]
    reqs = _requests(N, [4, 4, 4], 3)
    # a 4^3 solve is charged about 1.2 MB (P_C buffers, states, projection
    # scratch): a 1.9 MB budget admits one at a time
    big = (12, 12, 12)
    srv = L.DDServer(ds, hbm_budget_bytes=1_900_000, mode="bf16")
    try:
        tickets = [srv.submit(*r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
        _say("budget stats", st["peak_active"], st["peak_bytes"], st["budget_bytes"])
        assert st["peak_active"] == 1 and st["completed"] == 3
        assert st["peak_bytes"] <= st["budget_bytes"]
        for r, q in zip(res, reqs):
            _same(L.dd_solve(ds, *q, mode="bf16"), r)
        mask, force = ddsynth.box_bc(12, 100.0)
        with pytest.raises(L.DDError) as ex:
            srv.submit(big, mask, force, np.zeros(8 * 12 ** 3, np.int64))
        assert ex.value.status == 6
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()


def test_cancel_failures_and_limits(L, data):
    """Cancelled and iteration-limited solves end with their status while the
    others finish normally; invalid requests are refused at submit."""
    N, ds = data["N"], data["ds"]
    reqs = _requests(N, [3, 4, 3, 2], 4)
    alone = L.dd_solve(ds, *reqs[0], mode="bf16")
    srv = L.DDServer(ds, mode="bf16", max_active=1)
    try:
        t0 = srv.submit(*reqs[0])
        t1 = srv.submit(*reqs[1])
        t2 = srv.submit(*reqs[2], max_iter=1)
        t3 = srv.submit(*reqs[3])
        srv.cancel(t1)                                    # queued behind t0 (one slot)
        r1 = srv.wait(t1, raise_on_error=False)
        assert r1["status"] == 7
        _same(alone, srv.wait(t0))
        r2 = srv.wait(t2, raise_on_error=False)
        assert r2["status"] == 5 and r2["iterations"] == 1 and not r2["converged"]
        r3 = srv.wait(t3)
        assert r3["converged"]
        bad = list(reqs[0])
        bad[3] = np.full(8 * 27, N, np.int64)             # out-of-range association
        with pytest.raises(L.DDError) as ex:
            srv.submit(*bad)
        assert ex.value.status == 1
        with pytest.raises(L.DDError):
            srv.wait(123456789)                           # unknown ticket
        st = srv.stats()
        assert st["cancelled"] == 1 and st["completed"] == 3
    finally:
        srv.close()


def test_destroy_with_work_in_flight(L, data):
    """Destroying a server with queued and running solves returns cleanly."""
    N, ds = data["N"], data["ds"]
    srv = L.DDServer(ds, mode="bf16", max_active=2)
    for r in _requests(N, [4, 4, 4, 4, 4], 5):
        srv.submit(*r)
    time.sleep(0.01)
    srv.close()
