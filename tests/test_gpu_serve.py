"""GPU tests of the serving loop (dd_server_*): concurrent DD solves of
different meshes against one resident dataset, projections batched across
solves, admission by device footprint, through the C ABI."""
import sys
import time

import numpy as np
import pytest

import ddsynth
from oracle import fe
from gpu_util import assert_matches_oracle_solve, to_dev

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
    return dict(N=N, ds=ds, e=e, s=s)


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


def test_served_solves_match_oracle(L, data, C0):
    """Solves served in a mix of 2^3 and 3^3 meshes (staggered arrivals, one
    server) follow the oracle's DD loop from the same initial association:
    same iteration count and final association, u, strains and stresses to
    1e-10 of their maxima, distances to 1e-9."""
    N, ds, e, s = data["N"], data["ds"], data["e"], data["s"]
    rng = np.random.default_rng(21)
    probs = []
    for k, n in enumerate((2, 3, 2, 3, 3, 2)):
        m = fe.Mesh(n)
        t = float(rng.uniform(50.0, 200.0))
        probs.append((m, m.clamp_mask(), m.traction_x1(t),
                      ddsynth.indices(m.n_mp, N, 700 + k)))
    srv = L.DDServer(ds, mode="bf16")
    try:
        tickets = []
        for k, (m, mask, f, init) in enumerate(probs):
            n = m.n
            tickets.append(srv.submit((n, n, n), mask, f, init))
            if k % 2 == 1:
                time.sleep(0.002)
        served = [srv.wait(t) for t in tickets]
        assert srv.stats()["peak_active"] > 1
    finally:
        srv.close()
    for (m, mask, f, init), got in zip(probs, served):
        ref = fe.dd_solve(e, s, C0, m, mask, f, init)
        _say(f"served {m.n}^3 vs oracle: {got['iterations']} / {ref.iterations} iterations")
        assert got["status"] == 0 and got["converged"] and ref.converged
        assert_matches_oracle_solve(got, ref, history=False)


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


def _reserve(L, ds, **kw):
    """The fixed reserve of a server of these options (batch buffers and the
    scratch of a full projection batch)."""
    probe = L.DDServer(ds, **kw)
    try:
        return probe.stats()["reserve_bytes"]
    finally:
        probe.close()


def test_admission_by_footprint(L, data):
    """A budget that holds one solve at a time beside the server's reserve
    admits them one by one (all finish); a solve larger than the whole budget
    is rejected at submit; a budget below the reserve is refused at creation."""
    N, ds = data["N"], data["ds"]
    reqs = _requests(N, [4, 4, 4], 3)
    # a 4^3 solve's P_C buffers and states take about 0.57 MB: 0.9 MB beside the
    # reserve admit one at a time
    big = (12, 12, 12)
    r = _reserve(L, ds, mode="bf16", max_batch=1024)
    assert r > 0
    with pytest.raises(L.DDError) as ex:
        L.DDServer(ds, hbm_budget_bytes=r - 1, mode="bf16", max_batch=1024)
    assert ex.value.status == 6
    srv = L.DDServer(ds, hbm_budget_bytes=r + 900_000, mode="bf16", max_batch=1024)
    try:
        tickets = [srv.submit(*r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
        _say("budget stats", st["peak_active"], st["peak_bytes"], st["budget_bytes"])
        assert st["peak_active"] == 1 and st["completed"] == 3
        assert st["reserve_bytes"] == r and r < st["peak_bytes"] <= st["budget_bytes"]
        for r, q in zip(res, reqs):
            _same(L.dd_solve(ds, *q, mode="bf16"), r)
        mask, force = ddsynth.box_bc(12, 100.0)
        with pytest.raises(L.DDError) as ex:
            srv.submit(big, mask, force, np.zeros(8 * 12 ** 3, np.int64))
        assert ex.value.status == 6
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()


def test_inverse_beyond_budget_runs_by_cg(L, C0):
    """An 8^3 solve's buffers (3.7 MB) fit 20 MB beside the server's reserve but
    its K^-1 (40 MB) does not: on a dataset that has not formed that inverse,
    the server runs the solve by CG (the trajectory of dd_solve with
    DD_SOLVE_CG, bit for bit) and never charges more than the budget."""
    N = 1 << 16
    e, s = ddsynth.data_points(N, 1030)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | BF16)
    mask, force = ddsynth.box_bc(8, 120.0)
    init = ddsynth.indices(8 * 8 ** 3, N, 31)
    r = _reserve(L, ds, mode="bf16", max_batch=4096)
    srv = L.DDServer(ds, hbm_budget_bytes=r + 20_000_000, mode="bf16", max_batch=4096)
    try:
        got = srv.wait(srv.submit((8, 8, 8), mask, force, init))
        st = srv.stats()
    finally:
        srv.close()
    _say("cg fallback", st["peak_bytes"], st["budget_bytes"], got["cg_iterations"])
    assert got["cg_iterations"] > 0 and st["peak_bytes"] <= st["budget_bytes"]
    _same(L.dd_solve(ds, (8, 8, 8), mask, force, init, mode="bf16", cg=True, graph=False), got)
    ds.close()


def test_inverse_formed_off_the_scheduler_and_charged(L, C0):
    """Solves whose K^-1 the dataset does not hold yet: the server forms the
    inverses on a builder thread while the other solves run, charges them
    against the budget, and every result equals dd_solve's (which then finds
    the same inverses in the dataset's cache)."""
    N = 1 << 16
    e, s = ddsynth.data_points(N, 1031)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | BF16)
    reqs = _requests(N, [8, 3, 2, 3], 7)
    srv = L.DDServer(ds, mode="bf16")
    try:
        got = [srv.wait(t) for t in [srv.submit(*r) for r in reqs]]
        st = srv.stats()
    finally:
        srv.close()
    _say("async inverses", st["peak_bytes"], st["peak_active"])
    n_pad = (3 * 9 ** 3 + 63) // 64 * 64
    assert st["peak_bytes"] >= st["reserve_bytes"] + 8 * n_pad * n_pad   # the 8^3 inverse was charged
    for r, g in zip(reqs, got):
        assert g["cg_iterations"] == 0
        _same(L.dd_solve(ds, *r, mode="bf16"), g)
    ds.close()


@pytest.mark.parametrize("mode", ["fp64", "direct", "fp32", "bf16", "fp16", "ann", "kmeans"])
def test_every_mode_served_from_the_reserve(L, C0, mode):
    """In every projection mode the batch projections carve their scratch from
    the server's fixed reserve (no allocation, and a call that needed more would
    fail) and every served solve equals dd_solve alone."""
    N = 1 << 14
    e, s = ddsynth.data_points(N, 1040)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x2 | 0x4 | 0x8 | 0x10 | 0x20)
    reqs = _requests(N, [3, 2, 4], 41)
    alone = [L.dd_solve(ds, *r, mode=mode) for r in reqs]
    srv = L.DDServer(ds, mode=mode, max_batch=2048)
    try:
        got = [srv.wait(t) for t in [srv.submit(*r) for r in reqs]]
        st = srv.stats()
    finally:
        srv.close()
    _say(f"served {mode}: reserve {st['reserve_bytes']}, peak {st['peak_bytes']}")
    assert st["failed"] == 0 and 0 < st["reserve_bytes"] < st["peak_bytes"] <= st["budget_bytes"]
    for a, b in zip(alone, got):
        _same(a, b)
    ds.close()


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
