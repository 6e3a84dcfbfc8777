"""GPU tests of the k-means tree index (DD_PACK_KMEANS, mode DD_KMEANS): its
build on the device and the walk over it, through the C ABI.  The exact walk
(no budget, f_d = 1) must give the oracle's nearest neighbours; approximate
walks (a budget, f_d < 1) are checked for what holds at any size: never
nearer than the exact answer, never farther than the warm start."""
import sys
import time

import numpy as np
import pytest

import ddsynth
import oracle
from oracle import fe
from gpu_util import assert_matches_oracle_solve, compare_to_oracle, to_dev

pytestmark = pytest.mark.gpu

FP64, BF16, ANN, KMEANS = 0x1, 0x4, 0x10, 0x20


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_00357_amd import _lib
    return _lib


@pytest.mark.parametrize("n", [1, 64, 65, 129, 4097, 70001])
def test_kmeans_exact_small_and_ragged(L, C0, n):
    """Trees of one leaf, of one split, and ragged sizes: cold and warm-started
    exact walks equal the oracle; the tree has the documented shape."""
    import torch
    _say("kmeans n =", n)
    e, s = ddsynth.data_points(n, 300 + n)
    qe, qs, base = ddsynth.queries(e, s, 300, 400 + n)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    info = L.dd_dataset_index_info(ds)
    _say("index", info)
    assert info["kmeans_leaves"] >= (n + 63) // 64
    assert info["kmeans_nodes"] >= 1
    assert info["kmeans_records"] == info["kmeans_leaves"] + info["kmeans_nodes"] - 1
    states = to_dev(ddsynth.states(qe, qs))
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    idx, dist = L.dd_project(ds, states, mode="kmeans")
    compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), oi, od, o2)
    i2, d2 = L.dd_project(ds, states, warm_start_idx=to_dev(base % n), mode="kmeans")
    assert torch.equal(i2, idx) and torch.equal(d2, dist)


@pytest.fixture(scope="module")
def config0(L, C0):
    e, s = ddsynth.data_points(65536, 1000)
    qe, qs, base = ddsynth.queries(e, s, 4096, 2000)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | ANN | KMEANS)
    return dict(e=e, s=s, oi=oi, od=od, o2=o2, base=base, ds=ds,
                states=to_dev(ddsynth.states(qe, qs)))


def test_kmeans_exact_equals_oracle_and_box_tree(L, config0):
    """The k-means walk and the box-tree walk are two exact methods: both equal
    the oracle and each other, with or without a warm start."""
    import torch
    ds, states = config0["ds"], config0["states"]
    idx, dist, st = L.dd_project(ds, states, mode="kmeans", stats=True)
    ia, da, sa = L.dd_project(ds, states, mode="ann", stats=True)
    _say("kmeans", st, "\nbox tree", sa)
    compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), config0["oi"], config0["od"],
                      config0["o2"])
    assert torch.equal(idx, ia) and torch.equal(dist, da)
    assert st["visited"] > 0 and st["leaves"] > 0 and 0 < st["leaf_boxes"] <= st["boxes"]
    assert st["nodes"] >= 1 and sa["nodes"] == 0          # k-means nodes expanded (root first)
    assert st["overflowed"] == 0 and sa["overflowed"] == 0    # no FP64 fallback
    for warm in (to_dev(config0["base"]), to_dev(np.zeros(4096, np.int64)), idx.clone()):
        i2, d2, s2 = L.dd_project(ds, states, warm_start_idx=warm, mode="kmeans", stats=True)
        assert torch.equal(i2, idx) and torch.equal(d2, dist)
        assert s2["overflowed"] == 0
    assert s2["visited"] <= st["visited"]          # warm start at the answer: less work


def test_kmeans_build_is_deterministic(L, C0, config0):
    """Two builds from the same data give the same tree (fixed-point centroid
    sums): same shape and the same work for every query."""
    import torch
    ds, states = config0["ds"], config0["states"]
    ds2 = L.dd_dataset_create(to_dev(config0["e"]), to_dev(config0["s"]), C0, packs=FP64 | KMEANS)
    assert L.dd_dataset_index_info(ds2)["kmeans_records"] == \
        L.dd_dataset_index_info(ds)["kmeans_records"]
    i1, d1, s1 = L.dd_project(ds, states, mode="kmeans", ann_budget=3, stats=True)
    i2, d2, s2 = L.dd_project(ds2, states, mode="kmeans", ann_budget=3, stats=True)
    assert torch.equal(i1, i2) and torch.equal(d1, d2)
    assert (s1["visited"], s1["boxes"], s1["leaves"]) == (s2["visited"], s2["boxes"], s2["leaves"])


def test_kmeans_budget_and_fd_are_approximate_within_bounds(L, config0, C0):
    """Budgets and f_d < 1 (the ball test |q - c| - f_d r of Section 4) give
    approximate answers that are never nearer than the exact one and never
    farther than the warm start; the reported distance is exact for the
    returned point.  Recall is reported."""
    ds, states = config0["ds"], config0["states"]
    st_np = states.cpu().numpy()
    rng = np.random.default_rng(15)
    warm = rng.integers(0, 65536, 4096).astype(np.int64)
    wd = oracle.pair_dist_raw(st_np[:, :6], st_np[:, 6:], config0["e"][warm], config0["s"][warm], C0)
    for budget, fd in ((1, 1.0), (4, 1.0), (64, 1.0), (0, 0.0), (0, 0.25), (0, 0.5), (0, 0.8),
                       (4, 0.5)):
        idx, dist, st = L.dd_project(ds, states, warm_start_idx=to_dev(warm), mode="kmeans",
                                     ann_budget=budget, ann_fd=fd, stats=True)
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        got = oracle.pair_dist_raw(st_np[:, :6], st_np[:, 6:], config0["e"][idx],
                                   config0["s"][idx], C0)
        recall = float(np.mean(idx == config0["oi"]))
        _say(f"budget {budget} f_d {fd}: recall {recall:.4f}, leaves/query "
             f"{st['leaves'] / 4096:.2f}, visited/query {st['visited'] / 4096:.1f}")
        if budget:
            assert st["leaves"] <= budget * 4096
        np.testing.assert_allclose(dist, got, rtol=1e-12)
        assert np.all(got <= wd * (1 + 1e-12))
        assert np.all(got >= config0["od"] * (1 - 1e-12))
    with pytest.raises(L.DDError):
        L.dd_project(ds, states, mode="kmeans", ann_fd=1.5)


def test_kmeans_fd_search_descends_past_a_good_warm_start(L, C0, config0):
    """With f_d < 1 the warm start bounds no branch (Section 4.2: the search
    descends to the nearest centre's leaf first, then backtracks by the ball
    test against its own best).  Warm-started from each query's second
    nearest point, f_d = 0 must still find the nearest point for many
    queries, and never return a point farther than the warm start."""
    ds, states = config0["ds"], config0["states"]
    e, s = config0["e"], config0["s"]
    qs_np = states.cpu().numpy()
    wq = oracle.whiten(qs_np[:, :6], qs_np[:, 6:], C0)
    wd = oracle.whiten(e, s, C0)
    # the nearest point after the oracle's nearest (brute force)
    second = np.empty(len(wq), np.int64)
    n2 = np.einsum("ij,ij->i", wd, wd)
    for a in range(0, len(wq), 512):
        d = n2[None, :] - 2.0 * wq[a:a + 512] @ wd.T
        d[np.arange(len(d)), config0["oi"][a:a + 512]] = np.inf
        second[a:a + 512] = np.argmin(d, axis=1)
    warm_d = oracle.pair_dist_raw(qs_np[:, :6], qs_np[:, 6:], e[second], s[second], C0)
    for fd in (0.0, 0.5):
        idx, dist = L.dd_project(ds, states, warm_start_idx=to_dev(second), mode="kmeans",
                                 ann_fd=fd)
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        recall = float(np.mean(idx == config0["oi"]))
        _say(f"f_d {fd}, warm = second nearest: recall {recall:.4f}")
        assert np.all(dist <= warm_d * (1 + 1e-12))
        assert recall >= 0.25


def test_kmeans_mode_needs_its_pack(L, C0):
    """The k-means mode on a dataset without the tree is refused (status 8);
    a dataset without trees reports an empty index."""
    e, s = ddsynth.data_points(1000, 61)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | ANN)
    info = L.dd_dataset_index_info(ds)
    assert info["kmeans_nodes"] == 0 and info["kmeans_leaves"] == 0 and info["ann_levels"] >= 1
    qe, qs, _ = ddsynth.queries(e, s, 10, 62)
    with pytest.raises(L.DDError) as ex:
        L.dd_project(ds, to_dev(ddsynth.states(qe, qs)), mode="kmeans")
    assert ex.value.status == 8
    ds2 = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64)
    assert all(v == 0 for v in L.dd_dataset_index_info(ds2).values())
    ds3 = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    for fd in (-0.5, 1.0000001):
        with pytest.raises(L.DDError) as ex:
            L.dd_project(ds3, to_dev(ddsynth.states(qe, qs)), mode="kmeans", ann_fd=fd)
        assert ex.value.status == 1


def test_kmeans_repeated_points(L, C0):
    """Data with three distinct points repeated (every split degenerate: the
    build falls back to equal runs): exact answers, ties to the lowest index."""
    e0, s0 = ddsynth.data_points(3, 55)
    pick = ddsynth.indices(5000, 3, 56)
    e, s = e0[pick], s0[pick]
    qe, qs, _ = ddsynth.queries(e0, s0, 200, 57)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    _say("repeated points", L.dd_dataset_index_info(ds))
    idx, dist = L.dd_project(ds, to_dev(ddsynth.states(qe, qs)), mode="kmeans")
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    assert np.array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_allclose(dist.cpu().numpy(), od, rtol=1e-12)


@pytest.mark.parametrize("n", [4, 8])
def test_dd_solve_kmeans_equals_fp64_trajectory(L, C0, n):
    """DD solves projecting by the exact k-means walk (with and without the
    skipping of unmoved points) follow the FP64 scan's trajectory bit for bit;
    at 4^3 the skipping solve also follows the oracle's DD loop."""
    e, s = ddsynth.data_points(200000, 1010)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    mask, force = ddsynth.box_bc(n, 100.0)
    init = ddsynth.indices(8 * n ** 3, 200000, 11)
    a = L.dd_solve(ds, (n, n, n), mask, force, init, mode="kmeans", history=True)
    b = L.dd_solve(ds, (n, n, n), mask, force, init, mode="kmeans", history=True, skip=True)
    c = L.dd_solve(ds, (n, n, n), mask, force, init, mode="fp64", history=True)
    _say(f"{n}^3: {a['iterations']} iterations, {a['elapsed_ms']:.1f} ms; skipping "
         f"{b['skipped']} projections, {b['elapsed_ms']:.1f} ms; fp64 {c['elapsed_ms']:.1f} ms")
    for r in (b, c):
        assert np.array_equal(a["history"], r["history"])
        assert np.array_equal(a["u"], r["u"])
        assert np.array_equal(a["d_full"], r["d_full"])
    if n == 4:
        ref = fe.dd_solve(e, s, C0, fe.Mesh(n), mask, force, init, record_history=True)
        assert ref.converged and b["converged"]
        assert_matches_oracle_solve(b, ref)


def test_dd_solve_kmeans_fd_schedule(L, C0):
    """The f_d schedule of Section 4.5 in dd_solve: with f_d^f = 1 the ramp
    changes nothing (the exact trajectory); with f_d^f < 1 no stopping rule
    fires before the ramp ends, and every point of the last projection lies
    between its exact nearest neighbour and its previous association.  f_d
    with another projection mode is refused."""
    n = 4
    e, s = ddsynth.data_points(200000, 1011)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    mask, force = ddsynth.box_bc(n, 100.0)
    init = ddsynth.indices(8 * n ** 3, 200000, 12)
    exact = L.dd_solve(ds, (n, n, n), mask, force, init, mode="kmeans", history=True)
    same = L.dd_solve(ds, (n, n, n), mask, force, init, mode="kmeans", history=True,
                      ann_fd=1.0, ann_ramp=6)
    assert np.array_equal(exact["history"], same["history"])
    assert same["project_ms"] > 0
    for fd, ramp in ((0.0, 0), (0.0, 6), (0.4, 6), (0.8, 3)):
        r = L.dd_solve(ds, (n, n, n), mask, force, init, mode="kmeans", history=True,
                       ann_fd=fd, ann_ramp=ramp)
        k = r["iterations"]
        _say(f"f_d^f {fd}, ramp {ramp}: {k} iterations (stop {r['stop_reason']}), final "
             f"distance {r['d_full'][-1]:.6g} (exact walk {exact['d_full'][-1]:.6g}), "
             f"search {r['project_ms']:.2f} ms")
        assert r["stop_reason"] in (1, 2)
        assert k >= ramp
        hist = r["history"]
        assert hist.min() >= 0 and hist.max() < 200000
        got = oracle.pair_dist_raw(r["eps"], r["sig"], e[hist[k]], s[hist[k]], C0)
        prev = oracle.pair_dist_raw(r["eps"], r["sig"], e[hist[k - 1]], s[hist[k - 1]], C0)
        _, od, _ = oracle.pd_raw(e, s, C0, r["eps"], r["sig"])
        assert np.all(got >= od * (1 - 1e-12))
        assert np.all(got <= prev * (1 + 1e-12))
    with pytest.raises(L.DDError) as ex:
        L.dd_solve(ds, (n, n, n), mask, force, init, mode="fp64", ann_fd=0.5)
    assert ex.value.status == 1


@pytest.mark.parametrize("mode,kw", [("kmeans", dict(ann_fd=0.4, ann_ramp=6)),
                                     ("kmeans", dict(ann_fd=0.0, ann_ramp=0)),
                                     ("ann", dict(ann_budget=2, ann_ramp=6)),
                                     ("ann", dict(ann_budget=1, ann_ramp=0))])
def test_dd_solve_local_accuracy(L, C0, mode, kw):
    """DD_SOLVE_LOCAL_ACCURACY (accuracy from the local and the global distance
    and the iteration): every point of the last projection lies between its
    exact nearest neighbour (oracle) and its previous association, the stopping
    rules of approximate solves apply, and with an exact walk the flag changes
    nothing."""
    n = 4
    e, s = ddsynth.data_points(200000, 1012)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | ANN | KMEANS)
    mask, force = ddsynth.box_bc(n, 100.0)
    init = ddsynth.indices(8 * n ** 3, 200000, 13)
    base = L.dd_solve(ds, (n, n, n), mask, force, init, mode=mode, history=True, **kw)
    r = L.dd_solve(ds, (n, n, n), mask, force, init, mode=mode, history=True,
                   local_accuracy=True, **kw)
    k = r["iterations"]
    _say(f"{mode} {kw}: local {k} iterations (stop {r['stop_reason']}), final distance "
         f"{r['d_full'][-1]:.6g}, search {r['project_ms']:.2f} ms; schedule alone "
         f"{base['iterations']} iterations, {base['d_full'][-1]:.6g}, {base['project_ms']:.2f} ms")
    assert r["stop_reason"] in (1, 2) and k >= kw["ann_ramp"]
    hist = r["history"]
    assert hist.min() >= 0 and hist.max() < 200000
    got = oracle.pair_dist_raw(r["eps"], r["sig"], e[hist[k]], s[hist[k]], C0)
    prev = oracle.pair_dist_raw(r["eps"], r["sig"], e[hist[k - 1]], s[hist[k - 1]], C0)
    _, od, _ = oracle.pd_raw(e, s, C0, r["eps"], r["sig"])
    assert np.all(got >= od * (1 - 1e-12))
    assert np.all(got <= prev * (1 + 1e-12))
    # the first iteration has no previous distance: it follows the schedule alone
    assert np.array_equal(r["history"][1], base["history"][1])
    exact = L.dd_solve(ds, (n, n, n), mask, force, init, mode=mode, history=True)
    same = L.dd_solve(ds, (n, n, n), mask, force, init, mode=mode, history=True,
                      local_accuracy=True)
    assert np.array_equal(exact["history"], same["history"])


def test_dd_solve_unknown_flag_is_refused(L, C0):
    e, s = ddsynth.data_points(1000, 1013)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64)
    mask, force = ddsynth.box_bc(2, 100.0)
    init = ddsynth.indices(64, 1000, 14)
    opts = L.dd_solve_opts(0, 0, 0, 0x40, 0.0, 0, 0, None, 0.0)
    res = L.dd_solve_result()
    import ctypes
    m = L.dd_mesh(2, 2, 2, 1.0, 1.0, 1.0)
    mask = np.ascontiguousarray(mask, np.uint8)
    st = L.lib().dd_solve(ds.handle, ctypes.byref(m), mask.ctypes.data, force.ctypes.data,
                          init.ctypes.data, ctypes.byref(opts), ctypes.byref(res), None)
    assert st == 1


def test_server_kmeans_mode(L, C0):
    """The serving loop accepts the k-means mode and returns dd_solve's results."""
    e, s = ddsynth.data_points(1 << 16, 1020)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=FP64 | KMEANS)
    reqs = []
    for k, n in enumerate((3, 4, 2)):
        mask, force = ddsynth.box_bc(n, 120.0)
        reqs.append(((n, n, n), mask, force, ddsynth.indices(8 * n ** 3, 1 << 16, 30 + k)))
    alone = [L.dd_solve(ds, *r, mode="kmeans") for r in reqs]
    srv = L.DDServer(ds, mode="kmeans")
    try:
        got = [srv.wait(t) for t in [srv.submit(*r) for r in reqs]]
    finally:
        srv.close()
    for a, b in zip(alone, got):
        assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["u"], b["u"])


def test_kmeans_1e9_equals_bf16_scan(L, C0):
    """N = 10^9 points from the device generator: the k-means tree builds on
    the device and its exact walk equals the BF16 scan (an independent exact
    method) on 32768 queries; the box tree's figures for the same queries are
    in the benchmark."""
    import torch
    N, m = 1_000_000_000, 32768
    gen = ddsynth.DevicePoints(1003)
    t = time.time()
    ds = L.dd_dataset_create_streamed(N, C0, gen.fill_fn, gen.user, packs=FP64 | BF16 | KMEANS)
    torch.cuda.synchronize()
    info = L.dd_dataset_index_info(ds)
    _say(f"1e9 kmeans: dataset in {time.time() - t:.1f}s, {ds.info()[1] / 1e9:.1f} GB, {info}")
    qe, qs, base = ddsynth.queries_generated(N, 1003, m, 2003)
    states = torch.from_numpy(ddsynth.states(qe, qs)).cuda()
    ik, dk, st = L.dd_project(ds, states, mode="kmeans", stats=True)
    _say(f"1e9 kmeans exact: {st['scan_ms']:.1f} ms walk, {st['visited'] / m:.0f} points/query, "
         f"{st['leaves'] / m:.1f} leaves/query")
    ib, db = L.dd_project(ds, states, mode="bf16")
    assert torch.equal(ik, ib) and torch.equal(dk, db)
    iw, dw, sw = L.dd_project(ds, states, warm_start_idx=torch.from_numpy(base).cuda(),
                              mode="kmeans", stats=True)
    _say(f"1e9 kmeans warm: {sw['scan_ms']:.1f} ms walk, {sw['visited'] / m:.0f} points/query")
    assert torch.equal(iw, ik) and torch.equal(dw, dk)
    ds.close()
