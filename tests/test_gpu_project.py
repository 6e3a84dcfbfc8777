"""GPU parity of dd_project against the CPU oracle (through the C ABI)."""
import sys

import numpy as np
import pytest

import ddsynth
import oracle
from gpu_util import compare_to_oracle, to_dev

pytestmark = pytest.mark.gpu

MODES = ["direct", "fp64", "fp32", "bf16", "fp16", "ann"]
ALL_PACKS = 0x1 | 0x2 | 0x4 | 0x8 | 0x10


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_00357_amd import _lib
    return _lib


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_mfma_lane_layouts(L, kind):
    """The matrix-instruction lane layouts the scans assume reproduce A B."""
    _say("selftest kind", kind)
    rng = np.random.default_rng(kind)
    if kind == 2:
        A = rng.integers(-8, 9, (16, 4)).astype(float)
        B = rng.integers(-8, 9, (4, 16)).astype(float)
    else:
        A = rng.integers(-8, 9, (32, 16)).astype(float)
        B = rng.integers(-8, 9, (16, 32)).astype(float)
    D = L.dd_selftest_mfma(kind, A, B)
    np.testing.assert_array_equal(D, A @ B)


def test_mfma_fp32_lane_layout_with_accumulator_input(L):
    """The FP32 scan's layouts, its norms entering as the accumulator input."""
    rng = np.random.default_rng(5)
    A = rng.integers(-8, 9, (32, 2)).astype(float)
    B = rng.integers(-8, 9, (2, 32)).astype(float)
    D = L.dd_selftest_mfma(5, A, B)
    np.testing.assert_array_equal(D, A @ B + np.arange(32.0)[:, None])


def _bf16_rne(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("kind", [3, 4])
def test_query_operand_rounding_is_nearest_even(L, kind):
    """The error bound of the 16-bit scans assumes round-to-nearest-even
    conversions of the centred query operands."""
    rng = np.random.default_rng(10 + kind)
    x = np.concatenate([rng.normal(size=300) * 0.3, rng.normal(size=200) * 1e-3,
                        # exact ties between two representable neighbours
                        (1.0 + (np.arange(12) * 2 + 1) * 2.0 ** -8) if kind == 3
                        else (1.0 + (np.arange(12) * 2 + 1) * 2.0 ** -11)]).astype(np.float32)
    D = L.dd_selftest_mfma(kind, x.astype(np.float64), None)
    want = _bf16_rne(x) if kind == 3 else x.astype(np.float16).astype(np.float32)
    np.testing.assert_array_equal(D.astype(np.float32), want)


@pytest.fixture(scope="module")
def config0(L, C0):
    """N = 65536 data points, m = 4096 queries (the exact-projection workload)."""
    e, s = ddsynth.data_points(65536, 1000)
    qe, qs, _ = ddsynth.queries(e, s, 4096, 2000)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=ALL_PACKS)
    states = to_dev(ddsynth.states(qe, qs))
    return dict(e=e, s=s, qe=qe, qs=qs, oi=oi, od=od, o2=o2, ds=ds, states=states)


@pytest.mark.parametrize("mode", MODES)
def test_config0_parity(L, config0, mode):
    _say("config0 mode", mode)
    idx, dist, st = L.dd_project(config0["ds"], config0["states"], mode=mode, stats=True)
    ties = compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), config0["oi"], config0["od"],
                             config0["o2"])
    _say(f"  mode {mode}: near ties {ties}, stats {st}")


@pytest.mark.parametrize("mode", MODES)
def test_warm_start_and_determinism(L, config0, mode):
    import torch
    _say("warm/determinism mode", mode)
    ds, states = config0["ds"], config0["states"]
    i1, d1 = L.dd_project(ds, states, mode=mode)
    i2, d2 = L.dd_project(ds, states, mode=mode)
    assert torch.equal(i1, i2) and torch.equal(d1, d2)
    rng = np.random.default_rng(4)
    warm = to_dev(rng.integers(0, 65536, 4096).astype(np.int64))
    i3, d3 = L.dd_project(ds, states, warm_start_idx=warm, mode=mode)
    assert torch.equal(i1, i3) and torch.equal(d1, d3)
    i4, d4 = L.dd_project(ds, states, warm_start_idx=i1.clone(), mode=mode)
    assert torch.equal(i1, i4) and torch.equal(d1, d4)


@pytest.mark.parametrize("n,m,tile", [(1, 5, 256), (31, 7, 256), (1000, 77, 128), (5003, 300, 512),
                                      (20000, 1000, 512)])
@pytest.mark.parametrize("mode", MODES)
def test_ragged_sizes(L, C0, n, m, tile, mode):
    _say("ragged", n, m, tile, mode)
    e, s = ddsynth.data_points(n, 3000 + n)
    qe, qs, _ = ddsynth.queries(e, s, m, 4000 + n)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=ALL_PACKS, tile=tile)
    idx, dist = L.dd_project(ds, to_dev(ddsynth.states(qe, qs)), mode=mode)
    compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), oi, od, o2)


@pytest.mark.parametrize("mode", MODES)
def test_queries_on_data_points_and_duplicates(L, C0, mode):
    """A query equal to a data point is at distance 0; among duplicates (more of
    them than any candidate list holds, so the overflow fallback runs) the
    lowest index wins."""
    _say("duplicates", mode)
    n = 6000
    e, s = ddsynth.data_points(n, 77)
    dup_of = 1234
    dup_at = np.arange(2000, 2000 + 70)            # 70 copies of point 1234, all above it
    e[dup_at], s[dup_at] = e[dup_of], s[dup_of]
    e[10], s[10] = e[5000], s[5000]                # one copy of 5000 below it
    picks = np.array([dup_of, 2005, 5000, 10, 0, n - 1, 3333])
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=ALL_PACKS)
    states = to_dev(ddsynth.states(e[picks], s[picks]))
    idx, dist = L.dd_project(ds, states, mode=mode)
    assert idx.cpu().tolist() == [dup_of, dup_of, 10, 10, 0, n - 1, 3333]
    assert np.all(dist.cpu().numpy() == 0.0)


@pytest.mark.parametrize("mode", MODES)
def test_si_units_padded_tail_and_far_queries(L, C0, mode):
    """Stresses and metric in Pa (whitened coordinates about 1000 times those in
    MPa, tile offsets whose squared norms exceed the FP16 range unless the
    16-bit scans rescale), a last tile padded past N, queries on points of that
    tile, and queries so far from the data that their centred coordinates would
    overflow FP16 (answered by the FP64 fallback): every mode equals the oracle."""
    _say("SI units", mode)
    n = 5003
    e, s = ddsynth.data_points(n, 6100)
    s = s * 1e6
    C = C0 * 1e6
    qe, qs, _ = ddsynth.queries(e, s / 1e6, 200, 6101)
    qs = qs * 1e6
    tail = np.arange(n - 5, n)
    qe = np.concatenate([qe, e[tail], qe[:8] * 1e4, qe[:4] * 1e9])
    qs = np.concatenate([qs, s[tail], qs[:8] * 1e4, qs[:4] * 1e9])
    oi, od, o2 = oracle.pd_raw(e, s, C, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C, packs=ALL_PACKS, tile=1024)
    idx, dist, st = L.dd_project(ds, to_dev(ddsynth.states(qe, qs)), mode=mode, stats=True)
    _say(f"  {mode}: overflowed {st['overflowed']}, candidates {st['candidates']}")
    compare_to_oracle(idx.cpu().numpy(), dist.cpu().numpy(), oi, od, o2)
    assert np.array_equal(idx.cpu().numpy()[200:205], tail)


@pytest.mark.parametrize("mode", MODES + ["kmeans"])
def test_degenerate_data_sets(L, C0, mode):
    """Degenerate data: every point the same (tiles of radius 0, so the 16-bit
    scale is at its cap and most queries fall back), and points that differ in
    one strain component only (a data set on a line): every mode equals the
    oracle, ties to the lowest index."""
    _say("degenerate", mode)
    packs = ALL_PACKS | (0x20 if mode == "kmeans" else 0)
    e0, s0 = ddsynth.data_points(1, 91)
    qe, qs, _ = ddsynth.queries(*ddsynth.data_points(64, 92), 40, 93)
    for n, make in ((3000, lambda: (np.repeat(e0, 3000, 0), np.repeat(s0, 3000, 0))),
                    (2500, lambda: (np.repeat(e0, 2500, 0) + np.linspace(-1e-3, 1e-3, 2500)[:, None]
                                    * np.array([[1.0, 0, 0, 0, 0, 0]]), np.repeat(s0, 2500, 0)))):
        e, s = make()
        q_e = np.concatenate([qe, e[[0, n // 2, n - 1]]])
        q_s = np.concatenate([qs, s[[0, n // 2, n - 1]]])
        oi, od, o2 = oracle.pd_raw(e, s, C0, q_e, q_s)
        ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=packs, tile=512)
        idx, dist = L.dd_project(ds, to_dev(ddsynth.states(q_e, q_s)), mode=mode)
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        if n == 3000:
            assert np.all(idx == 0)                       # all points tie: the lowest index
        compare_to_oracle(idx, dist, oi, od, o2)
        ds.close()


def test_passes_out_of_range_is_refused(L, config0):
    for passes in (-1, 3):
        with pytest.raises(L.DDError) as ex:
            L.dd_project(config0["ds"], config0["states"][:4].contiguous(), mode="bf16",
                         passes=passes)
        assert ex.value.status == 1


@pytest.mark.parametrize("mode", ["fp64", "bf16", "ann"])
def test_scratch_reuse_across_sizes_streams_and_threads(L, C0, mode):
    """Projections reuse the dataset's scratch arenas: calls that grow the block,
    calls on another stream and calls from two threads at once give the same
    indices and distances as the first call; the footprint grows by the kept
    scratch only."""
    import threading
    import torch
    _say("scratch reuse", mode)
    e, s = ddsynth.data_points(20000, 5101)
    qe, qs, _ = ddsynth.queries(e, s, 3000, 5102)
    oi, od, o2 = oracle.pd_raw(e, s, C0, qe, qs)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4 | 0x10)
    _, b0 = L.dd_dataset_info(ds)
    states = to_dev(ddsynth.states(qe, qs))
    i1, d1 = L.dd_project(ds, states, mode=mode)
    compare_to_oracle(i1.cpu().numpy(), d1.cpu().numpy(), oi, od, o2)
    def same(i, d, reps, n=None):
        # another batch size may merge the split lists with the other merge
        # kernel: equal indices, distances to rounding
        ri, rd = i1.cpu()[:n].repeat(reps), d1.cpu()[:n].repeat(reps)
        assert torch.equal(i.cpu(), ri)
        np.testing.assert_allclose(d.cpu().numpy(), rd.numpy(), rtol=1e-14, atol=0)

    big = states.repeat(4, 1).contiguous()
    for q, reps, n in [(states[:37].contiguous(), 1, 37), (big, 4, None)]:
        same(*L.dd_project(ds, q, mode=mode), reps, n)
    i, d = L.dd_project(ds, states, mode=mode)
    assert torch.equal(i, i1) and torch.equal(d, d1)
    other = torch.cuda.Stream()
    with torch.cuda.stream(other):
        i, d = L.dd_project(ds, big, mode=mode, stream=other)
        other.synchronize()
    same(i, d, 4)
    out, errs = {}, []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for r in range(3):
                    q = big if (k + r) % 2 else states
                    i, d = L.dd_project(ds, q, mode=mode, stream=st)
                    st.synchronize()
                    out[(k, r)] = (q is big, i.cpu(), d.cpu())
        except Exception as ex:   # reported below, in the test's thread
            errs.append(repr(ex))

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=100)
    assert not errs and len(out) == 6, errs
    for is_big, i, d in out.values():
        if is_big:
            same(i, d, 4)
        else:
            assert torch.equal(i, i1.cpu()) and torch.equal(d, d1.cpu())
    _, b1 = L.dd_dataset_info(ds)
    _say(f"  device bytes {b0} -> {b1}")
    assert b0 < b1 <= b0 + 8 * (1 << 30)


@pytest.mark.parametrize("mode", MODES)
def test_invalid_states_and_empty(L, config0, mode):
    import torch
    states = config0["states"][:9].clone()
    states[3, 4] = float("nan")
    states[7, 11] = float("inf")
    idx, dist = L.dd_project(config0["ds"], states, mode=mode)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert idx[3] == -1 and idx[7] == -1 and np.isnan(dist[3]) and np.isnan(dist[7])
    ok = [0, 1, 2, 4, 5, 6, 8]
    assert np.array_equal(idx[ok], config0["oi"][ok])
    empty = torch.empty((0, 12), dtype=torch.float64, device="cuda")
    i0, d0 = L.dd_project(config0["ds"], empty, mode=mode)
    assert i0.numel() == 0


def test_error_paths(L, C0):
    import torch
    e, s = ddsynth.data_points(100, 5)
    bad_C = C0.copy()
    bad_C[0, 0] = -1.0
    with pytest.raises(L.DDError) as ex:
        L.dd_dataset_create(to_dev(e), to_dev(s), bad_C)
    assert ex.value.status == 2
    asym = C0.copy()
    asym[0, 1] += 1.0
    with pytest.raises(L.DDError) as ex:
        L.dd_dataset_create(to_dev(e), to_dev(s), asym)
    assert ex.value.status == 2
    e2 = e.copy()
    e2[50, 2] = np.nan
    with pytest.raises(L.DDError) as ex:
        L.dd_dataset_create(to_dev(e2), to_dev(s), C0)
    assert ex.value.status == 1
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1)
    for mode in ("fp32", "bf16", "fp16", "ann"):
        with pytest.raises(L.DDError) as ex:
            L.dd_project(ds, torch.zeros((3, 12), dtype=torch.float64, device="cuda"), mode=mode)
        assert ex.value.status == 8
    ds2 = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x10)
    with pytest.raises(L.DDError) as ex:
        L.dd_project(ds2, torch.zeros((3, 12), dtype=torch.float64, device="cuda"), mode="ann",
                     ann_budget=-1)
    assert ex.value.status == 1
