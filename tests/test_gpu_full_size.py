"""Parity at the full sizes of the measured workloads, on sampled outputs the
CPU oracle computes one by one (through the C ABI, in the launch configuration
the benchmark times).

* N = 2^27 data points, m = 65536 queries: the BF16, FP16 and FP32 scans with
  FP64 rerank equal the FP64 MFMA scan on every query (indices and distances),
  and the BF16 scan equals the oracle on a 1024-query sample (the
  oracle's whitened brute force, which equals its raw-metric brute force on
  the 4096 queries of the N = 65536 workload, a CPU test).
* N = 10^9 data points generated on the device, 16^3 hexahedra (32768
  material points): the exact ANN walk inside dd_solve equals oracle brute
  force over all 10^9 points on sampled material points, the ANN walk equals
  the BF16 exact scan on 32768 queries, and budgeted walks report their recall
  and the DD displacement error.
"""
import sys
import time

import numpy as np
import pytest

import ddsynth
import oracle
from gpu_util import NEAR_TIE, to_dev

pytestmark = pytest.mark.gpu

FP64, FP32, BF16, FP16, ANN = 0x1, 0x2, 0x4, 0x8, 0x10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_00357_amd import _lib
    return _lib


def _oracle_over_chunks(gen, N, C, qe, qs, chunk=1 << 25):
    """Oracle brute force over a data set streamed in chunks from the seeded
    generator: lexicographic (distance, index) minimum and the runner-up value
    over all chunks."""
    m = qe.shape[0]
    best = np.full(m, np.inf)
    bi = np.full(m, -1, np.int64)
    vals = [[] for _ in range(m)]
    for f in range(0, N, chunk):
        n = min(chunk, N - f)
        e, s = gen(f, n)
        oi, od, o2 = oracle.pd_raw(e, s, C, qe, qs)
        for q in range(m):
            vals[q] += [od[q], o2[q]]
            if od[q] < best[q]:          # earlier chunks hold lower indices
                best[q], bi[q] = od[q], oi[q] + f
    second = np.array([sorted(v)[1] for v in vals])
    return bi, best, second


@pytest.mark.timeout(900)
def test_config2_bf16_equals_fp64_and_oracle_2e27(L, C0):
    import torch
    N, m = 1 << 27, 65536
    t = time.time()
    e, s = ddsynth.data_points(N, 1002)
    qe, qs, _ = ddsynth.queries(e, s, m, 2002)
    ds = L.dd_dataset_create(torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda(), C0,
                             packs=FP64 | FP32 | BF16 | FP16)
    torch.cuda.empty_cache()
    states = torch.from_numpy(ddsynth.states(qe, qs)).cuda()
    ib, db = L.dd_project(ds, states, mode="bf16")
    i6, d6 = L.dd_project(ds, states, mode="fp64")
    assert torch.equal(ib, i6)
    assert torch.equal(db, d6)
    for mode in ("fp16", "fp32"):
        im, dm = L.dd_project(ds, states, mode=mode)
        assert torch.equal(im, i6), mode
        assert torch.equal(dm, d6), mode
    _say(f"2^27: bf16 == fp16 == fp32 == fp64 on all {m} queries ({time.time() - t:.0f}s)")
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(m, 1024, replace=False))
    t1 = time.time()
    W = oracle.whiten(e, s, C0)
    del e, s
    oi, od, o2 = oracle.pd_white(W, oracle.whiten(qe[sample], qs[sample], C0))
    del W
    clear = o2 > od * (1 + NEAR_TIE)
    got = ib.cpu().numpy()[sample]
    assert np.array_equal(got[clear], oi[clear])
    np.testing.assert_allclose(db.cpu().numpy()[sample], od, rtol=1e-12, atol=0)
    _say(f"2^27: 1024 sampled queries equal the oracle ({(~clear).sum()} near ties, oracle "
         f"{time.time() - t1:.0f}s on {oracle.threads()} threads), {time.time() - t:.0f}s")
    ds.close()


@pytest.fixture(scope="module")
def config3(L, C0):
    import torch
    N = 1_000_000_000
    gen = ddsynth.DevicePoints(1003)
    t = time.time()
    ds = L.dd_dataset_create_streamed(N, C0, gen.fill_fn, gen.user, packs=FP64 | BF16 | ANN)
    torch.cuda.synchronize()
    _say(f"1e9: dataset created in {time.time() - t:.1f}s, {ds.info()[1] / 1e9:.1f} GB")
    yield dict(N=N, gen=gen, ds=ds)
    ds.close()


def test_config3_ann_equals_bf16_scan_1e9(L, config3):
    """Two independent exact methods agree bit for bit at N = 10^9."""
    import torch
    N, ds = config3["N"], config3["ds"]
    qe, qs, base = ddsynth.queries_generated(N, 1003, 32768, 2003)
    states = torch.from_numpy(ddsynth.states(qe, qs)).cuda()
    ia, da, st = L.dd_project(ds, states, mode="ann", stats=True)
    _say(f"1e9 ann exact: {st['scan_ms']:.1f} ms walk, {st['visited'] / 32768:.0f} points/query, "
         f"{st['candidates'] / 32768:.2f} candidates/query, {st['overflowed']} overflowed")
    # The pruning bound is tight: no list overflows, and the certified band
    # around the nearest distance holds few other points (1.06 per query
    # measured).  A bound that is valid but too loose (a wrong wave minimum)
    # keeps every answer exact through the FP64 fallback and shows only here.
    assert st["overflowed"] == 0 and st["candidates"] <= 1.5 * 32768
    ib, db = L.dd_project(ds, states, mode="bf16")
    assert torch.equal(ia, ib) and torch.equal(da, db)
    warm = torch.from_numpy(base).cuda()
    for budget in (4, 64):
        ix, dx, st = L.dd_project(ds, states, warm_start_idx=warm, mode="ann", ann_budget=budget,
                                  stats=True)
        recall = float((ix == ia).double().mean())
        excess = float(((dx - da) / da).mean())
        _say(f"1e9 ann budget {budget}: recall {recall:.4f}, mean relative distance excess "
             f"{excess:.3e}, {st['scan_ms']:.2f} ms")
        assert bool((dx >= da * (1 - 1e-12)).all())


@pytest.mark.timeout(600)
def test_config3_dd_solve_ann_1e9(L, config3, C0):
    """16^3 hexahedra, clamp + 100 MPa, N = 10^9: the exact ANN solve's final
    association equals oracle brute force over every data point on sampled
    material points; budgeted solves report their displacement error."""
    import torch
    N, ds, gen = config3["N"], config3["ds"], config3["gen"]
    n = 16
    mask, force = ddsynth.box_bc(n, 100.0)
    init = ddsynth.indices(8 * n ** 3, N, 3)
    t = time.time()
    r = L.dd_solve(ds, (n, n, n), mask, force, init, mode="ann")
    _say(f"1e9 dd_solve exact ann: {r['iterations']} iterations, converged {r['converged']}, "
         f"{time.time() - t:.2f}s")
    assert r["converged"]
    tol = 1e-12 * r["d_half"][0]
    for i in range(r["iterations"]):
        assert r["d_full"][i] <= r["d_half"][i] + tol
    rng = np.random.default_rng(13)
    sample = rng.choice(8 * n ** 3, 16, replace=False)
    qe, qs = r["eps"][sample], r["sig"][sample]

    def chunk(f, k):
        e, s = gen.generate(f, k)
        torch.cuda.synchronize()
        return e.cpu().numpy(), s.cpu().numpy()

    t = time.time()
    oi, od, o2 = _oracle_over_chunks(chunk, N, C0, qe, qs)
    clear = o2 > od * (1 + NEAR_TIE)
    _say(f"1e9 oracle over 16 sampled material points: {time.time() - t:.0f}s, "
         f"{(~clear).sum()} near ties")
    assert np.array_equal(r["idx"][sample][clear], oi[clear])
    for budget in (16,):
        rb = L.dd_solve(ds, (n, n, n), mask, force, init, mode="ann", ann_budget=budget)
        err = np.linalg.norm(rb["u"] - r["u"]) / np.linalg.norm(r["u"])
        _say(f"1e9 dd_solve ann budget {budget}: {rb['iterations']} iterations (stop "
             f"{rb['stop_reason']}), |u - u_exact| / |u_exact| = {err:.3e}")
        assert rb["stop_reason"] in (1, 2)
