"""GPU parity of dd_solve (the DD fixed-point loop) against the CPU oracle."""
import numpy as np
import pytest

import ddsynth
import oracle
from oracle import fe
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_00357_amd import _lib
    return _lib


def _problem(n, N, seed, traction=100.0):
    e, s = ddsynth.data_points(N, seed)
    m = fe.Mesh(n)
    mask, f = m.clamp_mask(), m.traction_x1(traction)
    init = ddsynth.indices(m.n_mp, N, seed + 1)
    return e, s, m, mask, f, init


@pytest.mark.parametrize("mode", ["fp64", "bf16", "ann"])
def test_dd_solve_matches_oracle_trajectory(L, C0, mode):
    """Same association at every iteration, same iteration count, same u (the
    ANN walk without a budget is exact)."""
    e, s, m, mask, f, init = _problem(3, 20000, 51)
    ref = fe.dd_solve(e, s, C0, m, mask, f, init, record_history=True)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4 | 0x10)
    got = L.dd_solve(ds, (3, 3, 3), mask, f, init, mode=mode, history=True)
    print(f"iters oracle {ref.iterations} gpu {got['iterations']}, cg {got['cg_iterations']}, "
          f"res {got['cg_max_residual']:.2e}, {got['elapsed_ms']:.1f} ms", flush=True)
    assert got["converged"] and ref.converged
    assert got["iterations"] == ref.iterations
    for i, h in enumerate(ref.history):
        assert np.array_equal(got["history"][i], h), f"association differs at iteration {i}"
    np.testing.assert_allclose(got["u"], ref.u, rtol=0, atol=1e-10 * np.abs(ref.u).max())
    np.testing.assert_allclose(got["d_half"], ref.d_half, rtol=1e-9)
    np.testing.assert_allclose(got["d_full"], ref.d_full, rtol=1e-9)
    assert list(got["changed"]) == ref.changed
    np.testing.assert_allclose(got["eps"], ref.eps, rtol=0, atol=1e-10 * np.abs(ref.eps).max())
    np.testing.assert_allclose(got["sig"], ref.sig, rtol=0, atol=1e-9 * np.abs(ref.sig).max())


@pytest.mark.parametrize("mode", ["fp64", "ann"])
def test_dd_solve_resumes_from_a_checkpoint(L, C0, mode):
    """The association alone fixes the next iterate (Section 2): a solve cut
    after k iterations and resumed from its association (the checkpoint)
    follows the uninterrupted trajectory bit for bit."""
    e, s, m, mask, f, init = _problem(4, 50000, 71)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x10)
    full = L.dd_solve(ds, (4, 4, 4), mask, f, init, mode=mode, history=True)
    K = full["iterations"]
    assert full["converged"] and K >= 3
    k = K // 2
    cut = L.dd_solve(ds, (4, 4, 4), mask, f, init, mode=mode, history=True, max_iter=k)
    assert cut["iterations"] == k and not cut["converged"]
    assert np.array_equal(cut["history"], full["history"][:k + 1])
    rest = L.dd_solve(ds, (4, 4, 4), mask, f, cut["idx"], mode=mode, history=True)
    assert rest["iterations"] == K - k and rest["converged"]
    assert np.array_equal(rest["history"], full["history"][k:])
    assert np.array_equal(rest["u"], full["u"]) and np.array_equal(rest["idx"], full["idx"])
    assert np.array_equal(rest["d_full"], full["d_full"][k:])


def test_dd_solve_monotone_and_deterministic(L, C0):
    e, s, m, mask, f, init = _problem(4, 50000, 61)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4)
    a = L.dd_solve(ds, (4, 4, 4), mask, f, init, history=True)
    b = L.dd_solve(ds, (4, 4, 4), mask, f, init, history=True)
    assert np.array_equal(a["history"], b["history"]) and np.array_equal(a["u"], b["u"])
    tol = 1e-12 * a["d_half"][0]
    for i in range(a["iterations"]):
        assert a["d_full"][i] <= a["d_half"][i] + tol
        if i:
            assert a["d_half"][i] <= a["d_full"][i - 1] + tol


def test_dd_solve_linear_law_planted(L, C0):
    """Noise-free linear-law data with the exact uniaxial state planted: from the
    planted association the loop stops after one iteration with zero distance
    and the exact linear displacement (rollers, traction on x = 1)."""
    E, nu, t = ddsynth.E_MODULUS, ddsynth.POISSON, 60.0
    m = fe.Mesh(2)
    mask, f = m.roller_mask(), m.traction_x1(t)
    e, s = ddsynth.data_points(3000, 41, noise_std=0.0)
    e[1234] = (t / E) * np.array([1.0, -nu, -nu, 0, 0, 0])
    s[1234] = np.array([t, 0, 0, 0, 0, 0.0])
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4)
    got = L.dd_solve(ds, (2, 2, 2), mask, f, np.full(m.n_mp, 1234))
    assert got["converged"] and got["iterations"] == 1
    assert got["d_half"][0] <= 1e-24 and got["d_full"][0] <= 1e-24
    x = m.coords
    want = (t / E) * np.stack([x[:, 0], -nu * x[:, 1], -nu * x[:, 2]], 1).ravel()
    np.testing.assert_allclose(got["u"], want, atol=1e-15)


@pytest.mark.parametrize("mode", ["bf16", "fp64"])
def test_dd_solve_config1_stepwise(L, C0, mode):
    """8^3 mesh, N = 1e6, clamp + 100 MPa, in the BF16 and the FP64 mode: every
    P_C of the GPU trajectory is recomputed by the oracle from the GPU's
    association, and every P_D is checked on 48 sampled material points by
    oracle brute force."""
    e, s, m, mask, f, init = _problem(8, 1_000_000, 1001)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4)
    got = L.dd_solve(ds, (8, 8, 8), mask, f, init, mode=mode, history=True)
    print(f"config 1 ({mode}): {got['iterations']} iterations, converged {got['converged']}, "
          f"{got['elapsed_ms']:.1f} ms, cg {got['cg_iterations']}", flush=True)
    assert got["converged"]
    pc = fe.ConstraintProjector(m, C0, mask, f)
    rng = np.random.default_rng(7)
    sample = rng.choice(m.n_mp, 48, replace=False)
    hist = got["history"]
    for i in range(got["iterations"]):
        z = hist[i]
        u, _, eps, sig = pc(e[z], s[z])
        dh = m.w * np.sum(oracle.pair_dist_raw(eps, sig, e[z], s[z], C0))
        assert dh == pytest.approx(got["d_half"][i], rel=1e-9)
        oi, od, o2 = oracle.pd_raw(e, s, C0, eps[sample], sig[sample])
        clear = o2 > od * (1 + 1e-12)
        assert np.array_equal(hist[i + 1][sample][clear], oi[clear]), f"P_D differs at iteration {i}"
    np.testing.assert_allclose(got["u"], u, rtol=0, atol=1e-10 * np.abs(u).max())


def test_dd_solve_graph_replays_equal_eager(L, C0):
    """The captured CG batches (replayed many times per solve, with eager work
    and synchronisations between replays) give bitwise the eager result."""
    e, s, m, mask, f, init = _problem(4, 30000, 71)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4)
    a = L.dd_solve(ds, (4, 4, 4), mask, f, init, history=True, graph=True, cg=True)
    b = L.dd_solve(ds, (4, 4, 4), mask, f, init, history=True, graph=False, cg=True)
    assert a["cg_iterations"] > 100
    assert np.array_equal(a["history"], b["history"])
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["d_half"], b["d_half"])


@pytest.mark.parametrize("n", [3, 8, 16])
def test_dd_solve_inverse_equals_cg(L, C0, n):
    """P_C by the cached K^-1 and by CG give the same trajectory; u agrees to the
    CG tolerance.  The second solve on the same mesh reuses the inverse."""
    e, s, m, mask, f, init = _problem(n, 100000, 81 + n)
    ds = L.dd_dataset_create(to_dev(e), to_dev(s), C0, packs=0x1 | 0x4)
    cg = L.dd_solve(ds, (n, n, n), mask, f, init, mode="bf16", history=True, cg=True)
    inv1 = L.dd_solve(ds, (n, n, n), mask, f, init, mode="bf16", history=True)
    inv2 = L.dd_solve(ds, (n, n, n), mask, f, init, mode="bf16", history=True)
    print(f"{n}^3: cg {cg['elapsed_ms']:.1f} ms ({cg['cg_iterations']} CG iterations), inverse "
          f"{inv1['elapsed_ms']:.1f} ms first, {inv2['elapsed_ms']:.1f} ms cached", flush=True)
    assert inv1["cg_iterations"] == 0 and cg["cg_iterations"] > 0
    assert np.array_equal(cg["history"], inv1["history"])
    assert np.array_equal(inv1["history"], inv2["history"]) and np.array_equal(inv1["u"], inv2["u"])
    np.testing.assert_allclose(inv1["u"], cg["u"], rtol=0, atol=1e-10 * np.abs(cg["u"]).max())
