"""Pins of the CPU oracle against facts other than itself (closed forms,
hand-worked values, invariants of the method).  CPU only."""
import os

import numpy as np
import pytest

import ddsynth
import oracle
from oracle import fe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Generator
# ----------------------------------------------------------------------------
def test_philox_known_answers():
    """Philox4x32-10 known-answer vectors of its published reference implementation."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = ddsynth.philox_np(np.array([ctr], np.uint32), np.array(key, np.uint32))[0]
        assert tuple(int(x) for x in got) == want
    items = np.arange(257, dtype=np.uint64) * 1000003 + (1 << 33)
    ctr = np.stack([(items & 0xFFFFFFFF).astype(np.uint32), (items >> 32).astype(np.uint32),
                    np.full(items.size, 9, np.uint32), np.zeros(items.size, np.uint32)], -1)
    assert np.array_equal(ddsynth.philox(123456789012, items, 9),
                          ddsynth.philox_np(ctr, np.array([123456789012 & 0xFFFFFFFF,
                                                           123456789012 >> 32], np.uint32)))


def test_generator_elementary_functions():
    """The generator's own log and cos/sin(2 pi u) (shared by its host and GPU
    builds) agree with the C library to a few units in the last place."""
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.random(200000), [2.0 ** -53, 0.25, 0.5, 0.75, 1.0 - 2.0 ** -53],
                        np.arange(1, 64) / 64.0])
    el = ddsynth.elementary(u)
    ref_log = np.log(u)
    assert np.all(np.abs(el[:, 0] - ref_log) <= 4 * np.spacing(np.abs(ref_log)) + 1e-300)
    # 2 pi u is itself rounded in the library reference: compare absolutely
    assert np.abs(el[:, 1] - np.cos(2 * np.pi * u)).max() < 2e-15
    assert np.abs(el[:, 2] - np.sin(2 * np.pi * u)).max() < 2e-15
    assert el[u == 0.25, 1][0] == 0.0 and el[u == 0.5, 2][0] == 0.0
    z = ddsynth.box_muller(rng.random(400000), rng.random(400000)).ravel()
    assert abs(z.mean()) < 5e-3 and abs(z.std() - 1.0) < 5e-3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_generated_queries_match_stored_queries():
    e, s = ddsynth.data_points(5000, 91)
    a = ddsynth.queries(e, s, 700, 92)
    b = ddsynth.queries_generated(5000, 91, 700, 92)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_generator_moments(C0):
    e, s = ddsynth.data_points(200000, 1000)
    assert e.min() >= -1e-3 and e.max() < 1e-3
    assert abs(e.mean()) < 1e-5 and abs(e.std() - 2e-3 / np.sqrt(12)) < 5e-6
    noise = s - e @ C0.T
    assert abs(noise.std() - 2.0) < 0.02 and abs(noise.mean()) < 0.02
    qe, qs, base = ddsynth.queries(e, s, 20000, 2000)
    assert abs((qe - e[base]).std() - 5e-5) < 1e-6 and abs((qs - s[base]).std() - 10.0) < 0.2


# ----------------------------------------------------------------------------
# P_D
# ----------------------------------------------------------------------------
def _read_hand():
    data, queries = [], []
    diag = None
    with open(os.path.join(GOLDEN, "pd_hand.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "metric_diag":
                diag = np.array([float(x) for x in tok[1:]])
            elif tok[0] == "data":
                data.append([float(x) for x in tok[1:]])
            elif tok[0] == "query":
                k = tok.index("expect")
                queries.append(([float(x) for x in tok[1:k]], int(tok[k + 1]), float(tok[k + 2]),
                                float(tok[k + 3])))
    return np.diag(diag), np.array(data), queries


def test_pd_hand_worked():
    C, data, queries = _read_hand()
    q = np.array([x[0] for x in queries])
    idx, dist, second = oracle.pd_raw(data[:, :6], data[:, 6:], C, q[:, :6], q[:, 6:])
    for k, (_, i, d, d2) in enumerate(queries):
        assert idx[k] == i
        assert dist[k] == pytest.approx(d, rel=1e-15)
        assert second[k] == pytest.approx(d2, rel=1e-15)
    # the whitened form reaches the same answer
    iw, dw, _ = oracle.pd_white(oracle.whiten(data[:, :6], data[:, 6:], C),
                                oracle.whiten(q[:, :6], q[:, 6:], C))
    assert np.array_equal(iw, idx) and np.allclose(dw, dist, rtol=1e-14)


def _mandel(v, stress: bool):
    """Voigt (engineering shear strain / plain shear stress) -> Mandel components."""
    v = np.array(v, dtype=float)
    out = v.copy()
    out[..., 3:] = v[..., 3:] * (np.sqrt(2.0) if stress else 1.0 / np.sqrt(2.0))
    return out


def test_metric_isotropic_closed_form(C0):
    """Isotropic metric through the volumetric/deviatoric projectors (Mandel form):
    de.C de = 3K |P_vol de|^2 + 2mu |P_dev de|^2,  ds.C^-1 ds = |P_vol ds|^2/3K + |P_dev ds|^2/2mu."""
    E, nu = ddsynth.E_MODULUS, ddsynth.POISSON
    K = E / (3.0 * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    one = np.array([1.0, 1, 1, 0, 0, 0])
    Pv = np.outer(one, one) / 3.0
    Pd = np.eye(6) - Pv
    rng = np.random.default_rng(5)
    a_e, b_e = rng.uniform(-1e-3, 1e-3, (2, 500, 6))
    a_s, b_s = rng.uniform(-300, 300, (2, 500, 6))
    got = oracle.pair_dist_raw(a_e, a_s, b_e, b_s, C0)
    de, ds = _mandel(a_e - b_e, False), _mandel(a_s - b_s, True)
    want = 0.5 * (3 * K * np.sum((de @ Pv) ** 2, 1) + 2 * mu * np.sum((de @ Pd) ** 2, 1)) \
        + 0.5 * (np.sum((ds @ Pv) ** 2, 1) / (3 * K) + np.sum((ds @ Pd) ** 2, 1) / (2 * mu))
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # and the whitened map reproduces the same squared norm
    w = 0.5 * np.sum((oracle.whiten(a_e, a_s, C0) - oracle.whiten(b_e, b_s, C0)) ** 2, 1)
    np.testing.assert_allclose(w, want, rtol=1e-12)


def test_metric_scaling_separates_terms(C0):
    """C -> aC scales the strain term by a and the stress term by 1/a."""
    rng = np.random.default_rng(6)
    a_e, b_e = rng.uniform(-1e-3, 1e-3, (2, 50, 6))
    a_s, b_s = rng.uniform(-300, 300, (2, 50, 6))
    zero = np.zeros((50, 6))
    de1 = oracle.pair_dist_raw(a_e, zero, b_e, zero, C0)
    de3 = oracle.pair_dist_raw(a_e, zero, b_e, zero, 3.0 * C0)
    ds1 = oracle.pair_dist_raw(zero, a_s, zero, b_s, C0)
    ds3 = oracle.pair_dist_raw(zero, a_s, zero, b_s, 3.0 * C0)
    np.testing.assert_allclose(de3, 3.0 * de1, rtol=1e-13)
    np.testing.assert_allclose(ds3, ds1 / 3.0, rtol=1e-13)
    both = oracle.pair_dist_raw(a_e, a_s, b_e, b_s, C0)
    np.testing.assert_allclose(both, de1 + ds1, rtol=1e-13)


def test_pd_query_is_data_point_and_duplicates(C0):
    e, s = ddsynth.data_points(3000, 11)
    # plant duplicates of point 17 at higher indices, of point 2500 at a lower one
    e[1200], s[1200] = e[17], s[17]
    e[2999], s[2999] = e[17], s[17]
    e[40], s[40] = e[2500], s[2500]
    picks = np.array([17, 1200, 2999, 2500, 40, 0, 2998])
    idx, dist, second = oracle.pd_raw(e, s, C0, e[picks], s[picks])
    assert np.all(dist == 0.0)
    assert list(idx) == [17, 17, 17, 40, 40, 0, 2998]
    assert second[0] == 0.0 and second[3] == 0.0 and second[5] > 0.0


def test_pd_permutation_equivariance(C0):
    e, s = ddsynth.data_points(5000, 12)
    qe, qs, _ = ddsynth.queries(e, s, 300, 13)
    i1, d1, s1 = oracle.pd_raw(e, s, C0, qe, qs)
    perm = np.random.default_rng(3).permutation(5000)
    i2, d2, _ = oracle.pd_raw(e[perm], s[perm], C0, qe, qs)
    clear = s1 > d1 * (1 + 1e-12)
    assert clear.mean() > 0.99
    assert np.array_equal(perm[i2][clear], i1[clear])
    np.testing.assert_allclose(d2, d1, rtol=1e-13)


def test_pd_second_is_second_order_statistic(C0):
    e, s = ddsynth.data_points(2000, 14)
    qe, qs, _ = ddsynth.queries(e, s, 25, 15)
    idx, dist, second = oracle.pd_raw(e, s, C0, qe, qs)
    for q in range(25):
        all_d = oracle.pair_dist_raw(np.repeat(qe[q:q + 1], 2000, 0), np.repeat(qs[q:q + 1], 2000, 0),
                                     e, s, C0)
        srt = np.sort(all_d)
        assert dist[q] == srt[0] and second[q] == srt[1]
        assert idx[q] == np.flatnonzero(all_d == srt[0])[0]


def test_pd_few_queries_path_matches_many_queries_path(C0):
    """The data-split path (few queries) and the per-query path agree exactly."""
    e, s = ddsynth.data_points(20000, 16)
    qe, qs, _ = ddsynth.queries(e, s, 200, 17)
    ia, da, sa = oracle.pd_raw(e, s, C0, qe, qs)
    for q in (0, 7, 199):
        ib, db, sb = oracle.pd_raw(e, s, C0, qe[q:q + 1], qs[q:q + 1])
        assert ib[0] == ia[q] and db[0] == da[q] and sb[0] == sa[q]
    w, qw = oracle.whiten(e, s, C0), oracle.whiten(qe, qs, C0)
    iw, dw, _ = oracle.pd_white(w, qw)
    iw1, dw1, _ = oracle.pd_white(w, qw[5:6])
    assert iw1[0] == iw[5] and dw1[0] == dw[5]
    i32, d32, _ = oracle.pd_white_f32data(w.astype(np.float32), qw[:3])
    ref = oracle.pd_white(w.astype(np.float32).astype(np.float64), qw[:3])
    assert np.array_equal(i32, ref[0]) and np.array_equal(d32, ref[1])


def test_pd_whitened_equals_raw_on_exact_projection_workload(C0):
    """The oracle's whitened brute force (the timed CPU baseline and the check of
    the 2^27 sample) gives the raw-metric brute force's answer on the whole
    N = 65536, m = 4096 workload: equal indices wherever the raw best is clear
    of the runner-up by 1e-12, distances within 1e-13 relative (the two forms
    differ only in rounding)."""
    e, s = ddsynth.data_points(65536, 1000)
    qe, qs, _ = ddsynth.queries(e, s, 4096, 2000)
    ri, rd, r2 = oracle.pd_raw(e, s, C0, qe, qs)
    wi, wd, w2 = oracle.pd_white(oracle.whiten(e, s, C0), oracle.whiten(qe, qs, C0))
    clear = r2 > rd * (1 + 1e-12)
    assert clear.mean() > 0.99
    assert np.array_equal(wi[clear], ri[clear])
    np.testing.assert_allclose(wd, rd, rtol=1e-13, atol=0)
    np.testing.assert_allclose(w2, r2, rtol=1e-13, atol=0)


# ----------------------------------------------------------------------------
# Finite elements
# ----------------------------------------------------------------------------
def test_fe_patch_test():
    """A linear displacement field gives the exact constant strain everywhere."""
    m = fe.Mesh(3)
    A = np.random.default_rng(1).normal(size=(3, 3)) * 1e-3
    u = (m.coords @ A.T).ravel()
    eps = m.strains(u)
    want = np.array([A[0, 0], A[1, 1], A[2, 2], A[1, 2] + A[2, 1], A[0, 2] + A[2, 0],
                     A[0, 1] + A[1, 0]])
    np.testing.assert_allclose(eps, np.tile(want, (m.n_mp, 1)), atol=1e-15)
    assert m.w * m.n_mp == pytest.approx(1.0, rel=1e-14)      # weights sum to the volume


def test_fe_rigid_modes_in_kernel(C0):
    m = fe.Mesh(2)
    K = m.stiffness(C0)
    assert abs(K - K.T).max() <= 1e-9 * abs(K).max()
    x = m.coords
    modes = []
    for c in range(3):
        t = np.zeros_like(x)
        t[:, c] = 1.0
        modes.append(t.ravel())
    for axis in np.eye(3):
        modes.append(np.cross(axis, x).ravel())
    for r in modes:
        assert np.abs(K @ r).max() <= 1e-9 * abs(K).max()
        assert np.abs(m.strains(r)).max() <= 1e-12


def test_fe_traction_resultant():
    m = fe.Mesh(5)
    f = m.traction_x1(37.0)
    assert f[0::3].sum() == pytest.approx(37.0, rel=1e-14)
    assert f[1::3].sum() == 0.0 and f[2::3].sum() == 0.0
    loaded = np.flatnonzero(f)
    assert np.allclose(m.coords[loaded // 3, 0], 1.0)


def test_fe_homogeneous_tension_closed_form(C0):
    """Rollers on x=0, y=0, z=0 and traction t on x=1: uniaxial stress state,
    u = (t/E) (x, -nu y, -nu z) exactly."""
    E, nu, t = ddsynth.E_MODULUS, ddsynth.POISSON, 80.0
    m = fe.Mesh(3)
    mask, f = m.roller_mask(), m.traction_x1(t)
    pc = fe.ConstraintProjector(m, C0, mask, f)
    u = pc.solve(f)                    # linear elasticity K u = f
    x = m.coords
    want = (t / E) * np.stack([x[:, 0], -nu * x[:, 1], -nu * x[:, 2]], 1).ravel()
    np.testing.assert_allclose(u, want, atol=1e-15)
    eps = m.strains(u)
    np.testing.assert_allclose(eps @ C0.T, np.tile([t, 0, 0, 0, 0, 0], (m.n_mp, 1)), atol=1e-9)


def _objective(m, C, eps, sig, ze, zs):
    return m.w * np.sum(oracle.pair_dist_raw(eps, sig, ze, zs, C))


def test_pc_properties(C0):
    """P_C output is compatible, equilibrated, a fixed point, and minimises the
    weighted distance over admissible perturbations."""
    m = fe.Mesh(2)
    mask, f = m.clamp_mask(), m.traction_x1(100.0)
    pc = fe.ConstraintProjector(m, C0, mask, f)
    de, ds = ddsynth.data_points(4000, 21)
    idx = ddsynth.indices(m.n_mp, 4000, 22)
    ze, zs = de[idx], ds[idx]
    u, eta, eps, sig = pc(ze, zs)
    np.testing.assert_allclose(eps, m.strains(u), atol=0)                  # compatibility
    res = m.assemble_vector(sig) - f
    assert np.abs(res[pc.free]).max() <= 1e-10 * np.abs(f).max()           # equilibrium
    assert np.all(u[mask] == 0.0) and np.all(eta[mask] == 0.0)
    u2, _, eps2, sig2 = pc(eps, sig)                                       # idempotence
    np.testing.assert_allclose(u2, u, rtol=1e-10, atol=1e-18)
    np.testing.assert_allclose(sig2, sig, rtol=1e-10, atol=1e-9)
    J0 = _objective(m, C0, eps, sig, ze, zs)
    rng = np.random.default_rng(7)
    # admissible displacement perturbations keep equilibrium untouched
    for _ in range(5):
        du = rng.normal(size=m.n_dof) * 1e-5
        du[mask] = 0.0
        for t in (1.0, -1.0, 0.1):
            assert _objective(m, C0, m.strains(u + t * du), sig, ze, zs) >= J0 * (1 - 1e-13)
    # self-equilibrated stress perturbations: null space of the free rows of A_e{w B^T .}
    n_s = m.n_mp * 6
    Bt = np.zeros((m.n_dof, n_s))
    for k in range(n_s):
        e = np.zeros(n_s)
        e[k] = 1.0
        Bt[:, k] = m.assemble_vector(e.reshape(m.n_mp, 6))
    Af = Bt[pc.free]
    _, sv, vt = np.linalg.svd(Af)
    null = vt[np.sum(sv > 1e-12 * sv[0]):]
    for k in range(5):
        dsig = (null.T @ rng.normal(size=null.shape[0])).reshape(m.n_mp, 6) * 5.0
        assert np.abs(Af @ dsig.ravel()).max() < 1e-9
        for t in (1.0, -1.0, 0.1):
            assert _objective(m, C0, eps, sig + t * dsig, ze, zs) >= J0 * (1 - 1e-13)


# ----------------------------------------------------------------------------
# DD loop
# ----------------------------------------------------------------------------
def test_dd_monotone_and_terminates(C0):
    """Alternating minimisation: D_full_i <= D_half_i <= D_full_{i-1}."""
    m = fe.Mesh(3)
    de, ds = ddsynth.data_points(20000, 31)
    init = ddsynth.indices(m.n_mp, 20000, 32)
    r = fe.dd_solve(de, ds, C0, m, m.clamp_mask(), m.traction_x1(100.0), init)
    assert r.converged and r.changed[-1] == 0
    tol = 1e-12 * r.d_half[0]
    for i in range(r.iterations):
        assert r.d_full[i] <= r.d_half[i] + tol
        if i > 0:
            assert r.d_half[i] <= r.d_full[i - 1] + tol
    assert r.d_full[-1] < 0.2 * r.d_half[0]


def test_dd_linear_law_planted_homogeneous(C0):
    """Noise-free linear-law data containing the exact uniaxial state: from the
    planted initial association the loop stops at once with zero distance and
    the exact linear displacement; from a random start it still converges."""
    E, nu, t = ddsynth.E_MODULUS, ddsynth.POISSON, 60.0
    m = fe.Mesh(2)
    mask, f = m.roller_mask(), m.traction_x1(t)
    de, ds = ddsynth.data_points(3000, 41, noise_std=0.0)
    exact_e = (t / E) * np.array([1.0, -nu, -nu, 0, 0, 0])
    exact_s = np.array([t, 0, 0, 0, 0, 0.0])
    de[1234], ds[1234] = exact_e, exact_s
    r = fe.dd_solve(de, ds, C0, m, mask, f, np.full(m.n_mp, 1234))
    assert r.converged and r.iterations == 1
    assert r.d_half[0] <= 1e-24 and r.d_full[0] <= 1e-24
    x = m.coords
    want = (t / E) * np.stack([x[:, 0], -nu * x[:, 1], -nu * x[:, 2]], 1).ravel()
    np.testing.assert_allclose(r.u, want, atol=1e-15)
    r2 = fe.dd_solve(de, ds, C0, m, mask, f, ddsynth.indices(m.n_mp, 3000, 42))
    assert r2.converged                      # may stop at a local minimum (Section 2)
    assert r2.d_full[-1] < 0.1 * r2.d_half[0]


def test_dd_planted_fe_solution_clamped(C0):
    """Data plus the states (B u_FE, C B u_FE) of the linear FE solution: started
    from them, DD is at a fixed point after one iteration with u = u_FE."""
    m = fe.Mesh(2)
    mask, f = m.clamp_mask(), m.traction_x1(100.0)
    pc = fe.ConstraintProjector(m, C0, mask, f)
    u_fe = pc.solve(f)
    pe = m.strains(u_fe)
    ps = pe @ C0.T
    de, ds = ddsynth.data_points(2000, 43)
    de = np.concatenate([de, pe])
    ds = np.concatenate([ds, ps])
    init = 2000 + np.arange(m.n_mp)
    r = fe.dd_solve(de, ds, C0, m, mask, f, init)
    assert r.converged and r.iterations == 1
    np.testing.assert_allclose(r.u, u_fe, rtol=1e-10, atol=1e-16)
    assert r.d_full[0] <= 1e-20


def test_input_bc_matches_oracle_mesh():
    """The benchmark's boundary conditions describe the same problem as the
    oracle's mesh helpers (clamped x = 0, traction on x = 1)."""
    for n in (1, 3, 8):
        mask, f = ddsynth.box_bc(n, 100.0)
        m = fe.Mesh(n)
        assert np.array_equal(mask.astype(bool), m.clamp_mask())
        np.testing.assert_allclose(f, m.traction_x1(100.0), rtol=1e-15, atol=0)


# ----------------------------------------------------------------------------
# The paper's example (Section 3): nonlinear law, PCA metric, torsion
# ----------------------------------------------------------------------------
def test_nonlinear_law_closed_forms():
    """Uniaxial strain and simple shear of the reference law, by hand."""
    E, a = ddsynth.PAPER_E, ddsynth.PAPER_ALPHA
    x = 0.02
    s = ddsynth.nonlinear_stress(np.array([x, 0, 0, 0, 0, 0]))[0]
    k = x + a * x ** 3
    np.testing.assert_allclose(s, [1.5 * E * k, 0.5 * E * k, 0.5 * E * k, 0, 0, 0], rtol=1e-14,
                               atol=1e-12)
    g = 0.03                                 # engineering shear 12: tensor component g/2
    s = ddsynth.nonlinear_stress(np.array([0, 0, 0, 0, 0, g]))[0]
    np.testing.assert_allclose(s, [0, 0, 0, 0, 0, E * (g / 2 + a * (g / 2) ** 3)], rtol=1e-14,
                               atol=1e-12)
    e, s = ddsynth.data_points_nonlinear(1000, 3)
    assert np.abs(e).max() <= 0.025 and np.array_equal(ddsynth.nonlinear_stress(e), s)


def test_pca_metric_closed_forms(C0):
    """Linear noise-free data give back their stiffness; at vanishing amplitude
    the nonlinear law gives its tangent E (I + 1/2 11^T) (normal) and E/2
    (shear); the metric is invariant under reordering and scales with stress."""
    e, s = ddsynth.data_points(40000, 5, noise_std=0.0)
    np.testing.assert_allclose(oracle.pca_metric(e, s), C0, rtol=0, atol=1e-9 * C0.max())
    E = ddsynth.PAPER_E
    T = np.zeros((6, 6))
    T[:3, :3] = 0.5 * E
    T[:3, :3] += E * np.eye(3)
    T[3:, 3:] = 0.5 * E * np.eye(3)
    e, s = ddsynth.data_points_nonlinear(40000, 6, eps_amp=1e-6)
    np.testing.assert_allclose(oracle.pca_metric(e, s), T, rtol=0, atol=1e-6 * E)
    e, s = ddsynth.data_points_nonlinear(20000, 7)
    C = oracle.pca_metric(e, s)
    p = np.random.default_rng(0).permutation(20000)
    tol = 1e-12 * np.abs(C).max()
    np.testing.assert_allclose(oracle.pca_metric(e[p], s[p]), C, rtol=0, atol=tol)
    np.testing.assert_allclose(oracle.pca_metric(e, 3.0 * s), 3.0 * C, rtol=0, atol=3 * tol)
    assert np.allclose(C, C.T) and np.linalg.eigvalsh(C).min() > 0


def test_torsion_boundary_conditions():
    m = fe.Mesh(4, size=10.0)
    mask, val = m.torsion(2.0)
    top = np.where(np.isclose(m.coords[:, 2], 10.0))[0]
    bot = np.where(np.isclose(m.coords[:, 2], 0.0))[0]
    assert mask.sum() == 3 * (len(top) + len(bot))
    th = np.deg2rad(2.0)
    corner = top[np.argmax(m.coords[top, 0] + m.coords[top, 1])]   # (10, 10, 10)
    want = np.array([5 * np.cos(th) - 5 * np.sin(th) - 5, 5 * np.sin(th) + 5 * np.cos(th) - 5, 0])
    np.testing.assert_allclose(val[3 * corner:3 * corner + 3], want, rtol=1e-14, atol=1e-15)
    assert np.all(val[3 * bot[0]:3 * bot[0] + 3] == 0)
    gm, gv, gf = ddsynth.torsion_bc(4, 10.0, 2.0)
    assert np.array_equal(gm.astype(bool), mask) and np.allclose(gv, val, rtol=0, atol=1e-14)
    assert not gf.any()


def test_pc_with_prescribed_affine_displacement(C0):
    """Patch test with prescribed displacements: u = G x on every boundary node
    and data planted at the uniform strain of G; P_C returns u = G x at every
    node (interior included) and that strain at every material point."""
    m = fe.Mesh(3, size=2.0)
    G = np.array([[1e-3, 2e-4, -1e-4], [3e-4, -5e-4, 2e-4], [-2e-4, 1e-4, 7e-4]])
    exact = (m.coords @ G.T).ravel()
    bnd = np.any(np.isclose(m.coords, 0.0) | np.isclose(m.coords, 2.0), axis=1)
    mask = np.repeat(bnd, 3)
    eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[1, 2] + G[2, 1], G[0, 2] + G[2, 0],
                    G[0, 1] + G[1, 0]])
    es, ss = np.tile(eps, (m.n_mp, 1)), np.tile(C0 @ eps, (m.n_mp, 1))
    f = np.zeros(m.n_dof)
    pc = fe.ConstraintProjector(m, C0, mask, f, exact)
    u, eta, e_out, s_out = pc(es, ss)
    np.testing.assert_allclose(u, exact, rtol=0, atol=1e-15)
    np.testing.assert_allclose(e_out, es, rtol=0, atol=1e-15)
    np.testing.assert_allclose(s_out, ss, rtol=0, atol=1e-9)


def test_dd_torsion_descends():
    """The DD loop on the paper's problem (nonlinear data, PCA metric, torsion)
    decreases the global distance monotonically and converges."""
    m = fe.Mesh(2, size=10.0)
    mask, val = m.torsion(2.0)
    e, s = ddsynth.data_points_nonlinear(3000, 12)
    C = oracle.pca_metric(e, s)
    r = fe.dd_solve(e, s, C, m, mask, np.zeros(m.n_dof), ddsynth.indices(m.n_mp, 3000, 13),
                    u_dirichlet=val)
    assert r.converged
    tol = 1e-12 * r.d_half[0]
    for i in range(r.iterations):
        assert r.d_full[i] <= r.d_half[i] + tol
        if i:
            assert r.d_half[i] <= r.d_full[i - 1] + tol
    top = np.where(np.isclose(m.coords[:, 2], 10.0))[0]
    np.testing.assert_allclose(r.u[3 * top], val[3 * top], rtol=0, atol=1e-15)
