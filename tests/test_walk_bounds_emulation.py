"""CPU emulation of the tree walk's certified leaf distances and box bounds.

A compact leaf stores, in principal-axis coordinates y = V^T x (V orthonormal,
so distances are those of the whitened space), its FP32 centre c, its radius r
(max |y - c| rounded up) with 1/r in FP32, and per point the FP16 offset
(y - c) / r.  The walk forms, in FP32, q'' = (y_q - c) / r and
s~ = r sqrt(sum (q'' - x'')^2), and certifies |s~ - |q - x|| <= E with
E = 2^-20 |q| + 2^-20 (2 s~ + 2 r) + 1.001 (2^-11 + 2^-22) r.  A box (FP32,
rounded outward) bounds its points from below by
sqrt(sum gap^2) (1 - 2^-19) - 2^-22 (|q| + max |x|); a leaf box stored as
bytes inside its parent box is decoded outward by 2^-20 (|lo| + |hi|) of the
parent first.  This test rebuilds all three from FP64 data, evaluates them as
the walk does (FP32 operations, with and without fused multiply-adds, FP16
offsets, and a square root that may be one unit in the last place off either
way, as v_sqrt_f32 is), and checks the inequalities against the FP64
distances for ordinary, far and coincident queries, with E shrunk by 1e-6 so
that its own rounding cannot decide the outcome.
"""
import numpy as np

import ddsynth
import oracle

EPS20 = np.float32(2.0 ** -20)
EPS22 = np.float32(2.0 ** -22)
LEAF_REL = np.float32((2.0 ** -11 + 2.0 ** -22) * 1.001)
LB_SHRINK = np.float32(1.0 - 2.0 ** -19)


def principal_axes(w):
    X = w - w.mean(0)
    _, _, Vt = np.linalg.svd(X, full_matrices=False)
    return Vt.T                      # columns: axes (orthonormal, FP64)


def pack_leaves(y):
    """Leaves of 64 consecutive rows: FP32 centre, radius (rounded up), 1/r, FP16 offsets."""
    L = y.reshape(-1, 64, 12)
    c = (L.sum(1) / 64.0).astype(np.float32)
    r = np.sqrt(((L - c[:, None, :].astype(np.float64)) ** 2).sum(2)).max(1)
    rf = np.nextafter((r * (1.0 + 1e-12)).astype(np.float32), np.float32(np.inf))
    rf = np.maximum(rf, np.float32(2.0 ** -20))
    inv = 1.0 / rf.astype(np.float64)
    h = ((L - c[:, None, :].astype(np.float64)) * inv[:, None, None]).astype(np.float16)
    return c, rf, inv.astype(np.float32), h


def sqrt_ulp(x, ulp):
    """FP32 square root moved `ulp` units in the last place (the walk's
    v_sqrt_f32 is within one)."""
    r = np.sqrt(np.asarray(x, np.float32))
    if ulp > 0:
        r = np.nextafter(r, np.float32(np.inf))
    elif ulp < 0:
        r = np.maximum(np.nextafter(r, np.float32(0)), np.float32(0))
    return r.astype(np.float32)


def leaf_distances(yq, c, rf, invf, h, fused=False, ulp=0):
    """s~ of every (query, leaf point) pair, in FP32 as the walk computes it:
    unfused (q'' rounded, then q'' - x'', then each square) or fused (the scale
    and the FP16 offset in one fused multiply-add, the squares accumulated by
    fused multiply-adds)."""
    diff = (yq[:, None, :] - c[None, :, :]).astype(np.float32)          # [query][leaf][12]
    x = h.astype(np.float32)                                            # [leaf][64][12]
    if fused:
        t = (diff[:, :, None, :].astype(np.float64) * invf[None, :, None, None].astype(np.float64)
             - x[None].astype(np.float64)).astype(np.float32)
    else:
        qs = (diff * invf[None, :, None]).astype(np.float32)
        t = (qs[:, :, None, :] - x[None]).astype(np.float32)
    d = np.zeros(t.shape[:-1], np.float32)
    for k in range(12):
        tk = t[..., k].astype(np.float64)
        if fused:
            d = (d.astype(np.float64) + tk * tk).astype(np.float32)
        else:
            d = (d + (t[..., k] * t[..., k]).astype(np.float32)).astype(np.float32)
    return (rf[None, :, None] * sqrt_ulp(d, ulp)).astype(np.float32)


def test_leaf_distance_certificate(C0):
    e, s = ddsynth.data_points(4096, 4201)
    qe, qs, _ = ddsynth.queries(e, s, 64, 4202)
    w = oracle.whiten(e, s, C0)
    q = oracle.whiten(qe, qs, C0)
    q = np.concatenate([q, w[:8], 8.0 * q[:8]])             # coincident and far queries
    V = principal_axes(w)
    y = w @ V
    yq = (q @ V).astype(np.float32)
    qnorm = np.sqrt((q ** 2).sum(1)).astype(np.float32)
    c, rf, invf, h = pack_leaves(y)
    worst = 0.0
    for fused in (False, True):
        for ulp in (-1, 0, 1):
            st = leaf_distances(yq, c, rf, invf, h, fused, ulp)       # [query][leaf][64]
            true = np.sqrt(((q[:, None, :] - w[None, :, :]) ** 2).sum(2)).reshape(st.shape)
            E = (EPS20 * qnorm[:, None, None] + EPS20 * (np.float32(2.0) * st + np.float32(2.0) * rf[None, :, None])
                 + LEAF_REL * rf[None, :, None]).astype(np.float64) * (1.0 - 1e-6)
            err = np.abs(st.astype(np.float64) - true)
            assert np.all(err <= E), (fused, ulp, float((err - E).max()))
            worst = max(worst, float((err / E).max()))
    # the bound is not loose by orders of magnitude: errors use a visible part of it
    assert worst > 0.05


def test_box_lower_bound(C0):
    e, s = ddsynth.data_points(4096, 4203)
    qe, qs, _ = ddsynth.queries(e, s, 64, 4204)
    w = oracle.whiten(e, s, C0)
    q = oracle.whiten(qe, qs, C0)
    q = np.concatenate([q, w[:8], 8.0 * q[:8]])
    V = principal_axes(w)
    y = (w @ V).reshape(-1, 64, 12)
    lo = np.nextafter(y.min(1).astype(np.float32), np.float32(-np.inf))
    hi = np.nextafter(y.max(1).astype(np.float32), np.float32(np.inf))
    lo = np.where(lo.astype(np.float64) <= y.min(1), lo, np.nextafter(lo, np.float32(-np.inf)))
    hi = np.where(hi.astype(np.float64) >= y.max(1), hi, np.nextafter(hi, np.float32(np.inf)))
    yq = (q @ V).astype(np.float32)
    qnorm = np.sqrt((q ** 2).sum(1)).astype(np.float32)
    xmax = np.float32(np.sqrt((w ** 2).sum(1)).max())
    slack = (EPS22 * (qnorm + xmax) + np.float32(1e-30)).astype(np.float32)
    true = np.sqrt(((q[:, None, :] - w[None, :, :]) ** 2).sum(2)).reshape(len(q), -1, 64).min(2)
    lb = box_bound(lo[None], hi[None], yq[:, None], slack[:, None], ulp=1)
    assert np.all(lb <= true), float((lb - true).max())
    assert np.mean(lb > 0) > 0.5          # the bound prunes: most boxes are bounded away from 0


def box_bound(lo, hi, yq, slack, ulp):
    """sqrt(sum gap^2) (1 - 2^-19) - slack in FP32 (fused squares), the square
    root `ulp` units off."""
    g = np.maximum(np.maximum(lo - yq, yq - hi), np.float32(0)).astype(np.float32)
    ss = np.zeros(g.shape[:-1], np.float32)
    for k in range(12):
        gk = g[..., k].astype(np.float64)
        ss = (ss.astype(np.float64) + gk * gk).astype(np.float32)
    return (sqrt_ulp(ss, ulp) * LB_SHRINK - slack).astype(np.float32).astype(np.float64)


def test_box_bound_margins_cover_query_rounding():
    """Boxes with a data point on a corner and queries just outside one face:
    the true distance equals the gap to the box, and the query's FP32
    coordinates round it up about half the time.  The slack 2^-22 (|q| +
    max |x|) and the shrink 1 - 2^-19 keep the bound below the distance; without
    them it exceeds the distance for some of these pairs."""
    rng = np.random.default_rng(7)
    n = 4000
    hi = rng.uniform(40.0, 60.0, (n, 12)).astype(np.float32)
    lo = (hi - rng.uniform(0.1, 2.0, (n, 12))).astype(np.float32)
    gap = rng.uniform(1e-6, 1e-3, n)
    q64 = hi.astype(np.float64)
    q64[:, 0] += gap                                 # the nearest point: the corner hi
    true = gap
    yq = q64.astype(np.float32)
    qnorm = np.sqrt((q64 ** 2).sum(1)).astype(np.float32)
    xmax = np.float32(np.sqrt((hi.astype(np.float64) ** 2).sum(1)).max())
    slack = (EPS22 * (qnorm + xmax) + np.float32(1e-30)).astype(np.float32)
    lb = box_bound(lo, hi, yq, slack, ulp=1)
    assert np.all(lb <= true)
    bare = box_bound(lo, hi, yq, np.float32(0.0), ulp=1) / float(LB_SHRINK)
    assert np.any(bare > true)


def test_quantised_leaf_box_lower_bound(C0):
    """Leaf boxes stored as bytes inside their parent box (the FP32 box of 64
    leaves): quantised down / up in FP64 at creation, decoded in FP32 as
    lo = fma(ql, step, plo) - delta, hi = fma(qh, step, plo) + delta with
    step = (phi - plo) / 255 and delta = 2^-20 max(|plo| + |phi|); the decoded
    box must still hold every point of the leaf, and its bound stay below the
    distance to them.  The points sit on the FP32 grid, so that the boxes are
    tight, and data shifted far from the origin make the roundings largest."""
    e, s = ddsynth.data_points(64 * 64 * 4, 4205)
    qe, qs, _ = ddsynth.queries(e, s, 48, 4206)
    for shift in (0.0, 50.0):
        w = oracle.whiten(e, s, C0) + shift
        q = oracle.whiten(qe, qs, C0) + shift
        q = np.concatenate([q, w[::997][:8], 4.0 * (q[:8] - shift) + shift])
        V = principal_axes(w)
        y = (w @ V).astype(np.float32).astype(np.float64).reshape(-1, 64, 12)   # [leaf][64][12]
        lo, hi = y.min(1).astype(np.float32), y.max(1).astype(np.float32)         # exact
        dlo, dhi = decode_leaf_boxes(lo, hi, EPS20)
        assert np.all(dlo.astype(np.float64) <= y.min(1)) and np.all(dhi.astype(np.float64) >= y.max(1))
        yq64 = q @ V
        yq = yq64.astype(np.float32)
        qnorm = np.sqrt((q ** 2).sum(1)).astype(np.float32)
        xmax = np.float32(np.sqrt((w ** 2).sum(1)).max())
        slack = (EPS22 * (qnorm + xmax) + np.float32(1e-30)).astype(np.float32)
        lb = box_bound(dlo[None], dhi[None], yq[:, None], slack[:, None], ulp=1)
        true = np.sqrt(((yq64[:, None, None, :] - y[None]) ** 2).sum(3)).min(2)
        assert np.all(lb <= true), (shift, float((lb - true).max()))
        assert np.mean(lb > 0) > 0.3


def test_leaf_box_decoding_margin():
    """Leaf boxes whose edges fall on the quantisation levels of their parent
    (lo = plo + k (phi - plo) / 255 in FP32): decoded without the margin, some
    come out inside the stored box (the FP32 step is rounded up), so a point on
    their edge would be cut off; with delta = 2^-20 (|plo| + |phi|) every one
    contains its stored box."""
    parents = [(0.0, 1.0), (1.0, 3.0), (-2.5, 7.25), (50.0, 57.0), (10.0, 10.5), (-80.0, -79.0)]
    short = 0
    for plo, phi in parents:
        k = np.arange(0, 256)
        edge = (plo + (phi - plo) * k / 255.0).astype(np.float32)
        lo = np.repeat(edge[:, None], 12, 1)                    # 256 leaves, the same edge on each axis
        hi = np.repeat(np.concatenate([edge[1:], edge[-1:]])[:, None], 12, 1)
        lo[0], hi[-1] = np.float32(plo), np.float32(phi)        # the parent is exactly [plo, phi]
        lo, hi = lo.reshape(-1, 12), hi.reshape(-1, 12)
        # every leaf in one parent of 256 leaves: the decoding below groups by 64, so tile the parent
        for g in range(4):
            sl = slice(64 * g, 64 * g + 64)
            l, h = lo[sl].copy(), hi[sl].copy()
            l[0], h[-1] = np.float32(plo), np.float32(phi)
            dlo, dhi = decode_leaf_boxes(l, h, EPS20)
            assert np.all(dlo <= l) and np.all(dhi >= h), (plo, phi, g)
            nlo, nhi = decode_leaf_boxes(l, h, np.float32(0.0))
            short += int(np.sum(nlo > l) + np.sum(nhi < h))
    assert short > 0


def decode_leaf_boxes(lo, hi, eps):
    """Quantise FP32 leaf boxes inside their parents (64 leaves each) as the
    dataset build does, then decode them as the walk does with margin
    eps (|plo| + |phi|)."""
    n_leaf = lo.shape[0]
    plo = lo.reshape(-1, 64, 12).min(1)
    phi = hi.reshape(-1, 64, 12).max(1)
    par = np.arange(n_leaf) // 64
    P_lo, P_hi = plo[par].astype(np.float64), phi[par].astype(np.float64)
    ext = P_hi - P_lo
    with np.errstate(divide="ignore", invalid="ignore"):
        ql = np.where(ext > 0, np.floor((lo - P_lo) / ext * 255.0), 0.0)
        qh = np.where(ext > 0, np.ceil((hi - P_lo) / ext * 255.0), 255.0)
    ql, qh = np.clip(ql, 0, 255), np.clip(qh, 0, 255)
    plo32, phi32 = plo[par], phi[par]
    step = ((phi32 - plo32).astype(np.float32) * np.float32(1.0 / 255.0)).astype(np.float32)
    amax = (np.abs(plo32) + np.abs(phi32)).astype(np.float32).max(1)
    delta = (eps * amax + np.float32(1e-30)).astype(np.float32)[:, None]
    dlo = ((ql * step.astype(np.float64) + plo32.astype(np.float64)).astype(np.float32) - delta).astype(np.float32)
    dhi = ((qh * step.astype(np.float64) + plo32.astype(np.float64)).astype(np.float32) + delta).astype(np.float32)
    return dlo, dhi


def f32_ru(x):
    """FP64 -> FP32 rounded up."""
    f = np.asarray(x, np.float64).astype(np.float32)
    return np.where(f.astype(np.float64) < x, np.nextafter(f, np.float32(np.inf)), f).astype(np.float32)


def ball_bound(qf, c, r, slack, ulp=1):
    """The k-means walk's ball bound sqrt(sum (q - c)^2) (1 - 2^-19) - slack - r
    in FP32 (f_d = 1), the square root `ulp` units off."""
    t = (qf[:, None, :] - c[None]).astype(np.float32)
    ss = np.zeros(t.shape[:-1], np.float32)
    for k in range(12):
        tk = t[..., k].astype(np.float64)
        ss = (ss.astype(np.float64) + tk * tk).astype(np.float32)
    dc = (sqrt_ulp(ss, ulp) * LB_SHRINK - slack[:, None]).astype(np.float32)
    return (dc - r[None]).astype(np.float32).astype(np.float64)


def test_kmeans_ball_lower_bound(C0):
    """A k-means child record bounds its points by the ball (FP32 centre c,
    radius r = max |x - c| rounded up): |q - c| (1 - 2^-19) - 2^-22 (|q| +
    max |x|) - r, evaluated in FP32 from the query's FP32 whitened
    coordinates, stays below the distance to every point of the record, on
    ordinary data shifted far from the origin and on points placed on the
    sphere with queries just outside it along the same ray (where the true
    distance equals the gap); without the slack and the shrink the bound exceeds
    the distance for some of those."""
    e, s = ddsynth.data_points(64 * 64, 4207)
    qe, qs, _ = ddsynth.queries(e, s, 64, 4208)
    for shift in (0.0, 40.0):
        w = oracle.whiten(e, s, C0) + shift
        q = oracle.whiten(qe, qs, C0) + shift
        q = np.concatenate([q, w[::331][:8]])
        grp = w.reshape(-1, 64, 12)
        c = grp.mean(1).astype(np.float32)
        r = f32_ru(np.sqrt(((grp - c[:, None, :].astype(np.float64)) ** 2).sum(2)).max(1) * (1.0 + 1e-12))
        qnorm = np.sqrt((q ** 2).sum(1)).astype(np.float32)
        xmax = np.float32(np.sqrt((w ** 2).sum(1)).max())
        slack = (EPS22 * (qnorm + xmax) + np.float32(1e-30)).astype(np.float32)
        lb = ball_bound(q.astype(np.float32), c, r, slack)
        true = np.sqrt(((q[:, None, None, :] - grp[None]) ** 2).sum(3)).min(2)
        assert np.all(lb <= true), (shift, float((lb - true).max()))
    # points on a sphere, queries just outside along their rays
    rng = np.random.default_rng(8)
    n = 2000
    c = rng.uniform(30.0, 50.0, (n, 12)).astype(np.float32)
    u = rng.normal(size=(n, 12))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = rng.uniform(0.5, 3.0, n)
    gap = rng.uniform(1e-6, 1e-3, n)
    p = c.astype(np.float64) + rad[:, None] * u                   # the record's point on the ray
    q64 = c.astype(np.float64) + (rad + gap)[:, None] * u
    r = f32_ru(rad * (1.0 + 1e-12))
    qnorm = np.sqrt((q64 ** 2).sum(1)).astype(np.float32)
    xmax = np.float32(np.sqrt((p ** 2).sum(1)).max())
    slack = (EPS22 * (qnorm + xmax) + np.float32(1e-30)).astype(np.float32)
    qf = q64.astype(np.float32)
    true = np.sqrt(((q64 - p) ** 2).sum(1))
    lb = np.diagonal(ball_bound(qf, c, r, slack))
    assert np.all(lb <= true)
    bare = np.diagonal(ball_bound(qf, c, r, np.zeros(n, np.float32))) / float(LB_SHRINK)
    assert np.any(bare > true)
