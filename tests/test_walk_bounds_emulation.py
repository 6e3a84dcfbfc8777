"""CPU emulation of the tree walk's certified leaf distances and box bounds.

A compact leaf stores, in principal-axis coordinates y = V^T x (V orthonormal,
so distances are those of the whitened space), its FP32 centre c, its radius r
(max |y - c| rounded up) with 1/r in FP32, and per point the FP16 offset
(y - c) / r.  The walk forms, in FP32, q'' = (y_q - c) / r and
s~ = r sqrt(sum (q'' - x'')^2), and certifies |s~ - |q - x|| <= E with
E = 2^-20 |q| + 2^-20 (2 s~ + 2 r) + 1.001 (2^-11 + 2^-22) r.  A box (FP32,
rounded outward) bounds its points from below by
sqrt(sum gap^2) (1 - 2^-19) - 2^-22 (|q| + max |x|).  This test rebuilds both
from FP64 data, evaluates them as the walk does (FP32 operations, FP16
offsets), and checks the inequalities against the FP64 distances for ordinary,
far and coincident queries, with E shrunk by 1e-6 so that its own rounding
cannot decide the outcome.
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


def leaf_distances(yq, c, rf, invf, h):
    """s~ of every (query, leaf point) pair, in FP32 as the walk computes it."""
    qs = ((yq[:, None, :] - c[None, :, :]).astype(np.float32) * invf[None, :, None]).astype(np.float32)
    x = h.astype(np.float32)                                   # [leaf][64][12]
    t = (qs[:, :, None, :] - x[None]).astype(np.float32)
    d = np.zeros(t.shape[:-1], np.float32)
    for k in range(12):
        d = (d + (t[..., k] * t[..., k]).astype(np.float32)).astype(np.float32)
    return (rf[None, :, None] * np.sqrt(d)).astype(np.float32)


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
    st = leaf_distances(yq, c, rf, invf, h)                   # [query][leaf][64]
    true = np.sqrt(((q[:, None, :] - w[None, :, :]) ** 2).sum(2)).reshape(st.shape)
    E = (EPS20 * qnorm[:, None, None] + EPS20 * (np.float32(2.0) * st + np.float32(2.0) * rf[None, :, None])
         + LEAF_REL * rf[None, :, None]).astype(np.float64) * (1.0 - 1e-6)
    err = np.abs(st.astype(np.float64) - true)
    assert np.all(err <= E), float((err - E).max())
    # the bound is not loose by orders of magnitude: errors use a visible part of it
    assert (err / E).max() > 0.05


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
    g = np.maximum(np.maximum(lo[None] - yq[:, None], yq[:, None] - hi[None]), np.float32(0))
    ss = np.zeros(g.shape[:2], np.float32)
    for k in range(12):
        ss = (ss + (g[..., k] * g[..., k]).astype(np.float32)).astype(np.float32)
    lb = (np.sqrt(ss) * LB_SHRINK - slack[:, None]).astype(np.float64)
    true = np.sqrt(((q[:, None, :] - w[None, :, :]) ** 2).sum(2)).reshape(len(q), -1, 64).min(2)
    assert np.all(lb <= true), float((lb - true).max())
    assert np.mean(lb > 0) > 0.5          # the bound prunes: most boxes are bounded away from 0
