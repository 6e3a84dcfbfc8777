"""CPU emulation of the FP32 MFMA scan's certified band (DD_MIXED_FP32).

The FP32 scan stores the whitened data as x^ = fl32(x) with the norms
n^ = fl32(|x^|^2), takes the query column -2 q^ with q^ = fl32(q), starts the
matrix-core accumulation at n^ and adds the twelve products q^_k x^_k times -2
in an order the hardware does not document, then adds o = fl32(|q^|^2):
d~ = (n^ - 2 q^.x^) + o approximates d = |q - x|^2.  It keeps point j while
d~_j - a <= U, U = min_i (d~_i + a), with the band

    a = 2^-18 (Q + X)^2,   Q = fl32(|q|), X >= max |x|,

evaluated in FP32.  This test rebuilds those operands, accumulates in several
orders (one FP32 rounding per addition, with exact and with rounded products:
fused and unfused hardware), and checks |d~ - d| <= a (a shrunk by 1e-6) on
ordinary queries, queries on data points, far queries and data shifted far from
the origin (where the cancellation in n^ - 2 q^.x^ + o is largest), then that
the kernel's FP32 comparisons keep the exact nearest point of every query.  The
observed error reaches about 1.4 u (Q + X)^2 (u = 2^-24) against the 64 u of the
band and the 22 u of the worst-case analysis; a band of one unit roundoff fails
on the same pairs, so the check has teeth.
"""
import numpy as np
import pytest

import ddsynth
import oracle

BAND = np.float32(2.0 ** -18)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def operands(w, q):
    xh = f32(w)
    nh = f32((xh.astype(np.float64) ** 2).sum(1))
    qh = f32(q)
    b = (np.float32(-2.0) * qh).astype(np.float32)      # exact scaling
    o = f32((qh.astype(np.float64) ** 2).sum(1))
    return xh, nh, b, o


def accumulate(xh, nh, b, order, fused):
    """FP32 accumulation of n^ and the twelve products in the given order."""
    prod = xh[None, :, :].astype(np.float64) * b[:, None, :].astype(np.float64)   # exact
    if not fused:
        prod = prod.astype(np.float32).astype(np.float64)
    acc = np.broadcast_to(nh[None, :], prod.shape[:2]).astype(np.float32)
    if order == "pairwise":
        t = prod.astype(np.float32) if not fused else prod
        # products summed pairwise (exact products rounded once per level), then the norm
        while t.shape[-1] > 1:
            if t.shape[-1] % 2:
                t = np.concatenate([t, np.zeros(t.shape[:-1] + (1,), t.dtype)], axis=-1)
            t = f32(t[..., 0::2].astype(np.float64) + t[..., 1::2].astype(np.float64))
        return f32(acc.astype(np.float64) + t[..., 0].astype(np.float64))
    for k in order:
        acc = f32(acc.astype(np.float64) + prod[..., k])
    return acc


def orders(seed):
    rng = np.random.default_rng(seed)
    yield list(range(12))
    yield list(range(11, -1, -1))
    yield "pairwise"
    for _ in range(3):
        yield list(rng.permutation(12))


def band(q, xmax):
    qa = (f32(np.sqrt((np.asarray(q, np.float64) ** 2).sum(1))) + np.float32(xmax)).astype(np.float32)
    return ((BAND * qa) * qa + np.float32(1e-30)).astype(np.float32)


def workload(C0, shift):
    e, s = ddsynth.data_points(1024, 5101)
    qe, qs, _ = ddsynth.queries(e, s, 64, 5102)
    w = oracle.whiten(e, s, C0) + shift
    q = oracle.whiten(qe, qs, C0) + shift
    q = np.concatenate([q, w[:16], 6.0 * q[:8], np.tile(w.mean(0), (2, 1))])
    return w, q


@pytest.mark.parametrize("shift", [0.0, 40.0])
@pytest.mark.parametrize("fused", [True, False])
def test_fp32_band_contains_distance(C0, shift, fused):
    w, q = workload(C0, shift)
    xh, nh, b, o = operands(w, q)
    xmax = float(np.sqrt((w ** 2).sum(1)).max()) * (1.0 + 1e-6)
    a = band(q, xmax).astype(np.float64) * (1.0 - 1e-6)
    d = ((q[:, None, :] - w[None, :, :]) ** 2).sum(2)
    worst = 0.0
    for order in orders(7 + int(shift) + fused):
        dt = f32(accumulate(xh, nh, b, order, fused).astype(np.float64) + o[:, None].astype(np.float64))
        err = np.abs(dt.astype(np.float64) - d)
        assert (err <= a[:, None]).all(), (order, float((err / a[:, None]).max()))
        worst = max(worst, float((err / a[:, None]).max()))
    # the check is not vacuous: at the shifted data the error exceeds one unit roundoff of (Q + X)^2
    if shift > 0:
        assert worst > 1.0 / 64.0, worst


def test_fp32_band_of_one_roundoff_fails(C0):
    """Plant a mistake in the band (2^-24 instead of 2^-18): some pair of the
    shifted workload escapes it."""
    w, q = workload(C0, 40.0)
    xh, nh, b, o = operands(w, q)
    xmax = float(np.sqrt((w ** 2).sum(1)).max()) * (1.0 + 1e-6)
    a = band(q, xmax).astype(np.float64) / 64.0
    d = ((q[:, None, :] - w[None, :, :]) ** 2).sum(2)
    escaped = False
    for order in orders(3):
        for fused in (True, False):
            dt = f32(accumulate(xh, nh, b, order, fused).astype(np.float64) + o[:, None].astype(np.float64))
            escaped |= bool((np.abs(dt.astype(np.float64) - d) > a[:, None]).any())
    assert escaped


@pytest.mark.parametrize("shift", [0.0, 40.0])
def test_fp32_candidates_keep_the_exact_nearest_point(C0, shift):
    """The kernel's FP32 tests (U = min fl32(d~ + a), keep fl32(d~ - a) <= U)
    keep the FP64 nearest point (lowest index on ties) of every query."""
    w, q = workload(C0, shift)
    xh, nh, b, o = operands(w, q)
    xmax = float(np.sqrt((w ** 2).sum(1)).max()) * (1.0 + 1e-6)
    a = band(q, xmax)
    d = ((q[:, None, :] - w[None, :, :]) ** 2).sum(2)
    best = np.argmin(d, axis=1)
    for order in orders(11):
        dt = f32(accumulate(xh, nh, b, order, True).astype(np.float64) + o[:, None].astype(np.float64))
        U = (dt + a[:, None]).astype(np.float32).min(1)
        keep = (dt - a[:, None]).astype(np.float32) <= U[:, None]
        assert keep[np.arange(len(q)), best].all()
        assert keep.sum(1).max() < len(w)      # the band prunes
