"""CPU emulation of the 16-bit scans' certified distance bounds.

The BF16 / FP16 MFMA scans score a data point x of tile T against a query q as
d~ = (|x'|^2 - 2 q'.x') + |q'|^2 with x' = round16(x - c_T) and
q' = round16(fl32(q) - c_T), the sum taken in FP32 in an order the hardware
does not document, and certify, in square-root space,

    sqrt(max(d~ - alpha, 0)) (1 - 2^-20) - eta  <=  |q - x|  <=  (sqrt(d~ + alpha) + eta) (1 + 2^-20)

with eta = (u (1.0043 |q'| + r_T) + 1.8e-7 (|q| + |q'|) + 8 a) (1 + 2^-20) and
alpha = 2^-18 (|q'| + r_T)^2 + 16 a (u: unit roundoff of the 16-bit format,
a: its subnormal half-step).  Every point that the lower bound does not exclude
stays a candidate, so the exact nearest point survives whenever these
inequalities hold.  This test rebuilds the pack and the query operands as the
scan does (round-to-nearest-even conversions, the norm split in three 16-bit
terms), accumulates the 16 products in several orders, and checks both
inequalities against the FP64 distance on ordinary, far and coincident queries,
with the margins eta and alpha shrunk by a factor 1 - 1e-6 so that rounding in
their own evaluation cannot decide the outcome.
"""
import numpy as np
import pytest

import ddsynth
import oracle

REL_UP = np.float32(1.0 + 2.0 ** -20)
REL_DN = np.float32(1.0 - 2.0 ** -20)
FORMATS = {
    # name: (unit roundoff of double -> float -> 16-bit, subnormal half-step)
    "bf16": (np.float32(0.00390625 * (1.0 + 3.0517578125e-05)), np.float32(0.0)),
    "fp16": (np.float32(0.00048828125 + 5.9604645e-08), np.float32(2.9802322e-08)),
}


def round16(x, fmt):
    """Round FP32 values to the 16-bit format (nearest even), returned as FP32."""
    x = np.asarray(x, np.float32)
    if fmt == "fp16":
        return x.astype(np.float16).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def tile_pack(w, fmt, n_real=None):
    """Centre, radius and A operand rows (-2x', n_hi, n_mid, n_lo, 0) of one tile;
    with n_real, rows from n_real on are padding (copies of the last real row)
    and the centre and radius cover the real rows only."""
    n_real = len(w) if n_real is None else n_real
    w = np.concatenate([w[:n_real], np.repeat(w[n_real - 1:n_real], len(w) - n_real, 0)])
    c = (w[:n_real].sum(0) / n_real).astype(np.float32)
    r = np.sqrt(((w[:n_real] - c.astype(np.float64)) ** 2).sum(1)).max()
    r = np.nextafter(np.float32(r * (1.0 + 1e-12) + 1e-30), np.float32(np.inf))
    xf = (w - c.astype(np.float64)).astype(np.float32)
    v = round16(xf, fmt)
    nn = (v.astype(np.float64) ** 2).sum(1)
    hi = round16(nn.astype(np.float32), fmt)
    r1 = nn - hi.astype(np.float64)
    mid = round16(r1.astype(np.float32), fmt)
    r2 = r1 - mid.astype(np.float64)
    lo = round16(r2.astype(np.float32), fmt)
    A = np.concatenate([round16(np.float32(-2.0) * v, fmt), hi[:, None], mid[:, None], lo[:, None],
                        np.zeros((len(w), 1), np.float32)], axis=1)
    return c, np.float32(r), A


def sum_fp32(terms, order):
    """FP32 sum of terms[..., k] in the given order of k (one rounding per addition)."""
    acc = np.zeros(terms.shape[:-1], np.float32)
    for k in order:
        acc = (acc + terms[..., k]).astype(np.float32)
    return acc


def pairwise_fp32(terms):
    t = terms
    while t.shape[-1] > 1:
        t = (t[..., 0::2] + t[..., 1::2]).astype(np.float32)
    return t[..., 0]


def bounds(qw, tile_w, fmt, order, n_real=None):
    """(lower, upper) sqrt-space bounds of every (query, point) pair of one tile."""
    unit, absf = FORMATS[fmt]
    c, rad, A = tile_pack(tile_w, fmt, n_real)
    qf = qw.astype(np.float32)
    qp = round16((qf - c).astype(np.float32), fmt)
    B = np.concatenate([qp, np.ones((len(qw), 3), np.float32), np.zeros((len(qw), 1), np.float32)],
                       axis=1)
    prod = (B[:, None, :] * A[None, :, :]).astype(np.float32)   # exact: 16-bit x 16-bit
    score = pairwise_fp32(prod) if order == "pairwise" else sum_fp32(prod, order)
    o = sum_fp32((qp * qp).astype(np.float32), range(12))
    d = (score + o[:, None]).astype(np.float32)
    so = np.sqrt(o).astype(np.float32)
    qabs = np.sqrt((qw.astype(np.float64) ** 2).sum(1)).astype(np.float32)
    eta = ((unit * (np.float32(1.0043) * so + rad) + np.float32(1.8e-7) * (qabs + so)
            + np.float32(8.0) * absf) * REL_UP).astype(np.float32)
    sr = (so + rad).astype(np.float32)
    alpha = (np.float32(3.814697265625e-06) * sr * sr + np.float32(16.0) * absf
             + np.float32(1e-30)).astype(np.float32)
    shrink = np.float32(1.0 - 1e-6)
    eta, alpha = eta * shrink, alpha * shrink
    lo = np.sqrt(np.maximum(d - alpha[:, None], 0)) * REL_DN - eta[:, None]
    hi = (np.sqrt(d + alpha[:, None]) + eta[:, None]) * REL_UP
    return lo.astype(np.float64), hi.astype(np.float64)


def orders(seed):
    rng = np.random.default_rng(seed)
    yield list(range(16))
    yield list(range(15, -1, -1))
    yield "pairwise"
    for _ in range(3):
        yield list(rng.permutation(16))


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_sqrt_space_bounds_hold(fmt, C0):
    e, s = ddsynth.data_points(2048, 4101)
    qe, qs, base = ddsynth.queries(e, s, 96, 4102)
    w = oracle.whiten(e, s, C0)
    q = oracle.whiten(qe, qs, C0)
    # adversarial queries: data points themselves, far from the data, at a tile centre
    q = np.concatenate([q, w[:16], 6.0 * q[:16], np.tile(w[:1024].mean(0), (4, 1))])
    tile = 1024
    for t0 in range(0, len(w), tile):
        tw = w[t0:t0 + tile]
        true = np.sqrt(((q[:, None, :] - tw[None, :, :]) ** 2).sum(2))
        for order in orders(t0 + (fmt == "fp16")):
            lo, hi = bounds(q, tw, fmt, order)
            assert np.all(lo <= true), (fmt, t0, order, float((lo - true).max()))
            assert np.all(true <= hi), (fmt, t0, order, float((true - hi).max()))


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_candidates_keep_the_exact_nearest_point(fmt, C0):
    """U = min over the scanned points of the upper bound; every point whose
    lower bound is <= U stays a candidate; the exact minimiser (lowest index on
    ties) is always among them, and the candidate lists stay short."""
    e, s = ddsynth.data_points(4096, 4103)
    qe, qs, _ = ddsynth.queries(e, s, 128, 4104)
    w = oracle.whiten(e, s, C0)
    q = oracle.whiten(qe, qs, C0)
    oi, _, _ = oracle.pd_raw(e, s, C0, qe, qs)
    tile = 1024
    lo_all, hi_all = [], []
    for t0 in range(0, len(w), tile):
        lo, hi = bounds(q, w[t0:t0 + tile], fmt, "pairwise")
        lo_all.append(lo)
        hi_all.append(hi)
    lo_all, hi_all = np.concatenate(lo_all, 1), np.concatenate(hi_all, 1)
    U = hi_all.min(1)
    cand = lo_all <= U[:, None]
    assert np.all(cand[np.arange(len(q)), oi])
    assert np.median(cand.sum(1)) <= 8


def scale16(w, tile):
    """The 16-bit scans' power-of-two scale: the largest tile radius into [1, 2)."""
    rmax = 0.0
    for t0 in range(0, len(w), tile):
        tw = w[t0:t0 + tile]
        c = (tw.sum(0) / len(tw)).astype(np.float32).astype(np.float64)
        rmax = max(rmax, float(np.sqrt(((tw - c) ** 2).sum(1)).max()))
    return 2.0 ** -np.floor(np.log2(rmax))


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_si_units_scaled_pack_and_padded_tail(fmt, C0):
    """Stresses and metric in Pa: whitened offsets inside a tile reach squared
    norms beyond the FP16 range (65504), so the packs are built from the data
    multiplied by the power of two that brings the largest tile radius into
    [1, 2) (exact, so the bounds hold in scaled units).  The last tile is padded
    with copies of the last point: the scores of the padding rows are distances
    to a real point, so U stays an upper bound of the true minimum, and the
    exact nearest point (lowest index on ties) is always a candidate."""
    n, tile = 2048 + 300, 1024
    e, s = ddsynth.data_points(n, 4105)
    s = s * 1e6
    C = C0 * 1e6
    qe, qs, _ = ddsynth.queries(e, s / 1e6, 96, 4106)
    qs = qs * 1e6
    qe = np.concatenate([qe, e[-3:]])
    qs = np.concatenate([qs, s[-3:]])
    w = oracle.whiten(e, s, C)
    q = oracle.whiten(qe, qs, C)
    oi, _, _ = oracle.pd_raw(e, s, C, qe, qs)
    # unscaled, the FP16 norm slot of this data would overflow
    c0 = (w[:tile].sum(0) / tile).astype(np.float32).astype(np.float64)
    assert ((w[:tile] - c0) ** 2).sum(1).max() > 65504.0
    sc = scale16(w, tile)
    ws, qsc = w * sc, q * sc
    lo_all, hi_all = [], []
    for t0 in range(0, n, tile):
        real = min(tile, n - t0)
        tw = np.concatenate([ws[t0:t0 + real], np.zeros((tile - real, 12))])
        for order in ("pairwise", list(range(16))):
            lo, hi = bounds(qsc, tw, fmt, order, n_real=real)
            padded = np.concatenate([ws[t0:t0 + real], np.repeat(ws[t0 + real - 1:t0 + real],
                                                                  tile - real, 0)])
            true = np.sqrt(((qsc[:, None, :] - padded[None, :, :]) ** 2).sum(2))
            assert np.all(lo <= true) and np.all(true <= hi), (fmt, t0, order)
        lo_all.append(lo[:, :real])
        hi_all.append(hi)              # padding rows take part in U (distances to a real point)
    U = np.concatenate(hi_all, 1).min(1)
    cand = np.concatenate(lo_all, 1) <= U[:, None]
    assert np.all(cand[np.arange(len(q)), oi])
    assert np.array_equal(oi[-3:], np.arange(n - 3, n))


def test_extraction_screen_passes_every_kept_score():
    """The extraction of the 16-bit scans screens a score s in score space,
    s <= T with a = (U + eta)(1 + 2^-18), T = (a^2 + alpha - o)
    + 2^-18 (a^2 + alpha + |o|), before it evaluates the FP32 lower bound
    lb = sqrt(max(s + o - alpha, 0)) (1 - 2^-20) - eta and keeps s if lb <= U.
    Every score the lower-bound test keeps must pass the screen: checked in
    FP32 on scores drawn around the boundary for near, far and coincident
    queries, with the square root perturbed by one ulp either way (the GPU's
    is correct to 1 ulp)."""
    rng = np.random.default_rng(4107)
    f = np.float32
    n = 200000
    for o_scale in (1e-6, 1e-2, 1.0, 1e3):
        o = (rng.random(n) * o_scale).astype(f)
        U = (rng.random(n) * np.sqrt(o_scale) * 2).astype(f)
        eta = (U * rng.random(n) * 1e-2).astype(f)
        alpha = (rng.random(n) * 1e-5 * o_scale).astype(f)
        # scores around the boundary sqrt(s + o - alpha) ~ U + eta
        edge = ((U.astype(np.float64) + eta) ** 2 + alpha - o).astype(f)
        s = (edge * (1 + (rng.random(n) - 0.5) * 1e-5)
             + (rng.random(n) - 0.5) * 1e-6 * np.abs(o)).astype(f)
        a = ((U + eta) * f(1.0 + 2.0 ** -18)).astype(f)
        sa = (a * a + alpha).astype(f)
        T = ((sa - o) + f(2.0 ** -18) * (sa + np.abs(o)) + f(1e-30)).astype(f)
        x = np.maximum((s + o).astype(f) - alpha, f(0)).astype(f)
        r = np.sqrt(x).astype(f)
        for ulp in (-1, 0, 1):
            rr = r if ulp == 0 else np.nextafter(r, f(np.inf) if ulp > 0 else f(0))
            lb = ((rr * f(1.0 - 2.0 ** -20)).astype(f) - eta).astype(f)
            kept = lb <= U
            assert kept.any() and (~kept).any()
            assert np.all(s[kept] <= T[kept]), o_scale
