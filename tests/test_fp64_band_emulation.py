"""CPU emulation of the FP64 MFMA scan's certified band (DD_EXACT_FP64).

The FP64 scan stores the whitened rows x with their norms n = |x|^2 (an FP64
fused multiply-add chain), takes the query column -2 q, starts each
16 x 16 x 4 matrix-core accumulation at n and adds the twelve products in three
steps of four, in an order (and with a fusion) the hardware does not document,
then adds |q|^2: d~ = (n - 2 q.x) + |q|^2 approximates d = |q - x|^2.  It keeps
point j while d~_j - a <= U, U = min_i (d~_i + a), with the band

    a = 2^-48 (Q + X)^2,   Q = |q|, X >= max |x|.

This test evaluates d~ in exact rational arithmetic rounded to FP64 after every
operation (one rounding per addition, with the products either exact, as in a
fused step, or rounded first), in several orders, and checks |d~ - d| <= a
against the exact d on ordinary queries, queries on data points and data
shifted far from the origin (where the cancellation is largest).  A band of one
unit roundoff (2^-53) fails on the shifted pairs, so the check has teeth.
"""
from fractions import Fraction

import numpy as np
import pytest

import ddsynth
import oracle


def rnd(x):
    """Round a rational to the nearest FP64 value (ties to even)."""
    return Fraction(float(x))


def fma_chain(v):
    s = Fraction(0)
    for t in v:
        s = rnd(s + t * t)
    return s


def accumulate(x, b, n, order, fused):
    acc = n
    for k in order:
        p = x[k] * b[k]
        acc = rnd(acc + (p if fused else rnd(p)))
    return acc


def orders(seed):
    rng = np.random.default_rng(seed)
    yield list(range(12))
    yield list(range(11, -1, -1))
    yield [0, 4, 8, 1, 5, 9, 2, 6, 10, 3, 7, 11]   # the three k-steps of four, interleaved
    for _ in range(2):
        yield [int(k) for k in rng.permutation(12)]


def workload(C0, shift, nq=12, nx=64):
    e, s = ddsynth.data_points(256, 6101)
    qe, qs, _ = ddsynth.queries(e, s, nq, 6102)
    w = oracle.whiten(e, s, C0)[:nx] + shift
    q = oracle.whiten(qe, qs, C0) + shift
    q = np.concatenate([q, w[:4]])
    return w, q


def errors(w, q, fused, order_seed, band_exp):
    X = float(np.sqrt((w ** 2).sum(1)).max()) * (1.0 + 1e-6)
    worst = 0.0
    escaped = False
    wf = [[Fraction(float(v)) for v in row] for row in w]
    norms = [fma_chain(row) for row in wf]
    for qrow in q:
        qf = [Fraction(float(v)) for v in qrow]
        b = [-2 * v for v in qf]                       # exact
        qn = fma_chain(qf)
        Q = float(np.sqrt((qrow ** 2).sum()))
        a = Fraction(2.0 ** band_exp) * Fraction((Q + X) ** 2)
        for xi, xr in enumerate(wf):
            d = sum((qk - xk) ** 2 for qk, xk in zip(qf, xr))
            for order in orders(order_seed + xi):
                dt = rnd(accumulate(xr, b, norms[xi], order, fused) + qn)
                err = abs(dt - d)
                worst = max(worst, float(err / a))
                escaped |= err > a
    return worst, escaped


@pytest.mark.parametrize("shift", [0.0, 30.0])
@pytest.mark.parametrize("fused", [True, False])
def test_fp64_band_contains_distance(C0, shift, fused):
    worst, escaped = errors(*workload(C0, shift), fused, 3, -48)
    assert not escaped and worst <= 1.0 - 1e-6, worst
    if shift > 0:
        # not vacuous: at the shifted data the error reaches a few unit roundoffs of (Q + X)^2
        assert worst > 2.0 ** -6, worst


def test_fp64_band_of_one_roundoff_fails(C0):
    """Plant a mistake in the band (2^-53 instead of 2^-48): some shifted pair
    escapes it."""
    w, q = workload(C0, 30.0, nq=6, nx=32)
    _, escaped = errors(w, q, True, 5, -53)
    assert escaped
