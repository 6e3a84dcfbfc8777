"""CPU oracle for the data-driven (DD) projection hot path — TEST INFRASTRUCTURE.

This package is the slow, plain, obviously-correct FP64 reference that the GPU
library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library neither imports nor
links anything from here, and the two share no code (only the seeded input
arrays from `ddsynth`).

Contents
  * P_D  — brute-force nearest neighbour under the paper's metric
           (Section 2, eq. "distmetric", with the 1/2 of the global distance),
           ties to the lowest index (linear search, Section 1); C code in pd.c.
  * whitening — the map q = (C^1/2 eps, C^-1/2 sig) of Section 3.2, with
           C^1/2 taken as the transposed Cholesky factor (any F with F^T F = C
           gives the same squared norm).
  * FE / P_C / DD loop — fe.py (Section 2, eqs. "KuE", "KeS" and the
           alternating iteration z_{i+1} = P_D(P_C(z_i))).

Parity pins (tests/test_oracle_*.py) tie every function here to something other
than itself: closed forms, hand-worked values, invariants and brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_pd.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile pd.c (gcc, OpenMP, no FMA contraction) into liboracle_pd.so."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_pd_raw.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp]
        lib.oracle_pd_white.argtypes = [vp, i64, vp, i64, vp, vp, vp]
        lib.oracle_pd_white_f32data.argtypes = [vp, i64, vp, i64, vp, vp, vp]
        lib.oracle_pair_dist_raw.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
        for f in ("oracle_pd_raw", "oracle_pd_white", "oracle_pd_white_f32data",
                  "oracle_pair_dist_raw"):
            getattr(lib, f).restype = None
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def threads() -> int:
    """OpenMP threads the C oracle uses."""
    return int(_load().oracle_threads())


def metric_inverse(C: np.ndarray) -> np.ndarray:
    """C^-1 of the (symmetric positive definite) metric, by a library inverse."""
    C = _c(C)
    return _c(np.linalg.inv(C))


def pd_raw(data_eps, data_sig, C, q_eps, q_sig):
    """P_D by brute force under the raw metric.

    Returns (idx[m] int64, dist[m], second[m]) where dist is the local distance
    1/2 d_e^2 and second the next value of the distance multiset.
    """
    de, ds, qe, qs = _c(data_eps), _c(data_sig), _c(q_eps), _c(q_sig)
    C = _c(C)
    Ci = metric_inverse(C)
    N, m = de.shape[0], qe.shape[0]
    assert de.shape == (N, 6) and ds.shape == (N, 6) and qe.shape == (m, 6) and qs.shape == (m, 6)
    idx = np.empty(m, np.int64)
    dist = np.empty(m)
    second = np.empty(m)
    _load().oracle_pd_raw(de.ctypes.data, ds.ctypes.data, N, C.ctypes.data, Ci.ctypes.data,
                          qe.ctypes.data, qs.ctypes.data, m, idx.ctypes.data, dist.ctypes.data,
                          second.ctypes.data)
    return idx, dist, second


def whitening_factors(C):
    """(F, G) with F^T F = C and G^T G = C^-1: F = L^T, G = L^-1 (C = L L^T)."""
    L = np.linalg.cholesky(_c(C))
    Linv = np.linalg.inv(L)
    return L.T.copy(), Linv.copy()


def whiten(eps, sig, C):
    """Whitened 12-component points (F eps, G sig) (Section 3.2)."""
    F, G = whitening_factors(C)
    eps, sig = _c(eps), _c(sig)
    return _c(np.concatenate([eps @ F.T, sig @ G.T], axis=1))


def pd_white(data_w, q_w):
    """P_D by brute force on whitened points: 1/2 |q - x|^2, ties to the lowest index."""
    x, q = _c(data_w), _c(q_w)
    N, m = x.shape[0], q.shape[0]
    assert x.shape == (N, 12) and q.shape == (m, 12)
    idx = np.empty(m, np.int64)
    dist = np.empty(m)
    second = np.empty(m)
    _load().oracle_pd_white(x.ctypes.data, N, q.ctypes.data, m, idx.ctypes.data,
                            dist.ctypes.data, second.ctypes.data)
    return idx, dist, second


def pd_white_f32data(data_w32, q_w):
    """P_D over single-precision stored whitened points (promoted exactly to FP64)."""
    x = _c(data_w32, np.float32)
    q = _c(q_w)
    N, m = x.shape[0], q.shape[0]
    assert x.shape == (N, 12) and q.shape == (m, 12)
    idx = np.empty(m, np.int64)
    dist = np.empty(m)
    second = np.empty(m)
    _load().oracle_pd_white_f32data(x.ctypes.data, N, q.ctypes.data, m, idx.ctypes.data,
                                    dist.ctypes.data, second.ctypes.data)
    return idx, dist, second


def pair_dist_raw(a_eps, a_sig, b_eps, b_sig, C):
    """Raw-metric local distance 1/2 d_e^2 for m paired states."""
    ae, as_, be, bs = _c(a_eps), _c(a_sig), _c(b_eps), _c(b_sig)
    C = _c(C)
    Ci = metric_inverse(C)
    m = ae.shape[0]
    out = np.empty(m)
    _load().oracle_pair_dist_raw(ae.ctypes.data, as_.ctypes.data, be.ctypes.data,
                                 bs.ctypes.data, m, C.ctypes.data, Ci.ctypes.data,
                                 out.ctypes.data)
    return out


def pca_metric(eps, sig):
    """The metric of the paper's example (Section 3): principal components of
    the data, the 12 components centred and scaled by their standard
    deviations; the 6 leading principal vectors, unscaled, are the columns of
    A = [A_eps; A_sig]; C = sym(A_sig A_eps^-1).  The paper writes the product
    as A_eps^-1 A_sig, a similar matrix but not the slope: on data lying on
    sig = C0 eps the principal subspace is {(v, C0 v)}, so that A_sig = C0 A_eps
    and only A_sig A_eps^-1 returns C0."""
    X = np.concatenate([_c(eps), _c(sig)], axis=1)
    X = X - X.mean(axis=0)
    cov = X.T @ X / X.shape[0]
    sd = np.sqrt(np.diag(cov))
    R = cov / np.outer(sd, sd)
    w, V = np.linalg.eigh(R)                 # ascending
    A = V[:, np.argsort(w)[::-1][:6]] * sd[:, None]
    Ae, As = A[:6], A[6:]
    C = As @ np.linalg.inv(Ae)
    return 0.5 * (C + C.T)


from . import fe  # noqa: E402,F401  (finite elements, P_C and the DD loop)
