"""Seeded synthetic inputs for the DD projection workloads.

Input generation only: a counter-based generator (Philox4x32-10) and the recipes
that turn it into material data points, query states and initial assignments.
Nothing here computes the DD metric, a projection or a finite-element quantity;
the CPU oracle and the GPU library both consume the arrays produced here.

Workload recipe (every configuration):
  * strain components i.i.d. uniform in [-1e-3, 1e-3] (6 Voigt components,
    engineering shear order 11, 22, 33, 23, 13, 12);
  * stress = C0 strain + N(0, 2^2) MPa per component, C0 isotropic with
    E = 200000 MPa, nu = 0.3 (1 % of the stress scale E * 1e-3 = 200 MPa);
  * queries: a uniformly drawn data point plus N(0, (5e-5)^2) on each strain
    component and N(0, 10^2) MPa on each stress component (5 % of the scales).

The C core (gen.c) is compiled with gcc on first use; `build()` forces it and
also compiles the GPU twin of the data-point recipe (gen_dev.hip, hipcc for
gfx950), which writes the same bits on the device (`DevicePoints`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libddsynth.so")
_DEV_SRC = os.path.join(_HERE, "gen_dev.hip")
_DEV_LIB_PATH = os.path.join(_HERE, "libddsynth_dev.so")
_lib = None
_dev_lib = None

E_MODULUS = 200000.0
POISSON = 0.3
EPS_AMP = 1.0e-3
STRESS_SCALE = E_MODULUS * EPS_AMP          # 200 MPa
DATA_NOISE_STD = 0.01 * STRESS_SCALE         # 2 MPa
QUERY_EPS_STD = 0.05 * EPS_AMP               # 5e-5
QUERY_SIG_STD = 0.05 * STRESS_SCALE          # 10 MPa


def build(force: bool = True, device: bool = True) -> str:
    """Compile gen.c into libddsynth.so next to it (gcc, OpenMP) and, with
    `device`, gen_dev.hip into libddsynth_dev.so (hipcc, gfx950)."""
    global _lib, _dev_lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    if device and (force or not os.path.exists(_DEV_LIB_PATH)):
        tmp = _DEV_LIB_PATH + ".tmp"
        hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                               "-o", tmp, _DEV_SRC])
        os.replace(tmp, _DEV_LIB_PATH)
        _dev_lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i64, u32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
        vp = ctypes.c_void_p
        lib.ddsynth_philox.argtypes = [u64, u64, u32, vp]
        lib.ddsynth_philox_many.argtypes = [u64, u32, vp, i64, vp]
        lib.ddsynth_points.argtypes = [u64, i64, i64, dbl, vp, dbl, vp, vp]
        lib.ddsynth_queries.argtypes = [u64, i64, vp, vp, i64, dbl, dbl, vp, vp, vp]
        lib.ddsynth_indices.argtypes = [u64, i64, i64, vp]
        lib.ddsynth_uniform.argtypes = [u64, i64, dbl, dbl, vp]
        lib.ddsynth_box_muller.argtypes = [vp, vp, i64, vp]
        lib.ddsynth_queries_gen.argtypes = [u64, i64, u64, i64, dbl, vp, dbl, dbl, dbl, vp, vp, vp]
        lib.ddsynth_points_nonlinear.argtypes = [u64, i64, i64, dbl, dbl, dbl, vp, vp]
        lib.ddsynth_nonlinear_stress.argtypes = [vp, i64, dbl, dbl, vp]
        lib.ddsynth_elementary.argtypes = [vp, i64, vp]
        for f in ("ddsynth_philox", "ddsynth_philox_many", "ddsynth_points",
                  "ddsynth_queries", "ddsynth_indices", "ddsynth_uniform",
                  "ddsynth_box_muller", "ddsynth_elementary", "ddsynth_queries_gen",
                  "ddsynth_points_nonlinear", "ddsynth_nonlinear_stress"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# --------------------------------------------------------------------------
# Philox4x32-10 in numpy (used to cross-check the C core and device copies).
# --------------------------------------------------------------------------
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)


def philox_np(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 on counters ctr[..., 4] (uint32) with key[2] (uint32)."""
    c = [ctr[..., i].astype(np.uint64) for i in range(4)]
    k0, k1 = np.uint32(key[0]), np.uint32(key[1])
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        n0 = hi1 ^ c[1] ^ np.uint64(k0)
        n2 = hi0 ^ c[3] ^ np.uint64(k1)
        c = [n0, lo1, n2, lo0]
        k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
        k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def philox(seed: int, items: np.ndarray, stream: int) -> np.ndarray:
    """C-core Philox blocks [n][4] for (item, stream) under seed."""
    items = np.ascontiguousarray(items, dtype=np.uint64)
    out = np.empty((items.size, 4), dtype=np.uint32)
    _load().ddsynth_philox_many(seed, stream, _ptr(items), items.size, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Recipes
# --------------------------------------------------------------------------
def isotropic_stiffness(E: float = E_MODULUS, nu: float = POISSON) -> np.ndarray:
    """Isotropic 6x6 stiffness in Voigt order (11,22,33,23,13,12), engineering shear."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    for i in range(3):
        C[i, i] = lam + 2.0 * mu
        C[3 + i, 3 + i] = mu
    return C


def data_points(n: int, seed: int, first: int = 0, S0: np.ndarray | None = None,
                eps_amp: float = EPS_AMP, noise_std: float = DATA_NOISE_STD):
    """(strain[n][6], stress[n][6]) float64 for items first..first+n-1."""
    S0 = isotropic_stiffness() if S0 is None else np.ascontiguousarray(S0, dtype=np.float64)
    strain = np.empty((n, 6), dtype=np.float64)
    stress = np.empty((n, 6), dtype=np.float64)
    _load().ddsynth_points(seed, first, n, eps_amp, _ptr(S0), noise_std, _ptr(strain),
                           _ptr(stress))
    return strain, stress


def queries(strain: np.ndarray, stress: np.ndarray, m: int, seed: int,
            eps_std: float = QUERY_EPS_STD, sig_std: float = QUERY_SIG_STD):
    """(q_strain[m][6], q_stress[m][6], base[m]) around uniformly drawn data points."""
    strain = np.ascontiguousarray(strain, dtype=np.float64)
    stress = np.ascontiguousarray(stress, dtype=np.float64)
    qe = np.empty((m, 6), dtype=np.float64)
    qs = np.empty((m, 6), dtype=np.float64)
    base = np.empty(m, dtype=np.int64)
    _load().ddsynth_queries(seed, m, _ptr(strain), _ptr(stress), strain.shape[0], eps_std,
                            sig_std, _ptr(qe), _ptr(qs), _ptr(base))
    return qe, qs, base


# The paper's example (Section 3): nonlinear isotropic law, strains in +-0.025.
PAPER_E = 1000.0
PAPER_ALPHA = 500.0
PAPER_EPS_AMP = 0.025


def data_points_nonlinear(n: int, seed: int, first: int = 0, eps_amp: float = PAPER_EPS_AMP,
                          E: float = PAPER_E, alpha: float = PAPER_ALPHA):
    """(strain[n][6], stress[n][6]) of the paper's example: Voigt strains uniform in
    [-eps_amp, eps_amp], stress from the nonlinear reference law (no noise)."""
    strain = np.empty((n, 6), dtype=np.float64)
    stress = np.empty((n, 6), dtype=np.float64)
    _load().ddsynth_points_nonlinear(seed, first, n, eps_amp, E, alpha, _ptr(strain), _ptr(stress))
    return strain, stress


def nonlinear_stress(strain: np.ndarray, E: float = PAPER_E, alpha: float = PAPER_ALPHA):
    strain = np.ascontiguousarray(strain, dtype=np.float64).reshape(-1, 6)
    out = np.empty_like(strain)
    _load().ddsynth_nonlinear_stress(_ptr(strain), strain.shape[0], E, alpha, _ptr(out))
    return out


def torsion_bc(n: int, size: float = 10.0, theta_deg: float = 2.0):
    """The paper's boundary conditions on an n^3 cube of edge `size` (Section 3):
    nodes on z = 0 fixed; nodes on z = size rotated by theta about the vertical
    axis through the face centre and fixed in z.  Returns (mask uint8 [ndof],
    prescribed displacement float64 [ndof], zero nodal force [ndof])."""
    n1 = n + 1
    ndof = 3 * n1 ** 3
    mask = np.zeros(ndof, dtype=np.uint8)
    val = np.zeros(ndof)
    h = size / n
    th = np.deg2rad(theta_deg)
    c, s = np.cos(th), np.sin(th)
    for j in range(n1):
        for i in range(n1):
            mask[3 * (i + n1 * j) + np.arange(3)] = 1                  # z = 0
            nid = i + n1 * (j + n1 * n)                                # z = size
            x, y = i * h - 0.5 * size, j * h - 0.5 * size
            mask[3 * nid + np.arange(3)] = 1
            val[3 * nid] = (c - 1.0) * x - s * y
            val[3 * nid + 1] = s * x + (c - 1.0) * y
    return mask, val, np.zeros(ndof)


def queries_generated(n_data: int, data_seed: int, m: int, seed: int,
                      S0: np.ndarray | None = None, eps_amp: float = EPS_AMP,
                      noise_std: float = DATA_NOISE_STD, eps_std: float = QUERY_EPS_STD,
                      sig_std: float = QUERY_SIG_STD):
    """As `queries` for the data set data_points(n_data, data_seed) without
    holding it: each base point is regenerated from its index.  The result
    equals queries(*data_points(n_data, data_seed), m, seed)."""
    S0 = isotropic_stiffness() if S0 is None else np.ascontiguousarray(S0, dtype=np.float64)
    qe = np.empty((m, 6), dtype=np.float64)
    qs = np.empty((m, 6), dtype=np.float64)
    base = np.empty(m, dtype=np.int64)
    _load().ddsynth_queries_gen(seed, m, data_seed, n_data, eps_amp, _ptr(S0), noise_std, eps_std,
                                sig_std, _ptr(qe), _ptr(qs), _ptr(base))
    return qe, qs, base


def indices(n: int, n_data: int, seed: int) -> np.ndarray:
    """Uniform random indices in [0, n_data) (e.g. a random initial DD assignment)."""
    out = np.empty(n, dtype=np.int64)
    _load().ddsynth_indices(seed, n, n_data, _ptr(out))
    return out


def uniform(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().ddsynth_uniform(seed, n, lo, hi, _ptr(out))
    return out


def box_muller(ua: np.ndarray, ub: np.ndarray) -> np.ndarray:
    """Pairs of standard normals [n][2] from uniforms ua, ub (the shared transform)."""
    ua = np.ascontiguousarray(ua, dtype=np.float64)
    ub = np.ascontiguousarray(ub, dtype=np.float64)
    z = np.empty((ua.size, 2))
    _load().ddsynth_box_muller(_ptr(ua), _ptr(ub), ua.size, _ptr(z))
    return z


def elementary(x: np.ndarray) -> np.ndarray:
    """[n][3] = (log x, cos 2 pi x, sin 2 pi x) from the shared generator core."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty((x.size, 3))
    _load().ddsynth_elementary(_ptr(x), x.size, _ptr(out))
    return out


class _PointParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("eps_amp", ctypes.c_double),
                ("S0", ctypes.c_double * 36), ("noise_std", ctypes.c_double)]


class _NonlinearParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("eps_amp", ctypes.c_double), ("E", ctypes.c_double),
                ("alpha", ctypes.c_double)]


class DevicePoints:
    """The data-point recipe on the GPU (same bits as `data_points`, or as
    `data_points_nonlinear` with law="nonlinear").

    `fill_fn` / `user` form a producer for dd_dataset_create_streamed:
    fill(user, first, count, strain_dev, stress_dev, hip_stream) -> 0 on success.
    `generate(first, n)` returns device tensors (strain, stress) [n][6].
    """

    def __init__(self, seed: int, S0: np.ndarray | None = None, eps_amp: float = EPS_AMP,
                 noise_std: float = DATA_NOISE_STD, law: str = "linear"):
        global _dev_lib
        if _dev_lib is None:
            if not os.path.exists(_DEV_LIB_PATH):
                raise RuntimeError("libddsynth_dev.so is not built (ddsynth.build())")
            import torch  # noqa: F401  (one HIP runtime per process: torch's)
            lib = ctypes.CDLL(_DEV_LIB_PATH)
            lib.ddsynth_dev_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            lib.ddsynth_dev_fill.restype = ctypes.c_int
            lib.ddsynth_dev_params_bytes.restype = ctypes.c_int
            lib.ddsynth_dev_fill_nonlinear.argtypes = lib.ddsynth_dev_fill.argtypes
            lib.ddsynth_dev_fill_nonlinear.restype = ctypes.c_int
            if lib.ddsynth_dev_params_bytes() != ctypes.sizeof(_PointParams):
                raise RuntimeError("libddsynth_dev.so parameter layout mismatch")
            _dev_lib = lib
        self.lib = _dev_lib
        if law == "nonlinear":
            self.params = _NonlinearParams(seed, PAPER_EPS_AMP if eps_amp == EPS_AMP else eps_amp,
                                           PAPER_E, PAPER_ALPHA)
            self._fill = _dev_lib.ddsynth_dev_fill_nonlinear
        else:
            S0 = isotropic_stiffness() if S0 is None else np.asarray(S0, dtype=np.float64)
            self.params = _PointParams(seed, eps_amp,
                                       (ctypes.c_double * 36)(*S0.ravel().tolist()), noise_std)
            self._fill = _dev_lib.ddsynth_dev_fill
        self.fill_fn = ctypes.cast(self._fill, ctypes.c_void_p).value
        self.user = ctypes.addressof(self.params)

    def generate(self, first: int, n: int, stream: int = 0):
        import torch
        e = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        s = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        if stream == 0:
            stream = torch.cuda.current_stream().cuda_stream
        rc = self._fill(self.user, first, n, e.data_ptr(), s.data_ptr(), stream)
        if rc != 0:
            raise RuntimeError(f"ddsynth_dev_fill failed ({rc})")
        return e, s


def states(strain: np.ndarray, stress: np.ndarray) -> np.ndarray:
    """Pack (strain, stress) into phase-space states [n][12]."""
    return np.ascontiguousarray(np.concatenate([strain, stress], axis=1))


# Workload configurations (sizes of the measured cases).
CONFIGS = {
    0: dict(name="exact-fp64 N=65536 m=4096", N=65536, m=4096, data_seed=1000, query_seed=2000),
    1: dict(name="dd-solve 8^3 hex N=1e6 traction 100 MPa", N=1_000_000, mesh=8,
            traction=100.0, data_seed=1001),
    2: dict(name="mixed-precision N=2^27 m=65536", N=1 << 27, m=65536, data_seed=1002,
            query_seed=2002),
    3: dict(name="ann N=1e9 16^3 hex", N=1_000_000_000, mesh=16, traction=100.0,
            data_seed=1003),
    4: dict(name="serving N=2^26 hex 4^3/8^3/16^3/24^3", N=1 << 26, meshes=(4, 8, 16, 24),
            traction=(50.0, 200.0), data_seed=1004),
}


def box_bc(n: int, traction: float):
    """Boundary-value problem of the measured DD solves on the unit cube with
    n^3 hexahedra (node (i,j,k) id i + (n+1)(j + (n+1)k), DOF 3 id + c):
    all DOFs of the nodes on x = 0 fixed; uniform normal traction `traction`
    (+x) on x = 1 as nodal loads, each face quad passing t h^2 / 4 to its nodes.
    Returns (mask uint8 [ndof], force float64 [ndof])."""
    n1 = n + 1
    ndof = 3 * n1 ** 3
    mask = np.zeros(ndof, dtype=np.uint8)
    force = np.zeros(ndof)
    h = 1.0 / n
    for k in range(n1):
        for j in range(n1):
            mask[3 * (0 + n1 * (j + n1 * k)) + np.arange(3)] = 1
    for k in range(n):
        for j in range(n):
            for dj, dk in ((0, 0), (1, 0), (0, 1), (1, 1)):
                nid = n + n1 * ((j + dj) + n1 * (k + dk))
                force[3 * nid] += traction * h * h / 4.0
    return mask, force
