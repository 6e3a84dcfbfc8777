"""ctypes binding of libdd.so: the C-ABI entry points under the same names.

Only argument marshalling happens here (torch tensors -> device pointers and
the current HIP stream).  Every step of the computation runs in the library's
HIP kernels; if libdd.so is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdd.so")

DD_OK = 0
STATUS = {0: "DD_OK", 1: "DD_ERR_ARG", 2: "DD_ERR_NOT_SPD", 3: "DD_ERR_OOM", 4: "DD_ERR_DEVICE",
          5: "DD_ERR_NOT_CONVERGED", 6: "DD_ERR_TOO_LARGE", 7: "DD_ERR_CANCELLED",
          8: "DD_ERR_UNSUPPORTED", 9: "DD_ERR_TIMEOUT"}

(DD_EXACT_FP64, DD_MIXED_FP32, DD_MIXED_BF16, DD_ANN, DD_DIRECT_FP64, DD_MIXED_FP16,
 DD_KMEANS) = range(7)
MODES = {"fp64": DD_EXACT_FP64, "fp32": DD_MIXED_FP32, "bf16": DD_MIXED_BF16, "ann": DD_ANN,
         "direct": DD_DIRECT_FP64, "fp16": DD_MIXED_FP16, "kmeans": DD_KMEANS}

DD_PACK_FP64, DD_PACK_FP32, DD_PACK_BF16, DD_PACK_FP16, DD_PACK_ANN, DD_PACK_KMEANS = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20)


class DDError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {message}")


class dd_dataset_opts(ctypes.Structure):
    _fields_ = [("packs", ctypes.c_uint32), ("tile", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class dd_project_stats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("overflowed", ctypes.c_int64),
                ("visited", ctypes.c_int64), ("scan_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("slow_tiles", ctypes.c_int64),
                ("boxes", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("leaf_boxes", ctypes.c_int64), ("nodes", ctypes.c_int64)]


class dd_index_info(ctypes.Structure):
    _fields_ = [("ann_levels", ctypes.c_int32), ("kmeans_levels", ctypes.c_int32),
                ("ann_leaves", ctypes.c_int64), ("kmeans_nodes", ctypes.c_int64),
                ("kmeans_leaves", ctypes.c_int64), ("kmeans_records", ctypes.c_int64)]


class dd_project_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("splits", ctypes.c_int32), ("ann_budget", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("stats", ctypes.POINTER(dd_project_stats)),
                ("ann_radius_discount", ctypes.c_double)]


def _load():
    # torch ships its own HIP runtime (same SONAME as ROCm's).  Loading torch
    # first makes libdd bind to that runtime; the other order would put two HIP
    # (and HSA) runtimes in the process, and torch's streams and allocations
    # would belong to the other one.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2012_00357_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.dd_dataset_create.argtypes = [vp, vp, i64, vp, ctypes.POINTER(dd_dataset_opts), vp,
                                      ctypes.POINTER(vp)]
    lib.dd_dataset_create_streamed.argtypes = [i64, vp, vp, vp, ctypes.POINTER(dd_dataset_opts),
                                               vp, ctypes.POINTER(vp)]
    lib.dd_dataset_destroy.argtypes = [vp]
    lib.dd_dataset_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.dd_dataset_index_info.argtypes = [vp, ctypes.POINTER(dd_index_info)]
    lib.dd_project.argtypes = [vp, vp, i64, vp, ctypes.POINTER(dd_project_opts), vp, vp, vp]
    lib.dd_selftest_mfma.argtypes = [i32, vp, vp, vp]
    lib.dd_metric_pca.argtypes = [vp, vp, i64, vp, vp]
    for f in ("dd_dataset_create", "dd_dataset_create_streamed", "dd_dataset_destroy",
              "dd_dataset_info", "dd_dataset_index_info", "dd_project", "dd_selftest_mfma",
              "dd_metric_pca"):
        getattr(lib, f).restype = ctypes.c_int
    lib.dd_last_error.restype = ctypes.c_char_p
    lib.dd_version.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def dd_last_error() -> str:
    return _lib.dd_last_error().decode()


def dd_version() -> str:
    return _lib.dd_version().decode()


def _check(status: int, where: str):
    if status != DD_OK:
        raise DDError(status, where, dd_last_error())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, shape_tail=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n]{list(shape_tail)}, got {list(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Dataset:
    """Owning handle of a dd_dataset (released by dd_dataset_destroy)."""

    def __init__(self, handle: int, n: int):
        self._h = ctypes.c_void_p(handle)
        self.n = n

    @property
    def handle(self):
        return self._h

    def info(self):
        n, b = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.dd_dataset_info(self._h, ctypes.byref(n), ctypes.byref(b)), "dd_dataset_info")
        return n.value, b.value

    def close(self):
        if self._h is not None and self._h.value:
            _lib.dd_dataset_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DD_DATASET_HOST_INPUT = 0x1


def dd_dataset_create(strain, stress, C, packs: int = 0, tile: int = 0,
                      stream=None) -> Dataset:
    """dd_dataset_create: strain/stress float64 [N][6], both device tensors or both
    host (numpy) arrays (DD_DATASET_HOST_INPUT); C a 6x6 host array."""
    import torch
    n = int(strain.shape[0])
    flags = 0
    if isinstance(strain, np.ndarray) or isinstance(stress, np.ndarray):
        e = np.ascontiguousarray(strain, dtype=np.float64)
        t = np.ascontiguousarray(stress, dtype=np.float64)
        if e.shape != (n, 6) or t.shape != (n, 6):
            raise ValueError("strain and stress must be [N][6]")
        ps, pt, flags = ctypes.c_void_p(e.ctypes.data), ctypes.c_void_p(t.ctypes.data), DD_DATASET_HOST_INPUT
    else:
        ps = _dev_ptr(strain, torch.float64, (6,), "strain")
        pt = _dev_ptr(stress, torch.float64, (6,), "stress")
    Cm = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(36))
    opts = dd_dataset_opts(packs, tile, flags)
    out = ctypes.c_void_p()
    _check(_lib.dd_dataset_create(ps, pt, n, Cm.ctypes.data, ctypes.byref(opts), _stream(stream),
                                  ctypes.byref(out)), "dd_dataset_create")
    return Dataset(out.value, n)


def dd_dataset_create_streamed(n: int, C, fill_fn: int, user: int, packs: int = 0, tile: int = 0,
                               stream=None) -> Dataset:
    """dd_dataset_create_streamed: fill_fn is the address of a C producer with the
    dd_fill_fn signature, user its opaque argument (e.g. ddsynth.DevicePoints)."""
    Cm = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(36))
    opts = dd_dataset_opts(packs, tile, 0)
    out = ctypes.c_void_p()
    _check(_lib.dd_dataset_create_streamed(int(n), Cm.ctypes.data, ctypes.c_void_p(fill_fn),
                                           ctypes.c_void_p(user), ctypes.byref(opts),
                                           _stream(stream), ctypes.byref(out)),
           "dd_dataset_create_streamed")
    return Dataset(out.value, int(n))


def dd_dataset_destroy(ds: Dataset):
    ds.close()


def dd_project(ds: Dataset, states, warm_start_idx=None, mode="fp64", splits: int = 0,
               ann_budget: int = 0, idx_out=None, dist_out=None, stream=None, stats: bool = False,
               passes: int = 0, ann_fd: float | None = None):
    """dd_project: states device float64 [m][12] -> (idx int64 [m], dist float64 [m][, stats]).

    ann_fd is the k-means walk's f_d (None = 1, exact); it is passed as
    ann_radius_discount = 1 - f_d."""
    import torch
    m = int(states.shape[0])
    ps = _dev_ptr(states, torch.float64, (12,), "states")
    if idx_out is None:
        idx_out = torch.empty(m, dtype=torch.int64, device=states.device)
    if dist_out is None:
        dist_out = torch.empty(m, dtype=torch.float64, device=states.device)
    pi = _dev_ptr(idx_out, torch.int64, None, "idx_out")
    pd = _dev_ptr(dist_out, torch.float64, None, "dist_out")
    pw = None
    if warm_start_idx is not None:
        pw = _dev_ptr(warm_start_idx, torch.int64, None, "warm_start_idx")
    st = dd_project_stats()
    opts = dd_project_opts(MODES[mode] if isinstance(mode, str) else int(mode), splits, ann_budget,
                           passes, ctypes.pointer(st) if stats else None,
                           0.0 if ann_fd is None else 1.0 - float(ann_fd))
    _check(_lib.dd_project(ds.handle, ps, m, pw, ctypes.byref(opts), pi, pd, _stream(stream)),
           "dd_project")
    if stats:
        return idx_out, dist_out, {"candidates": st.candidates, "overflowed": st.overflowed,
                                   "visited": st.visited, "scan_ms": st.scan_ms,
                                   "total_ms": st.total_ms, "slow_tiles": st.slow_tiles,
                                   "boxes": st.boxes, "leaves": st.leaves,
                                   "leaf_boxes": st.leaf_boxes, "nodes": st.nodes}
    return idx_out, dist_out


_lib.dd_project_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.POINTER(dd_project_opts),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
_lib.dd_project_noalloc.restype = ctypes.c_int
DD_NOALLOC_MAX_QUERIES = 65536


def dd_project_noalloc(ds: Dataset, states, warm_start_idx=None, mode="fp64",
                       ann_budget: int = 0, ann_fd: float | None = None, idx_out=None,
                       dist_out=None, stream=None):
    """dd_project_noalloc: as dd_project (modes fp64, ann, kmeans) with the library's
    scratch array instead of allocations; the outputs are allocated here unless given."""
    import torch
    m = int(states.shape[0])
    sp = _dev_ptr(states, torch.float64, (12,), "states")
    wp = _dev_ptr(warm_start_idx, torch.int64, (), "warm_start_idx") if warm_start_idx is not None else None
    idx = idx_out if idx_out is not None else torch.empty(m, dtype=torch.int64, device=states.device)
    dist = dist_out if dist_out is not None else torch.empty(m, dtype=torch.float64, device=states.device)
    pi = _dev_ptr(idx, torch.int64, None, "idx_out")
    pd = _dev_ptr(dist, torch.float64, None, "dist_out")
    opts = dd_project_opts(MODES[mode] if isinstance(mode, str) else int(mode), 0, ann_budget, 0,
                           None, 0.0 if ann_fd is None else 1.0 - float(ann_fd))
    _check(_lib.dd_project_noalloc(ds.handle, sp, m, wp, ctypes.byref(opts), pi, pd,
                                   _stream(stream)), "dd_project_noalloc")
    return idx, dist


def dd_metric_pca(strain, stress, stream=None) -> np.ndarray:
    """dd_metric_pca: device float64 [N][6] strain/stress -> the 6x6 PCA metric (host)."""
    import torch
    n = int(strain.shape[0])
    ps = _dev_ptr(strain, torch.float64, (6,), "strain")
    pt = _dev_ptr(stress, torch.float64, (6,), "stress")
    C = np.zeros(36)
    _check(_lib.dd_metric_pca(ps, pt, n, C.ctypes.data, _stream(stream)), "dd_metric_pca")
    return C.reshape(6, 6)


def dd_selftest_mfma(kind: int, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(np.zeros(1) if B is None else B, dtype=np.float64)
    shape = (16, 16) if kind == 2 else ((512,) if kind in (3, 4) else (32, 32))
    D = np.zeros(shape, dtype=np.float64)
    _check(_lib.dd_selftest_mfma(kind, A.ctypes.data, B.ctypes.data, D.ctypes.data),
           "dd_selftest_mfma")
    return D


def dd_dataset_info(ds: Dataset):
    """dd_dataset_info: (number of points, device bytes held)."""
    return ds.info()


def dd_dataset_index_info(ds: Dataset) -> dict:
    """dd_dataset_index_info: shape of the dataset's search trees."""
    info = dd_index_info()
    _check(_lib.dd_dataset_index_info(ds.handle, ctypes.byref(info)), "dd_dataset_index_info")
    return {k: getattr(info, k) for k, _ in info._fields_}


class dd_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class dd_solve_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("cg_max_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("ann_budget", ctypes.c_int32),
                ("ann_ramp", ctypes.c_int32), ("dirichlet_values", ctypes.c_void_p),
                ("ann_radius_discount", ctypes.c_double)]


class dd_solve_result(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("eps", ctypes.c_void_p),
                ("sig", ctypes.c_void_p), ("d_half", ctypes.c_void_p), ("d_full", ctypes.c_void_p),
                ("changed", ctypes.c_void_p), ("history", ctypes.c_void_p),
                ("history_capacity", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("cg_iterations", ctypes.c_int64), ("cg_max_residual", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("skipped", ctypes.c_int64),
                ("project_ms", ctypes.c_double)]


_lib.dd_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(dd_mesh), ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.POINTER(dd_solve_opts),
                          ctypes.POINTER(dd_solve_result), ctypes.c_void_p]
_lib.dd_solve.restype = ctypes.c_int


def dd_solve(ds: Dataset, mesh, dirichlet_mask, nodal_force, init_idx, mode="fp64",
             max_iter: int = 500, history: bool = False, cg_tol: float = 0.0,
             cg_max_iter: int = 0, graph: bool = True, ann_budget: int = 0, cg: bool = False,
             ann_ramp: int = 0, skip: bool = False, dirichlet_values=None, stream=None,
             ann_fd: float | None = None, local_accuracy: bool = False):
    """dd_solve: mesh = (nx, ny, nz[, lx, ly, lz]); host numpy mask/force/init arrays.

    ann_fd is the final f_d of the k-means walk (None = 1, exact), passed as
    ann_radius_discount = 1 - f_d; with ann_ramp it is reached linearly from 0.
    local_accuracy sets DD_SOLVE_LOCAL_ACCURACY (per-point accuracy from the
    local and global distances).

    Returns a dict with u, idx, eps, sig, d_half, d_full, changed, history
    (when requested), iterations, converged, cg_iterations, cg_max_residual,
    elapsed_ms, project_ms.  Not converging within max_iter is reported, not raised."""
    nx, ny, nz = mesh[:3]
    lx, ly, lz = (mesh[3:] if len(mesh) > 3 else (1.0, 1.0, 1.0))
    m = dd_mesh(nx, ny, nz, lx, ly, lz)
    n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    n_mp = 8 * nx * ny * nz
    mask = np.ascontiguousarray(np.asarray(dirichlet_mask, dtype=np.uint8).reshape(n_dof))
    force = np.ascontiguousarray(np.asarray(nodal_force, dtype=np.float64).reshape(n_dof))
    init = np.ascontiguousarray(np.asarray(init_idx, dtype=np.int64).reshape(n_mp))
    cap = max_iter
    out = {"u": np.zeros(n_dof), "idx": np.zeros(n_mp, np.int64), "eps": np.zeros((n_mp, 6)),
           "sig": np.zeros((n_mp, 6)), "d_half": np.zeros(cap), "d_full": np.zeros(cap),
           "changed": np.zeros(cap, np.int64)}
    hist = np.zeros((cap + 1, n_mp), np.int64) if history else None
    res = dd_solve_result(out["u"].ctypes.data, out["idx"].ctypes.data, out["eps"].ctypes.data,
                          out["sig"].ctypes.data, out["d_half"].ctypes.data,
                          out["d_full"].ctypes.data, out["changed"].ctypes.data,
                          hist.ctypes.data if history else None, cap, 0, 0, 0, 0, 0.0, 0.0, 0,
                          0.0)
    dv = None
    if dirichlet_values is not None:
        dv = np.ascontiguousarray(np.asarray(dirichlet_values, dtype=np.float64).reshape(n_dof))
    opts = dd_solve_opts(max_iter, MODES[mode] if isinstance(mode, str) else int(mode),
                         cg_max_iter, (0 if graph else 1) | (2 if cg else 0) | (4 if skip else 0)
                         | (8 if local_accuracy else 0),
                         cg_tol, ann_budget, ann_ramp, dv.ctypes.data if dv is not None else None,
                         0.0 if ann_fd is None else 1.0 - float(ann_fd))
    st = _lib.dd_solve(ds.handle, ctypes.byref(m), mask.ctypes.data, force.ctypes.data,
                       init.ctypes.data, ctypes.byref(opts), ctypes.byref(res), _stream(stream))
    if st not in (DD_OK, 5):
        raise DDError(st, "dd_solve", dd_last_error())
    it = res.iterations
    for k in ("d_half", "d_full", "changed"):
        out[k] = out[k][:it]
    if history:
        out["history"] = hist[:it + 1]
    out.update(iterations=it, converged=bool(res.converged), stop_reason=res.stop_reason,
               skipped=res.skipped, cg_iterations=res.cg_iterations,
               cg_max_residual=res.cg_max_residual, elapsed_ms=res.elapsed_ms,
               project_ms=res.project_ms)
    return out


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
class dd_server_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("ann_budget", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class dd_solve_request(ctypes.Structure):
    _fields_ = [("mesh", dd_mesh), ("dirichlet_mask", ctypes.c_void_p),
                ("nodal_force", ctypes.c_void_p), ("init_idx", ctypes.c_void_p),
                ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("deadline_s", ctypes.c_double)]


class dd_server_statistics(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("submitted", "completed", "failed", "rejected", "cancelled", "active", "queued",
                 "batches", "queries", "peak_active", "peak_bytes", "budget_bytes")] + \
               [(k, ctypes.c_double) for k in
                ("proj_p50_ms", "proj_p99_ms", "solve_p50_ms", "solve_p99_ms", "queue_p50_ms",
                 "queue_p99_ms", "queries_per_s", "elapsed_s")] + \
               [("reserve_bytes", ctypes.c_int64)]


_lib.dd_server_create.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(dd_server_opts),
                                  ctypes.POINTER(ctypes.c_void_p)]
_lib.dd_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(dd_solve_request),
                                  ctypes.POINTER(ctypes.c_uint64)]
_lib.dd_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(dd_solve_result),
                                ctypes.c_double]
_lib.dd_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
_lib.dd_server_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(dd_server_statistics)]
_lib.dd_server_destroy.argtypes = [ctypes.c_void_p]
for _f in ("dd_server_create", "dd_server_submit", "dd_server_wait", "dd_server_cancel",
           "dd_server_stats", "dd_server_destroy"):
    getattr(_lib, _f).restype = ctypes.c_int


class DDServer:
    """Owning handle of a dd_server: submit(...) -> ticket, wait(ticket) -> result dict."""

    def __init__(self, ds: Dataset, hbm_budget_bytes: int = 0, mode="bf16", max_active: int = 0,
                 max_batch: int = 0, max_queue: int = 0, ann_budget: int = 0):
        self.ds = ds   # keeps the dataset alive for the server's lifetime
        opts = dd_server_opts(MODES[mode] if isinstance(mode, str) else int(mode), max_active,
                              max_batch, max_queue, ann_budget, 0)
        h = ctypes.c_void_p()
        _check(_lib.dd_server_create(ds.handle, hbm_budget_bytes, ctypes.byref(opts),
                                     ctypes.byref(h)), "dd_server_create")
        self._h = h
        self._pending = {}

    def submit(self, mesh, dirichlet_mask, nodal_force, init_idx, max_iter: int = 0,
               deadline_s: float = 0.0) -> int:
        nx, ny, nz = mesh[:3]
        lx, ly, lz = (mesh[3:] if len(mesh) > 3 else (1.0, 1.0, 1.0))
        n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
        n_mp = 8 * nx * ny * nz
        mask = np.ascontiguousarray(np.asarray(dirichlet_mask, dtype=np.uint8).reshape(n_dof))
        force = np.ascontiguousarray(np.asarray(nodal_force, dtype=np.float64).reshape(n_dof))
        init = np.ascontiguousarray(np.asarray(init_idx, dtype=np.int64).reshape(n_mp))
        req = dd_solve_request(dd_mesh(nx, ny, nz, lx, ly, lz), mask.ctypes.data,
                               force.ctypes.data, init.ctypes.data, max_iter, 0, deadline_s)
        t = ctypes.c_uint64()
        _check(_lib.dd_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "dd_server_submit")
        self._pending[t.value] = (n_dof, n_mp, max_iter if max_iter > 0 else 500)
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0, raise_on_error: bool = True):
        if ticket not in self._pending:
            _check(_lib.dd_server_wait(self._h, ticket, None, 0.0), "dd_server_wait")
        n_dof, n_mp, cap = self._pending[ticket]
        out = {"u": np.zeros(n_dof), "idx": np.zeros(n_mp, np.int64), "eps": np.zeros((n_mp, 6)),
               "sig": np.zeros((n_mp, 6)), "d_half": np.zeros(cap), "d_full": np.zeros(cap),
               "changed": np.zeros(cap, np.int64)}
        res = dd_solve_result(out["u"].ctypes.data, out["idx"].ctypes.data, out["eps"].ctypes.data,
                              out["sig"].ctypes.data, out["d_half"].ctypes.data,
                              out["d_full"].ctypes.data, out["changed"].ctypes.data, None, cap,
                              0, 0, 0, 0, 0.0, 0.0, 0, 0.0)
        st = _lib.dd_server_wait(self._h, ticket, ctypes.byref(res), float(timeout_s))
        if st == 9:   # DD_ERR_TIMEOUT: the ticket stays valid
            raise DDError(st, "dd_server_wait", dd_last_error())
        del self._pending[ticket]
        it = res.iterations
        for k in ("d_half", "d_full", "changed"):
            out[k] = out[k][:it]
        out.update(status=st, iterations=it, converged=bool(res.converged),
                   stop_reason=res.stop_reason, cg_iterations=res.cg_iterations,
                   cg_max_residual=res.cg_max_residual, elapsed_ms=res.elapsed_ms)
        if st not in (DD_OK, 5) and raise_on_error:
            raise DDError(st, "dd_server_wait", dd_last_error())
        return out

    def cancel(self, ticket: int):
        _check(_lib.dd_server_cancel(self._h, ticket), "dd_server_cancel")

    def stats(self) -> dict:
        s = dd_server_statistics()
        _check(_lib.dd_server_stats(self._h, ctypes.byref(s)), "dd_server_stats")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            _lib.dd_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dd_server_create(ds: Dataset, hbm_budget_bytes: int = 0, **kw) -> DDServer:
    return DDServer(ds, hbm_budget_bytes, **kw)


def dd_server_destroy(srv: DDServer):
    srv.close()


def dd_server_submit(srv: DDServer, *a, **kw) -> int:
    return srv.submit(*a, **kw)


def dd_server_wait(srv: DDServer, ticket: int, timeout_s: float = -1.0):
    return srv.wait(ticket, timeout_s)


def dd_server_cancel(srv: DDServer, ticket: int):
    srv.cancel(ticket)


def dd_server_stats(srv: DDServer) -> dict:
    return srv.stats()
