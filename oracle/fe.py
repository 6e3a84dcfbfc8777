"""Oracle finite elements, constraint-set projection P_C and the DD loop (CPU, FP64).

TEST INFRASTRUCTURE: part of the oracle package; never used by the GPU library.

Discretisation (the paper's setting of Section 2 on a structured cube):
  * cube [0,L]^3 (L = 1 unless given) split into n^3 trilinear hexahedra of edge h = L/n;
    node (i, j, k) has id i + (n+1)(j + (n+1)k); DOF = 3 * node + component;
  * element (ex, ey, ez) has id ex + n(ey + n ez);
  * 2x2x2 Gauss points at +-1/sqrt(3) with unit weights, point a + 2(b + 2c)
    (a, b, c = 0 for the negative abscissa); integration-point weight
    w_e = det J = (h/2)^3 (the "volumes" of the global distance, Section 2);
  * material-point order: element-major, then Gauss point;
  * strain-displacement operator B (6 x 24) in Voigt order
    (11, 22, 33, 23, 13, 12) with engineering shear strains.

P_C (Section 2, eqs. "KuE" and "KeS"): given data states z* = (eps*, sig*),
    K u   = E = A_e { w B^T C eps* }
    K eta = S = f - A_e { w B^T sig* }
    eps = B u,  sig = sig* + C B eta
with the prescribed displacements (zero unless given) on u and homogeneous
conditions on eta at the constrained DOFs: the free part of u solves
K_ff u_f = E_f - K_fd u_D.
K = A_e { w B^T C B } is factorised once (Section 2, after eq. "KeS"); the
factorisation is a library sparse LU (SuperLU through scipy), used only as the
"solve K x = b" step.

DD loop (Section 2): random initial association, then z_{i+1} = P_D(P_C(z_i))
until the association no longer changes (the exact-projection stopping rule).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GAUSS = 1.0 / np.sqrt(3.0)


def node_id(n, i, j, k):
    return i + (n + 1) * (j + (n + 1) * k)


def shape_gradients(h: float) -> np.ndarray:
    """dN_a/dx at the 8 Gauss points: array [8 gauss][8 nodes][3]."""
    out = np.zeros((8, 8, 3))
    for g in range(8):
        xi = np.array([(g & 1) * 2 - 1, ((g >> 1) & 1) * 2 - 1, ((g >> 2) & 1) * 2 - 1]) * GAUSS
        for a in range(8):
            s = np.array([(a & 1) * 2 - 1, ((a >> 1) & 1) * 2 - 1, ((a >> 2) & 1) * 2 - 1],
                         dtype=float)
            f = 1.0 + s * xi                       # (1 + s_x xi)(1 + s_y eta)(1 + s_z zeta) / 8
            dxi = np.array([s[0] * f[1] * f[2], f[0] * s[1] * f[2], f[0] * f[1] * s[2]]) / 8.0
            out[g, a] = dxi * (2.0 / h)            # d xi / d x = 2 / h
    return out


def strain_operators(h: float) -> np.ndarray:
    """B matrices [8 gauss][6][24] (Voigt 11,22,33,23,13,12; engineering shear)."""
    G = shape_gradients(h)
    B = np.zeros((8, 6, 24))
    for g in range(8):
        for a in range(8):
            dx, dy, dz = G[g, a]
            c = 3 * a
            B[g, 0, c + 0] = dx
            B[g, 1, c + 1] = dy
            B[g, 2, c + 2] = dz
            B[g, 3, c + 1] = dz
            B[g, 3, c + 2] = dy
            B[g, 4, c + 0] = dz
            B[g, 4, c + 2] = dx
            B[g, 5, c + 0] = dy
            B[g, 5, c + 1] = dx
    return B


@dataclass
class Mesh:
    """Structured n^3 hexahedral mesh of the cube [0, size]^3."""
    n: int
    size: float = 1.0
    h: float = field(init=False)
    n_nodes: int = field(init=False)
    n_dof: int = field(init=False)
    n_el: int = field(init=False)
    n_mp: int = field(init=False)
    edofs: np.ndarray = field(init=False, repr=False)     # [n_el][24]
    coords: np.ndarray = field(init=False, repr=False)    # [n_nodes][3]
    B: np.ndarray = field(init=False, repr=False)         # [8][6][24]
    w: float = field(init=False)

    def __post_init__(self):
        n = self.n
        self.h = self.size / n
        self.n_nodes = (n + 1) ** 3
        self.n_dof = 3 * self.n_nodes
        self.n_el = n ** 3
        self.n_mp = 8 * self.n_el
        ii, jj, kk = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1),
                                 indexing="ij")
        coords = np.zeros((self.n_nodes, 3))
        ids = node_id(n, ii, jj, kk).ravel()
        coords[ids, 0] = ii.ravel() * self.h
        coords[ids, 1] = jj.ravel() * self.h
        coords[ids, 2] = kk.ravel() * self.h
        self.coords = coords
        edofs = np.zeros((self.n_el, 24), dtype=np.int64)
        for ez in range(n):
            for ey in range(n):
                for ex in range(n):
                    e = ex + n * (ey + n * ez)
                    for a in range(8):
                        nid = node_id(n, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1))
                        edofs[e, 3 * a:3 * a + 3] = 3 * nid + np.arange(3)
        self.edofs = edofs
        self.B = strain_operators(self.h)
        self.w = (self.h / 2.0) ** 3

    # ---- boundary conditions ------------------------------------------
    def clamp_mask(self, face_x0: bool = True) -> np.ndarray:
        """Dirichlet mask: all three components of the nodes on x = 0."""
        mask = np.zeros(self.n_dof, dtype=bool)
        nodes = np.where(np.isclose(self.coords[:, 0], 0.0))[0]
        for c in range(3):
            mask[3 * nodes + c] = True
        return mask

    def roller_mask(self) -> np.ndarray:
        """u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on z = 0."""
        mask = np.zeros(self.n_dof, dtype=bool)
        for c in range(3):
            nodes = np.where(np.isclose(self.coords[:, c], 0.0))[0]
            mask[3 * nodes + c] = True
        return mask

    def torsion(self, theta_deg: float):
        """The paper's boundary conditions (Section 3): the face z = 0 fixed, the
        face z = size rotated by theta about the vertical axis through its
        centre and fixed in z.  Returns (mask, prescribed displacement)."""
        mask = np.zeros(self.n_dof, dtype=bool)
        val = np.zeros(self.n_dof)
        th = np.deg2rad(theta_deg)
        rot = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        for z, turn in ((0.0, False), (self.size, True)):
            nodes = np.where(np.isclose(self.coords[:, 2], z))[0]
            for c in range(3):
                mask[3 * nodes + c] = True
            if turn:
                r = self.coords[nodes, :2] - 0.5 * self.size
                d = r @ rot.T - r
                val[3 * nodes] = d[:, 0]
                val[3 * nodes + 1] = d[:, 1]
        return mask, val

    def traction_x1(self, t: float) -> np.ndarray:
        """Consistent nodal forces of a uniform normal traction t (+x) on the face x = 1."""
        f = np.zeros(self.n_dof)
        n, h = self.n, self.h
        for k in range(n):
            for j in range(n):
                for (dj, dk) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                    nid = node_id(n, n, j + dj, k + dk)
                    f[3 * nid] += t * h * h / 4.0
        return f

    # ---- operators -------------------------------------------------------
    def strains(self, u: np.ndarray) -> np.ndarray:
        """eps = B u at every material point: [n_mp][6]."""
        ue = u[self.edofs]                                  # [n_el][24]
        out = np.einsum("gij,ej->egi", self.B, ue)          # [n_el][8][6]
        return out.reshape(self.n_mp, 6)

    def assemble_vector(self, s: np.ndarray) -> np.ndarray:
        """A_e { w B^T s_e } for a field s [n_mp][6]."""
        s = s.reshape(self.n_el, 8, 6)
        ce = self.w * np.einsum("gij,egi->ej", self.B, s)   # [n_el][24]
        return np.bincount(self.edofs.ravel(), weights=ce.ravel(), minlength=self.n_dof)

    def stiffness(self, C: np.ndarray) -> sp.csr_matrix:
        """K = A_e { w B^T C B } (sparse, all DOFs)."""
        Ke = self.w * np.einsum("gki,kl,glj->ij", self.B, C, self.B)
        rows = np.repeat(self.edofs, 24, axis=1).ravel()
        cols = np.tile(self.edofs, (1, 24)).ravel()
        vals = np.tile(Ke.ravel(), self.n_el)
        return sp.coo_matrix((vals, (rows, cols)), shape=(self.n_dof, self.n_dof)).tocsr()


class ConstraintProjector:
    """P_C for a fixed mesh, metric C, Dirichlet mask (with prescribed
    displacements u_D, zero by default) and load f (K factorised once)."""

    def __init__(self, mesh: Mesh, C: np.ndarray, mask: np.ndarray, f: np.ndarray,
                 u_dirichlet: np.ndarray | None = None):
        self.mesh = mesh
        self.C = np.asarray(C, dtype=np.float64)
        self.mask = np.asarray(mask, dtype=bool)
        self.f = np.asarray(f, dtype=np.float64)
        self.free = np.where(~self.mask)[0]
        K = mesh.stiffness(self.C)
        self.K = K
        Kff = K[self.free][:, self.free].tocsc()
        self.lu = spla.splu(Kff)
        self.uD = np.zeros(mesh.n_dof)
        if u_dirichlet is not None:
            self.uD[self.mask] = np.asarray(u_dirichlet, dtype=np.float64)[self.mask]
        self.lift = K @ self.uD      # K_fd u_D on the free rows

    def solve(self, rhs: np.ndarray, prescribed: np.ndarray | None = None) -> np.ndarray:
        x = np.zeros(self.mesh.n_dof)
        if prescribed is None:
            x[self.free] = self.lu.solve(rhs[self.free])
        else:
            x[self.free] = self.lu.solve(rhs[self.free] - self.lift[self.free])
            x[self.mask] = prescribed[self.mask]
        return x

    def __call__(self, eps_star: np.ndarray, sig_star: np.ndarray):
        """(u, eta, eps, sig) = P_C(eps*, sig*)."""
        m = self.mesh
        E = m.assemble_vector(eps_star @ self.C.T)
        S = self.f - m.assemble_vector(sig_star)
        u = self.solve(E, self.uD)
        eta = self.solve(S)
        eps = m.strains(u)
        sig = sig_star + m.strains(eta) @ self.C.T
        return u, eta, eps, sig


@dataclass
class DDResult:
    u: np.ndarray
    eps: np.ndarray
    sig: np.ndarray
    idx: np.ndarray
    iterations: int
    converged: bool
    d_half: list
    d_full: list
    changed: list
    history: list          # assignment arrays idx_0, idx_1, ... (when recorded)


def dd_solve(data_eps, data_sig, C, mesh: Mesh, mask, f, init_idx, max_iter=500,
             project=None, record_history=False, u_dirichlet=None) -> DDResult:
    """Plain DD fixed-point loop (Section 2): z_{i+1} = P_D(P_C(z_i)).

    project(eps, sig) -> (idx, dist) is the P_D step; by default the brute-force
    raw-metric oracle.  Per iteration i:
        y_i       = P_C(z_i)
        D_half_i  = sum_e w_e dist(y_e, z_i,e)
        z_{i+1}   = P_D(y_i)
        D_full_i  = sum_e w_e dist(y_e, z_{i+1},e)
        changed_i = #{e : idx_{i+1,e} != idx_{i,e}}
    stopping when changed_i = 0 (converged) or after max_iter iterations.  The
    result is the constraint-set state of the last P_C.
    """
    from . import pair_dist_raw, pd_raw

    data_eps = np.ascontiguousarray(data_eps, dtype=np.float64)
    data_sig = np.ascontiguousarray(data_sig, dtype=np.float64)
    if project is None:
        def project(e, s):
            i, d, _ = pd_raw(data_eps, data_sig, C, e, s)
            return i, d
    pc = ConstraintProjector(mesh, C, mask, f, u_dirichlet)
    idx = np.asarray(init_idx, dtype=np.int64).copy()
    d_half, d_full, changed, hist = [], [], [], []
    if record_history:
        hist.append(idx.copy())
    converged = False
    it = 0
    u = eps = sig = None
    for it in range(1, max_iter + 1):
        zs_e, zs_s = data_eps[idx], data_sig[idx]
        u, _, eps, sig = pc(zs_e, zs_s)
        dh = mesh.w * pair_dist_raw(eps, sig, zs_e, zs_s, C)
        new_idx, new_dist = project(eps, sig)
        d_half.append(float(np.sum(dh)))
        d_full.append(float(np.sum(mesh.w * new_dist)))
        ch = int(np.count_nonzero(new_idx != idx))
        changed.append(ch)
        idx = np.asarray(new_idx, dtype=np.int64).copy()
        if record_history:
            hist.append(idx.copy())
        if ch == 0:
            converged = True
            break
    return DDResult(u=u, eps=eps, sig=sig, idx=idx, iterations=it, converged=converged,
                    d_half=d_half, d_full=d_full, changed=changed, history=hist)
