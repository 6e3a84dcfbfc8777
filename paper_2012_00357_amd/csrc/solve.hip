// dd_solve: the data-driven fixed-point loop z_{i+1} = P_D(P_C(z_i)) of
// Section 2 on one GPU, for a structured hexahedral mesh of a box.
//
// States are kept in whitened coordinates w = (F eps, G sig) with F = L^T,
// G = L^-1 (C = L L^T), the coordinates in which P_D is evaluated.  P_C
// (eqs. "KuE", "KeS") needs C eps* = L w_eps* and sig* = L w_sig*, and returns
// eps = B u, sig = sig* + C B eta, i.e. w_eps = L^T B u, w_sig = w_sig* + L^T B eta.
//
// K = A_e{ w B^T C B } is assembled once (host, CSR over all DOFs with identity
// rows at Dirichlet DOFs) and both systems K u = E, K eta = S are solved
// together by a Jacobi-preconditioned conjugate-gradient kernel running in one
// workgroup, warm-started from the previous iterate.  All reductions run in a
// fixed order, so a solve is bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "pack16.h"
#include "scan.h"
#include "solve.h"

namespace dd {

// ---------------------------------------------------------------------------
// Host finite-element operators of the structured mesh
// ---------------------------------------------------------------------------
static const double kGauss = 0.57735026918962576451;   // 1/sqrt(3)

void FEMesh::init(const dd_mesh& m) {
  nx = m.nx;
  ny = m.ny;
  nz = m.nz;
  hx = m.lx / nx;
  hy = m.ly / ny;
  hz = m.lz / nz;
  n_nodes = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  n_dof = 3 * n_nodes;
  n_el = (int64_t)nx * ny * nz;
  n_mp = 8 * n_el;
  w = (hx / 2) * (hy / 2) * (hz / 2);
  // trilinear shape-function gradients at the 2x2x2 Gauss points
  for (int g = 0; g < 8; ++g) {
    double xi[3] = {((g & 1) ? 1 : -1) * kGauss, (((g >> 1) & 1) ? 1 : -1) * kGauss,
                    (((g >> 2) & 1) ? 1 : -1) * kGauss};
    for (int i = 0; i < 6 * 24; ++i) B[g][i] = 0.0;
    for (int a = 0; a < 8; ++a) {
      double s[3] = {(a & 1) ? 1.0 : -1.0, ((a >> 1) & 1) ? 1.0 : -1.0, ((a >> 2) & 1) ? 1.0 : -1.0};
      double f[3] = {1 + s[0] * xi[0], 1 + s[1] * xi[1], 1 + s[2] * xi[2]};
      double dx = s[0] * f[1] * f[2] / 8.0 * (2.0 / hx);
      double dy = f[0] * s[1] * f[2] / 8.0 * (2.0 / hy);
      double dz = f[0] * f[1] * s[2] / 8.0 * (2.0 / hz);
      int c = 3 * a;
      B[g][0 * 24 + c + 0] = dx;
      B[g][1 * 24 + c + 1] = dy;
      B[g][2 * 24 + c + 2] = dz;
      B[g][3 * 24 + c + 1] = dz;   // gamma_23
      B[g][3 * 24 + c + 2] = dy;
      B[g][4 * 24 + c + 0] = dz;   // gamma_13
      B[g][4 * 24 + c + 2] = dx;
      B[g][5 * 24 + c + 0] = dy;   // gamma_12
      B[g][5 * 24 + c + 1] = dx;
    }
  }
}

int64_t FEMesh::node(int i, int j, int k) const {
  return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
}

// Element stiffness Ke = w sum_g B_g^T C B_g (24 x 24).
static void element_stiffness(const FEMesh& M, const double* C, double* Ke) {
  std::fill(Ke, Ke + 24 * 24, 0.0);
  for (int g = 0; g < 8; ++g) {
    const double* B = M.B[g];
    double CB[6 * 24];
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 24; ++c) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += C[6 * r + k] * B[24 * k + c];
        CB[24 * r + c] = s;
      }
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += B[24 * k + i] * CB[24 * k + j];
        Ke[24 * i + j] += M.w * s;
      }
  }
}

// CSR of K over all DOFs; rows and columns of Dirichlet DOFs are replaced by the
// identity so that the systems can be solved on full vectors.
static void assemble_csr(const FEMesh& M, const double* C, const uint8_t* mask,
                         std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                         std::vector<double>& val, std::vector<double>& dinv) {
  double Ke[24 * 24];
  element_stiffness(M, C, Ke);
  const int64_t nd = M.n_dof;
  rowptr.assign(nd + 1, 0);
  col.clear();
  val.clear();
  dinv.assign(nd, 0.0);
  std::vector<double> rowv;
  std::vector<int32_t> rowc;
  for (int k = 0; k <= M.nz; ++k)
    for (int j = 0; j <= M.ny; ++j)
      for (int i = 0; i <= M.nx; ++i) {
        const int64_t nd0 = M.node(i, j, k);
        for (int comp = 0; comp < 3; ++comp) {
          const int64_t row = 3 * nd0 + comp;
          // neighbouring nodes in index order; values summed over the elements
          // sharing both nodes, in element order
          std::vector<std::pair<int64_t, double>> entries;
          if (mask[row]) {
            entries.push_back({row, 1.0});
          } else {
            for (int dk = -1; dk <= 1; ++dk)
              for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                  int ii = i + di, jj = j + dj, kk = k + dk;
                  if (ii < 0 || jj < 0 || kk < 0 || ii > M.nx || jj > M.ny || kk > M.nz) continue;
                  const int64_t nb = M.node(ii, jj, kk);
                  for (int c2 = 0; c2 < 3; ++c2) {
                    const int64_t cdof = 3 * nb + c2;
                    if (mask[cdof]) continue;
                    double s = 0.0;
                    bool any = false;
                    for (int ez = std::max(k, kk) - 1; ez <= std::min(k, kk); ++ez)
                      for (int ey = std::max(j, jj) - 1; ey <= std::min(j, jj); ++ey)
                        for (int ex = std::max(i, ii) - 1; ex <= std::min(i, ii); ++ex) {
                          if (ex < 0 || ey < 0 || ez < 0 || ex >= M.nx || ey >= M.ny || ez >= M.nz)
                            continue;
                          int a = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
                          int b = (ii - ex) + 2 * (jj - ey) + 4 * (kk - ez);
                          s += Ke[24 * (3 * a + comp) + 3 * b + c2];
                          any = true;
                        }
                    if (any) entries.push_back({cdof, s});
                  }
                }
            std::sort(entries.begin(), entries.end(),
                      [](const std::pair<int64_t, double>& x, const std::pair<int64_t, double>& y) {
                        return x.first < y.first;
                      });
          }
          for (auto& e : entries) {
            col.push_back((int32_t)e.first);
            val.push_back(e.second);
            if (e.first == row) dinv[row] = 1.0 / e.second;
          }
          rowptr[row + 1] = (int32_t)col.size();
        }
      }
}

// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------
struct Mat6 {
  double a[36];
};
struct BOps {
  double B[8][6 * 24];
};

__device__ inline int64_t dnode(int nx, int ny, int i, int j, int k) {
  return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
}

// Per material point: the assigned data point's whitened state z_w (from the
// sorted FP64 pack), and (C eps*, sig*) = (L w_eps*, L w_sig*).
__global__ void gather_z_kernel(const int64_t* __restrict__ idx, int64_t n_mp, int64_t N,
                                const uint32_t* __restrict__ iperm, const double* __restrict__ w64,
                                Mat6 L, double* __restrict__ zw, double* __restrict__ zc,
                                int* __restrict__ bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_mp) return;
  int64_t j = idx[e];
  if (j < 0 || j >= N) {   // a non-finite admissible state upstream: report, stay in bounds
    atomicOr(bad, 1);
    j = 0;
  }
  const int64_t p = iperm[j];
  double z[12];
  for (int k = 0; k < 12; ++k) {
    z[k] = w64[12 * p + k];
    zw[12 * e + k] = z[k];
  }
  for (int r = 0; r < 6; ++r) {
    double a = 0.0, b = 0.0;
    for (int c = 0; c < 6; ++c) {
      a = fma(L.a[6 * r + c], z[c], a);
      b = fma(L.a[6 * r + c], z[6 + c], b);
    }
    zc[12 * e + r] = a;       // C eps*
    zc[12 * e + 6 + r] = b;   // sig*
  }
}

// RHS by gathering, per DOF, the contributions of its (<= 8) elements and their
// Gauss points: one wavefront per DOF, lane 8 a + g taking Gauss point g of the
// element whose local node a is the DOF's node, then a fixed-order wave sum.
// E = A_e{w B^T C eps*} - K_fd u_D on free DOFs and u_D on Dirichlet DOFs (the
// identity rows of K carry the prescribed displacement), S = f - A_e{w B^T sig*}
// on free DOFs and 0 on Dirichlet DOFs (eta vanishes there).  uD and lift may be
// null (homogeneous conditions).
__global__ __launch_bounds__(256) void assemble_rhs_kernel(
    int nx, int ny, int nz, double w, BOps Bo, const double* __restrict__ zc,
    const uint8_t* __restrict__ mask, const double* __restrict__ f, const double* __restrict__ uD,
    const double* __restrict__ lift, double* __restrict__ E, double* __restrict__ S) {
  const int lane = threadIdx.x & 63;
  const int64_t dof = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_dof = 3 * (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  if (dof >= n_dof) return;   // wave-uniform
  if (mask[dof]) {
    if (lane == 0) {
      E[dof] = uD ? uD[dof] : 0.0;
      S[dof] = 0.0;
    }
    return;
  }
  const int comp = (int)(dof % 3);
  const int64_t nd = dof / 3;
  const int i = (int)(nd % (nx + 1));
  const int j = (int)((nd / (nx + 1)) % (ny + 1));
  const int k = (int)(nd / ((int64_t)(nx + 1) * (ny + 1)));
  const int a = lane >> 3, g = lane & 7;
  const int ex = i - (a & 1), ey = j - ((a >> 1) & 1), ez = k - (a >> 2);
  double se = 0.0, ss = 0.0;
  if (ex >= 0 && ey >= 0 && ez >= 0 && ex < nx && ey < ny && ez < nz) {
    const int64_t el = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
    const double* z = zc + 12 * (8 * el + g);
    for (int r = 0; r < 6; ++r) {
      const double bv = Bo.B[g][24 * r + 3 * a + comp];
      se = fma(bv, z[r], se);
      ss = fma(bv, z[6 + r], ss);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_xor(se, off);
    ss += __shfl_xor(ss, off);
  }
  if (lane == 0) {
    E[dof] = lift ? w * se - lift[dof] : w * se;
    S[dof] = f[dof] - w * ss;
  }
}

// ---------------------------------------------------------------------------
// Conjugate gradients for the two systems K u = E, K eta = S (Jacobi
// preconditioner), spread over many workgroups.  One iteration = three kernels:
//   cg_spmv     q = K p and per-block partial sums of p.q
//   cg_update   alpha = rz / p.q (every block sums the partials in the same
//               order), x += alpha p, r -= alpha q, z = D^-1 r, partials of
//               r.z and r.r
//   cg_pupdate  beta = rz_new / rz, p = z + beta p; block 0 stores the scalars
//               of the next iteration (double-buffered by iteration parity)
// A system whose residual |r| <= tol |b| is frozen; the host polls the flags
// every few iterations.  All sums run in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kCgBlock = 256;
constexpr int kCgPoll = 16;   // CG iterations per convergence poll (even)

struct CGState {
  double rz[2][2];     // [parity][system]
  int active[2][2];
  double bb[2];
  double rr[2];
  int iters[2];
};

__device__ inline void block_reduce(double* v, int k, double* red) {
  // sums v[0..k) over the block (k <= 6); result in v for every thread
  const int t = threadIdx.x;
  for (int j = 0; j < k; ++j) red[j * kCgBlock + t] = v[j];
  __syncthreads();
  for (int off = kCgBlock / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int j = 0; j < k; ++j) red[j * kCgBlock + t] += red[j * kCgBlock + t + off];
    __syncthreads();
  }
  for (int j = 0; j < k; ++j) v[j] = red[j * kCgBlock];
  __syncthreads();
}

// every block sums the per-block partials (k <= 6 values per block): thread t
// adds partials t, t + 256, ..., then a fixed-order tree over the block, so all
// blocks obtain bitwise the same sums
__device__ inline void sum_partials(const double* __restrict__ part, int nb, int k, double* out,
                                    double* red) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += kCgBlock)
    for (int j = 0; j < k; ++j) v[j] += part[b * 8 + j];
  block_reduce(v, k, red);
  for (int j = 0; j < k; ++j) out[j] = v[j];
}

__device__ inline double spmv_row(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                  const double* __restrict__ val, const double* __restrict__ v,
                                  int64_t i) {
  double s = 0.0;
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s = fma(val[e], v[col[e]], s);
  return s;
}

__global__ __launch_bounds__(kCgBlock) void cg_init_kernel(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ dinv, const double* __restrict__ b,
    const double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
    double* __restrict__ p, double* __restrict__ part) {
  __shared__ double red[6 * kCgBlock];
  const int64_t i = (int64_t)blockIdx.x * kCgBlock + threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};   // bb0 bb1 rz0 rz1 rr0 rr1
  if (i < n) {
    for (int s = 0; s < 2; ++s) {
      const double bi = b[s * n + i];
      const double ri = bi - spmv_row(rowptr, col, val, x + s * n, i);
      const double zi = dinv[i] * ri;
      r[s * n + i] = ri;
      z[s * n + i] = zi;
      p[s * n + i] = zi;
      v[s] = bi * bi;
      v[2 + s] = ri * zi;
      v[4 + s] = ri * ri;
    }
  }
  block_reduce(v, 6, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < 6; ++j) part[blockIdx.x * 8 + j] = v[j];
}

__global__ __launch_bounds__(kCgBlock) void cg_init_finish_kernel(const double* __restrict__ part,
                                                                  int nb, double tol,
                                                                  CGState* __restrict__ st) {
  __shared__ double red[6 * kCgBlock];
  double v[6];
  sum_partials(part, nb, 6, v, red);
  if (threadIdx.x != 0) return;
  for (int s = 0; s < 2; ++s) {
    st->bb[s] = v[s];
    st->rz[0][s] = v[2 + s];
    st->rr[s] = v[4 + s];
    st->active[0][s] = v[4 + s] > tol * tol * v[s] ? 1 : 0;
    st->iters[s] = 0;
  }
}

// q = K p for both systems, 16 lanes per row (rows have up to 81 entries), and
// per-block partial sums of p.q.  Partial-sum order is fixed, so the result is
// deterministic.
constexpr int kRowLanes = 16;
constexpr int kRowsPerBlock = kCgBlock / kRowLanes;

__global__ __launch_bounds__(kCgBlock) void cg_spmv_kernel(
    int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ p, double* __restrict__ q,
    double* __restrict__ part, const CGState* __restrict__ st, int parity) {
  __shared__ double red[2 * kCgBlock];
  if (!st->active[parity][0] && !st->active[parity][1]) return;
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kRowLanes;
  double s0 = 0.0, s1 = 0.0;
  if (i < n) {
    const int32_t e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int32_t e = e0 + sub; e < e1; e += kRowLanes) {
      const double v = val[e];
      const int32_t c = col[e];
      s0 = fma(v, p[c], s0);
      s1 = fma(v, p[n + c], s1);
    }
  }
  // reduce over the 16 lanes of the row (fixed butterfly order)
  for (int off = kRowLanes / 2; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, kRowLanes);
    s1 += __shfl_xor(s1, off, kRowLanes);
  }
  double v[2] = {0.0, 0.0};
  if (i < n && sub == 0) {
    q[i] = s0;
    q[n + i] = s1;
    v[0] = p[i] * s0;
    v[1] = p[n + i] * s1;
  }
  block_reduce(v, 2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 8 + 0] = v[0];
    part[blockIdx.x * 8 + 1] = v[1];
  }
}

__global__ __launch_bounds__(kCgBlock) void cg_update_kernel(
    int64_t n, int nb, const double* __restrict__ dinv, double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ z, const double* __restrict__ p,
    const double* __restrict__ q, const double* __restrict__ part_pq, double* __restrict__ part,
    const CGState* __restrict__ st, int parity) {
  __shared__ double red[4 * kCgBlock];
  const int a0 = st->active[parity][0], a1 = st->active[parity][1];
  if (!a0 && !a1) return;
  double pq[2];
  sum_partials(part_pq, nb, 2, pq, red);
  const double alpha[2] = {a0 ? st->rz[parity][0] / pq[0] : 0.0, a1 ? st->rz[parity][1] / pq[1] : 0.0};
  const int64_t i = (int64_t)blockIdx.x * kCgBlock + threadIdx.x;
  double v[4] = {0, 0, 0, 0};   // rz0 rz1 rr0 rr1
  if (i < n) {
    for (int s = 0; s < 2; ++s) {
      if (!(s ? a1 : a0)) continue;
      x[s * n + i] = fma(alpha[s], p[s * n + i], x[s * n + i]);
      const double ri = fma(-alpha[s], q[s * n + i], r[s * n + i]);
      const double zi = dinv[i] * ri;
      r[s * n + i] = ri;
      z[s * n + i] = zi;
      v[s] = ri * zi;
      v[2 + s] = ri * ri;
    }
  }
  block_reduce(v, 4, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < 4; ++j) part[blockIdx.x * 8 + j] = v[j];
}

__global__ __launch_bounds__(kCgBlock) void cg_pupdate_kernel(
    int64_t n, int nb, const double* __restrict__ z, double* __restrict__ p,
    const double* __restrict__ part, CGState* __restrict__ st, int parity, double tol) {
  const int a0 = st->active[parity][0], a1 = st->active[parity][1];
  if (!a0 && !a1) {
    // both frozen: carry the state into the other parity slot
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      for (int s = 0; s < 2; ++s) {
        st->rz[parity ^ 1][s] = st->rz[parity][s];
        st->active[parity ^ 1][s] = 0;
      }
    }
    return;
  }
  __shared__ double red[4 * kCgBlock];
  double v[4];
  sum_partials(part, nb, 4, v, red);
  const int act[2] = {a0, a1};
  double beta[2];
  for (int s = 0; s < 2; ++s) beta[s] = act[s] ? v[s] / st->rz[parity][s] : 0.0;
  const int64_t i = (int64_t)blockIdx.x * kCgBlock + threadIdx.x;
  if (i < n) {
    for (int s = 0; s < 2; ++s)
      if (act[s]) p[s * n + i] = fma(beta[s], p[s * n + i], z[s * n + i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int s = 0; s < 2; ++s) {
      if (act[s]) {
        st->rz[parity ^ 1][s] = v[s];
        st->rr[s] = v[2 + s];
        st->iters[s] += 1;
        st->active[parity ^ 1][s] = v[2 + s] > tol * tol * st->bb[s] ? 1 : 0;
      } else {
        st->rz[parity ^ 1][s] = st->rz[parity][s];
        st->active[parity ^ 1][s] = 0;
      }
    }
  }
}

// Admissible state at every material point from u, eta (whitened):
//   w_eps = L^T B u,  w_sig = w_sig* + L^T B eta;  optionally raw eps = B u,
//   sig = sig* + C B eta with C B eta = L (L^T B eta).
// Eight lanes per material point, lane a taking element node a.  The node
// sums meet in an xor butterfly, which leaves the same sums in all eight lanes
// (each step adds the same two values on both partners); lane r < 6 then
// writes row r.
__global__ __launch_bounds__(256) void recover_kernel(int nx, int ny, int nz, BOps Bo, Mat6 LT,
                                                      Mat6 L,
                                                      const double* __restrict__ x /*[2][n_dof]*/,
                                                      int64_t n_dof, const double* __restrict__ zw,
                                                      const double* __restrict__ zc,
                                                      double* __restrict__ yw,
                                                      double* __restrict__ eps_raw,
                                                      double* __restrict__ sig_raw) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mp = gid >> 3;
  const int a = (int)(gid & 7);
  const int64_t n_mp = 8 * (int64_t)nx * ny * nz;
  if (mp >= n_mp) return;   // whole groups of eight leave together
  const int g = (int)(mp % 8);
  const int64_t el = mp / 8;
  const int ex = (int)(el % nx), ey = (int)((el / nx) % ny), ez = (int)(el / ((int64_t)nx * ny));
  double eu[6] = {0, 0, 0, 0, 0, 0}, ee[6] = {0, 0, 0, 0, 0, 0};
  const int64_t nd = dnode(nx, ny, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
  for (int c = 0; c < 3; ++c) {
    const double uv = x[3 * nd + c], ev = x[n_dof + 3 * nd + c];
    for (int r = 0; r < 6; ++r) {
      const double bv = Bo.B[g][24 * r + 3 * a + c];
      eu[r] = fma(bv, uv, eu[r]);
      ee[r] = fma(bv, ev, ee[r]);
    }
  }
  for (int m = 1; m < 8; m <<= 1) {
    for (int r = 0; r < 6; ++r) {
      eu[r] += __shfl_xor(eu[r], m, 8);
      ee[r] += __shfl_xor(ee[r], m, 8);
    }
  }
  if (a >= 6) return;
  const int r = a;
  double we = 0.0, ws = 0.0, eur = 0.0;
  for (int c = 0; c < 6; ++c) {
    we = fma(LT.a[6 * r + c], eu[c], we);
    ws = fma(LT.a[6 * r + c], ee[c], ws);
    eur = (c == r) ? eu[c] : eur;
  }
  yw[12 * mp + r] = we;
  yw[12 * mp + 6 + r] = zw[12 * mp + 6 + r] + ws;
  if (eps_raw) {
    double cb = 0.0;
    for (int c = 0; c < 6; ++c) {
      double wsc = 0.0;
      for (int k = 0; k < 6; ++k) wsc = fma(LT.a[6 * c + k], ee[k], wsc);
      cb = fma(L.a[6 * r + c], wsc, cb);
    }
    eps_raw[6 * mp + r] = eur;
    sig_raw[6 * mp + r] = zc[12 * mp + 6 + r] + cb;
  }
}

// Deterministic per-iteration scalars over the material points:
//   out[0] = sum_e w 1/2 |y_e - z_e|^2 (D_half), out[1] = sum_e w dist_e (D_full),
//   out[2] = #{idx_new != idx_old}.
// out[3] holds a ticket (u32, zero between launches) and out[4 + 3b ..] the
// partial sums of block b.  Block b sums a fixed range of material points (the
// squared differences read as one flat, coalesced array), its waves reduce in a
// fixed shuffle order and the block stores its partials; the block that takes
// the last ticket adds the partials in block order and resets the ticket, so
// the result does not depend on which block finishes last.
constexpr int kScalBlocks = 32;
__global__ __launch_bounds__(256) void iter_scalars_kernel(
    int64_t n_mp, double w, const double* __restrict__ yw, const double* __restrict__ zw,
    const double* __restrict__ dist, const int64_t* __restrict__ idx_new,
    const int64_t* __restrict__ idx_old, double* out) {
  const int t = threadIdx.x;
  const int64_t chunk = (n_mp + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = min(n_mp, (int64_t)blockIdx.x * chunk);
  const int64_t e1 = min(n_mp, e0 + chunk);
  double dh = 0.0, df = 0.0, ch = 0.0;
  for (int64_t f = 12 * e0 + t; f < 12 * e1; f += 256) {
    const double d = yw[f] - zw[f];
    dh = fma(d, d, dh);
  }
  for (int64_t e = e0 + t; e < e1; e += 256) {
    df += dist[e];
    ch += (idx_new[e] != idx_old[e]) ? 1.0 : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    dh += __shfl_down(dh, off);
    df += __shfl_down(df, off);
    ch += __shfl_down(ch, off);
  }
  __shared__ double ws[3][4];
  __shared__ int last;
  if ((t & 63) == 0) {
    ws[0][t >> 6] = dh;
    ws[1][t >> 6] = df;
    ws[2][t >> 6] = ch;
  }
  __syncthreads();
  if (t == 0) {
    double* part = out + 4 + 3 * blockIdx.x;
    for (int k = 0; k < 3; ++k) part[k] = ((ws[k][0] + ws[k][1]) + ws[k][2]) + ws[k][3];
    __threadfence();
    last = atomicAdd(reinterpret_cast<unsigned*>(out + 3), 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (t < 3) {
    const volatile double* part = out + 4;
    double sum = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) sum += part[3 * b + t];
    out[t] = t == 0 ? 0.5 * w * sum : (t == 1 ? w * sum : sum);
  }
  if (t == 0) *reinterpret_cast<volatile unsigned*>(out + 3) = 0u;
}

// Unmoved material points (exact ANN projections).  If the state y moved by
// delta < (d2 - d1)/2 from the reference state q at which the nearest (d1) and
// second nearest (d2) distances were certified, every other data point stays
// farther from y than the nearest one: d(y, x) >= d2 - delta > d1 + delta >=
// d(y, p1).  gap holds (d2 - d1)/2 less a margin far above the FP64 rounding of
// the distances; NaN or negative = no certified gap.  Skipped points keep their
// association and get the FP64 direct-form distance of the projection's rerank;
// the others are compacted (list order does not affect any result).
__global__ void skip_kernel(int64_t nm, const double* __restrict__ yw,
                            const double* __restrict__ qref, const double* __restrict__ gap,
                            const int64_t* __restrict__ idx, const uint32_t* __restrict__ iperm,
                            const double* __restrict__ w64, int64_t* __restrict__ idx_new,
                            double* __restrict__ dist, int* __restrict__ list, int* __restrict__ cnt,
                            double* __restrict__ qc, int64_t* __restrict__ wc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nm) return;
  double y[12], dl = 0.0;
  for (int k = 0; k < 12; ++k) {
    y[k] = yw[12 * e + k];
    const double t = y[k] - qref[12 * e + k];
    dl = fma(t, t, dl);
  }
  const double g = gap[e];
  if (g > 0.0 && dl < g * g) {
    const int64_t j = idx[e];
    const int64_t p = iperm[j];
    double d = 0.0;
    for (int k = 0; k < 12; ++k) {
      const double t = y[k] - w64[12 * p + k];
      d = fma(t, t, d);
    }
    idx_new[e] = j;
    dist[e] = 0.5 * d;
  } else {
    const int k = atomicAdd(cnt, 1);
    list[k] = (int)e;
    for (int c = 0; c < 12; ++c) qc[12 * (int64_t)k + c] = y[c];
    wc[k] = idx[e];
  }
}

__global__ void unskip_kernel(int n, const int* __restrict__ list, const int64_t* __restrict__ ic,
                              const double* __restrict__ dc, const double* __restrict__ d2c,
                              const double* __restrict__ qc, int64_t* __restrict__ idx_new,
                              double* __restrict__ dist, double* __restrict__ qref,
                              double* __restrict__ gap) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t e = list[k];
  idx_new[e] = ic[k];
  dist[e] = dc[k];
  for (int c = 0; c < 12; ++c) qref[12 * e + c] = qc[12 * (int64_t)k + c];
  if (d2c[k] >= 0.0 && ic[k] >= 0) {
    const double d1 = sqrt(2.0 * dc[k]), d2 = sqrt(2.0 * d2c[k]);
    gap[e] = 0.5 * (d2 - d1) - 1e-9 * d2 - 1e-12;
  } else {
    gap[e] = -1.0;
  }
}

// Accuracy of each material point's search from its latest local distance
// d_e (the distance of the previous projection) and the latest global one
// (the mean local distance dbar = D_full / sum of the weights) at an iteration
// whose schedule gives the radius factor f and the leaf budget b (Section 4's
// accuracy parameter as a function of the global distance, the local distance
// and the iteration).  With rho = d_e / dbar, points at least as far from the
// data as the mean keep (f, b); nearer points get more accuracy, up to the
// exact search at the data: f_e = f + (1 - f)(1 - rho), b_e = b ceil(1 / rho)
// (at most 16 b).
__global__ void local_accuracy_kernel(int64_t nm, const double* __restrict__ dist, double inv_dbar,
                                      float f, int b, float* __restrict__ fdq,
                                      int* __restrict__ bq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nm) return;
  const double rho = dist[e] * inv_dbar;
  const double near = rho < 1.0 ? 1.0 - rho : 0.0;
  fdq[e] = (float)fmin(1.0, (double)f + (1.0 - (double)f) * near);
  int be = b;
  if (b > 0 && rho < 1.0) be = b * (int)fmin(16.0, ceil(1.0 / fmax(rho, 1.0 / 16.0)));
  bq[e] = be;
}

static unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---------------------------------------------------------------------------
// Solver object
// ---------------------------------------------------------------------------
dd_status DDSolver::setup(const Dataset& D, const dd_mesh& mesh, const uint8_t* mask,
                          const double* force, const dd_solve_opts* opts, hipStream_t st) {
  if (!(D.packs & DD_PACK_FP64))
    return set_error(DD_ERR_UNSUPPORTED, "dd_solve needs the dataset's FP64 pack");
  if (mesh.nx < 1 || mesh.ny < 1 || mesh.nz < 1 || !(mesh.lx > 0) || !(mesh.ly > 0) ||
      !(mesh.lz > 0))
    return set_error(DD_ERR_ARG, "mesh needs nx, ny, nz >= 1 and positive edge lengths");
  if ((int64_t)mesh.nx * mesh.ny * mesh.nz > (1 << 24))
    return set_error(DD_ERR_TOO_LARGE, "mesh too large");
  ds = &D;
  M.init(mesh);
  this->st = st;
  mode = opts ? opts->mode : DD_EXACT_FP64;
  ann_budget = opts ? opts->ann_budget : 0;
  ann_ramp = opts ? opts->ann_ramp : 0;
  if (ann_budget < 0 || ann_ramp < 0)
    return set_error(DD_ERR_ARG, "dd_solve_opts: ann_budget and ann_ramp must be >= 0");
  {
    const double discount = opts ? opts->ann_radius_discount : 0.0;
    if (!(discount >= 0.0 && discount <= 1.0))
      return set_error(DD_ERR_ARG, "dd_solve_opts: ann_radius_discount must be in [0, 1]");
    if (discount > 0.0 && mode != DD_KMEANS)
      return set_error(DD_ERR_ARG, "dd_solve_opts: ann_radius_discount applies to DD_KMEANS only");
    ann_fd = 1.0 - discount;
  }
  if (opts && (opts->flags & ~(DD_SOLVE_NO_GRAPH | DD_SOLVE_CG | DD_SOLVE_SKIP |
                               DD_SOLVE_LOCAL_ACCURACY)))
    return set_error(DD_ERR_ARG, "dd_solve_opts: unknown flag bits");
  use_graph = !(opts && (opts->flags & DD_SOLVE_NO_GRAPH));
  cg_tol = (opts && opts->cg_tol > 0) ? opts->cg_tol : 1e-13;
  cg_max_iter = (opts && opts->cg_max_iter > 0) ? opts->cg_max_iter : 20000;
  // Cholesky factor of the metric for the whitened/raw conversions
  double Lm[36], LT[36];
  cholesky6(D.C, Lm);
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) LT[6 * r + c] = Lm[6 * c + r];
  std::memcpy(L, Lm, sizeof(L));
  std::memcpy(Lt, LT, sizeof(Lt));
  const int64_t nd = M.n_dof, nm = M.n_mp;
  const bool want_dense = nd <= kDenseMaxDof && !(opts && (opts->flags & DD_SOLVE_CG));
  if (want_dense) dense = dense_inverse_cached(D, M, mask);
  // the CSR matrix is needed by CG, or once to form K^-1
  const bool need_csr = !dense;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val, dinv;
  if (need_csr) assemble_csr(M, D.C, mask, rowptr, col, val, dinv);
  nnz = (int64_t)col.size();
  const int64_t nb = (nd + kCgBlock - 1) / kCgBlock;
  const int64_t nbs = (nd + kRowsPerBlock - 1) / kRowsPerBlock;
  // one device allocation carved into the solver's buffers (256-byte aligned)
  struct Part {
    DevBuf* buf;
    size_t bytes;
  };
  // prescribed displacements: u_D on Dirichlet DOFs and the lifting K_fd u_D
  std::vector<double> uD, lift;
  const double* vals = opts ? opts->dirichlet_values : nullptr;
  if (vals) {
    uD.assign(nd, 0.0);
    lift.assign(nd, 0.0);
    bool any = false;
    for (int64_t d = 0; d < nd; ++d) {
      if (!std::isfinite(vals[d])) return set_error(DD_ERR_ARG, "non-finite Dirichlet value");
      if (mask[d] && vals[d] != 0.0) {
        uD[d] = vals[d];
        any = true;
      }
    }
    if (any) {
      double Ke[24 * 24];
      element_stiffness(M, D.C, Ke);
      for (int ez = 0; ez < M.nz; ++ez)
        for (int ey = 0; ey < M.ny; ++ey)
          for (int ex = 0; ex < M.nx; ++ex) {
            int64_t g[24];
            double ue[24];
            bool nz = false;
            for (int a = 0; a < 8; ++a) {
              const int64_t nid = M.node(ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
              for (int c = 0; c < 3; ++c) {
                g[3 * a + c] = 3 * nid + c;
                ue[3 * a + c] = uD[3 * nid + c];
                nz = nz || ue[3 * a + c] != 0.0;
              }
            }
            if (!nz) continue;
            for (int i = 0; i < 24; ++i) {
              if (mask[g[i]]) continue;
              double acc = 0.0;
              for (int j = 0; j < 24; ++j) acc += Ke[24 * i + j] * ue[j];
              lift[g[i]] += acc;
            }
          }
    } else {
      uD.clear();
      lift.clear();
    }
  }
  std::vector<Part> parts = {
      {&d_mask, (size_t)nd}, {&d_f, sizeof(double) * nd}, {&d_b, sizeof(double) * 2 * nd},
      {&d_x, sizeof(double) * 2 * nd}, {&d_idx, sizeof(int64_t) * nm},
      {&d_idx_new, sizeof(int64_t) * nm}, {&d_dist, sizeof(double) * nm},
      {&d_zw, sizeof(double) * 12 * nm}, {&d_zc, sizeof(double) * 12 * nm},
      {&d_yw, sizeof(double) * 12 * nm}, {&d_scal, sizeof(double) * (4 + 3 * kScalBlocks)},
      {&d_cgstat, 64}};
  if (!uD.empty()) {
    parts.push_back({&d_uD, sizeof(double) * nd});
    parts.push_back({&d_lift, sizeof(double) * nd});
  }
  if (need_csr) {
    parts.push_back({&d_rowptr, sizeof(int32_t) * (nd + 1)});
    parts.push_back({&d_col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)});
    parts.push_back({&d_val, sizeof(double) * std::max<int64_t>(nnz, 1)});
  }
  if (!want_dense) {   // CG state
    parts.push_back({&d_dinv, sizeof(double) * nd});
    parts.push_back({&d_work, sizeof(double) * 8 * nd});
    parts.push_back({&d_part, sizeof(double) * 8 * (nb + nbs)});
    parts.push_back({&d_cgstate, sizeof(CGState)});
  }
  size_t total = 0;
  for (const Part& q : parts) total += (q.bytes + 255) / 256 * 256;
  DD_TRY(arena.alloc(total));
  {
    char* base = arena.as<char>();
    for (const Part& q : parts) {
      q.buf->view(base, q.bytes);
      base += (q.bytes + 255) / 256 * 256;
    }
  }
  if (need_csr) {
    DD_HIP(hipMemcpyAsync(d_rowptr.p, rowptr.data(), sizeof(int32_t) * (nd + 1),
                          hipMemcpyHostToDevice, st));
    if (nnz) {
      DD_HIP(hipMemcpyAsync(d_col.p, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
      DD_HIP(hipMemcpyAsync(d_val.p, val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
    }
  }
  if (!want_dense)
    DD_HIP(hipMemcpyAsync(d_dinv.p, dinv.data(), sizeof(double) * nd, hipMemcpyHostToDevice, st));
  if (!uD.empty()) {
    DD_HIP(hipMemcpyAsync(d_uD.p, uD.data(), sizeof(double) * nd, hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(d_lift.p, lift.data(), sizeof(double) * nd, hipMemcpyHostToDevice, st));
  }
  DD_HIP(hipMemcpyAsync(d_mask.p, mask, nd, hipMemcpyHostToDevice, st));
  DD_HIP(hipMemcpyAsync(d_f.p, force, sizeof(double) * nd, hipMemcpyHostToDevice, st));
  DD_HIP(hipMemsetAsync(d_x.p, 0, sizeof(double) * 2 * nd, st));
  DD_HIP(hipMemsetAsync(d_cgstat.p, 0, 64, st));
  DD_HIP(hipMemsetAsync(d_scal.p, 0, d_scal.bytes, st));   // the scalars kernel's ticket
  if (want_dense && !dense)
    DD_TRY(dense_inverse_for(D, M, mask, d_rowptr.as<int32_t>(), d_col.as<int32_t>(),
                             d_val.as<double>(), dense, st));
  skip_on = (walk_mode(mode) && ann_budget == 0 && fd_at(1) >= 1.0 && opts &&
             (opts->flags & DD_SOLVE_SKIP));
  local_on = walk_mode(mode) && opts && (opts->flags & DD_SOLVE_LOCAL_ACCURACY) &&
             (ann_budget > 0 || ann_fd < 1.0);
  last_full = INFINITY;
  if (local_on) {
    DD_TRY(d_fdq.alloc(sizeof(float) * nm));
    DD_TRY(d_budq.alloc(sizeof(int) * nm));
  }
  if (skip_on) {
    DD_TRY(d_qref.alloc(sizeof(double) * 12 * nm));
    DD_TRY(d_gap.alloc(sizeof(double) * nm));
    DD_TRY(d_list.alloc(sizeof(int) * nm));
    DD_TRY(d_cnt.alloc(sizeof(int)));
    DD_TRY(d_qc.alloc(sizeof(double) * 12 * nm));
    DD_TRY(d_wc.alloc(sizeof(int64_t) * nm));
    DD_TRY(d_ic.alloc(sizeof(int64_t) * nm));
    DD_TRY(d_dc.alloc(sizeof(double) * nm));
    DD_TRY(d_d2c.alloc(sizeof(double) * nm));
    DD_HIP(hipMemsetAsync(d_gap.p, 0xFF, sizeof(double) * nm, st));   // NaN: no gap yet
    DD_HIP(hipMemsetAsync(d_qref.p, 0, sizeof(double) * 12 * nm, st));
  }
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

dd_status DDSolver::project_step(int it) {
  const int64_t nm = M.n_mp;
  if (local_on && approximate_at(it) && std::isfinite(last_full) && last_full > 0.0) {
    const double dbar = last_full / ((double)nm * M.w);
    hipLaunchKernelGGL(local_accuracy_kernel, dim3(g256(nm)), dim3(256), 0, st, nm,
                       d_dist.as<double>(), 1.0 / dbar, (float)fd_at(it), budget_at(it),
                       d_fdq.as<float>(), d_budq.as<int>());
    DD_HIP(hipGetLastError());
    return project_whitened(*ds, d_yw.as<double>(), nm, d_idx.as<int64_t>(), mode, budget_at(it),
                            d_idx_new.as<int64_t>(), d_dist.as<double>(), st, nullptr, fd_at(it),
                            0, d_fdq.as<float>(), d_budq.as<int>());
  }
  if (!skip_on)
    return project_whitened(*ds, d_yw.as<double>(), nm, d_idx.as<int64_t>(), mode, budget_at(it),
                            d_idx_new.as<int64_t>(), d_dist.as<double>(), st, nullptr, fd_at(it),
                            scan_passes(it));
  DD_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(skip_kernel, dim3(g256(nm)), dim3(256), 0, st, nm, d_yw.as<double>(),
                     d_qref.as<double>(), d_gap.as<double>(), d_idx.as<int64_t>(),
                     ds->iperm.as<uint32_t>(), ds->w64.as<double>(), d_idx_new.as<int64_t>(),
                     d_dist.as<double>(), d_list.as<int>(), d_cnt.as<int>(), d_qc.as<double>(),
                     d_wc.as<int64_t>());
  DD_HIP(hipGetLastError());
  int n = 0;
  DD_HIP(hipMemcpyAsync(&n, d_cnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  skipped_total += nm - n;
  if (n == 0) return DD_OK;
  DD_TRY(project_whitened(*ds, d_qc.as<double>(), n, d_wc.as<int64_t>(), mode, 0,
                          d_ic.as<int64_t>(), d_dc.as<double>(), st, d_d2c.as<double>()));
  hipLaunchKernelGGL(unskip_kernel, dim3(g256(n)), dim3(256), 0, st, n, d_list.as<int>(),
                     d_ic.as<int64_t>(), d_dc.as<double>(), d_d2c.as<double>(), d_qc.as<double>(),
                     d_idx_new.as<int64_t>(), d_dist.as<double>(), d_qref.as<double>(),
                     d_gap.as<double>());
  DD_HIP(hipGetLastError());
  return DD_OK;
}

DDSolver::~DDSolver() {
  if (cg_graph) (void)hipGraphExecDestroy(cg_graph);
  for (hipEvent_t e : {ev_cg, ev_ready, ev_scal})
    if (e) (void)hipEventDestroy(e);
  if (h_pin) (void)hipHostFree(h_pin);
}

// Device bytes setup() allocates for a mesh (the CSR pattern bounded by 81
// couplings per row: 27 nodes x 3 components).
int64_t DDSolver::footprint_bytes(const dd_mesh& m) {
  const int64_t nd = 3 * (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  const int64_t nm = 8 * (int64_t)m.nx * m.ny * m.nz;
  const int64_t nnz = 81 * nd;
  const int64_t nb = (nd + kCgBlock - 1) / kCgBlock, nbs = (nd + kRowsPerBlock - 1) / kRowsPerBlock;
  return 4 * (nd + 1) + 12 * nnz + (8 + 1 + 8 + 16 + 16 + 64) * nd + (8 + 8 + 8 + 3 * 96) * nm +
         8 * (4 + 3 * kScalBlocks) + 64 + 64 * (nb + nbs) + (int64_t)sizeof(CGState);
}

int64_t DDSolver::inverse_bytes(const dd_mesh& m) {
  const int64_t nd = 3 * (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  if (nd > kDenseMaxDof) return 0;
  const int64_t n_pad = (nd + 63) / 64 * 64;   // the Gauss-Jordan block size
  return n_pad * n_pad * (int64_t)sizeof(double);
}

bool DDSolver::inverse_cached(const Dataset& D, const dd_mesh& m, const uint8_t* mask) {
  std::unique_ptr<FEMesh> M(new FEMesh());
  M->init(m);
  return dense_inverse_cached(D, *M, mask) != nullptr;
}

dd_status DDSolver::prepare_inverse(const Dataset& D, const dd_mesh& m, const uint8_t* mask,
                                    hipStream_t st) {
  std::unique_ptr<FEMesh> M(new FEMesh());
  M->init(m);
  if (M->n_dof > kDenseMaxDof || dense_inverse_cached(D, *M, mask)) return DD_OK;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val, dinv;
  assemble_csr(*M, D.C, mask, rowptr, col, val, dinv);
  DevBuf r, c, v;
  DD_TRY(r.alloc(sizeof(int32_t) * rowptr.size()));
  DD_TRY(c.alloc(sizeof(int32_t) * std::max<size_t>(col.size(), 1)));
  DD_TRY(v.alloc(sizeof(double) * std::max<size_t>(val.size(), 1)));
  DD_HIP(hipMemcpyAsync(r.p, rowptr.data(), sizeof(int32_t) * rowptr.size(), hipMemcpyHostToDevice, st));
  if (!col.empty()) {
    DD_HIP(hipMemcpyAsync(c.p, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(v.p, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, st));
  }
  std::shared_ptr<DenseInverse> out;
  DD_TRY(dense_inverse_for(D, *M, mask, r.as<int32_t>(), c.as<int32_t>(), v.as<double>(), out, st));
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

// Pinned layout: [0, 128) CG state, [128, 152) iteration scalars, [160, 164) bad flag.
dd_status DDSolver::async_init() {
  static_assert(sizeof(CGState) <= 128, "CG state mirror");
  if (!h_pin) DD_HIP(hipHostMalloc((void**)&h_pin, 256, hipHostMallocDefault));
  for (hipEvent_t* e : {&ev_cg, &ev_ready, &ev_scal})
    if (!*e) DD_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return DD_OK;
}

dd_status DDSolver::pc_begin() {
  const int64_t nd = M.n_dof, nm = M.n_mp;
  Mat6 Lm;
  std::memcpy(Lm.a, L, sizeof(L));
  BOps Bo;
  std::memcpy(Bo.B, M.B, sizeof(Bo.B));
  hipLaunchKernelGGL(gather_z_kernel, dim3(g256(nm)), dim3(256), 0, st, d_idx.as<int64_t>(), nm,
                     ds->N, ds->iperm.as<uint32_t>(), ds->w64.as<double>(), Lm, d_zw.as<double>(),
                     d_zc.as<double>(), reinterpret_cast<int*>(d_cgstat.as<char>() + 32));
  hipLaunchKernelGGL(assemble_rhs_kernel, dim3(g256(64 * nd)), dim3(256), 0, st, M.nx, M.ny, M.nz, M.w,
                     Bo, d_zc.as<double>(), d_mask.as<uint8_t>(), d_f.as<double>(),
                     d_uD.as<double>(), d_lift.as<double>(), d_b.as<double>(),
                     d_b.as<double>() + nd);
  cg_it = 0;
  if (dense) {
    DD_TRY(dense_apply(*dense, d_b.as<double>(), d_x.as<double>(), st));
    return DD_OK;
  }
  const int nb = (int)((nd + kCgBlock - 1) / kCgBlock);
  double* wk = d_work.as<double>();
  hipLaunchKernelGGL(cg_init_kernel, dim3(nb), dim3(kCgBlock), 0, st, nd, d_rowptr.as<int32_t>(),
                     d_col.as<int32_t>(), d_val.as<double>(), d_dinv.as<double>(), d_b.as<double>(),
                     d_x.as<double>(), wk, wk + 2 * nd, wk + 4 * nd, d_part.as<double>());
  hipLaunchKernelGGL(cg_init_finish_kernel, dim3(1), dim3(kCgBlock), 0, st, d_part.as<double>(), nb,
                     cg_tol, d_cgstate.as<CGState>());
  DD_HIP(hipGetLastError());
  cg_it = 0;
  return DD_OK;
}

dd_status DDSolver::cg_batch() {
  if (dense) {   // the product was enqueued by pc_begin
    DD_HIP(hipEventRecord(ev_cg, st));
    return DD_OK;
  }
  const int64_t nd = M.n_dof;
  const int nb = (int)((nd + kCgBlock - 1) / kCgBlock);
  const int nbs = (int)((nd + kRowsPerBlock - 1) / kRowsPerBlock);
  double* wk = d_work.as<double>();
  double *r = wk, *z = wk + 2 * nd, *p = wk + 4 * nd, *q = wk + 6 * nd;
  double* part = d_part.as<double>();
  double* part2 = part + 8 * (int64_t)nb;
  CGState* cs = d_cgstate.as<CGState>();
  const int32_t *rp = d_rowptr.as<int32_t>(), *cl = d_col.as<int32_t>();
  const double* vl = d_val.as<double>();
  const int count = std::min(kCgPoll, cg_max_iter - cg_it);
  for (int k = 0; k < count; ++k) {
    const int par = (cg_it + k) & 1;
    hipLaunchKernelGGL(cg_spmv_kernel, dim3(nbs), dim3(kCgBlock), 0, st, nd, rp, cl, vl, p, q, part2,
                       cs, par);
    hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(kCgBlock), 0, st, nd, nbs,
                       d_dinv.as<double>(), d_x.as<double>(), r, z, p, q, part2, part, cs, par);
    hipLaunchKernelGGL(cg_pupdate_kernel, dim3(nb), dim3(kCgBlock), 0, st, nd, nb, z, p, part, cs,
                       par, cg_tol);
  }
  cg_it += count;
  DD_HIP(hipGetLastError());
  DD_HIP(hipMemcpyAsync(h_pin, cs, sizeof(CGState), hipMemcpyDeviceToHost, st));
  DD_HIP(hipEventRecord(ev_cg, st));
  return DD_OK;
}

bool DDSolver::cg_finished() const {
  if (dense) return true;
  CGState hs;
  std::memcpy(&hs, h_pin, sizeof(hs));
  return cg_it >= cg_max_iter || (!hs.active[cg_it & 1][0] && !hs.active[cg_it & 1][1]);
}

dd_status DDSolver::pc_end() {
  if (dense) {
    cg_last_iters[0] = cg_last_iters[1] = 0;
    cg_last_res[0] = cg_last_res[1] = 0.0;
  } else {
    CGState hs;
    std::memcpy(&hs, h_pin, sizeof(hs));
    cg_last_iters[0] = hs.iters[0];
    cg_last_iters[1] = hs.iters[1];
    cg_last_res[0] = hs.bb[0] > 0 ? std::sqrt(hs.rr[0] / hs.bb[0]) : 0.0;
    cg_last_res[1] = hs.bb[1] > 0 ? std::sqrt(hs.rr[1] / hs.bb[1]) : 0.0;
  }
  const int64_t nd = M.n_dof, nm = M.n_mp;
  Mat6 Lm, LTm;
  std::memcpy(Lm.a, L, sizeof(L));
  std::memcpy(LTm.a, Lt, sizeof(Lt));
  BOps Bo;
  std::memcpy(Bo.B, M.B, sizeof(Bo.B));
  hipLaunchKernelGGL(recover_kernel, dim3(g256(8 * nm)), dim3(256), 0, st, M.nx, M.ny, M.nz, Bo, LTm, Lm,
                     d_x.as<double>(), nd, d_zw.as<double>(), d_zc.as<double>(), d_yw.as<double>(),
                     (double*)nullptr, (double*)nullptr);
  DD_HIP(hipGetLastError());
  DD_HIP(hipEventRecord(ev_ready, st));
  return DD_OK;
}

dd_status DDSolver::scalars_begin() {
  const int64_t nm = M.n_mp;
  hipLaunchKernelGGL(iter_scalars_kernel, dim3(kScalBlocks), dim3(256), 0, st, nm, M.w, d_yw.as<double>(),
                     d_zw.as<double>(), d_dist.as<double>(), d_idx_new.as<int64_t>(),
                     d_idx.as<int64_t>(), d_scal.as<double>());
  DD_HIP(hipGetLastError());
  DD_HIP(hipMemcpyAsync(h_pin + 128, d_scal.p, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  DD_HIP(hipMemcpyAsync(h_pin + 160, d_cgstat.as<char>() + 32, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipEventRecord(ev_scal, st));
  return DD_OK;
}

void DDSolver::scalars_end(double sc[3], int* bad) {
  std::memcpy(sc, h_pin + 128, 3 * sizeof(double));
  std::memcpy(bad, h_pin + 160, sizeof(int));
  std::swap(d_idx.p, d_idx_new.p);
}

dd_status DDSolver::set_assignment(const int64_t* idx_host) {
  const int64_t nm = M.n_mp;
  for (int64_t e = 0; e < nm; ++e)
    if (idx_host[e] < 0 || idx_host[e] >= ds->N) return set_error(DD_ERR_ARG, "init_idx out of range");
  DD_HIP(hipMemcpyAsync(d_idx.p, idx_host, sizeof(int64_t) * nm, hipMemcpyHostToDevice, st));
  return DD_OK;
}

dd_status DDSolver::cg_solve() {
  if (dense) {
    DD_TRY(dense_apply(*dense, d_b.as<double>(), d_x.as<double>(), st));
    cg_last_iters[0] = cg_last_iters[1] = 0;
    cg_last_res[0] = cg_last_res[1] = 0.0;
    return DD_OK;
  }
  const int64_t nd = M.n_dof;
  const int nb = (int)((nd + kCgBlock - 1) / kCgBlock);
  const int nbs = (int)((nd + kRowsPerBlock - 1) / kRowsPerBlock);   // SpMV blocks
  double* wk = d_work.as<double>();
  double *r = wk, *z = wk + 2 * nd, *p = wk + 4 * nd, *q = wk + 6 * nd;
  double* part = d_part.as<double>();
  double* part2 = part + 8 * (int64_t)nb;
  CGState* cs = d_cgstate.as<CGState>();
  const int32_t *rp = d_rowptr.as<int32_t>(), *cl = d_col.as<int32_t>();
  const double* vl = d_val.as<double>();
  hipLaunchKernelGGL(cg_init_kernel, dim3(nb), dim3(kCgBlock), 0, st, nd, rp, cl, vl,
                     d_dinv.as<double>(), d_b.as<double>(), d_x.as<double>(), r, z, p, part);
  hipLaunchKernelGGL(cg_init_finish_kernel, dim3(1), dim3(kCgBlock), 0, st, part, nb, cg_tol, cs);
  DD_HIP(hipGetLastError());
  CGState hs;
  int it = 0;
  const int poll = kCgPoll;
  auto enqueue = [&](hipStream_t s, int it0, int count) {
    for (int k = 0; k < count; ++k) {
      const int par = (it0 + k) & 1;
      hipLaunchKernelGGL(cg_spmv_kernel, dim3(nbs), dim3(kCgBlock), 0, s, nd, rp, cl, vl, p, q,
                         part2, cs, par);
      hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(kCgBlock), 0, s, nd, nbs,
                         d_dinv.as<double>(), d_x.as<double>(), r, z, p, q, part2, part, cs, par);
      hipLaunchKernelGGL(cg_pupdate_kernel, dim3(nb), dim3(kCgBlock), 0, s, nd, nb, z, p, part, cs,
                         par, cg_tol);
    }
  };
  if (use_graph && !cg_graph) {
    // one batch of kCgPoll iterations (even start, so the parity sequence is
    // fixed) captured on a private stream, replayed on the solver's stream
    hipStream_t cap;
    DD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      enqueue(cap, 0, poll);
      e = hipStreamEndCapture(cap, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&cg_graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      cg_graph = nullptr;
      use_graph = false;   // fall back to eager launches
      (void)hipGetLastError();
    }
  }
  while (it < cg_max_iter) {
    if (use_graph && cg_graph && it + poll <= cg_max_iter) {
      DD_HIP(hipGraphLaunch(cg_graph, st));
      it += poll;
    } else {
      const int count = std::min(poll, cg_max_iter - it);
      enqueue(st, it, count);
      it += count;
    }
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpyAsync(&hs, cs, sizeof(hs), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    if (!hs.active[it & 1][0] && !hs.active[it & 1][1]) break;
  }
  cg_last_iters[0] = hs.iters[0];
  cg_last_iters[1] = hs.iters[1];
  cg_last_res[0] = hs.bb[0] > 0 ? std::sqrt(hs.rr[0] / hs.bb[0]) : 0.0;
  cg_last_res[1] = hs.bb[1] > 0 ? std::sqrt(hs.rr[1] / hs.bb[1]) : 0.0;
  return DD_OK;
}

dd_status DDSolver::constraint_projection() {
  const int64_t nd = M.n_dof, nm = M.n_mp;
  Mat6 Lm, LTm;
  std::memcpy(Lm.a, L, sizeof(L));
  std::memcpy(LTm.a, Lt, sizeof(Lt));
  BOps Bo;
  std::memcpy(Bo.B, M.B, sizeof(Bo.B));
  hipLaunchKernelGGL(gather_z_kernel, dim3(g256(nm)), dim3(256), 0, st, d_idx.as<int64_t>(), nm,
                     ds->N, ds->iperm.as<uint32_t>(), ds->w64.as<double>(), Lm, d_zw.as<double>(),
                     d_zc.as<double>(), reinterpret_cast<int*>(d_cgstat.as<char>() + 32));
  hipLaunchKernelGGL(assemble_rhs_kernel, dim3(g256(64 * nd)), dim3(256), 0, st, M.nx, M.ny, M.nz, M.w,
                     Bo, d_zc.as<double>(), d_mask.as<uint8_t>(), d_f.as<double>(),
                     d_uD.as<double>(), d_lift.as<double>(), d_b.as<double>(),
                     d_b.as<double>() + nd);
  DD_TRY(cg_solve());
  hipLaunchKernelGGL(recover_kernel, dim3(g256(8 * nm)), dim3(256), 0, st, M.nx, M.ny, M.nz, Bo, LTm, Lm,
                     d_x.as<double>(), nd, d_zw.as<double>(), d_zc.as<double>(), d_yw.as<double>(),
                     (double*)nullptr, (double*)nullptr);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

dd_status DDSolver::fetch_results(double* u, int64_t* idx, double* eps, double* sig) {
  const int64_t nd = M.n_dof, nm = M.n_mp;
  if (u) DD_HIP(hipMemcpyAsync(u, d_x.p, sizeof(double) * nd, hipMemcpyDeviceToHost, st));
  if (idx) DD_HIP(hipMemcpyAsync(idx, d_idx.p, sizeof(int64_t) * nm, hipMemcpyDeviceToHost, st));
  if (eps || sig) {
    // raw admissible state of the last P_C, recomputed from u, eta and the z*
    // that P_C used (kept in zc)
    DevBuf er, sr;
    DD_TRY(er.alloc(sizeof(double) * 6 * nm));
    DD_TRY(sr.alloc(sizeof(double) * 6 * nm));
    Mat6 Lm, LTm;
    std::memcpy(Lm.a, L, sizeof(L));
    std::memcpy(LTm.a, Lt, sizeof(Lt));
    BOps Bo;
    std::memcpy(Bo.B, M.B, sizeof(Bo.B));
    hipLaunchKernelGGL(recover_kernel, dim3(g256(8 * nm)), dim3(256), 0, st, M.nx, M.ny, M.nz, Bo, LTm,
                       Lm, d_x.as<double>(), nd, d_zw.as<double>(), d_zc.as<double>(),
                       d_yw.as<double>(), er.as<double>(), sr.as<double>());
    DD_HIP(hipGetLastError());
    if (eps) DD_HIP(hipMemcpyAsync(eps, er.p, sizeof(double) * 6 * nm, hipMemcpyDeviceToHost, st));
    if (sig) DD_HIP(hipMemcpyAsync(sig, sr.p, sizeof(double) * 6 * nm, hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
  }
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

namespace {
// two timing events, destroyed with the scope
struct StepEvents {
  hipEvent_t e[2] = {nullptr, nullptr};
  dd_status init() {
    for (auto& x : e) DD_HIP(hipEventCreate(&x));
    return DD_OK;
  }
  ~StepEvents() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};
}  // namespace

dd_status DDSolver::run(int max_iter, dd_solve_result* res) {
  const int64_t nm = M.n_mp;
  auto t0 = std::chrono::steady_clock::now();
  int it = 0;
  bool converged = false;
  int stop_reason = 0;
  double prev_full = INFINITY;
  int64_t cg_total = 0;
  double cg_res_max = 0.0;
  double project_ms = 0.0;
  StepEvents ev;
  DD_TRY(ev.init());
  DD_TRY(async_init());
  last_changed = -1;
  if (res && res->history) {
    DD_HIP(hipMemcpyAsync(res->history, d_idx.p, sizeof(int64_t) * nm, hipMemcpyDeviceToHost, st));
  }
  for (it = 1; it <= max_iter; ++it) {
    DD_TRY(constraint_projection());
    DD_HIP(hipEventRecord(ev.e[0], st));
    DD_TRY(project_step(it));
    DD_HIP(hipEventRecord(ev.e[1], st));
    hipLaunchKernelGGL(iter_scalars_kernel, dim3(kScalBlocks), dim3(256), 0, st, nm, M.w, d_yw.as<double>(),
                       d_zw.as<double>(), d_dist.as<double>(), d_idx_new.as<int64_t>(),
                       d_idx.as<int64_t>(), d_scal.as<double>());
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpyAsync(h_pin + 128, d_scal.p, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    DD_HIP(hipMemcpyAsync(h_pin + 160, d_cgstat.as<char>() + 32, sizeof(int), hipMemcpyDeviceToHost,
                          st));
    if (res && res->history && it <= res->history_capacity)
      DD_HIP(hipMemcpyAsync(res->history + (int64_t)it * nm, d_idx_new.p, sizeof(int64_t) * nm,
                            hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    float pms = 0.f;
    DD_HIP(hipEventElapsedTime(&pms, ev.e[0], ev.e[1]));
    project_ms += pms;
    int cg_it[2] = {cg_last_iters[0], cg_last_iters[1]};
    double cg_res[2] = {cg_last_res[0], cg_last_res[1]};
    double sc[3];
    int bad = 0;
    std::memcpy(sc, h_pin + 128, sizeof(sc));
    std::memcpy(&bad, h_pin + 160, sizeof(bad));
    if (bad) return set_error(DD_ERR_DEVICE, "dd_solve: the admissible state became non-finite");
    cg_total += cg_it[0] + cg_it[1];
    cg_res_max = std::max(cg_res_max, std::max(cg_res[0], cg_res[1]));
    last_changed = (int64_t)sc[2];
    if (res) {
      if (res->d_half && it <= res->history_capacity) res->d_half[it - 1] = sc[0];
      if (res->d_full && it <= res->history_capacity) res->d_full[it - 1] = sc[1];
      if (res->changed && it <= res->history_capacity) res->changed[it - 1] = (int64_t)sc[2];
    }
    // the new association becomes the current one
    std::swap(d_idx.p, d_idx_new.p);
    // under an accuracy schedule the stopping rules wait for its end
    const bool approximate = approximate_at(it);
    const bool scheduled = ann_ramp > 0 && it <= ann_ramp && approximate_at(1);
    if (sc[2] == 0.0 && !scheduled) {
      converged = true;
      stop_reason = 1;
      break;
    }
    // an approximate projection gives no descent guarantee: stop once the
    // distance to the data stops decreasing
    if (approximate && !scheduled && it > 1 && !(sc[1] < prev_full)) {
      stop_reason = 2;
      break;
    }
    prev_full = sc[1];
    last_full = sc[1];
  }
  if (it > max_iter) it = max_iter;
  if (res) {
    res->iterations = it;
    res->converged = converged ? 1 : 0;
    res->stop_reason = stop_reason;
    res->skipped = skipped_total;
    res->cg_iterations = cg_total;
    res->cg_max_residual = cg_res_max;
    res->project_ms = project_ms;
    DD_TRY(fetch_results(res->u, res->idx, res->eps, res->sig));
    res->elapsed_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return stop_reason != 0 ? DD_OK : set_error(DD_ERR_NOT_CONVERGED, "dd_solve reached max_iter");
}

}  // namespace dd

extern "C" dd_status dd_solve(const dd_dataset* ds, const dd_mesh* mesh,
                              const uint8_t* dirichlet_mask, const double* nodal_force,
                              const int64_t* init_idx, const dd_solve_opts* opts,
                              dd_solve_result* result, void* hip_stream) {
  using namespace dd;
  if (!ds || !mesh || !dirichlet_mask || !nodal_force || !init_idx)
    return set_error(DD_ERR_ARG, "dd_solve: NULL argument");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DDSolver S;
  DD_TRY(S.setup(ds->d, *mesh, dirichlet_mask, nodal_force, opts, st));
  DD_TRY(S.set_assignment(init_idx));
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 500;
  return S.run(max_iter, result);
}
