// P_C by an explicit inverse for small meshes.  K is constant over the DD
// iterations (Section 2: the paper factorises it once); for up to kDenseMaxDof
// DOFs its inverse is formed once on the GPU and kept per (mesh, Dirichlet
// pattern) on the dataset, and every P_C is then one product of K^-1 with the
// two right-hand sides (E and S of eqs. "KuE", "KeS") -- a stream of n^2
// doubles instead of hundreds of CG iterations.
//
// Inversion: blocked Gauss-Jordan without pivoting (K is symmetric positive
// definite, with identity rows and columns at Dirichlet DOFs), in place on the
// matrix padded to a multiple of 64 with identity.  For each diagonal block k:
//   A_kk <- A_kk^-1;  A_ik <- -A_ik A_kk (i != k);  A_ij <- A_ij + A_ik A_kj
//   (i, j != k);  A_kj <- A_kk A_kj (j != k).
#include <algorithm>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>

#include "solve.h"

namespace dd {

namespace {

constexpr int kB = 64;   // block size of the Gauss-Jordan sweep

__global__ void dense_from_csr_kernel(const int32_t* __restrict__ rowptr,
                                      const int32_t* __restrict__ col,
                                      const double* __restrict__ val, int64_t n, int64_t n_pad,
                                      double* __restrict__ A) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  if (r < n) {
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) A[r * n_pad + col[e]] = val[e];
  } else {
    A[r * n_pad + r] = 1.0;
  }
}

// Inverts the diagonal block [k0, k0+64)^2 in place (and copies it to Akk).
__global__ __launch_bounds__(256) void gj_diag_kernel(double* __restrict__ A, int64_t n_pad,
                                                      int64_t k0, double* __restrict__ Akk) {
  __shared__ double s[kB][kB + 1];
  __shared__ double colp[kB], rowp[kB];
  __shared__ double dpiv;
  const int t = threadIdx.x;
  for (int e = t; e < kB * kB; e += 256) s[e / kB][e % kB] = A[(k0 + e / kB) * n_pad + k0 + e % kB];
  __syncthreads();
  for (int p = 0; p < kB; ++p) {
    if (t < kB) {
      colp[t] = s[t][p];
      rowp[t] = s[p][t];
    }
    if (t == 0) dpiv = 1.0 / s[p][p];
    __syncthreads();
    const double d = dpiv;
    for (int e = t; e < kB * kB; e += 256) {
      const int i = e / kB, j = e % kB;
      double v;
      if (i == p && j == p)
        v = d;
      else if (i == p)
        v = d * rowp[j];
      else if (j == p)
        v = -colp[i] * d;
      else
        v = fma(-colp[i] * d, rowp[j], s[i][j]);
      s[i][j] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < kB * kB; e += 256) {
    const double v = s[e / kB][e % kB];
    A[(k0 + e / kB) * n_pad + k0 + e % kB] = v;
    Akk[e] = v;
  }
}

// Column panel: rows i outside the block, A[i, k] <- -A[i, k] Akk.  4 rows per block.
__global__ __launch_bounds__(256) void gj_col_kernel(double* __restrict__ A, int64_t n_pad,
                                                     int64_t k0, const double* __restrict__ Akk) {
  __shared__ double inv[kB][kB + 1];
  __shared__ double row[4][kB];
  const int t = threadIdx.x;
  for (int e = t; e < kB * kB; e += 256) inv[e / kB][e % kB] = Akk[e];
  const int ri = t / kB, c = t % kB;
  int64_t i = (int64_t)blockIdx.x * 4 + ri;      // index among rows outside the block
  if (i >= k0) i += kB;
  const bool v = i < n_pad;
  row[ri][c] = v ? A[i * n_pad + k0 + c] : 0.0;
  __syncthreads();
  if (!v) return;
  double acc = 0.0;
#pragma unroll 8
  for (int q = 0; q < kB; ++q) acc = fma(row[ri][q], inv[q][c], acc);
  A[i * n_pad + k0 + c] = -acc;
}

// Trailing update of one 64x64 tile outside block row/column k:
// A[I, J] += A[I, k] A[k, J].  Each thread computes a 4x4 sub-tile.
__global__ __launch_bounds__(256) void gj_update_kernel(double* __restrict__ A, int64_t n_pad,
                                                        int64_t k0) {
  __shared__ double a[kB][kB + 1];   // A[I, k]
  __shared__ double b[kB][kB + 1];   // A[k, J]
  const int64_t nb = n_pad / kB;
  int64_t bi = blockIdx.x % (nb - 1), bj = blockIdx.x / (nb - 1);
  const int64_t kb = k0 / kB;
  if (bi >= kb) ++bi;
  if (bj >= kb) ++bj;
  const int64_t I0 = bi * kB, J0 = bj * kB;
  const int t = threadIdx.x;
  for (int e = t; e < kB * kB; e += 256) {
    const int r = e / kB, c = e % kB;
    a[r][c] = A[(I0 + r) * n_pad + k0 + c];
    b[r][c] = A[(k0 + r) * n_pad + J0 + c];
  }
  __syncthreads();
  const int ty = t / 16, tx = t % 16;   // rows ty + 16 m, columns tx + 16 l
  double acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int l = 0; l < 4; ++l) acc[m][l] = 0.0;
  for (int q = 0; q < kB; ++q) {
    double av[4], bv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) av[m] = a[ty + 16 * m][q];
#pragma unroll
    for (int l = 0; l < 4; ++l) bv[l] = b[q][tx + 16 * l];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int l = 0; l < 4; ++l) acc[m][l] = fma(av[m], bv[l], acc[m][l]);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double* p = A + (I0 + ty + 16 * m) * n_pad + J0 + tx + 16 * l;
      *p += acc[m][l];
    }
}

// Row panel: columns j outside the block, A[k, j] <- Akk A[k, j].  4 columns per block.
__global__ __launch_bounds__(256) void gj_row_kernel(double* __restrict__ A, int64_t n_pad,
                                                     int64_t k0, const double* __restrict__ Akk) {
  __shared__ double inv[kB][kB + 1];
  __shared__ double colv[4][kB];
  const int t = threadIdx.x;
  for (int e = t; e < kB * kB; e += 256) inv[e / kB][e % kB] = Akk[e];
  const int cj = t / kB, r = t % kB;
  int64_t j = (int64_t)blockIdx.x * 4 + cj;
  if (j >= k0) j += kB;
  const bool v = j < n_pad;
  colv[cj][r] = v ? A[(k0 + r) * n_pad + j] : 0.0;
  __syncthreads();
  if (!v) return;
  double acc = 0.0;
#pragma unroll 8
  for (int q = 0; q < kB; ++q) acc = fma(inv[r][q], colv[cj][q], acc);
  A[(k0 + r) * n_pad + j] = acc;
}

// x_s = K^-1 b_s for the two systems; one wavefront per row, fixed reduction order.
__global__ __launch_bounds__(256) void dense_apply_kernel(const double* __restrict__ inv,
                                                          int64_t n_pad, int64_t n,
                                                          const double* __restrict__ b,
                                                          double* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const double* row = inv + r * n_pad;
  double a0 = 0.0, a1 = 0.0;
  // unrolled so that several iterations' loads are in flight; the FMA chain
  // keeps its order
#pragma unroll 8
  for (int64_t j = lane; j < n; j += 64) {
    const double k = row[j];
    a0 = fma(k, b[j], a0);
    a1 = fma(k, b[n + j], a1);
  }
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off);
    a1 += __shfl_xor(a1, off);
  }
  if (lane == 0) {
    x[r] = a0;
    x[n + r] = a1;
  }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Forms K^-1 (padded, row-major, n_pad x n_pad) from the CSR matrix on st.
static dd_status form_inverse(const int32_t* rowptr, const int32_t* col, const double* val,
                              int64_t n, DenseInverse& D, hipStream_t st) {
  const int64_t n_pad = (n + kB - 1) / kB * kB;
  D.n = n;
  D.n_pad = n_pad;
  DD_TRY(D.inv.alloc(sizeof(double) * (size_t)(n_pad * n_pad)));
  DevBuf akk;
  DD_TRY(akk.alloc(sizeof(double) * kB * kB));
  double* A = D.inv.as<double>();
  DD_HIP(hipMemsetAsync(A, 0, sizeof(double) * (size_t)(n_pad * n_pad), st));
  hipLaunchKernelGGL(dense_from_csr_kernel, dim3(blocks_for(n_pad, 256)), dim3(256), 0, st, rowptr,
                     col, val, n, n_pad, A);
  DD_HIP(hipGetLastError());
  const int64_t nb = n_pad / kB;
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t k0 = k * kB;
    hipLaunchKernelGGL(gj_diag_kernel, dim3(1), dim3(256), 0, st, A, n_pad, k0, akk.as<double>());
    if (nb > 1) {
      hipLaunchKernelGGL(gj_col_kernel, dim3(blocks_for(n_pad - kB, 4)), dim3(256), 0, st, A, n_pad,
                         k0, akk.as<double>());
      hipLaunchKernelGGL(gj_update_kernel, dim3((unsigned)((nb - 1) * (nb - 1))), dim3(256), 0, st, A,
                         n_pad, k0);
      hipLaunchKernelGGL(gj_row_kernel, dim3(blocks_for(n_pad - kB, 4)), dim3(256), 0, st, A, n_pad,
                         k0, akk.as<double>());
    }
    DD_HIP(hipGetLastError());
  }
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

std::shared_ptr<DenseInverse> dense_inverse_cached(const Dataset& ds, const FEMesh& M,
                                                   const uint8_t* mask) {
  const int64_t n = M.n_dof;
  auto same = [&](const DenseInverse& d) {
    return d.nx == M.nx && d.ny == M.ny && d.nz == M.nz && d.hx == M.hx && d.hy == M.hy &&
           d.hz == M.hz && (int64_t)d.mask.size() == n &&
           std::memcmp(d.mask.data(), mask, (size_t)n) == 0;
  };
  std::lock_guard<std::mutex> lk(ds.cache_mu);
  for (auto it = ds.pc_cache.begin(); it != ds.pc_cache.end(); ++it) {
    if (same(**it)) {
      ds.pc_cache.splice(ds.pc_cache.begin(), ds.pc_cache, it);   // most recently used first
      return ds.pc_cache.front();
    }
  }
  return nullptr;
}

dd_status dense_inverse_for(const Dataset& ds, const FEMesh& M, const uint8_t* mask,
                            const int32_t* rowptr, const int32_t* col, const double* val,
                            std::shared_ptr<DenseInverse>& out, hipStream_t st) {
  const int64_t n = M.n_dof;
  out = dense_inverse_cached(ds, M, mask);
  if (out) return DD_OK;
  auto d = std::make_shared<DenseInverse>();
  d->nx = M.nx;
  d->ny = M.ny;
  d->nz = M.nz;
  d->hx = M.hx;
  d->hy = M.hy;
  d->hz = M.hz;
  d->mask.assign(mask, mask + n);
  DD_TRY(form_inverse(rowptr, col, val, n, *d, st));
  std::lock_guard<std::mutex> lk(ds.cache_mu);
  ds.pc_cache.push_front(d);
  int64_t bytes = 0;
  for (auto it = ds.pc_cache.begin(); it != ds.pc_cache.end();) {
    bytes += (int64_t)(*it)->inv.bytes;
    if (bytes > kDenseCacheBytes && it != ds.pc_cache.begin())
      it = ds.pc_cache.erase(it);   // solvers still using it hold their own reference
    else
      ++it;
  }
  out = d;
  return DD_OK;
}

dd_status dense_apply(const DenseInverse& D, const double* b, double* x, hipStream_t st) {
  hipLaunchKernelGGL(dense_apply_kernel, dim3(blocks_for(D.n, 4)), dim3(256), 0, st,
                     D.inv.as<double>(), D.n_pad, D.n, b, x);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace dd
