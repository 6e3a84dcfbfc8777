// dd_metric_pca: the metric of the paper's example (Section 3) from a
// principal component analysis of the data set.  Two device passes with
// per-block partial sums (summed on the host in block order, so the result is
// reproducible): the 12 means, then the 78 centred second moments.  The
// 12x12 eigenproblem and the 6x6 algebra run on the host.
#include <cmath>
#include <cstring>
#include <vector>

#include "dd_internal.h"

namespace dd {

namespace {

constexpr int kPcaBlocks = 1024;
constexpr int kPcaThreads = 256;

__device__ inline void load_row(const double* __restrict__ e, const double* __restrict__ s,
                                int64_t i, double x[12]) {
  for (int k = 0; k < 6; ++k) {
    x[k] = e[6 * i + k];
    x[6 + k] = s[6 * i + k];
  }
}

// partial[b][k] = sum over the block's points of x_k
__global__ __launch_bounds__(kPcaThreads) void pca_mean_kernel(const double* __restrict__ e,
                                                               const double* __restrict__ s,
                                                               int64_t n, double* __restrict__ partial) {
  __shared__ double red[kPcaThreads];
  double acc[12] = {0};
  for (int64_t i = (int64_t)blockIdx.x * kPcaThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kPcaThreads) {
    double x[12];
    load_row(e, s, i, x);
    for (int k = 0; k < 12; ++k) acc[k] += x[k];
  }
  for (int k = 0; k < 12; ++k) {
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = kPcaThreads / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[12 * blockIdx.x + k] = red[0];
    __syncthreads();
  }
}

struct Mean12 {
  double m[12];
};

// partial[b][p] = sum over the block's points of (x_i - m_i)(x_j - m_j), p over i <= j
__global__ __launch_bounds__(kPcaThreads) void pca_cov_kernel(const double* __restrict__ e,
                                                              const double* __restrict__ s,
                                                              int64_t n, Mean12 M,
                                                              double* __restrict__ partial) {
  __shared__ double red[kPcaThreads];
  double acc[78] = {0};
  for (int64_t i = (int64_t)blockIdx.x * kPcaThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kPcaThreads) {
    double x[12];
    load_row(e, s, i, x);
    for (int k = 0; k < 12; ++k) x[k] -= M.m[k];
#pragma unroll
    for (int a = 0; a < 12; ++a)
#pragma unroll
      for (int b = a; b < 12; ++b) {
        const int p = a * 12 - a * (a - 1) / 2 + (b - a);   // position of (a, b), a <= b
        acc[p] = fma(x[a], x[b], acc[p]);
      }
  }
#pragma unroll
  for (int p = 0; p < 78; ++p) {
    red[threadIdx.x] = acc[p];
    __syncthreads();
    for (int off = kPcaThreads / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[78 * blockIdx.x + p] = red[0];
    __syncthreads();
  }
}

// In-place inverse of a 6x6 matrix by Gauss-Jordan with partial pivoting.
bool invert6(double* A) {
  double I[36] = {0};
  for (int i = 0; i < 6; ++i) I[7 * i] = 1.0;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(A[6 * r + c]) > std::fabs(A[6 * piv + c])) piv = r;
    if (!(std::fabs(A[6 * piv + c]) > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < 6; ++k) {
        std::swap(A[6 * c + k], A[6 * piv + k]);
        std::swap(I[6 * c + k], I[6 * piv + k]);
      }
    const double d = 1.0 / A[6 * c + c];
    for (int k = 0; k < 6; ++k) {
      A[6 * c + k] *= d;
      I[6 * c + k] *= d;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const double f = A[6 * r + c];
      for (int k = 0; k < 6; ++k) {
        A[6 * r + k] -= f * A[6 * c + k];
        I[6 * r + k] -= f * I[6 * c + k];
      }
    }
  }
  std::memcpy(A, I, sizeof(I));
  return true;
}

}  // namespace

}  // namespace dd

extern "C" dd_status dd_metric_pca(const double* strain_dev, const double* stress_dev, int64_t N,
                                   double* C_out, void* hip_stream) {
  using namespace dd;
  if (!strain_dev || !stress_dev || !C_out) return set_error(DD_ERR_ARG, "NULL pointer");
  if (N < 12) return set_error(DD_ERR_ARG, "dd_metric_pca needs N >= 12");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int blocks = (int)std::min<int64_t>(kPcaBlocks, (N + kPcaThreads - 1) / kPcaThreads);
  DevBuf part;
  DD_TRY(part.alloc(sizeof(double) * 78 * blocks));
  hipLaunchKernelGGL(pca_mean_kernel, dim3(blocks), dim3(kPcaThreads), 0, st, strain_dev,
                     stress_dev, N, part.as<double>());
  DD_HIP(hipGetLastError());
  std::vector<double> h(78 * (size_t)blocks);
  DD_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * 12 * blocks, hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  Mean12 M;
  for (int k = 0; k < 12; ++k) {
    double acc = 0.0;
    for (int b = 0; b < blocks; ++b) acc += h[12 * b + k];
    M.m[k] = acc / (double)N;
    if (!std::isfinite(M.m[k])) return set_error(DD_ERR_ARG, "non-finite data");
  }
  hipLaunchKernelGGL(pca_cov_kernel, dim3(blocks), dim3(kPcaThreads), 0, st, strain_dev,
                     stress_dev, N, M, part.as<double>());
  DD_HIP(hipGetLastError());
  DD_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * 78 * blocks, hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  double cov[144];
  {
    int p = 0;
    for (int a = 0; a < 12; ++a)
      for (int b = a; b < 12; ++b, ++p) {
        double acc = 0.0;
        for (int k = 0; k < blocks; ++k) acc += h[78 * k + p];
        cov[12 * a + b] = cov[12 * b + a] = acc / (double)N;
      }
  }
  double sd[12], R[144];
  for (int k = 0; k < 12; ++k) {
    sd[k] = std::sqrt(cov[13 * k]);
    if (!(sd[k] > 0.0)) return set_error(DD_ERR_ARG, "a data component has zero variance");
  }
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) R[12 * a + b] = cov[12 * a + b] / (sd[a] * sd[b]);
  double ev[12], V[144];
  sym_eigen(12, R, ev, V);   // eigenvalues descending, eigenvectors as columns
  double Ae[36], As[36];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      Ae[6 * r + c] = sd[r] * V[12 * r + c];
      As[6 * r + c] = sd[6 + r] * V[12 * (6 + r) + c];
    }
  if (!invert6(Ae)) return set_error(DD_ERR_ARG, "the strain block of the principal vectors is singular");
  double C[36];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 6; ++k) acc += As[6 * r + k] * Ae[6 * k + c];
      C[6 * r + c] = acc;
    }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) C_out[6 * r + c] = 0.5 * (C[6 * r + c] + C[6 * c + r]);
  double L[36];
  if (!cholesky6(C_out, L))
    return set_error(DD_ERR_NOT_SPD, "sym(A_sig A_eps^-1) is not positive definite");
  return DD_OK;
}
