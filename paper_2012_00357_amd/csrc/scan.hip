// Projection kernels for P_D (Section 2): nearest data point of every query
// under the metric of eq. "distmetric", evaluated in whitened coordinates
// (Section 3.2), where the metric is the plain squared Euclidean norm.
//
// Three scans share one certification scheme.  A scan evaluates approximate
// squared distances d~_j with a rigorous per-pair error bound and keeps, per
// query, every data point that could still be the exact minimiser:
//   * FP64 MFMA scan, d-space: |d~_j - d_j| <= a, keep j if d~_j - a <= U where
//     U = min_i d~_i + a is an upper bound of the true minimum;
//   * 16-bit MFMA scan, sqrt-space: |sqrt(d~_j) - sqrt(d_j)| is bounded through
//     the rounding of the centred operands (eta) and the FP32 accumulation
//     (alpha); keep j if sqrt(d~_j - alpha) - eta <= U, U = min_i sqrt(d~_i +
//     alpha) + eta_i.
// The exact minimiser always satisfies its own test, so reranking the kept
// points in FP64 direct form returns the FP64 nearest neighbour; ties resolve
// to the lowest original index.  Candidate lists that overflow send the query
// to the next, more precise scan.
#include <cmath>

#include "pack16.h"
#include "scan.h"

namespace dd {

static unsigned grid1(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

int choose_splits(int64_t n_query_blocks, int64_t n_tiles, int requested) {
  int64_t S;
  if (requested > 0) {
    S = requested;
  } else {
    // few query blocks: one round of workgroups; many: about 2048 workgroups
    const int64_t qb = std::max<int64_t>(n_query_blocks, 1);
    S = ((qb < 64 ? 512 : 2048) + qb - 1) / qb;
    if (S >= 8) S = (S + 7) / 8 * 8;   // all blocks of one split on one XCD
  }
  S = std::min<int64_t>(S, std::max<int64_t>(n_tiles, 1));
  S = std::min<int64_t>(S, 4096);
  return (int)std::max<int64_t>(S, 1);
}

int choose_splits16(int64_t n_query_blocks, int64_t n_tiles, int requested) {
  if (requested > 0) return choose_splits(n_query_blocks, n_tiles, requested);
  const int64_t qb = std::max<int64_t>(n_query_blocks, 1);
  const int64_t target = qb < 64 ? 256 : 1024;
  int64_t S = (target + qb - 1) / qb;
  if (S >= 8) S = (S + 7) / 8 * 8;
  S = std::min<int64_t>(S, std::max<int64_t>(n_tiles, 1));
  return (int)std::max<int64_t>(std::min<int64_t>(S, 4096), 1);
}

// ---------------------------------------------------------------------------
// Query preparation: whitening, warm-start bounds
// ---------------------------------------------------------------------------
struct Mats {
  double F[36];
  double G[36];
};

__global__ void prep_kernel(const double* __restrict__ states, int64_t m, Mats M,
                            const int64_t* __restrict__ warm, int64_t N,
                            const uint32_t* __restrict__ iperm, const double* __restrict__ w64,
                            const float* __restrict__ w32, double u32_scale,
                            double* __restrict__ qw, double* __restrict__ qn2,
                            double* __restrict__ u64, float* __restrict__ u32,
                            int* __restrict__ invalid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double y[12];
  bool ok = true;
  for (int k = 0; k < 12; ++k) {
    y[k] = states[12 * i + k];
    ok = ok && isfinite(y[k]);
  }
  double q[12];
  double n2 = 0.0;
  for (int r = 0; r < 6; ++r) {
    double a = 0.0, b = 0.0;
    for (int c = 0; c < 6; ++c) {
      a = fma(M.F[6 * r + c], y[c], a);
      b = fma(M.G[6 * r + c], y[6 + c], b);
    }
    q[r] = ok ? a : 0.0;
    q[6 + r] = ok ? b : 0.0;
  }
  for (int k = 0; k < 12; ++k) {
    qw[12 * i + k] = q[k];
    n2 = fma(q[k], q[k], n2);
  }
  qn2[i] = n2;
  invalid[i] = ok ? 0 : 1;
  double ub = INFINITY;
  float ub32 = INFINITY;
  if (ok && warm && (w64 || w32)) {
    int64_t wi = warm[i];
    if (wi >= 0 && wi < N) {
      int64_t p = iperm[wi];
      double d = 0.0;
      for (int k = 0; k < 12; ++k) {
        double x = w64 ? w64[12 * p + k] : (double)w32[12 * p + k];
        double t = q[k] - x;
        d = fma(t, t, d);
      }
      // the FP64 sum carries at most ~13 ulp of relative error: inflate by 2^-40
      ub = d * (1.0 + 0x1p-40) + 1e-300;
      ub32 = __double2float_ru(sqrt(ub) * (1.0 + 0x1p-40) * u32_scale);
    }
  }
  u64[i] = ub;
  u32[i] = ub32;
}

dd_status prepare_queries(const Dataset& D, const double* states, bool whitened, int64_t m,
                          const int64_t* warm, double u32_scale, QueryPrep& Q, hipStream_t st) {
  Mats M;
  for (int i = 0; i < 36; ++i) {
    const double id = (i % 7 == 0) ? 1.0 : 0.0;   // identity: states already whitened
    M.F[i] = whitened ? id : D.F[i];
    M.G[i] = whitened ? id : D.G[i];
  }
  hipLaunchKernelGGL(prep_kernel, dim3(grid1(m)), dim3(256), 0, st, states, m, M, warm, D.N,
                     D.iperm.as<uint32_t>(), D.w64.as<double>(), D.w32.as<float>(), u32_scale,
                     Q.qw, Q.qn2, Q.u64, Q.u32, Q.invalid);
  DD_HIP(hipGetLastError());
  return DD_OK;
}


// ---------------------------------------------------------------------------
// Bound-only pass reduction: u32[q] = min over splits of the split bounds.
// ---------------------------------------------------------------------------
__global__ void reduce_bounds_kernel(QueryList L, const float* __restrict__ U, int S,
                                     float* __restrict__ u32) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= list_len(L)) return;
  float u = INFINITY;
  for (int s = 0; s < S; ++s) u = fminf(u, U[p * S + s]);
  const int64_t q = list_query(L, p);
  u32[q] = fminf(u32[q], u);
}

dd_status launch_reduce_bounds(QueryList L, int64_t list_len_max, const float* U, int S, float* u32,
                               hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  hipLaunchKernelGGL(reduce_bounds_kernel, dim3(grid1(list_len_max)), dim3(256), 0, st, L, U, S, u32);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// Merge and FP64 rerank (direct form 1/2 |q - x|^2), lexicographic minimum of
// (distance, original index) over every certified candidate.  With few
// candidate slots per query (the 16-bit scans: one list per half-wave), one
// thread per query in large batches and, in small ones, one wavefront per query
// whose lanes take the (slot, entry) pairs; with many slots (the FP64 scan: one
// list per split and part), one wavefront per query, its lanes taking the
// slots in turn.  The wave then reduces; the minimum is order-independent, so
// every variant gives the result of a serial merge.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void merge_rerank_thread_kernel(
    QueryList L, CandBuf cb, const float* __restrict__ Uq, const double* __restrict__ qw,
    const int* __restrict__ invalid,
    const double* __restrict__ w64, const float* __restrict__ w32, const uint32_t* __restrict__ perm,
    Outputs out, int* __restrict__ fb_list, int* __restrict__ fb_count,
    unsigned long long* __restrict__ n_cand) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = p < list_len(L) ? list_query(L, p) : -1;
  unsigned long long nc = 0;
  if (q >= 0 && invalid[q]) {
    out.idx[q] = -1;
    if (out.dist) out.dist[q] = NAN;
  } else if (q >= 0) {
    const int S = cb.S, P = cb.P, K = cb.K;
    float Uf = INFINITY;
    if (Uq) {
      Uf = Uq[q];
    } else {
      for (int s = 0; s < S; ++s) Uf = fminf(Uf, cb.U[p * S + s]);
    }
    double qv[12];
    for (int k = 0; k < 12; ++k) qv[k] = qw[12 * q + k];
    double best = INFINITY;
    uint32_t bo = 0xFFFFFFFFu;
    bool ovf = false;
    for (int sl = 0; sl < S * P; ++sl) {
      const int64_t slot = p * (S * P) + sl;   // (p S + s) P + part with sl = s P + part
      const int c = cb.count[slot];
      const int raw = c & ~kOverflowBit;
      ovf = ovf || (c & kOverflowBit) || raw > K;
      const int n = raw < K ? raw : K;
      for (int e = 0; e < n; ++e) {
        if (cb.lb[slot * K + e] <= Uf) {
          const uint32_t j = cb.j[slot * K + e];
          double d = 0.0;
          for (int k = 0; k < 12; ++k) {
            double x = w64 ? w64[12 * (int64_t)j + k] : (double)w32[12 * (int64_t)j + k];
            double t = qv[k] - x;
            d = fma(t, t, d);
          }
          const uint32_t o = perm[j];
          if (d < best || (d == best && o < bo)) {
            best = d;
            bo = o;
          }
          ++nc;
        }
      }
    }
    if (ovf || bo == 0xFFFFFFFFu) {
      int k = atomicAdd(fb_count, 1);
      fb_list[k] = (int)q;
    } else {
      out.idx[q] = (int64_t)bo;
      if (out.dist) out.dist[q] = 0.5 * best;
    }
  }
  // one atomic add per wavefront for the candidate count
  for (int off = 32; off > 0; off >>= 1) nc += __shfl_xor(nc, off);
  if (n_cand && (threadIdx.x & 63) == 0 && nc) atomicAdd(n_cand, nc);
}

// FLAT: the lanes take (slot, entry) pairs instead of whole slots, for lists
// with few slots of many entries (the 16-bit scans' two half-wave lists).
template <bool FLAT>
__global__ __launch_bounds__(256) void merge_rerank_wave_kernel(
    QueryList L, CandBuf cb, const float* __restrict__ Uq, const double* __restrict__ qw,
    const int* __restrict__ invalid,
    const double* __restrict__ w64, const float* __restrict__ w32, const uint32_t* __restrict__ perm,
    Outputs out, int* __restrict__ fb_list, int* __restrict__ fb_count,
    unsigned long long* __restrict__ n_cand) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= list_len(L)) return;   // wave-uniform
  const int64_t q = list_query(L, p);
  if (invalid[q]) {
    if (lane == 0) {
      out.idx[q] = -1;
      if (out.dist) out.dist[q] = NAN;
    }
    return;
  }
  const int S = cb.S, P = cb.P, K = cb.K;
  float Uf = INFINITY;
  if (Uq) {
    Uf = Uq[q];
  } else {
    for (int s = lane; s < S; s += 64) Uf = fminf(Uf, cb.U[p * S + s]);
    for (int off = 32; off > 0; off >>= 1) Uf = fminf(Uf, __shfl_xor(Uf, off));
  }
  double qv[12];
  for (int k = 0; k < 12; ++k) qv[k] = qw[12 * q + k];
  double best = INFINITY;
  uint32_t bo = 0xFFFFFFFFu;
  bool ovf = false;
  unsigned long long nc = 0;
  const int slots = S * P;
  auto rerank = [&](int64_t slot, int e) __attribute__((always_inline)) {
    if (cb.lb[slot * K + e] <= Uf) {
      const uint32_t j = cb.j[slot * K + e];
      double d = 0.0;
      for (int k = 0; k < 12; ++k) {
        double x = w64 ? w64[12 * (int64_t)j + k] : (double)w32[12 * (int64_t)j + k];
        double t = qv[k] - x;
        d = fma(t, t, d);
      }
      const uint32_t o = perm[j];
      if (d < best || (d == best && o < bo)) {
        best = d;
        bo = o;
      }
      ++nc;
    }
  };
  if (FLAT) {
    for (int it = lane; it < slots * K; it += 64) {
      const int sl = it / K, e = it - sl * K;
      const int64_t slot = p * slots + sl;
      const int c = cb.count[slot];
      const int raw = c & ~kOverflowBit;
      if (e == 0) ovf = ovf || (c & kOverflowBit) || raw > K;
      if (e < (raw < K ? raw : K)) rerank(slot, e);
    }
  } else {
    for (int sl = lane; sl < slots; sl += 64) {
      const int64_t slot = p * slots + sl;   // (p S + s) P + part with sl = s P + part
      const int c = cb.count[slot];
      const int raw = c & ~kOverflowBit;
      ovf = ovf || (c & kOverflowBit) || raw > K;
      const int n = raw < K ? raw : K;
      for (int e = 0; e < n; ++e) rerank(slot, e);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const uint32_t oo = (uint32_t)__shfl_xor((int)bo, off);
    if (ob < best || (ob == best && oo < bo)) {
      best = ob;
      bo = oo;
    }
    nc += __shfl_xor(nc, off);
  }
  ovf = __any(ovf);
  if (lane == 0) {
    if (ovf || bo == 0xFFFFFFFFu) {
      int k = atomicAdd(fb_count, 1);
      fb_list[k] = (int)q;
    } else {
      out.idx[q] = (int64_t)bo;
      if (out.dist) out.dist[q] = 0.5 * best;
    }
    if (n_cand && nc) atomicAdd(n_cand, nc);
  }
}

dd_status launch_merge_rerank(const Dataset& D, const QueryPrep& Q, QueryList L,
                              int64_t list_len_max, const CandBuf& cb, const float* Uq,
                              Outputs out, int* fb_list, int* fb_count, unsigned long long* n_cand,
                              hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  // few slots: a thread per query for large batches, a wavefront per query
  // over the (slot, entry) pairs for small ones; many slots: a wavefront per
  // query over the slots
  if (cb.S * cb.P <= 8 && list_len_max < 16384 && cb.S * cb.P * cb.K <= 256)
    hipLaunchKernelGGL(merge_rerank_wave_kernel<true>, dim3(grid1(list_len_max, 4)), dim3(256), 0,
                       st, L, cb, Uq, Q.qw, Q.invalid, D.w64.as<double>(),
                       D.w64.p ? nullptr : D.w32.as<float>(), D.perm.as<uint32_t>(), out, fb_list,
                       fb_count, n_cand);
  else if (cb.S * cb.P <= 8)
    hipLaunchKernelGGL(merge_rerank_thread_kernel, dim3(grid1(list_len_max)), dim3(256), 0, st, L, cb,
                       Uq, Q.qw, Q.invalid, D.w64.as<double>(),
                       D.w64.p ? nullptr : D.w32.as<float>(), D.perm.as<uint32_t>(), out, fb_list,
                       fb_count, n_cand);
  else
    hipLaunchKernelGGL(merge_rerank_wave_kernel<false>, dim3(grid1(list_len_max, 4)), dim3(256), 0,
                       st, L, cb, Uq, Q.qw, Q.invalid, D.w64.as<double>(),
                       D.w64.p ? nullptr : D.w32.as<float>(), D.perm.as<uint32_t>(), out, fb_list,
                       fb_count, n_cand);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// Plain FP64 direct-form scan: one query per lane, data rows broadcast from LDS.
// ---------------------------------------------------------------------------
constexpr int kDirectRows = 128;

__global__ __launch_bounds__(256) void direct_kernel(
    const double* __restrict__ w64, const float* __restrict__ w32, const uint32_t* __restrict__ perm,
    int64_t n_tiles, int64_t N, const double* __restrict__ qw, QueryList L, int S,
    double* __restrict__ part_d, uint32_t* __restrict__ part_o) {
  __shared__ double xs[kDirectRows][12];
  __shared__ uint32_t os[kDirectRows];
  const int tid = threadIdx.x;
  const int split = blockIdx.x % S;
  const int64_t p = (int64_t)(blockIdx.x / S) * 256 + tid;
  const int64_t len = list_len(L);
  if ((int64_t)(blockIdx.x / S) * 256 >= len) return;
  const bool v = p < len;
  const int64_t q = v ? list_query(L, p) : 0;
  double qv[12];
  for (int k = 0; k < 12; ++k) qv[k] = v ? qw[12 * q + k] : 0.0;
  const int64_t t0 = (int64_t)split * n_tiles / S, t1 = (int64_t)(split + 1) * n_tiles / S;
  double best = INFINITY;
  uint32_t bo = 0xFFFFFFFFu;
  for (int64_t t = t0; t < t1; ++t) {
    for (int e = tid; e < kDirectRows * 12; e += 256) {
      int64_t row = t * kDirectRows + e / 12;
      double x = 0.0;
      if (row < N) x = w64 ? w64[12 * row + e % 12] : (double)w32[12 * row + e % 12];
      xs[e / 12][e % 12] = x;
    }
    if (tid < kDirectRows) {
      int64_t row = t * kDirectRows + tid;
      os[tid] = row < N ? perm[row] : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int r = 0; r < kDirectRows; ++r) {
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        double t2 = qv[k] - xs[r][k];
        d = fma(t2, t2, d);
      }
      const uint32_t o = os[r];
      if (o != 0xFFFFFFFFu && (d < best || (d == best && o < bo))) {
        best = d;
        bo = o;
      }
    }
    __syncthreads();
  }
  if (v) {
    part_d[p * S + split] = best;
    part_o[p * S + split] = bo;
  }
}

__global__ void merge_direct_kernel(QueryList L, int S, const double* __restrict__ part_d,
                                    const uint32_t* __restrict__ part_o,
                                    const int* __restrict__ invalid, Outputs out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= list_len(L)) return;
  const int64_t q = list_query(L, p);
  if (invalid[q]) {
    out.idx[q] = -1;
    if (out.dist) out.dist[q] = NAN;
    return;
  }
  double best = INFINITY;
  uint32_t bo = 0xFFFFFFFFu;
  for (int s = 0; s < S; ++s) {
    double d = part_d[p * S + s];
    uint32_t o = part_o[p * S + s];
    if (o != 0xFFFFFFFFu && (d < best || (d == best && o < bo))) {
      best = d;
      bo = o;
    }
  }
  out.idx[q] = bo == 0xFFFFFFFFu ? -1 : (int64_t)bo;
  if (out.dist) out.dist[q] = 0.5 * best;
}

int direct_splits(const Dataset& D, int64_t list_len) {
  return choose_splits((list_len + 255) / 256, (D.N + kDirectRows - 1) / kDirectRows, 0);
}

dd_status run_direct(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len_max, int S,
                     Outputs out, hipStream_t st, double* part_d, uint32_t* part_o) {
  if (list_len_max <= 0) return DD_OK;
  int64_t n_tiles = (D.N + kDirectRows - 1) / kDirectRows;
  int64_t qblocks = (list_len_max + 255) / 256;
  S = choose_splits(qblocks, n_tiles, S);
  const bool own = !(part_d && part_o);
  double* pd = part_d;
  uint32_t* po = part_o;
  if (own) {
    DD_HIP(hipMallocAsync((void**)&pd, sizeof(double) * (size_t)(list_len_max * S), st));
    DD_HIP(hipMallocAsync((void**)&po, sizeof(uint32_t) * (size_t)(list_len_max * S), st));
  }
  hipLaunchKernelGGL(direct_kernel, dim3((unsigned)(qblocks * S)), dim3(256), 0, st,
                     D.w64.as<double>(), D.w64.p ? nullptr : D.w32.as<float>(),
                     D.perm.as<uint32_t>(), n_tiles, D.N, Q.qw, L, S, pd, po);
  DD_HIP(hipGetLastError());
  hipLaunchKernelGGL(merge_direct_kernel, dim3(grid1(list_len_max)), dim3(256), 0, st, L, S, pd, po,
                     Q.invalid, out);
  DD_HIP(hipGetLastError());
  if (own) {
    DD_HIP(hipFreeAsync(pd, st));
    DD_HIP(hipFreeAsync(po, st));
  }
  return DD_OK;
}

}  // namespace dd
