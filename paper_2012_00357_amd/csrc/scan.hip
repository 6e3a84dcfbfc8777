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

constexpr float kRelUp = 1.0f + 9.5367431640625e-07f;   // 1 + 2^-20
constexpr float kRelDn = 1.0f - 9.5367431640625e-07f;   // 1 - 2^-20

static unsigned grid1(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

int choose_splits(int64_t n_query_blocks, int64_t n_tiles, int requested) {
  int64_t S;
  if (requested > 0) {
    S = requested;
  } else {
    S = (2048 + n_query_blocks - 1) / std::max<int64_t>(n_query_blocks, 1);
    if (S >= 8) S = (S + 7) / 8 * 8;   // all blocks of one split on one XCD
  }
  S = std::min<int64_t>(S, std::max<int64_t>(n_tiles, 1));
  S = std::min<int64_t>(S, 4096);
  return (int)std::max<int64_t>(S, 1);
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
                            const float* __restrict__ w32, double* __restrict__ qw,
                            double* __restrict__ qn2, double* __restrict__ u64,
                            float* __restrict__ u32, int* __restrict__ invalid) {
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
      ub32 = __double2float_ru(sqrt(ub) * (1.0 + 0x1p-40));
    }
  }
  u64[i] = ub;
  u32[i] = ub32;
}

dd_status prepare_queries(const Dataset& D, const double* states, int64_t m, const int64_t* warm,
                          QueryPrep& Q, hipStream_t st) {
  Mats M;
  for (int i = 0; i < 36; ++i) {
    M.F[i] = D.F[i];
    M.G[i] = D.G[i];
  }
  hipLaunchKernelGGL(prep_kernel, dim3(grid1(m)), dim3(256), 0, st, states, m, M, warm, D.N,
                     D.iperm.as<uint32_t>(), D.w64.as<double>(), D.w32.as<float>(), Q.qw, Q.qn2,
                     Q.u64, Q.u32, Q.invalid);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// Candidate list append with compaction
// ---------------------------------------------------------------------------
__device__ inline void cand_append(const CandBuf& cb, int64_t slot, int& cnt, bool& ovf, float lb,
                                   uint32_t j, float U) {
  if (ovf) return;
  float* L = cb.lb + slot * cb.K;
  uint32_t* J = cb.j + slot * cb.K;
  if (cnt == cb.K) {
    int k = 0;
    for (int c = 0; c < cb.K; ++c) {
      float v = L[c];
      if (v <= U) {
        uint32_t jj = J[c];
        L[k] = v;
        J[k] = jj;
        ++k;
      }
    }
    cnt = k;
    if (cnt == cb.K) {
      ovf = true;
      return;
    }
  }
  L[cnt] = lb;
  J[cnt] = j;
  ++cnt;
}

__device__ inline int64_t list_len(const QueryList& L) { return L.list ? (int64_t)*L.count : L.m; }
__device__ inline int64_t list_query(const QueryList& L, int64_t p) { return L.list ? (int64_t)L.list[p] : p; }

// ---------------------------------------------------------------------------
// FP64 MFMA scan.  v_mfma_f64_16x16x4: A (16 data rows x 4 k) one double per
// lane (row = lane%16, k = lane/16), B (4 k x 16 queries) one double per lane
// (query = lane%16, k = lane/16), D register i holds row lane/16 + 4 i of
// query lane%16.
// Score s_j = |x_j|^2 - 2 q.x_j over K = 12 (three MFMAs); d~ = s + |q|^2.
// ---------------------------------------------------------------------------
constexpr int kG64 = 4;                                  // 16-query groups per wave
constexpr int kQ64 = 4 * kG64 * 16;                      // queries per workgroup

__global__ __launch_bounds__(256) void scan64_kernel(
    const double* __restrict__ w64, const double* __restrict__ n64, int64_t n_tiles, int64_t N,
    const double* __restrict__ qw, const double* __restrict__ qn2, const double* __restrict__ u64,
    const int* __restrict__ invalid, double xmax, QueryList L, CandBuf cb) {
  __shared__ double xs[2][12][kTile64];
  __shared__ double ns[2][kTile64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int S = cb.S;
  const int split = blockIdx.x % S;
  const int64_t qbase = (int64_t)(blockIdx.x / S) * kQ64;
  const int64_t len = list_len(L);
  if (qbase >= len) return;
  const int64_t t0 = (int64_t)split * n_tiles / S, t1 = (int64_t)(split + 1) * n_tiles / S;

  double b[kG64][3], qn[kG64], U[kG64], alpha[kG64];
  bool valid[kG64];
  int64_t pos[kG64];
  int cnt[kG64];
  bool ovf[kG64];
#pragma unroll
  for (int g = 0; g < kG64; ++g) {
    int64_t p = qbase + wave * 16 * kG64 + g * 16 + col;
    bool v = p < len;
    int64_t q = v ? list_query(L, p) : 0;
    v = v && !invalid[q];
    valid[g] = v;
    pos[g] = p;
#pragma unroll
    for (int s = 0; s < 3; ++s) b[g][s] = v ? -2.0 * qw[12 * q + 4 * s + kq] : 0.0;
    qn[g] = v ? qn2[q] : 0.0;
    U[g] = v ? u64[q] : INFINITY;
    double qa = sqrt(qn[g]) + xmax;
    // |d~ - d| <= 15 roundings of terms bounded by (|q| + max|x|)^2
    alpha[g] = 0x1p-48 * qa * qa + 1e-300;
    cnt[g] = 0;
    ovf[g] = false;
  }

  if (t0 < t1) {
    auto load = [&](int64_t t, double (&reg)[6], double& nreg) {
      const double* src = w64 + t * kTile64 * 12;
#pragma unroll
      for (int r = 0; r < 6; ++r) reg[r] = src[tid + 256 * r];
      nreg = (tid < kTile64) ? n64[t * kTile64 + tid] : 0.0;
    };
    auto store = [&](int buf, const double (&reg)[6], double nreg) {
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        int e = tid + 256 * r;
        xs[buf][e % 12][e / 12] = reg[r];
      }
      if (tid < kTile64) ns[buf][tid] = nreg;
    };
    double reg[6], nreg;
    load(t0, reg, nreg);
    store(0, reg, nreg);
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
      const int cur = (int)((t - t0) & 1);
      const bool more = t + 1 < t1;
      if (more) load(t + 1, reg, nreg);
      double tm[kG64];
#pragma unroll
      for (int g = 0; g < kG64; ++g) tm[g] = INFINITY;
#pragma unroll 2
      for (int rb = 0; rb < kTile64 / 16; ++rb) {
        const int r0 = rb * 16 + col;
        double a0 = xs[cur][kq][r0], a1 = xs[cur][4 + kq][r0], a2 = xs[cur][8 + kq][r0];
        double nr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) nr[i] = ns[cur][rb * 16 + kq + 4 * i];
#pragma unroll
        for (int g = 0; g < kG64; ++g) {
          f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[g][0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b[g][1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b[g][2], acc, 0, 0, 0);
          double m01 = fmin(acc[0] + nr[0], acc[1] + nr[1]);
          double m23 = fmin(acc[2] + nr[2], acc[3] + nr[3]);
          tm[g] = fmin(tm[g], fmin(m01, m23));
        }
      }
#pragma unroll
      for (int g = 0; g < kG64; ++g) {
        double v = tm[g];
        v = fmin(v, __shfl_xor(v, 16));
        v = fmin(v, __shfl_xor(v, 32));
        double dmin = v + qn[g];
        double Un = fmin(U[g], dmin + alpha[g]);
        bool need = valid[g] && (dmin - alpha[g] <= Un);
        U[g] = Un;
        if (__any(need)) {
          const float Uf = __double2float_ru(U[g]);
          const int64_t slot = (pos[g] * S + split) * 4 + kq;
          for (int rb = 0; rb < kTile64 / 16; ++rb) {
            const int r0 = rb * 16 + col;
            f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][kq][r0], b[g][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][4 + kq][r0], b[g][1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][8 + kq][r0], b[g][2], acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = rb * 16 + kq + 4 * i;
              const int64_t j = t * kTile64 + row;
              double d = acc[i] + ns[cur][row] + qn[g];
              double lb = d - alpha[g];
              if (valid[g] && j < N && lb <= U[g])
                cand_append(cb, slot, cnt[g], ovf[g], __double2float_rd(lb), (uint32_t)j, Uf);
            }
          }
        }
      }
      if (more) store(cur ^ 1, reg, nreg);
      __syncthreads();
    }
  }
#pragma unroll
  for (int g = 0; g < kG64; ++g) {
    if (pos[g] < len) {
      const int64_t slot = (pos[g] * S + split) * 4 + kq;
      cb.count[slot] = cnt[g] | (ovf[g] ? kOverflowBit : 0);
      if (kq == 0) cb.U[pos[g] * S + split] = __double2float_ru(U[g]);
    }
  }
}

dd_status launch_scan64(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len_max,
                        const CandBuf& cb, hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  int64_t qblocks = (list_len_max + kQ64 - 1) / kQ64;
  int64_t n_tiles = D.n_pad64 / kTile64;
  hipLaunchKernelGGL(scan64_kernel, dim3((unsigned)(qblocks * cb.S)), dim3(256), 0, st,
                     D.w64.as<double>(), D.n64.as<double>(), n_tiles, D.N, Q.qw, Q.qn2, Q.u64,
                     Q.invalid, D.xmax, L, cb);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// 16-bit MFMA scan over tile-centred data.  v_mfma_f32_32x32x16_{bf16,f16}:
// A (32 data rows x 16 k): lane supplies row lane%32, k = 8*(lane/32)..+7;
// B (16 k x 32 queries): lane supplies query lane%32, same k range;
// D: lane holds rows 8*(i/4) + 4*(lane/32) + i%4 (i < 16) of query lane%32.
// Data row (-2 x', n_hi, n_mid, n_lo, 0), query column (q', 1, 1, 1, 0) with
// q' = round16(q - c_T): the MFMA yields |x'|^2 - 2 q'.x', and d~ = that + |q'|^2.
// ---------------------------------------------------------------------------
template <class T16> struct Vec16;
template <> struct Vec16<Bf16> {
  typedef bf16x8_t type;
  __device__ static inline f32x16_t mfma(type a, type b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Vec16<Fp16> {
  typedef f16x8_t type;
  __device__ static inline f32x16_t mfma(type a, type b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

__device__ inline float min16(const f32x16_t& a) {
  float m0 = fminf(fminf(a[0], a[1]), a[2]);
  float m1 = fminf(fminf(a[3], a[4]), a[5]);
  float m2 = fminf(fminf(a[6], a[7]), a[8]);
  float m3 = fminf(fminf(a[9], a[10]), a[11]);
  float m4 = fminf(fminf(a[12], a[13]), a[14]);
  float m5 = fminf(fminf(m0, m1), m2);
  float m6 = fminf(fminf(m3, m4), a[15]);
  return fminf(m5, m6);
}

constexpr int kG16 = 2;                                  // 32-query groups per wave
constexpr int kQ16 = 4 * kG16 * 32;                      // queries per workgroup

template <class T16, int TILE>
__global__ __launch_bounds__(256) void scan16_kernel(
    const uint4* __restrict__ wp, const float* __restrict__ centre, const float* __restrict__ radius,
    int64_t n_tiles, int64_t N, const double* __restrict__ qw, const double* __restrict__ qn2,
    const float* __restrict__ u32, const int* __restrict__ invalid, QueryList L, CandBuf cb) {
  typedef typename Vec16<T16>::type vec_t;
  constexpr int V = TILE * 2 / 256;   // uint4 per thread per tile
  static_assert(V >= 1 && TILE * 2 % 256 == 0, "tile");
  __shared__ uint4 lds[2][TILE * 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, col = lane & 31;
  const int S = cb.S;
  const int split = blockIdx.x % S;
  const int64_t qbase = (int64_t)(blockIdx.x / S) * kQ16;
  const int64_t len = list_len(L);
  if (qbase >= len) return;
  const int64_t t0 = (int64_t)split * n_tiles / S, t1 = (int64_t)(split + 1) * n_tiles / S;

  float qf[kG16][8], qabs[kG16], U[kG16];
  bool valid[kG16];
  int64_t pos[kG16];
  int cnt[kG16];
  bool ovf[kG16];
#pragma unroll
  for (int g = 0; g < kG16; ++g) {
    int64_t p = qbase + wave * 32 * kG16 + g * 32 + col;
    bool v = p < len;
    int64_t q = v ? list_query(L, p) : 0;
    v = v && !invalid[q];
    valid[g] = v;
    pos[g] = p;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      int k = 8 * h + i;
      qf[g][i] = (k < 12) ? (v ? (float)qw[12 * q + k] : 0.0f) : (k < 15 ? 1.0f : 0.0f);
    }
    qabs[g] = v ? (float)sqrt(qn2[q]) : 0.0f;
    U[g] = v ? u32[q] : INFINITY;
    cnt[g] = 0;
    ovf[g] = false;
  }

  if (t0 < t1) {
    uint4 pre[V];
    {
      const uint4* src = wp + t0 * TILE * 2;
#pragma unroll
      for (int v = 0; v < V; ++v) lds[0][tid + 256 * v] = src[tid + 256 * v];
    }
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
      const int cur = (int)((t - t0) & 1);
      const bool more = t + 1 < t1;
      if (more) {
        const uint4* src = wp + (t + 1) * TILE * 2;
#pragma unroll
        for (int v = 0; v < V; ++v) pre[v] = src[tid + 256 * v];
      }
      // centred query operands of this tile
      const float* cp = centre + 12 * t;
      const float rad = radius[t];
      float cs[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) cs[i] = h ? (i < 4 ? cp[8 + i] : 0.0f) : cp[i];
      vec_t B[kG16];
      float o[kG16], eta[kG16], alpha[kG16];
#pragma unroll
      for (int g = 0; g < kG16; ++g) {
        uint16_t bits[8];
        float rsq = 0.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          bits[i] = T16::from_float(qf[g][i] - cs[i]);
          float rv = T16::to_float(bits[i]);
          if (i < 4 || h == 0) rsq = fmaf(rv, rv, rsq);
        }
        o[g] = rsq + __shfl_xor(rsq, 32);
        uint4 pk;
        pk.x = bits[0] | ((uint32_t)bits[1] << 16);
        pk.y = bits[2] | ((uint32_t)bits[3] << 16);
        pk.z = bits[4] | ((uint32_t)bits[5] << 16);
        pk.w = bits[6] | ((uint32_t)bits[7] << 16);
        B[g] = __builtin_bit_cast(vec_t, pk);
        const float so = sqrtf(o[g]);
        // |q^' - (q - c)| <= u (|q - c| + ...) with |q - c| <= so / (1 - u); |x^' - x'| <= u r
        eta[g] = (T16::kUnit * (1.0043f * so + rad) + 1.8e-7f * (qabs[g] + so) + 8.0f * T16::kAbs) * kRelUp;
        const float sr = so + rad;
        alpha[g] = 3.814697265625e-06f * sr * sr + 16.0f * T16::kAbs;   // 2^-18 (|q'| + r)^2
      }
      float tm[kG16];
#pragma unroll
      for (int g = 0; g < kG16; ++g) tm[g] = INFINITY;
      const f32x16_t zero = {};
#pragma unroll 4
      for (int rb = 0; rb < TILE / 32; ++rb) {
        vec_t A = __builtin_bit_cast(vec_t, lds[cur][(rb * 32 + col) * 2 + h]);
#pragma unroll
        for (int g = 0; g < kG16; ++g) {
          f32x16_t acc = Vec16<T16>::mfma(A, B[g], zero);
          tm[g] = fminf(tm[g], min16(acc));
        }
      }
#pragma unroll
      for (int g = 0; g < kG16; ++g) {
        float v = fminf(tm[g], __shfl_xor(tm[g], 32));
        float dmin = v + o[g];
        float Uc = (sqrtf(dmin + alpha[g]) + eta[g]) * kRelUp;
        float Un = fminf(U[g], Uc);
        float lbmin = sqrtf(fmaxf(dmin - alpha[g], 0.0f)) * kRelDn - eta[g];
        bool need = valid[g] && (lbmin <= Un);
        U[g] = Un;
        if (__any(need)) {
          const int64_t slot = (pos[g] * S + split) * 2 + h;
          for (int rb = 0; rb < TILE / 32; ++rb) {
            vec_t A = __builtin_bit_cast(vec_t, lds[cur][(rb * 32 + col) * 2 + h]);
            f32x16_t acc = Vec16<T16>::mfma(A, B[g], zero);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int row = rb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
              const int64_t j = t * TILE + row;
              float d = acc[i] + o[g];
              float lb = sqrtf(fmaxf(d - alpha[g], 0.0f)) * kRelDn - eta[g];
              if (valid[g] && j < N && lb <= U[g])
                cand_append(cb, slot, cnt[g], ovf[g], lb, (uint32_t)j, U[g]);
            }
          }
        }
      }
      if (more) {
#pragma unroll
        for (int v = 0; v < V; ++v) lds[cur ^ 1][tid + 256 * v] = pre[v];
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int g = 0; g < kG16; ++g) {
    if (pos[g] < len) {
      const int64_t slot = (pos[g] * S + split) * 2 + h;
      cb.count[slot] = cnt[g] | (ovf[g] ? kOverflowBit : 0);
      if (h == 0) cb.U[pos[g] * S + split] = U[g];
    }
  }
}

template <class T16>
static dd_status launch16(const Dataset& D, const uint16_t* pack, const QueryPrep& Q, QueryList L,
                          int64_t list_len_max, const CandBuf& cb, hipStream_t st) {
  int64_t qblocks = (list_len_max + kQ16 - 1) / kQ16;
  dim3 grid((unsigned)(qblocks * cb.S));
  const uint4* wp = reinterpret_cast<const uint4*>(pack);
#define DD_SCAN16_CASE(TT)                                                                        \
  case TT:                                                                                        \
    hipLaunchKernelGGL((scan16_kernel<T16, TT>), grid, dim3(256), 0, st, wp, D.centre.as<float>(), \
                       D.radius.as<float>(), D.n_tiles, D.N, Q.qw, Q.qn2, Q.u32, Q.invalid, L, cb); \
    break;
  switch (D.tile) {
    DD_SCAN16_CASE(128)
    DD_SCAN16_CASE(256)
    DD_SCAN16_CASE(512)
    DD_SCAN16_CASE(1024)
    default:
      return set_error(DD_ERR_UNSUPPORTED, "16-bit scan supports tiles of 128, 256, 512 or 1024");
  }
#undef DD_SCAN16_CASE
  DD_HIP(hipGetLastError());
  return DD_OK;
}

dd_status launch_scan16(const Dataset& D, bool fp16, const QueryPrep& Q, QueryList L,
                        int64_t list_len_max, const CandBuf& cb, hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  if (fp16) return launch16<Fp16>(D, D.wfp16.as<uint16_t>(), Q, L, list_len_max, cb, st);
  return launch16<Bf16>(D, D.wbf16.as<uint16_t>(), Q, L, list_len_max, cb, st);
}

// ---------------------------------------------------------------------------
// Merge and FP64 rerank (direct form 1/2 |q - x|^2), lexicographic minimum of
// (distance, original index) over every certified candidate.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void merge_rerank_kernel(
    QueryList L, CandBuf cb, const double* __restrict__ qw, const int* __restrict__ invalid,
    const double* __restrict__ w64, const float* __restrict__ w32, const uint32_t* __restrict__ perm,
    Outputs out, int* __restrict__ fb_list, int* __restrict__ fb_count,
    unsigned long long* __restrict__ n_cand) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= list_len(L)) return;
  const int64_t q = list_query(L, p);
  if (invalid[q]) {
    out.idx[q] = -1;
    if (out.dist) out.dist[q] = NAN;
    return;
  }
  const int S = cb.S, P = cb.P, K = cb.K;
  float Uf = INFINITY;
  for (int s = 0; s < S; ++s) Uf = fminf(Uf, cb.U[p * S + s]);
  double qv[12];
  for (int k = 0; k < 12; ++k) qv[k] = qw[12 * q + k];
  double best = INFINITY;
  uint32_t bo = 0xFFFFFFFFu;
  bool ovf = false;
  unsigned long long nc = 0;
  for (int s = 0; s < S; ++s) {
    for (int part = 0; part < P; ++part) {
      const int64_t slot = (p * S + s) * P + part;
      const int c = cb.count[slot];
      ovf = ovf || (c & kOverflowBit);
      const int n = c & ~kOverflowBit;
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
  }
  if (ovf || bo == 0xFFFFFFFFu) {
    int k = atomicAdd(fb_count, 1);
    fb_list[k] = (int)q;
  } else {
    out.idx[q] = (int64_t)bo;
    if (out.dist) out.dist[q] = 0.5 * best;
  }
  if (n_cand && nc) atomicAdd(n_cand, nc);
}

dd_status launch_merge_rerank(const Dataset& D, const QueryPrep& Q, QueryList L,
                              int64_t list_len_max, const CandBuf& cb, bool /*sqrt_space*/,
                              Outputs out, int* fb_list, int* fb_count, unsigned long long* n_cand,
                              hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  hipLaunchKernelGGL(merge_rerank_kernel, dim3(grid1(list_len_max)), dim3(256), 0, st, L, cb, Q.qw,
                     Q.invalid, D.w64.as<double>(), D.w64.p ? nullptr : D.w32.as<float>(),
                     D.perm.as<uint32_t>(), out, fb_list, fb_count, n_cand);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

// ---------------------------------------------------------------------------
// Plain FP64 direct-form scan: one query per lane, data rows broadcast from LDS.
// ---------------------------------------------------------------------------
constexpr int kDirectRows = 128;

__global__ __launch_bounds__(256) void direct_kernel(
    const double* __restrict__ w64, const float* __restrict__ w32, const uint32_t* __restrict__ perm,
    int64_t n_tiles, int64_t N, const double* __restrict__ qw, const int* __restrict__ invalid,
    QueryList L, int S, double* __restrict__ part_d, uint32_t* __restrict__ part_o) {
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

dd_status run_direct(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len_max, int S,
                     Outputs out, hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  int64_t n_tiles = (D.N + kDirectRows - 1) / kDirectRows;
  int64_t qblocks = (list_len_max + 255) / 256;
  S = choose_splits(qblocks, n_tiles, S);
  double* pd = nullptr;
  uint32_t* po = nullptr;
  DD_HIP(hipMallocAsync((void**)&pd, sizeof(double) * (size_t)(list_len_max * S), st));
  DD_HIP(hipMallocAsync((void**)&po, sizeof(uint32_t) * (size_t)(list_len_max * S), st));
  hipLaunchKernelGGL(direct_kernel, dim3((unsigned)(qblocks * S)), dim3(256), 0, st,
                     D.w64.as<double>(), D.w64.p ? nullptr : D.w32.as<float>(),
                     D.perm.as<uint32_t>(), n_tiles, D.N, Q.qw, Q.invalid, L, S, pd, po);
  DD_HIP(hipGetLastError());
  hipLaunchKernelGGL(merge_direct_kernel, dim3(grid1(list_len_max)), dim3(256), 0, st, L, S, pd, po,
                     Q.invalid, out);
  DD_HIP(hipGetLastError());
  DD_HIP(hipFreeAsync(pd, st));
  DD_HIP(hipFreeAsync(po, st));
  return DD_OK;
}

}  // namespace dd
