// MFMA scans of the projection P_D (Section 2) in whitened coordinates
// (Section 3.2).  See scan.hip for the certification scheme they share.
//
// This translation unit is compiled with IEEE mode off and without NaN
// semantics (its inputs are finite: invalid queries are zeroed by the
// preparation kernel), so that min reductions of matrix-core results need no
// canonicalisation, and with matrix results kept in ordinary VGPRs.
#include <algorithm>
#include <cmath>

#include "pack16.h"
#include "scan.h"

namespace dd {

__device__ static inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }   // 1 ulp

// FP64 -> FP32 rounded up / down (finite or infinite inputs), in registers:
// the nearest conversion, moved one step when it fell on the wrong side.
__device__ inline float f32_next_up(float f) {
  if (f == 0.0f) return 0x1p-149f;
  const uint32_t u = __float_as_uint(f);
  return __uint_as_float(f > 0.0f ? u + 1u : u - 1u);
}
__device__ inline float f32_up(double d) {
  const float f = (float)d;
  return (double)f < d ? f32_next_up(f) : f;
}
__device__ inline float f32_down(double d) {
  const float f = (float)d;
  return (double)f > d ? -f32_next_up(-f) : f;
}

// Running minimum over 16 new values: 17 inputs, eight 3-input minima.
__device__ inline float min16(float run, const f32x16_t& a) {
  float m0 = fminf(fminf(a[0], a[1]), a[2]);
  float m1 = fminf(fminf(a[3], a[4]), a[5]);
  float m2 = fminf(fminf(a[6], a[7]), a[8]);
  float m3 = fminf(fminf(a[9], a[10]), a[11]);
  float m4 = fminf(fminf(a[12], a[13]), a[14]);
  float m5 = fminf(fminf(m0, m1), m2);
  float m6 = fminf(fminf(m3, m4), a[15]);
  return fminf(fminf(run, m5), m6);
}

// Split and query block of this workgroup in a grid of (query blocks x S)
// workgroups.  The command processor deals workgroups to the eight XCDs in
// turn (workgroup b runs on XCD b % 8), so the grid is renumbered to give XCD x
// the x-th eighth of the split-major order, every query block of one split
// before the next: the workgroups an XCD holds at once then stream the same
// data through its L2 instead of two or more splits competing for it.  A grid
// whose size is not a multiple of eight keeps the plain order.
__device__ inline void split_qblock(int S, int& split, int64_t& qblock) {
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned t = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
  const unsigned qblocks = G / (unsigned)S;
  split = (int)(t / qblocks);
  qblock = (int64_t)(t % qblocks);
}

// ---------------------------------------------------------------------------
// FP64 MFMA scan.  v_mfma_f64_16x16x4: A (16 data rows x 4 k) one double per
// lane (row = lane%16, k = lane/16), B (4 k x 16 queries) one double per lane
// (query = lane%16, k = lane/16), D register i holds row lane/16 + 4 i of
// query lane%16.  Score s_j = |x_j|^2 - 2 q.x_j over K = 12 (three MFMAs, the
// stored norm as the accumulator input of the first); d~ = s + |q|^2.
// ---------------------------------------------------------------------------
constexpr int kG64 = 4;                                  // 16-query groups per wave
constexpr int kQ64 = 4 * kG64 * 16;                      // queries per workgroup
// A tile is copied from HBM to LDS in 1 KB pieces, one 16-byte load per lane
// (global_load_lds_dwordx4: lane i's bytes land at the piece's LDS address
// plus 16 i): the rows (96 B each, row-major as in the pack), then the norms.
constexpr int kRowPieces64 = kTile64 * 12 * 8 / 1024;
constexpr int kPieces64 = kRowPieces64 + kTile64 * 8 / 1024;
static_assert(kTile64 * 8 % 1024 == 0, "whole 1 KB pieces of rows and norms");

typedef __attribute__((address_space(3))) unsigned char lds_byte;

// Copy a tile's rows and norms to LDS; the four waves of a workgroup take
// every fourth piece.  The copies complete asynchronously: a wait for the
// vector-memory counter and a barrier come before any wave reads them.
__device__ inline void tile_to_lds64(const double* __restrict__ w64, const double* __restrict__ n64,
                                     int64_t t, double* xs, double* ns, int wave, int lane) {
  const unsigned char* rows = reinterpret_cast<const unsigned char*>(w64 + t * kTile64 * 12);
  const unsigned char* norms = reinterpret_cast<const unsigned char*>(n64 + t * kTile64);
  for (int c = wave; c < kPieces64; c += 4) {   // a scalar loop: wave is uniform
    const bool r = c < kRowPieces64;
    const unsigned char* src = (r ? rows + 1024 * c : norms + 1024 * (c - kRowPieces64)) + 16 * lane;
    lds_byte* dst = (lds_byte*)(r ? (unsigned char*)xs + 1024 * c
                                  : (unsigned char*)ns + 1024 * (c - kRowPieces64));
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
  }
}

// s_waitcnt vmcnt(0): every copy this wave issued has reached LDS.
__device__ inline void wait_copies() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__global__ __launch_bounds__(256, 3) void scan64_kernel(
    const double* __restrict__ w64, const double* __restrict__ n64, int64_t n_tiles, int64_t N,
    const double* __restrict__ qw, const double* __restrict__ qn2, const double* __restrict__ u64,
    const int* __restrict__ invalid, double xmax, QueryList L, CandBuf cb) {
  // rows as in the pack (x of row r at xs[buf][12 r + k]), then their norms
  __shared__ __align__(16) double xs[2][kTile64 * 12];
  __shared__ __align__(16) double ns[2][kTile64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int S = cb.S;
  int split;
  int64_t qblock;
  split_qblock(S, split, qblock);
  const int64_t qbase = qblock * kQ64;
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
    // the wave index as a scalar, so that the copy loop and its LDS addresses are too
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    tile_to_lds64(w64, n64, t0, xs[0], ns[0], wu, lane);
    wait_copies();
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
      const int cur = (int)((t - t0) & 1);
      const bool more = t + 1 < t1;
      // the next tile goes to the other buffer, which every wave finished
      // reading before the barrier that ended the previous tile
      if (more) tile_to_lds64(w64, n64, t + 1, xs[cur ^ 1], ns[cur ^ 1], wu, lane);
      double tm[kG64];
#pragma unroll
      for (int g = 0; g < kG64; ++g) tm[g] = INFINITY;
#pragma unroll 2
      for (int rb = 0; rb < kTile64 / 16; ++rb) {
        const int r0 = rb * 16 + col;
        double a0 = xs[cur][12 * r0 + kq], a1 = xs[cur][12 * r0 + 4 + kq], a2 = xs[cur][12 * r0 + 8 + kq];
        double nr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) nr[i] = ns[cur][rb * 16 + kq + 4 * i];
        const f64x4_t cn = {nr[0], nr[1], nr[2], nr[3]};
#pragma unroll
        for (int g = 0; g < kG64; ++g) {
          // the rows' norms enter as the accumulator input: s = |x|^2 - 2 q.x
          f64x4_t acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b[g][0], cn, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b[g][1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b[g][2], acc, 0, 0, 0);
          tm[g] = fmin(tm[g], fmin(fmin(acc[0], acc[1]), fmin(acc[2], acc[3])));
        }
      }
#pragma unroll 1   // rolled: the rare candidate logging stays out of the code of every group
      for (int g = 0; g < kG64; ++g) {
        double v = tm[g];
        v = fmin(v, __shfl_xor(v, 16));
        v = fmin(v, __shfl_xor(v, 32));
        double dmin = v + qn[g];
        double Un = fmin(U[g], dmin + alpha[g]);
        bool need = valid[g] && (dmin - alpha[g] <= Un);
        U[g] = Un;
        if (__any(need)) {
          const float Uf = f32_up(U[g]);
          const int64_t slot = (pos[g] * S + split) * 4 + kq;
          for (int rb = 0; rb < kTile64 / 16; ++rb) {
            const int r0 = rb * 16 + col;
            f64x4_t acc;
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = ns[cur][rb * 16 + kq + 4 * i];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][12 * r0 + kq], b[g][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][12 * r0 + 4 + kq], b[g][1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[cur][12 * r0 + 8 + kq], b[g][2], acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = rb * 16 + kq + 4 * i;
              const int64_t j = t * kTile64 + row;
              double d = acc[i] + qn[g];
              double lb = d - alpha[g];
              if (valid[g] && j < N && lb <= U[g])
                cand_append(cb, slot, cnt[g], ovf[g], f32_down(lb), (uint32_t)j, Uf);
            }
          }
        }
      }
      wait_copies();
      __syncthreads();
    }
  }
#pragma unroll
  for (int g = 0; g < kG64; ++g) {
    if (pos[g] < len) {
      const int64_t slot = (pos[g] * S + split) * 4 + kq;
      cb.count[slot] = cnt[g] | (ovf[g] ? kOverflowBit : 0);
      if (kq == 0) cb.U[pos[g] * S + split] = f32_up(U[g]);
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
// FP32 MFMA scan.  v_mfma_f32_32x32x2_f32: A (32 data rows x 2 k): lane supplies
// row lane%32, k = lane/32; B (2 k x 32 queries): lane supplies query lane%32,
// k = lane/32; C and D: lane holds rows 8*(i/4) + 4*(lane/32) + i%4 (i < 16) of
// query lane%32.  Six MFMAs cover K = 12 with the data rows x^ = fl32(x) and
// the query column -2 q^, q^ = fl32(q); the accumulator input of the first is
// the rows' stored norms n^ = fl32(|x^|^2), so the matrix core returns
// s_j = n^_j - 2 q^.x^_j and d~_j = s_j + o, o = fl32(|q^|^2).
//
// Bound (d-space, u = 2^-24, Q = |q|, X >= max |x|): the stored operands move
// |q - x| by at most u (Q + X), hence |q - x|^2 by at most (2u + u^2)(Q + X)^2;
// the thirteen terms of the accumulation (twelve products and n^), the
// roundings of n^ and o and the final addition add at most 16.1 u (Q + X)^2 in
// any summation order; the FP32 evaluation of d~ +- a and of the minimum adds
// about 3 u (Q + X)^2.  a = 2^-18 (Q + X)^2 = 64 u (Q + X)^2 covers the sum
// (about 22 u) three times over.  A query with Q + X >= 2^60 (where (Q + X)^2
// could leave the FP32 range) is not scanned; the FP64 scan answers it.
// ---------------------------------------------------------------------------
constexpr int kG32 = 2;                                  // 32-query groups per wave
constexpr int kQ32 = 4 * kG32 * 32;                      // queries per workgroup (4 waves)
static_assert(kG32 == 2, "the inner loop interleaves two query groups");

__device__ inline f32x16_t mfma_f32(float a, float b, f32x16_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256, 3) void scan32_kernel(
    const float* __restrict__ w32, const float* __restrict__ n32, int64_t n_tiles, int64_t N,
    const double* __restrict__ qw, const double* __restrict__ qn2, const double* __restrict__ u64,
    const int* __restrict__ invalid, float xmax, QueryList L, CandBuf cb) {
  // xs[buf][s][h][row] = x^[row][2 s + h]; ns[buf][row] = n^[row]
  __shared__ float xs[2][6][2][kTile32];
  __shared__ __attribute__((aligned(16))) float ns[2][kTile32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, h = lane >> 5;
  const int S = cb.S;
  int split;
  int64_t qblock;
  split_qblock(S, split, qblock);
  const int64_t qbase = qblock * kQ32;
  const int64_t len = list_len(L);
  if (qbase >= len) return;
  const int64_t t0 = (int64_t)split * n_tiles / S, t1 = (int64_t)(split + 1) * n_tiles / S;

  float b[kG32][6], o[kG32], U[kG32], a[kG32];
  bool valid[kG32], ovf[kG32];
  int64_t pos[kG32];
  int cnt[kG32];
#pragma unroll
  for (int g = 0; g < kG32; ++g) {
    const int64_t p = qbase + wave * 32 * kG32 + g * 32 + col;
    bool v = p < len;
    const int64_t q = v ? list_query(L, p) : 0;
    const float qa = v ? (float)sqrt(qn2[q]) + xmax : 0.0f;
    v = v && !invalid[q] && qa < 0x1p60f;
    valid[g] = v;
    pos[g] = p;
    double oo = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double qk = v ? (double)(float)qw[12 * q + k] : 0.0;   // q^ = fl32(q)
      oo = fma(qk, qk, oo);
      if ((k & 1) == h) b[g][k >> 1] = (float)(-2.0 * qk);
    }
    o[g] = (float)oo;
    a[g] = 0x1p-18f * qa * qa + 1e-30f;
    U[g] = v ? f32_up(u64[q]) : INFINITY;
    cnt[g] = 0;
    ovf[g] = false;
  }

  if (t0 < t1) {
    // staging: thread t holds float4 number t + 256 v (v < 3) of the tile's
    // rows and the norm of row t
    auto load = [&](int64_t t, float4 (&reg)[3], float& nreg) {
      const float4* src = reinterpret_cast<const float4*>(w32 + t * kTile32 * 12);
#pragma unroll
      for (int v = 0; v < 3; ++v) reg[v] = src[tid + 256 * v];
      nreg = n32[t * kTile32 + tid];
    };
    auto store = [&](int buf, const float4 (&reg)[3], float nreg) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const int e = 4 * (tid + 256 * v), row = e / 12, k = e % 12;   // k in {0, 4, 8}
        xs[buf][k / 2][0][row] = reg[v].x;
        xs[buf][k / 2][1][row] = reg[v].y;
        xs[buf][k / 2 + 1][0][row] = reg[v].z;
        xs[buf][k / 2 + 1][1][row] = reg[v].w;
      }
      ns[buf][tid] = nreg;
    };
    static_assert(kTile32 == 256, "one staged row norm per thread");
    float4 reg[3];
    float nreg;
    load(t0, reg, nreg);
    store(0, reg, nreg);
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
      const int cur = (int)((t - t0) & 1);
      const bool more = t + 1 < t1;
      if (more) load(t + 1, reg, nreg);
      float tm0 = INFINITY, tm1 = INFINITY;
#pragma unroll 1
      for (int rb = 0; rb < kTile32 / 32; ++rb) {
        float A[6];
#pragma unroll
        for (int sk = 0; sk < 6; ++sk) A[sk] = xs[cur][sk][h][rb * 32 + col];
        f32x16_t cn;
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
          const float4 v4 = *reinterpret_cast<const float4*>(&ns[cur][rb * 32 + 8 * g4 + 4 * h]);
          cn[4 * g4 + 0] = v4.x;
          cn[4 * g4 + 1] = v4.y;
          cn[4 * g4 + 2] = v4.z;
          cn[4 * g4 + 3] = v4.w;
        }
        f32x16_t acc0 = mfma_f32(A[0], b[0][0], cn);
        f32x16_t acc1 = mfma_f32(A[0], b[1][0], cn);
#pragma unroll
        for (int sk = 1; sk < 6; ++sk) {
          acc0 = mfma_f32(A[sk], b[0][sk], acc0);
          acc1 = mfma_f32(A[sk], b[1][sk], acc1);
        }
        tm0 = min16(tm0, acc0);
        tm1 = min16(tm1, acc1);
      }
      const float tmg[kG32] = {tm0, tm1};
#pragma unroll
      for (int g = 0; g < kG32; ++g) {
        const float v = fminf(tmg[g], __shfl_xor(tmg[g], 32));
        const float dmin = v + o[g];
        const float Un = fminf(U[g], dmin + a[g]);
        const bool need = valid[g] && (dmin - a[g] <= Un);
        U[g] = Un;
        if (__any(need)) {
          // rare once the bound is tight: recompute the tile and log every row
          // whose lower bound d~ - a is within the bound
          const int64_t slot = (pos[g] * S + split) * 2 + h;
#pragma unroll 1
          for (int rb = 0; rb < kTile32 / 32; ++rb) {
            f32x16_t cn;
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
              const float4 v4 =
                  *reinterpret_cast<const float4*>(&ns[cur][rb * 32 + 8 * g4 + 4 * h]);
              cn[4 * g4 + 0] = v4.x;
              cn[4 * g4 + 1] = v4.y;
              cn[4 * g4 + 2] = v4.z;
              cn[4 * g4 + 3] = v4.w;
            }
            f32x16_t acc = cn;
#pragma unroll
            for (int sk = 0; sk < 6; ++sk) acc = mfma_f32(xs[cur][sk][h][rb * 32 + col], b[g][sk], acc);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int row = rb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
              const int64_t j = t * kTile32 + row;
              const float lb = (acc[i] + o[g]) - a[g];
              if (valid[g] && j < N && lb <= U[g])
                cand_append(cb, slot, cnt[g], ovf[g], lb, (uint32_t)j, U[g]);
            }
          }
        }
      }
      if (more) store(cur ^ 1, reg, nreg);
      __syncthreads();
    }
  }
#pragma unroll
  for (int g = 0; g < kG32; ++g) {
    if (pos[g] < len) {
      const int64_t slot = (pos[g] * S + split) * 2 + h;
      cb.count[slot] = cnt[g] | (ovf[g] ? kOverflowBit : 0);
      if (h == 0) cb.U[pos[g] * S + split] = U[g];
    }
  }
}

dd_status launch_scan32(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len_max,
                        const CandBuf& cb, hipStream_t st) {
  if (list_len_max <= 0) return DD_OK;
  if (cb.P != 2) return set_error(DD_ERR_ARG, "FP32 scan: two candidate lists per split");
  const int64_t qblocks = (list_len_max + kQ32 - 1) / kQ32;
  const int64_t n_tiles = D.n_pad32 / kTile32;
  hipLaunchKernelGGL(scan32_kernel, dim3((unsigned)(qblocks * cb.S)), dim3(256), 0, st,
                     D.w32.as<float>(), D.n32.as<float>(), n_tiles, D.N, Q.qw, Q.qn2, Q.u64,
                     Q.invalid, (float)D.xmax32, L, cb);
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
//
// Bounds per (query, tile), sqrt-space: |sqrt(d~) - sqrt(d)| <= eta + alpha terms
//   eta   = u (|q'| + r_T) + FP32 rounding of q and q - c_T (+ subnormal floor)
//   alpha = 2^-18 (|q'| + r_T)^2 >= the FP32 accumulation error of 16 terms
// EXTRACT = false: bound-only pass (no candidate lists).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

template <class T16> struct Vec16;
template <> struct Vec16<Bf16> {
  typedef bf16x8_t type;
  __device__ static inline f32x16_t mfma(type a, type b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  // two FP32 values -> packed pair, round to nearest even (v_cvt_pk_bf16_f32)
  __device__ static inline uint32_t pack2(float a, float b) {
    bf16x2_t v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
  }
  // FP32 dot of a packed pair with itself, accumulated (v_dot2c_f32_bf16)
  __device__ static inline float dot2(uint32_t p, float c) {
    bf16x2_t v = __builtin_bit_cast(bf16x2_t, p);
    return __builtin_amdgcn_fdot2_f32_bf16(v, v, c, false);
  }
};
template <> struct Vec16<Fp16> {
  typedef f16x8_t type;
  __device__ static inline f32x16_t mfma(type a, type b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  __device__ static inline uint32_t pack2(float a, float b) {
    f16x2_t v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
  }
  __device__ static inline float dot2(uint32_t p, float c) {
    f16x2_t v = __builtin_bit_cast(f16x2_t, p);
    return __builtin_amdgcn_fdot2(v, v, c, false);
  }
};

constexpr int kG16 = 2;                                  // 32-query groups per wave
constexpr int kW16 = 16;                                 // waves per workgroup
constexpr int kT16 = 64 * kW16;                          // threads per workgroup
constexpr int kQ16 = kW16 * kG16 * 32;                   // queries per workgroup
static_assert(kG16 == 2, "the pipelined inner loop is written for two query groups");

// Per-(query group, tile) operands of the 16-bit scans: centred query column
// q' = round16(q - c_T) packed for the MFMA B operand, o = |q'|^2 and the
// sqrt-space error terms eta, alpha of the bound described above.
template <class T16>
__device__ inline void tile_operands(const float (&qf)[8], float qabs, const float (&cs)[8],
                                     float rad, int h, typename Vec16<T16>::type& B, float& o,
                                     float& eta, float& alpha) {
  typedef Vec16<T16> VT;
  uint4 pk;
  pk.x = VT::pack2(qf[0] - cs[0], qf[1] - cs[1]);
  pk.y = VT::pack2(qf[2] - cs[2], qf[3] - cs[3]);
  pk.z = VT::pack2(qf[4] - cs[4], qf[5] - cs[5]);
  pk.w = VT::pack2(qf[6] - cs[6], qf[7] - cs[7]);
  B = __builtin_bit_cast(typename VT::type, pk);
  // lanes of the upper half hold coordinates 8..11 and the constant slots
  float lo = VT::dot2(pk.y, VT::dot2(pk.x, 0.0f));
  float hi = VT::dot2(pk.w, VT::dot2(pk.z, 0.0f));
  float part = h ? lo : lo + hi;
  o = part + __shfl_xor(part, 32);
  const float so = fsqrt(o);
  eta = (T16::kUnit * (1.0043f * so + rad) + 1.8e-7f * (qabs + so) + 8.0f * T16::kAbs) * kRelUp;
  const float sr = so + rad;
  alpha = 3.814697265625e-06f * sr * sr + 16.0f * T16::kAbs + 1e-30f;
}

// Lane's query coordinates for the B operand: lanes of half h hold k = 8h..8h+7
// (scaled coordinates 0..11, then the constant slots 1, 1, 1, 0).
__device__ inline void load_query_column(const double* __restrict__ qw, int64_t q, bool v, int h,
                                         double scale, float (&qf)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int k = 8 * h + i;
    qf[i] = (k < 12) ? (v ? (float)(qw[12 * q + k] * scale) : 0.0f) : (k < 15 ? 1.0f : 0.0f);
  }
}

// The query lies inside the radius around the data's mean within which its
// centred coordinates stay finite in the 16-bit format (see Scale16).
__device__ inline bool near16(const double* __restrict__ qw, int64_t q, const Scale16& sc) {
  float a = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const float t = (float)(qw[12 * q + k] * (double)sc.s) - sc.mean[k];
    a = fmaf(t, t, a);
  }
  return sc.far > 0.0f && a < sc.far * sc.far;
}

__device__ inline void centre_select(const float* __restrict__ cp, int h, float (&cs)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) cs[i] = h ? (i < 4 ? cp[8 + i] : 0.0f) : cp[i];
}

// Streaming pass of the 16-bit scan.  Every workgroup (sixteen waves: one
// workgroup with its double-buffered tile of 2048 rows, 128 KB of LDS, fills a
// CU with four waves per SIMD) covers 1024 queries (two 32-query groups per
// wave) against the tiles of its split; the split's tiles
// are visited with stride `stride` (1 = all; > 1 = a bound-seeding subsample).
// Tracks the sqrt-space bound U of each query; with MARK, appends a work item
// whenever some query of a group may have a candidate in the tile (its lower
// bound <= its running U).  Tiles are staged through LDS half-major (each lane
// reads 16 consecutive bytes of its row half: conflict-free 128-bit reads).
template <class T16, int TILE, bool MARK>
__global__ __launch_bounds__(kT16, 4) void scan16_pass_kernel(
    const uint4* __restrict__ wp, const float* __restrict__ centre, const float* __restrict__ radius,
    int64_t n_tiles, int stride, const double* __restrict__ qw, const double* __restrict__ qn2,
    const float* __restrict__ u32, const int* __restrict__ invalid, QueryList L, int S,
    float* __restrict__ U_out, WorkItem* __restrict__ items, unsigned* __restrict__ n_items,
    unsigned item_cap, Scale16 sc) {
  typedef Vec16<T16> VT;
  typedef typename VT::type vec_t;
  constexpr int V = (TILE * 2 + kT16 - 1) / kT16;   // uint4 per thread per tile
  constexpr int NB = TILE / 32;                     // 32-row blocks per tile
  static_assert(TILE * 2 % kT16 == 0 || TILE * 2 < kT16, "tile");
  auto staged = [](int e) { return TILE * 2 >= kT16 || e < TILE * 2; };
  __shared__ uint4 lds[2][2 * TILE];  // [buffer][half * TILE + row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, col = lane & 31;
  int split;
  int64_t qblock;
  split_qblock(S, split, qblock);
  const int64_t qbase = qblock * kQ16;
  const int64_t len = list_len(L);
  if (qbase >= len) return;
  const int64_t t0 = (int64_t)split * n_tiles / S, t1 = (int64_t)(split + 1) * n_tiles / S;

  float qf[kG16][8], qabs[kG16], U[kG16];
  bool valid[kG16];
  int64_t pos[kG16];
#pragma unroll
  for (int g = 0; g < kG16; ++g) {
    int64_t p = qbase + wave * 32 * kG16 + g * 32 + col;
    bool v = p < len;
    int64_t q = v ? list_query(L, p) : 0;
    v = v && !invalid[q] && near16(qw, q, sc);
    valid[g] = v;
    pos[g] = p;
    load_query_column(qw, q, v, h, (double)sc.s, qf[g]);
    qabs[g] = v ? (float)(sqrt(qn2[q]) * (double)sc.s) : 0.0f;
    U[g] = v ? u32[q] : INFINITY;
  }
  // element e of a tile (uint4 e = 2 row + half) lives at lds[half * TILE + row]
  auto lds_slot = [](int e) { return (e & 1) * TILE + (e >> 1); };

  if (t0 < t1) {
    {
      const uint4* src = wp + t0 * TILE * 2;
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (staged(tid + kT16 * v)) lds[0][lds_slot(tid + kT16 * v)] = src[tid + kT16 * v];
    }
    __syncthreads();
    int cur = 0;
    for (int64_t t = t0; t < t1; t += stride) {
      const int64_t tn = t + stride;
      const bool more = tn < t1;
      uint4 pre[V];
      {
        const uint4* src = wp + (more ? tn : t) * TILE * 2;
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (staged(tid + kT16 * v)) pre[v] = src[tid + kT16 * v];
      }
      float cs[8];
      centre_select(centre + 12 * t, h, cs);
      const float rad = radius[t];
      vec_t B[kG16];
      float o[kG16], eta[kG16], alpha[kG16];
#pragma unroll
      for (int g = 0; g < kG16; ++g) tile_operands<T16>(qf[g], qabs[g], cs, rad, h, B[g], o[g], eta[g], alpha[g]);
      // tile minimum of the scores: MFMA k = (row block k/2, group k%2); each
      // reduction lags two MFMAs behind its producer, so the wave never waits
      // on a result while the matrix core is busy
      float tm0 = INFINITY, tm1 = INFINITY;
      {
        const f32x16_t zero = {};
        const uint4* base = &lds[cur][h * TILE + col];
        f32x16_t acc[3];
        vec_t A = __builtin_bit_cast(vec_t, base[0]);
        vec_t An = A;
#pragma unroll
        for (int k = 0; k < 2 * NB + 2; ++k) {
          if (k < 2 * NB) {
            const int rb = k >> 1, g = k & 1;
            if (g == 0 && rb + 1 < NB) An = __builtin_bit_cast(vec_t, base[(rb + 1) * 32]);
            acc[k % 3] = VT::mfma(A, B[g], zero);
            if (g == 1) A = An;
          }
          if (k >= 2) {
            const int kk = k - 2;
            if (kk & 1)
              tm1 = min16(tm1, acc[kk % 3]);
            else
              tm0 = min16(tm0, acc[kk % 3]);
          }
        }
      }
      float tmg[kG16] = {tm0, tm1};
      unsigned mark = 0;
#pragma unroll
      for (int g = 0; g < kG16; ++g) {
        float v = fminf(tmg[g], __shfl_xor(tmg[g], 32));
        float dmin = v + o[g];
        U[g] = fminf(U[g], (fsqrt(dmin + alpha[g]) + eta[g]) * kRelUp);
        if (MARK) {
          float lbmin = fsqrt(fmaxf(dmin - alpha[g], 0.0f)) * kRelDn - eta[g];
          bool need = valid[g] && (lbmin <= U[g]);
          mark |= __any(need) ? (1u << g) : 0u;
        }
      }
      if (MARK && mark) {
        // rare: log the (group, tile) items; group ids are wave-uniform
        const uint32_t g0 = (uint32_t)((qbase + wave * 32 * kG16) / 32);
        if (lane == 0) {
          unsigned k = atomicAdd(n_items, (unsigned)__popc(mark));
          for (int g = 0; g < kG16; ++g)
            if ((mark >> g) & 1u) {
              if (k < item_cap) items[k] = WorkItem{g0 + (uint32_t)g, (uint32_t)t};
              ++k;
            }
        }
      }
      if (more) {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (staged(tid + kT16 * v)) lds[cur ^ 1][lds_slot(tid + kT16 * v)] = pre[v];
      }
      __syncthreads();
      cur ^= 1;
    }
  }
#pragma unroll
  for (int g = 0; g < kG16; ++g)
    if (pos[g] < len && h == 0) U_out[pos[g] * S + split] = U[g];
}

// Extraction: one wavefront per work item recomputes the item's 32 x TILE
// scores and appends every point whose sqrt-space lower bound is <= the query's
// final bound U to the query's candidate list (two lists per query, one per
// half-wave row set; slots claimed atomically, so only the order of a list
// varies between runs, never its content).
template <class T16, int TILE>
__global__ __launch_bounds__(256) void scan16_extract_kernel(
    const uint4* __restrict__ wp, const float* __restrict__ centre, const float* __restrict__ radius,
    int64_t N, const double* __restrict__ qw, const double* __restrict__ qn2,
    const float* __restrict__ u32, const int* __restrict__ invalid, QueryList L,
    const WorkItem* __restrict__ items, const unsigned* __restrict__ n_items, unsigned item_cap,
    CandBuf cb, Scale16 sc) {
  typedef Vec16<T16> VT;
  typedef typename VT::type vec_t;
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  const unsigned w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const unsigned total = min(*n_items, item_cap);
  if (w >= total) return;
  const WorkItem it = items[w];
  const int64_t len = list_len(L);
  const int64_t p = (int64_t)it.group * 32 + col;
  bool v = p < len;
  const int64_t q = v ? list_query(L, p) : 0;
  v = v && !invalid[q] && near16(qw, q, sc);
  float qf[8];
  load_query_column(qw, q, v, h, (double)sc.s, qf);
  const float qabs = v ? (float)(sqrt(qn2[q]) * (double)sc.s) : 0.0f;
  const float Uq = v ? u32[q] : -INFINITY;
  const int64_t t = it.tile;
  float cs[8];
  centre_select(centre + 12 * t, h, cs);
  vec_t B;
  float o, eta, alpha;
  tile_operands<T16>(qf, qabs, cs, radius[t], h, B, o, eta, alpha);
  const f32x16_t zero = {};
  const uint4* src = wp + t * TILE * 2;
  float* L0 = cb.lb + (p * 2 + h) * cb.K;
  uint32_t* J0 = cb.j + (p * 2 + h) * cb.K;
  // Score-space screen: a score whose lower bound
  //   lb = sqrt(max(s + o - alpha, 0)) (1 - 2^-20) - eta   (FP32 evaluation)
  // is <= U satisfies sqrt(max(s + o - alpha, 0)) <= a = (U + eta)(1 + 2^-18), hence
  // s <= a^2 + alpha - o, up to FP32 roundings of at most a few 2^-24 of
  // a^2 + alpha + |o|; the screen adds 2^-18 of that, so it passes every score
  // the lower-bound test keeps, and only those get the square root.
  const float a = (Uq + eta) * (1.0f + 0x1p-18f);
  const float sa = a * a + alpha;
  const float T = v ? (sa - o) + 0x1p-18f * (sa + fabsf(o)) + 1e-30f : -INFINITY;
  // row blocks in groups of kU: their operands are loaded together, and a row
  // block's scores are screened one by one only when their minimum passes
  constexpr int kU = TILE / 32 < 8 ? TILE / 32 : 8;
  for (int rb0 = 0; rb0 < TILE / 32; rb0 += kU) {
    vec_t A[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) A[u] = __builtin_bit_cast(vec_t, src[((rb0 + u) * 32 + col) * 2 + h]);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const f32x16_t acc = VT::mfma(A[u], B, zero);
      if (min16(INFINITY, acc) <= T) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (acc[i] <= T) {
            const int row = (rb0 + u) * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            const int64_t j = t * TILE + row;
            const float lb = fsqrt(fmaxf(acc[i] + o - alpha, 0.0f)) * kRelDn - eta;
            if (j < N && lb <= Uq) {
              int k = atomicAdd(&cb.count[p * 2 + h], 1);
              if (k < cb.K) {
                L0[k] = lb;
                J0[k] = (uint32_t)j;
              }
            }
          }
        }
      }
    }
  }
}

template <class T16, int TILE>
static dd_status launch16(const Dataset& D, const uint16_t* pack, const Scan16Call& c, hipStream_t st) {
  const uint4* wp = reinterpret_cast<const uint4*>(pack);
  const int64_t qblocks = (c.list_len_max + kQ16 - 1) / kQ16;
  Scale16 sc = D.sc16;
  const double limit = T16::kUnit < 0.001f ? kFarLimitFp16 : kFarLimitBf16;
  sc.far = (float)std::max(0.0, limit - D.span16);
  if (c.phase == Scan16Call::kExtract) {
    const unsigned waves = c.item_cap;   // grid sized for the capacity; extra waves exit
    const unsigned blocks = (unsigned)(((uint64_t)waves * 64 + 255) / 256);
    if (blocks == 0) return DD_OK;
    hipLaunchKernelGGL((scan16_extract_kernel<T16, TILE>), dim3(blocks), dim3(256), 0, st, wp,
                       D.centre.as<float>(), D.radius.as<float>(), D.N, c.Q->qw, c.Q->qn2,
                       c.Q->u32, c.Q->invalid, c.L, c.items, c.n_items, c.item_cap, c.cb, sc);
  } else if (c.phase == Scan16Call::kMark) {
    hipLaunchKernelGGL((scan16_pass_kernel<T16, TILE, true>), dim3((unsigned)(qblocks * c.S)),
                       dim3(kT16), 0, st, wp, D.centre.as<float>(), D.radius.as<float>(), D.n_tiles,
                       c.stride, c.Q->qw, c.Q->qn2, c.Q->u32, c.Q->invalid, c.L, c.S, c.U_out,
                       c.items, c.n_items, c.item_cap, sc);
  } else {
    hipLaunchKernelGGL((scan16_pass_kernel<T16, TILE, false>), dim3((unsigned)(qblocks * c.S)),
                       dim3(kT16), 0, st, wp, D.centre.as<float>(), D.radius.as<float>(), D.n_tiles,
                       c.stride, c.Q->qw, c.Q->qn2, c.Q->u32, c.Q->invalid, c.L, c.S, c.U_out,
                       c.items, c.n_items, c.item_cap, sc);
  }
  DD_HIP(hipGetLastError());
  return DD_OK;
}

template <class T16>
static dd_status launch16_tile(const Dataset& D, const uint16_t* pack, const Scan16Call& c,
                               hipStream_t st) {
  switch (D.tile) {
    case 128: return launch16<T16, 128>(D, pack, c, st);
    case 256: return launch16<T16, 256>(D, pack, c, st);
    case 512: return launch16<T16, 512>(D, pack, c, st);
    case 1024: return launch16<T16, 1024>(D, pack, c, st);
    case 2048: return launch16<T16, 2048>(D, pack, c, st);
    default:
      return set_error(DD_ERR_UNSUPPORTED,
                       "16-bit scan supports tiles of 128, 256, 512, 1024 or 2048");
  }
}

dd_status launch_scan16(const Dataset& D, bool fp16, const Scan16Call& c, hipStream_t st) {
  if (c.list_len_max <= 0) return DD_OK;
  if (fp16) return launch16_tile<Fp16>(D, D.wfp16.as<uint16_t>(), c, st);
  return launch16_tile<Bf16>(D, D.wbf16.as<uint16_t>(), c, st);
}

}  // namespace dd
