// DD_ANN: warm-started walk over the box tree of the dataset (P_D of Section 2
// by a search that starts from the previous association, as the graph walks of
// Section 4.3 do, and that may stop early under a budget, as the approximate
// searches of Section 4 trade accuracy for time).
//
// One wavefront per query.  The tree's level-0 boxes bound leaves of 64
// consecutive points of the spatially sorted data, each higher level bounds 64
// boxes of the level below; boxes live in principal-axis coordinates y = V^T x
// (a rotation of the whitened space, so box distances are lower bounds of
// whitened distances).  The walk is depth-first with the children of a node
// pushed farthest-first, so the nearest box is always expanded next; a box is
// skipped when its lower bound exceeds the current bound U.
//
// Leaves are stored compactly: per leaf its centre c and radius r (FP32), per
// point the FP16 offset (x - c) / r, both in the boxes' principal-axis
// coordinates (a rotation: distances are those of the whitened space, and
// the walk needs only the rotated query); a leaf's box is read quantised to 8 bits
// inside its parent's box, decoded outward.
//
// Certification.  s~ = r sqrt(sum (q'' - x'')^2) in FP32 with q'' = (q - c)/r
// differs from the exact whitened distance by at most
// E = r (2^-11 + 2^-22) 1.001 + 2^-20 (2 s~ + |q| + 2 r): the FP16 rounding of
// the offsets (2^-11 relative, 2^-25 absolute below the normal range, times r)
// plus the FP32 rounding of the query, the centring, 12 fused multiply-adds and
// the square root, with a wide margin.  U is the minimum of s~ + E over
// everything seen (and the exact warm-start distance);
// a point is kept as a candidate while s~ - E <= U.  Every point of a skipped
// box, and every dropped candidate, is strictly farther than U, which is at
// least the true minimum, so the kept candidates always contain every exact
// minimiser once the walk runs to completion (budget 0); they are reranked in
// FP64 direct form with ties to the lowest original index.  A candidate list
// that overflows sends the query to the FP64 scan.
#include <cmath>

#include "scan.h"

namespace dd {

namespace {

constexpr int kWaves = 4;                          // queries (wavefronts) per block
// depth-first stack entries per wave: at most 63 pending siblings per level,
// for the box tree's kAnnMaxLevels and the k-means tree's deeper cut
constexpr int kStack = kAnnFan * 10;
constexpr int kCand = 64;                          // candidate list entries per wave
constexpr int kBatch = 2;                          // leaves whose loads are issued together
constexpr int kRankSort = 16;                      // children ordered by rank up to this many
constexpr float kEps20 = 9.5367431640625e-07f;     // 2^-20
constexpr float kEps22 = 2.384185791015625e-07f;   // 2^-22
constexpr float kLbShrink = 1.0f - 1.9073486328125e-06f;   // 1 - 2^-19
constexpr float kLeafRel = (4.8828125e-04f + 2.384185791015625e-07f) * 1.001f;   // (2^-11 + 2^-22)

// Square root by the bare v_sqrt_f32 (within 1 ulp; a subnormal argument may
// give 0): the 2^-19 shrink of every box bound and the 2^-20 s~ term of the
// point error E cover it many times over, and a distance below 2^-63 r is far
// inside E's absolute terms.
__device__ inline float wsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

struct AnnArgs {
  const float* box[kAnnMaxLevels];
  int64_t n[kAnnMaxLevels];
  int levels;
  const float* meta;       // [n_leaf][16]: c[12], r, 1/r
  const uint8_t* q0;       // [n_leaf][24] quantised leaf boxes (levels >= 2)
  const uint16_t* h16;     // [n_leaf*64][12] FP16 scaled offsets
  const double* w64;
  const uint32_t* perm;
  const uint32_t* iperm;
  int64_t N;
  const float* yq;         // [m][12] queries on the principal axes (rotate_queries_kernel)
  float xmax;
  int budget;
  QueryList L;
  const double* qw;
  const double* qn2;
  const float* u32;
  const int* invalid;
  const int64_t* warm;
  Outputs out;
  // k-means tree (KMT): nodes, child records, slot <-> sorted position, f_d
  const int2* kmt_node;
  const float* kmt_nbox;
  const float* kmt_child;
  const uint32_t* slot_pos;
  const uint32_t* pos_slot;
  float fd;
  // optional per-query accuracy (indexed by query): radius factor of the
  // k-means walk and leaf budget, replacing fd and budget
  const float* fd_q;
  const int* budget_q;
  double* dist2;                  // TOP2: distance to the second nearest point (1/2 d^2)
  int* fb_list;
  int* fb_count;
  // kCounterSlots slots, kCounterStride u64 apart: [0] points visited, [1] boxes
  // tested, [2] leaves, [3] candidates, [4] leaf boxes tested, [5] nodes
  // expanded (k-means tree); block b adds into slot b % kCounterSlots
  // (one cache line each, so the per-wave atomics do not all meet on one line)
  unsigned long long* counters;
};

// The walk reads the tree and the leaves, which no kernel writes while it runs,
// through the constant address space where the address is the same in every
// lane (a leaf's centre and radius, a node's box and child range): such loads
// become scalar loads into SGPRs instead of 64 identical vector loads.
template <class T>
__device__ inline const __attribute__((address_space(4))) T* uniform_ptr(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// v from another lane of the same row of 16 (DPP control C); every lane active
template <int C>
__device__ inline float dpp_f(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), C, 0xF, 0xF, false));
}

__device__ inline float lane_f(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Minimum over the wavefront (every lane active): within rows of 16 by DPP
// (quad xor 1, quad xor 2, half-row mirror, row mirror), then the four rows.
__device__ inline float wave_min_f(float v) {
  v = fminf(v, dpp_f<0xB1>(v));
  v = fminf(v, dpp_f<0x4E>(v));
  v = fminf(v, dpp_f<0x141>(v));
  v = fminf(v, dpp_f<0x140>(v));
  return fminf(fminf(lane_f(v, 0), lane_f(v, 16)), fminf(lane_f(v, 32), lane_f(v, 48)));
}

__device__ inline int lanes_below(uint64_t mask, int lane) {
  return __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
}

__device__ inline float half_lo(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
}
__device__ inline float half_hi(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// Centred, scaled query of a leaf: qs = (q - c) / r (q in the leaves' frame:
// principal-axis coordinates for the box tree, whitened for the k-means tree).
__device__ inline void leaf_query(const float* __restrict__ meta, int64_t leaf, const float qf[12],
                                  float qs[12], float& r, uint32_t& count) {
  const auto* m = uniform_ptr(meta + 16 * leaf);
  r = m[12];
  const float inv_r = m[13];
  count = __builtin_bit_cast(uint32_t, m[14]);
#pragma unroll
  for (int k = 0; k < 12; ++k) qs[k] = (qf[k] - m[k]) * inv_r;
}

// s~ of stored point pos (FP16 scaled offsets, direct form, fixed order).
__device__ inline float leaf_point_dist(const uint16_t* __restrict__ h16, int64_t pos,
                                        const float qs[12], float r) {
  const uint2* p = reinterpret_cast<const uint2*>(h16 + 12 * pos);
  const uint2 a = p[0], b = p[1], c = p[2];
  const float x[12] = {half_lo(a.x), half_hi(a.x), half_lo(a.y), half_hi(a.y),
                       half_lo(b.x), half_hi(b.x), half_lo(b.y), half_hi(b.y),
                       half_lo(c.x), half_hi(c.x), half_lo(c.y), half_hi(c.y)};
  float d = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const float t = qs[k] - x[k];
    d = fmaf(t, t, d);
  }
  return r * wsqrt(d);
}

// s~ from a point's preloaded FP16 scaled offsets.
__device__ inline float leaf_point_dist_r(const uint2 (&xr)[3], const float qs[12], float r) {
  const uint2 a = xr[0], b = xr[1], c = xr[2];
  const float x[12] = {half_lo(a.x), half_hi(a.x), half_lo(a.y), half_hi(a.y),
                       half_lo(b.x), half_hi(b.x), half_lo(b.y), half_hi(b.y),
                       half_lo(c.x), half_hi(c.x), half_lo(c.y), half_hi(c.y)};
  float d = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const float t = qs[k] - x[k];
    d = fmaf(t, t, d);
  }
  return r * wsqrt(d);
}

// Lower bound from a box quantised inside its parent box (plo, step), given as
// its 24 bytes (lo[12], hi[12]) in six words, decoded outward by delta, which
// exceeds the FP32 rounding of the decoding.
__device__ __attribute__((always_inline)) inline float qbox_lb_words(const uint32_t (&v)[6], const float plo[12],
                                      const float step[12], float delta, const float yq[12],
                                      float slack) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const float ql = (float)((v[a >> 2] >> (8 * (a & 3))) & 0xFFu);
    const float qh = (float)((v[3 + (a >> 2)] >> (8 * (a & 3))) & 0xFFu);
    const float lo = fmaf(ql, step[a], plo[a]) - delta;
    const float hi = fmaf(qh, step[a], plo[a]) + delta;
    const float g = fmaxf(fmaxf(lo - yq[a], yq[a] - hi), 0.0f);
    s = fmaf(g, g, s);
  }
  return wsqrt(s) * kLbShrink - slack;
}

// The same with the parent box given by its corners (the step formed at use,
// so that only the corners stay live; uniform, they can sit in scalar registers).
__device__ __attribute__((always_inline)) inline float qbox_lb_corners(
    const uint32_t (&v)[6], const float plo[12], const float phi[12], float delta,
    const float yq[12], float slack) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const float step = (phi[a] - plo[a]) * (1.0f / 255.0f);
    const float ql = (float)((v[a >> 2] >> (8 * (a & 3))) & 0xFFu);
    const float qh = (float)((v[3 + (a >> 2)] >> (8 * (a & 3))) & 0xFFu);
    const float lo = fmaf(ql, step, plo[a]) - delta;
    const float hi = fmaf(qh, step, plo[a]) + delta;
    const float g = fmaxf(fmaxf(lo - yq[a], yq[a] - hi), 0.0f);
    s = fmaf(g, g, s);
  }
  return wsqrt(s) * kLbShrink - slack;
}

__device__ inline float qbox_lb(const uint8_t* __restrict__ q, const float plo[12],
                                const float step[12], float delta, const float yq[12],
                                float slack) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(q);
  uint32_t v[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = w[i];
  return qbox_lb_words(v, plo, step, delta, yq, slack);
}

// Lower bound of the whitened distance from the query to box b, minus the slack
// that covers the rounding of the query's rotated coordinates and of this sum.
__device__ inline float box_lb(const float* __restrict__ b, const float yq[12], float slack) {
  const float4* r = reinterpret_cast<const float4*>(b);
  const float4 l0 = r[0], l1 = r[1], l2 = r[2], h0 = r[3], h1 = r[4], h2 = r[5];
  const float lo[12] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w, l2.x, l2.y, l2.z, l2.w};
  const float hi[12] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x, h2.y, h2.z, h2.w};
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    const float g = fmaxf(fmaxf(lo[a] - yq[a], yq[a] - hi[a]), 0.0f);
    s = fmaf(g, g, s);
  }
  return wsqrt(s) * kLbShrink - slack;
}

// Lower bound of the whitened distance from the query to the points of a
// k-means tree child record: the ball (centre c, radius r >= max |x - c|)
// gives |q - c| - f_d r (|q - c| shrunk by the slack that covers the rounding
// of the query and of this sum), exact for f_d = 1 and the approximate test of
// Section 4.2 for f_d < 1; with f_d = 1 the bound is also at least the
// distance to the record's box in principal-axis coordinates (quantised inside
// the owner node's box plo, phi; decoding margin delta).  dc receives the
// shrunk |q - c| (the order in which the approximate search visits siblings).
__device__ __attribute__((always_inline)) inline float record_lb(
    const float* __restrict__ rec, const float qf[12], const float yq[12], float slack, float fd,
    const float plo[12], const float phi[12], float delta, uint32_t& code, float& dc) {
  const float4* m = reinterpret_cast<const float4*>(rec);
  const float4 a = m[0], b = m[1], c = m[2], e = m[3];
  const float cc[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const float t = qf[k] - cc[k];
    s = fmaf(t, t, s);
  }
  code = __builtin_bit_cast(uint32_t, e.y);
  dc = wsqrt(s) * kLbShrink - slack;
  const float ball = dc - fd * e.x;
  if (fd != 1.0f) return ball;
  const float4 f = m[4];
  const uint32_t v[6] = {__builtin_bit_cast(uint32_t, e.z), __builtin_bit_cast(uint32_t, e.w),
                         __builtin_bit_cast(uint32_t, f.x), __builtin_bit_cast(uint32_t, f.y),
                         __builtin_bit_cast(uint32_t, f.z), __builtin_bit_cast(uint32_t, f.w)};
  return fmaxf(ball, qbox_lb_corners(v, plo, phi, delta, yq, slack));
}

// Ascending bitonic sort of (key, val) across the 64 lanes of a wavefront;
// AUX: aux travels with its key.
template <bool AUX>
__device__ inline void wave_sort64(float& key, uint32_t& val, float& aux, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const float ok = __shfl_xor(key, j);
      const uint32_t ov = __shfl_xor(val, j);
      const float oa = AUX ? __shfl_xor(aux, j) : 0.0f;
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const bool take = (lower == up) ? (ok < key) : (ok > key);
      if (take) {
        key = ok;
        val = ov;
        if (AUX) aux = oa;
      }
    }
  }
}

// TOP2: certify the two nearest points instead of the nearest: the pruning
// bound is the second smallest of the per-point upper bounds seen (U2), so the
// candidates hold every point within the second-smallest distance.
//
// KMT: walk the k-means tree instead of the box tree (ball bounds, padded
// leaf blocks addressed by slot).  Siblings are visited nearest centre first
// (the exact walk too: a near centre finds a small distance sooner than the
// smallest lower bound does, so fewer branches stay open; the box tree has no
// centres above its leaves and keeps the bound order).  With f_d < 1 the walk
// is the approximate search of Section 4.2: a child is entered while
// |q - c| - f_d r stays below the best distance the walk itself has found (none
// at the start, so the first descent always reaches a leaf: the warm-start
// point bounds no branch), and the warm-start point remains a candidate, so the
// answer is never farther than the previous association.
//
// Occupancy: at least six waves per SIMD (at most 80 registers, no spills):
// a walk's pace is set by the latency of its dependent steps, which more waves
// hide.  The wave index is declared uniform, so that the query, its bounds and
// the per-wave statistics live in scalar registers.
template <bool TOP2, bool KMT>
__global__ __launch_bounds__(256, 6) void ann_walk_kernel(AnnArgs A) {
  __shared__ uint32_t s_code[kWaves][kStack];
  __shared__ float s_lb[kWaves][kStack];
  __shared__ uint32_t s_cpos[kWaves][kCand];
  __shared__ float s_clb[kWaves][kCand];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t p = (int64_t)blockIdx.x * kWaves + wv;
  if (p >= list_len(A.L)) return;
  const int64_t q = list_query(A.L, p);
  // one wave per query: the per-query accuracy is wave-uniform (scalar registers)
  float fd = A.fd;
  int budget = A.budget;
  if (KMT && A.fd_q)
    fd = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, A.fd_q[q])));
  if (A.budget_q) budget = __builtin_amdgcn_readfirstlane(A.budget_q[q]);
  if (A.invalid[q]) {
    if (lane == 0) {
      A.out.idx[q] = -1;
      // a quiet NaN by its bits: this file is compiled without NaN semantics
      const double nan64 = __builtin_bit_cast(double, 0x7FF8000000000000ull);
      if (A.out.dist) A.out.dist[q] = nan64;
      if (TOP2) A.dist2[q] = nan64;
    }
    return;
  }
  float qf[12], yq[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    qf[k] = (float)A.qw[12 * q + k];
    yq[k] = A.yq[12 * q + k];
  }
  const float qnorm = (float)sqrt(A.qn2[q]);
  const float ebase = kEps20 * qnorm;
  const float slack = kEps22 * (qnorm + A.xmax) + 1e-30f;
  // U: pruning bound (the smallest upper bound seen; with TOP2 the second
  // smallest over distinct points, U1 tracking the smallest)
  float U = TOP2 ? INFINITY : A.u32[q];
  float U1 = INFINITY;
  // approximate k-means search: Ua, the best upper bound over the points the
  // walk has evaluated, decides which branches are entered
  const bool approx = KMT && fd != 1.0f;
  float Ua = INFINITY;
  int nc = 0;
  bool ovf = false;

  // the warm-start point is the first candidate (TOP2: it is found by the walk,
  // which then counts it once)
  if (A.warm && !TOP2) {
    const int64_t wi = A.warm[q];
    if (wi >= 0 && wi < A.N) {
      const int64_t pos = KMT ? (int64_t)A.pos_slot[A.iperm[wi]] : (int64_t)A.iperm[wi];
      float qs[12], r;
      uint32_t count;
      leaf_query(A.meta, pos / kAnnLeaf, KMT ? qf : yq, qs, r, count);
      const float s = leaf_point_dist(A.h16, pos, qs, r);
      const float E = ebase + kEps20 * (2.0f * s + 2.0f * r) + kLeafRel * r;
      U = fminf(U, s + E);
      if (lane == 0) {
        s_cpos[wv][0] = (uint32_t)pos;
        s_clb[wv][0] = s - E;
      }
      nc = 1;
    }
  }

  // push the children [c0, c0 + cnt) of level lv that may hold candidates,
  // farthest first (so the nearest is on top of the stack)
  int sp = 0;
  uint32_t boxes = 0, leaves = 0, visited = 0, leaf_boxes = 0;   // per query: below 2^32
  uint32_t nodes = 0;
  auto expand = [&](int lv, int64_t c0, int cnt, uint32_t node) {
    float key = INFINITY;     // visiting order
    float bnd = INFINITY;     // entry test, kept on the stack (k-means tree; the box tree's is its key)
    uint32_t val = 0;
    if (KMT) {
      // child records [c0, c0 + cnt) of k-means tree node `node`; their boxes
      // are quantised inside the node's box; val is the code
      float plo[12], phi[12], amax = 0.0f;
      const auto* pb = uniform_ptr(A.kmt_nbox + 24 * (int64_t)node);
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        plo[a] = approx ? 0.0f : pb[a];
        phi[a] = approx ? 0.0f : pb[12 + a];
        amax = fmaxf(amax, fabsf(plo[a]) + fabsf(phi[a]));
      }
      const float delta = kEps20 * amax + 1e-30f;
      if (lane < cnt) {
        float dc;
        const float lb = record_lb(A.kmt_child + kKmtRecord * (c0 + lane), qf, yq, slack, fd,
                                   plo, phi, delta, val, dc);
        if (lb <= (approx ? Ua : U)) {
          bnd = fmaxf(lb, 0.0f);
          key = fmaxf(dc, 0.0f);
        }
      }
      leaf_boxes += (uint32_t)__popcll(__ballot(lane < cnt && (val >> 28) == 0));
    } else if (lv == 0 && A.levels >= 2) {
      // leaf boxes quantised inside their parent (the node being expanded)
      const auto* pb = uniform_ptr(A.box[1] + 24 * (c0 / kAnnFan));
      float plo[12], step[12], amax = 0.0f;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        const float lo = pb[a], hi = pb[12 + a];
        plo[a] = lo;
        step[a] = (hi - lo) * (1.0f / 255.0f);
        amax = fmaxf(amax, fabsf(lo) + fabsf(hi));
      }
      const float delta = kEps20 * amax + 1e-30f;
      if (lane < cnt) {
        const float lb = qbox_lb(A.q0 + 24 * (c0 + lane), plo, step, delta, yq, slack);
        if (lb <= U) key = fmaxf(lb, 0.0f);
        val = ((uint32_t)lv << 28) | (uint32_t)(c0 + lane);
      }
    } else if (lane < cnt) {
      const float lb = box_lb(A.box[lv] + 24 * (c0 + lane), yq, slack);
      if (lb <= U) key = fmaxf(lb, 0.0f);
      val = ((uint32_t)lv << 28) | (uint32_t)(c0 + lane);
    }
    if (!KMT) bnd = key;
    const uint64_t pass = __ballot(key != INFINITY);
    int k = __popcll(pass);
    // depth-first order keeps at most kAnnFan entries per level on the stack;
    // the guard only protects the shared array
    if (sp + k > kStack) {
      ovf = true;
      k = 0;
    }
    if (k <= kRankSort) {
      // few survivors: each takes its rank among them (ties by child order)
      int rank = 0;
      for (uint64_t m = pass; m != 0; m &= m - 1) {
        const int j = __builtin_ctzll(m);
        const float kj = lane_f(key, j);
        rank += (int)(kj < key) | ((int)(kj == key) & (int)(j < lane));
      }
      if (k > 0 && key != INFINITY) {
        s_code[wv][sp + k - 1 - rank] = val;
        s_lb[wv][sp + k - 1 - rank] = bnd;
      }
    } else {
      if (KMT) wave_sort64<true>(key, val, bnd, lane);
      else wave_sort64<false>(key, val, bnd, lane);
      if (lane < k) {
        s_code[wv][sp + k - 1 - lane] = val;
        s_lb[wv][sp + k - 1 - lane] = KMT ? bnd : key;
      }
    }
    __builtin_amdgcn_wave_barrier();
    sp += k;
    boxes += (uint32_t)cnt;
    if (!KMT && lv == 0) leaf_boxes += (uint32_t)cnt;
  };

  // one leaf: 64 consecutive sorted points, one per lane, data already loaded
  bool stop = false;
  auto leaf_step = [&](int64_t idx, const uint2 (&xr)[3]) {
    const int64_t pos = idx * kAnnLeaf + lane;
    float qs[12], r;
    uint32_t count;
    // the leaf index is the same in every lane: say so, for scalar loads
    leaf_query(A.meta, (int64_t)__builtin_amdgcn_readfirstlane((int)idx), KMT ? qf : yq, qs, r, count);
    const bool v = KMT ? lane < (int)count : pos < A.N;
    float s = INFINITY, E = 0.0f;
    if (v) {
      s = leaf_point_dist_r(xr, qs, r);
      E = ebase + kEps20 * (2.0f * s + 2.0f * r) + kLeafRel * r;
    }
    if (TOP2) {
      const float h = v ? s + E : INFINITY;
      const float m1 = wave_min_f(h);
      const uint64_t at1 = __ballot(h == m1);
      const int l1 = at1 ? __ffsll((long long)at1) - 1 : 0;
      const float m2 = wave_min_f(lane == l1 ? INFINITY : h);
      // the two smallest of {U1, U, m1, m2}
      const float lo = fminf(U1, m1);
      const float hi = fminf(fmaxf(U1, m1), fminf(U, m2));
      U1 = lo;
      U = hi;
    } else {
      const float mn = wave_min_f(v ? s + E : INFINITY);
      U = fminf(U, mn);
      Ua = fminf(Ua, mn);
    }
    const bool keep = v && (s - E <= U);
    const uint64_t km = __ballot(keep);
    const int cnt = __popcll(km);
    visited += (uint32_t)__popcll(__ballot(v));
    ++leaves;
    if (nc + cnt > kCand) {
      // drop the candidates the bound has excluded since they were kept
      uint32_t cp = 0;
      float cl = INFINITY;
      if (lane < nc) {
        cp = s_cpos[wv][lane];
        cl = s_clb[wv][lane];
      }
      const bool still = lane < nc && cl <= U;
      const uint64_t sm = __ballot(still);
      __builtin_amdgcn_wave_barrier();
      if (still) {
        const int at = lanes_below(sm, lane);
        s_cpos[wv][at] = cp;
        s_clb[wv][at] = cl;
      }
      __builtin_amdgcn_wave_barrier();
      nc = __popcll(sm);
      if (nc + cnt > kCand) {
        ovf = true;
        stop = true;
        return;
      }
    }
    if (keep) {
      const int at = nc + lanes_below(km, lane);
      s_cpos[wv][at] = (uint32_t)pos;
      s_clb[wv][at] = s - E;
    }
    __builtin_amdgcn_wave_barrier();
    nc += cnt;
    if (budget > 0 && leaves >= (uint32_t)budget) stop = true;
  };

  auto expand_node = [&](uint32_t node) __attribute__((always_inline)) {
    ++nodes;
    const auto* r = uniform_ptr(reinterpret_cast<const int*>(A.kmt_node) + 2 * (int64_t)node);
    expand(1, r[0], r[1] - r[0], node);
  };
  if (KMT) expand_node(0);
  else expand(A.levels - 1, 0, (int)A.n[A.levels - 1], 0);
  while (sp > 0 && !ovf && !stop) {
    // stack entries are the same in every lane: keep them in scalar registers
    const uint32_t code = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_code[wv][sp - 1]);
    const float lb = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, s_lb[wv][sp - 1])));
    if (lb > (approx ? Ua : U)) {
      --sp;
      continue;
    }
    const int lv = (int)(code >> 28);
    if (lv > 0) {
      --sp;
      if (KMT) {
        expand_node(code & 0x0FFFFFFFu);
      } else {
        const int64_t c0 = (int64_t)(code & 0x0FFFFFFFu) * kAnnFan;
        const int cnt = (int)min((int64_t)kAnnFan, A.n[lv - 1] - c0);
        expand(lv - 1, c0, cnt, 0);
      }
      continue;
    }
    // a batch of up to kBatch leaves from the top of the stack (nearest first):
    // their loads are issued together, then they are evaluated in order, each
    // against the bound as it stands
    int64_t bidx[kBatch];
    float blb[kBatch];
    int nb = 0;
    while (nb < kBatch && sp > 0) {
      const uint32_t c2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_code[wv][sp - 1]);
      if ((c2 >> 28) != 0) break;
      bidx[nb] = (int64_t)(c2 & 0x0FFFFFFFu);
      blb[nb] = __builtin_bit_cast(
          float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, s_lb[wv][sp - 1])));
      ++nb;
      --sp;
    }
    uint2 xr[kBatch][3];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int64_t pos = bidx[b < nb ? b : 0] * kAnnLeaf + lane;
      if (b < nb && (KMT || pos < A.N)) {
        const uint2* p = reinterpret_cast<const uint2*>(A.h16 + 12 * pos);
        xr[b][0] = p[0];
        xr[b][1] = p[1];
        xr[b][2] = p[2];
      } else {
        xr[b][0] = xr[b][1] = xr[b][2] = make_uint2(0u, 0u);
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (b < nb && !stop && blb[b] <= (approx ? Ua : U)) leaf_step(bidx[b], xr[b]);
    }
  }

  if (lane == 0) {
    unsigned long long* c = A.counters + kCounterStride * (blockIdx.x % kCounterSlots);
    atomicAdd(c + 0, (unsigned long long)visited);
    atomicAdd(c + 1, (unsigned long long)boxes);
    atomicAdd(c + 2, (unsigned long long)leaves);
    atomicAdd(c + 4, (unsigned long long)leaf_boxes);
    if (KMT) atomicAdd(c + 5, (unsigned long long)nodes);
  }
  if (ovf) {
    if (lane == 0) {
      const int k = atomicAdd(A.fb_count, 1);
      A.fb_list[k] = (int)q;
      if (TOP2) A.dist2[q] = -1.0;   // no second distance: never skipped
    }
    return;
  }
  // FP64 rerank of the surviving candidates (direct form, as every scan's merge)
  double d = INFINITY;
  uint32_t o = 0xFFFFFFFFu;
  const bool mine = lane < nc && s_clb[wv][lane] <= U;
  if (mine) {
    const int64_t j = KMT ? (int64_t)A.slot_pos[s_cpos[wv][lane]] : (int64_t)s_cpos[wv][lane];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double t = A.qw[12 * q + k] - A.w64[12 * j + k];
      acc = fma(t, t, acc);
    }
    d = acc;
    o = A.perm[j];
  }
  const uint64_t mine_mask = __ballot(mine);
  if (lane == 0)
    atomicAdd(A.counters + kCounterStride * (blockIdx.x % kCounterSlots) + 3,
              (unsigned long long)__popcll(mine_mask));
  const double dm = d;
  const uint32_t om = o;
  for (int off = 32; off > 0; off >>= 1) {
    const double od = __shfl_xor(d, off);
    const uint32_t oo = __shfl_xor(o, off);
    if (od < d || (od == d && oo < o)) {
      d = od;
      o = oo;
    }
  }
  if (TOP2) {
    // second smallest: the minimum over the other candidates (points are distinct)
    double d2 = (om == o) ? INFINITY : dm;
    for (int off = 32; off > 0; off >>= 1) d2 = fmin(d2, __shfl_xor(d2, off));
    if (lane == 0) A.dist2[q] = 0.5 * d2;
  }
  if (lane == 0) {
    A.out.idx[q] = (int64_t)o;
    if (A.out.dist) A.out.dist[q] = 0.5 * d;
  }
}

// Queries on the principal axes of the trees: yq[q][a] = sum_k V[k][a] q[k]
// (FP64, rounded to FP32), one thread per (query, axis).
__global__ void rotate_queries_kernel(const double* __restrict__ qw, int64_t m,
                                      const double* __restrict__ V, float* __restrict__ yq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 12 * m) return;
  const int64_t q = i / 12;
  const int a = (int)(i - 12 * q);
  double y = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) y = fma(V[12 * k + a], qw[12 * q + k], y);
  yq[i] = (float)y;
}

}  // namespace

dd_status launch_ann_walk(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t len_max,
                          const int64_t* warm, int budget, Outputs out, int* fb_list, int* fb_count,
                          unsigned long long* counters, double* dist2, hipStream_t st, bool kmt,
                          double fd, const float* fd_q, const int* budget_q) {
  if (dist2 && (budget != 0 || (kmt && fd != 1.0) || fd_q || budget_q))
    return set_error(DD_ERR_ARG, "second distances need the exact walk");
  if (!(fd >= 0.0 && fd <= 1.0)) return set_error(DD_ERR_ARG, "f_d must be in [0, 1]");
  if (len_max <= 0) return DD_OK;
  AnnArgs A{};
  if (kmt) {
    if (D.kmt_nodes < 1) return set_error(DD_ERR_UNSUPPORTED, "dataset has no k-means tree");
    A.meta = D.kmt_meta.as<float>();
    A.h16 = D.kmt_h16.as<uint16_t>();
    A.kmt_node = D.kmt_node.as<int2>();
    A.kmt_nbox = D.kmt_nbox.as<float>();
    A.kmt_child = D.kmt_child.as<float>();
    A.slot_pos = D.kmt_pos.as<uint32_t>();
    A.pos_slot = D.kmt_slot.as<uint32_t>();
    A.fd = (float)fd;
  } else {
    if (D.ann_levels < 1 || D.ann_levels > kAnnMaxLevels || D.ann_n[D.ann_levels - 1] > kAnnFan)
      return set_error(DD_ERR_UNSUPPORTED, "dataset has no ANN tree");
    for (int l = 0; l < D.ann_levels; ++l) {
      A.box[l] = D.ann_box[l].as<float>();
      A.n[l] = D.ann_n[l];
    }
    A.levels = D.ann_levels;
    A.meta = D.ann_meta.as<float>();
    A.q0 = D.ann_q0.as<uint8_t>();
    A.h16 = D.ann_h16.as<uint16_t>();
  }
  A.w64 = D.w64.as<double>();
  A.perm = D.perm.as<uint32_t>();
  A.iperm = D.iperm.as<uint32_t>();
  A.N = D.N;
  // the walk runs over all states of the call (the identity list), whose
  // rotated coordinates are formed first
  if (L.list || !Q.yq || !D.vrot.p)
    return set_error(DD_ERR_ARG, "walk: identity query list and room for the rotated queries");
  hipLaunchKernelGGL(rotate_queries_kernel, dim3((unsigned)((12 * L.m + 255) / 256)), dim3(256), 0,
                     st, Q.qw, L.m, D.vrot.as<double>(), Q.yq);
  DD_HIP(hipGetLastError());
  A.yq = Q.yq;
  A.xmax = __builtin_nextafterf((float)D.xmax, INFINITY);
  A.budget = budget;
  A.fd_q = kmt ? fd_q : nullptr;
  A.budget_q = budget_q;
  A.L = L;
  A.qw = Q.qw;
  A.qn2 = Q.qn2;
  A.u32 = Q.u32;
  A.invalid = Q.invalid;
  A.warm = warm;
  A.out = out;
  A.fb_list = fb_list;
  A.fb_count = fb_count;
  A.counters = counters;
  const unsigned blocks = (unsigned)((len_max + kWaves - 1) / kWaves);
  A.dist2 = dist2;
  if (kmt) {
    if (dist2)
      hipLaunchKernelGGL((ann_walk_kernel<true, true>), dim3(blocks), dim3(kWaves * 64), 0, st, A);
    else
      hipLaunchKernelGGL((ann_walk_kernel<false, true>), dim3(blocks), dim3(kWaves * 64), 0, st, A);
  } else {
    if (dist2)
      hipLaunchKernelGGL((ann_walk_kernel<true, false>), dim3(blocks), dim3(kWaves * 64), 0, st, A);
    else
      hipLaunchKernelGGL((ann_walk_kernel<false, false>), dim3(blocks), dim3(kWaves * 64), 0, st,
                         A);
  }
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace dd
