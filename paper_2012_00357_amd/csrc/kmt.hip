// DD_KMEANS index: the k-means tree of Section 4 (recursive k-means with k = 4;
// a node stands for its points through their centroid and covering radius)
// built on the device, one level of splits at a time over every node of more
// than 64 points.
//
// A split of a node of n points into k = min(4, ceil(n / 64)) children:
//   * seeds: k points spread evenly along the node's current order (the data
//     arrive spatially sorted, so these are far apart);
//   * Lloyd iterations: nearest-centroid labels from FP64 distances, centroid
//     sums in 64-bit fixed point, so that the sums (and the tree) do not depend
//     on the order of the atomic additions;
//   * a split that leaves more than 90 % of the points in one child (repeated
//     points, a degenerate start) is replaced by k equal runs of the current
//     order, which bounds the depth;
//   * a stable partition of the node's points by label.
// Nodes of at most 64 points become leaves.  The walk reads a 64-ary cut of
// the 4-ary tree: a stored node lists a frontier of its descendants (at most 64
// children, each with the ball (FP32 centre, radius rounded up) of its points
// and their box in the dataset's principal-axis coordinates, rounded outward).
// Nodes are stored three 4-means levels apart counted from the leaves; every
// other node is absorbed into the frontier of the stored node above it while
// that frontier stays within 64 entries, and stored when it would not.  Leaves
// are stored as padded blocks of 64 slots in the compact form of the box tree
// (FP32 centre and radius, FP16 scaled offsets), empty slots +inf.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dd_internal.h"
#include "sort.h"

namespace dd {

namespace {

constexpr int kK = 4;                 // children per split
constexpr int kLloyd = 6;             // Lloyd iterations per split
constexpr int kThreads = 256;         // threads per block in the split passes
constexpr int kItems = 16;            // positions per thread
constexpr int kChunk = kThreads * kItems;
constexpr int kWavesPerBlock = kThreads / 64;
constexpr int kFan = 64;              // children per stored node
constexpr int kMaxRounds = 200;
constexpr int kAcc = kK * 13;         // fixed-point sums (12) and count per child
// build-time child record (floats): c[12], r, code (bits), 0, 0, box lo[12],
// hi[12] in FP32; the walk's records (kKmtRecord) carry the box as bytes
constexpr int kKmtBuild = 40;

struct Axes {                         // principal axes: V[12 k + a] = component k of axis a
  double V[144];
};

// Order-preserving map of floats to unsigned integers (atomic min / max).
__device__ inline uint32_t fkey(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float fkey_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// y = V^T x rounded outward to FP32 (lo rounded down, hi up).
__device__ inline void rotate_out(const Axes& R, const double (&x)[12], float (&lo)[12],
                                  float (&hi)[12]) {
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) y = fma(R.V[12 * k + a], x[k], y);
    lo[a] = __double2float_rd(y);
    hi[a] = __double2float_ru(y);
  }
}

unsigned grid_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// segment of chunk b: the last s with cbase[s] <= b
__device__ inline int64_t chunk_segment(const uint32_t* __restrict__ cbase, int64_t S, uint32_t b) {
  int64_t lo = 0, hi = S - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (cbase[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// run of position offset o among k equal runs of cnt positions (run j holds
// offsets [floor(cnt j / k), floor(cnt (j + 1) / k)))
__device__ inline int equal_run(uint32_t o, uint32_t cnt, int k) {
  int j = (int)(((uint64_t)o * (uint64_t)k) / cnt);
  if (j > k - 1) j = k - 1;
  while (j > 0 && ((uint64_t)cnt * (uint64_t)j) / (uint64_t)k > o) --j;
  while (j + 1 < k && ((uint64_t)cnt * (uint64_t)(j + 1)) / (uint64_t)k <= o) ++j;
  return j;
}

struct Segs {            // the nodes split in one round (structure of arrays)
  uint32_t* start;
  uint32_t* cnt;
  uint32_t* owner;       // stored node the node's children are listed under
  float* mean;           // [S][12] centroid of the node's points
  int* k;                // children of this split
};

// Lloyd pass over one chunk of one node: labels by the nearest centroid
// (ties to the lower child), fixed-point sums and counts per child.
template <bool FINAL>
__global__ __launch_bounds__(kThreads) void lloyd_kernel(const uint32_t* __restrict__ ids,
                                                         const double* __restrict__ w64, Segs G,
                                                         int64_t S, const uint32_t* __restrict__ cbase,
                                                         const float* __restrict__ cent,
                                                         unsigned long long* __restrict__ acc,
                                                         uint8_t* __restrict__ labels, double fix) {
  __shared__ float c_l[kK][12];
  __shared__ unsigned long long a_l[kWavesPerBlock][kAcc];
  const int t = threadIdx.x, wave = t >> 6;
  const int64_t s = chunk_segment(cbase, S, blockIdx.x);
  const uint32_t kc = blockIdx.x - cbase[s];
  const int k = G.k[s];
  if (t < kK * 12) c_l[t / 12][t % 12] = cent[(s * kK) * 12 + t];
  for (int i = t; i < kWavesPerBlock * kAcc; i += kThreads) (&a_l[0][0])[i] = 0ull;
  __syncthreads();
  const int64_t first = (int64_t)G.start[s] + (int64_t)kc * kChunk;
  const int64_t end = min((int64_t)G.start[s] + (int64_t)G.cnt[s], first + kChunk);
  for (int it = 0; it < kItems; ++it) {
    const int64_t p = first + (int64_t)it * kThreads + t;
    if (p >= end) break;
    const int64_t id = ids[p];
    double x[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) x[a] = w64[12 * id + a];
    int best = 0;
    double bd = INFINITY;
    for (int j = 0; j < k; ++j) {
      double d = 0.0;
#pragma unroll
      for (int a = 0; a < 12; ++a) {
        const double u = x[a] - (double)c_l[j][a];
        d = fma(u, u, d);
      }
      if (d < bd) {
        bd = d;
        best = j;
      }
    }
    if (FINAL) labels[p] = (uint8_t)best;
#pragma unroll
    for (int a = 0; a < 12; ++a)
      atomicAdd(&a_l[wave][best * 13 + a], (unsigned long long)llrint(x[a] * fix));
    atomicAdd(&a_l[wave][best * 13 + 12], 1ull);
  }
  __syncthreads();
  if (t < kAcc) {
    unsigned long long v = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) v += a_l[w][t];
    if (v != 0ull) atomicAdd(&acc[s * kAcc + t], v);
  }
}

// New centroids from the sums (an empty child keeps its centroid); the final
// pass also records the children's counts and centroids.  Clears the sums.
template <bool FINAL>
__global__ void update_kernel(Segs G, int64_t S, unsigned long long* __restrict__ acc,
                              float* __restrict__ cent, uint32_t* __restrict__ ccnt,
                              float* __restrict__ cmean, double fix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * kK) return;
  const int64_t s = i / kK;
  const int j = (int)(i % kK);
  unsigned long long* a = acc + s * kAcc + j * 13;
  const long long n = (long long)a[12];
  if (j < G.k[s] && n > 0) {
    for (int c = 0; c < 12; ++c)
      cent[i * 12 + c] = (float)((double)(long long)a[c] / ((double)n * fix));
  }
  if (FINAL) {
    ccnt[i] = (j < G.k[s]) ? (uint32_t)n : 0u;
    for (int c = 0; c < 12; ++c) cmean[i * 12 + c] = cent[i * 12 + c];
  }
  for (int c = 0; c < 13; ++c) a[c] = 0ull;
}

// Splits that keep more than 90 % of the points in one child become k equal
// runs of the current order (children centred on the parent's centroid).
__global__ void balance_kernel(Segs G, int64_t S, uint32_t* __restrict__ ccnt,
                               float* __restrict__ cmean, uint8_t* __restrict__ forced) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t n = G.cnt[s];
  const int k = G.k[s];
  uint32_t mx = 0;
  for (int j = 0; j < k; ++j) mx = max(mx, ccnt[s * kK + j]);
  const bool f = (double)mx > 0.9 * (double)n;
  forced[s] = f ? 1 : 0;
  if (!f) return;
  for (int j = 0; j < k; ++j) {
    ccnt[s * kK + j] = (uint32_t)(((uint64_t)n * (j + 1)) / k - ((uint64_t)n * j) / k);
    for (int c = 0; c < 12; ++c) cmean[(s * kK + j) * 12 + c] = G.mean[s * 12 + c];
  }
}

__device__ inline int label_at(const Segs& G, int64_t s, const uint8_t* forced,
                               const uint8_t* labels, int64_t p) {
  return forced[s] ? equal_run((uint32_t)(p - G.start[s]), G.cnt[s], G.k[s]) : (int)labels[p];
}

// Per chunk and child: points of that child in the chunk, at
// H[4 cbase[s] + j nch[s] + kc] (node-major, child-major, chunk-minor, so that
// one exclusive scan gives every run's output offset).
__global__ __launch_bounds__(kThreads) void hist_kernel(Segs G, int64_t S,
                                                        const uint32_t* __restrict__ cbase,
                                                        const uint8_t* __restrict__ forced,
                                                        const uint8_t* __restrict__ labels,
                                                        uint32_t* __restrict__ H) {
  __shared__ uint32_t cnt[kK];
  const int t = threadIdx.x;
  const int64_t s = chunk_segment(cbase, S, blockIdx.x);
  const uint32_t kc = blockIdx.x - cbase[s];
  if (t < kK) cnt[t] = 0;
  __syncthreads();
  const int64_t first = (int64_t)G.start[s] + (int64_t)kc * kChunk;
  const int64_t end = min((int64_t)G.start[s] + (int64_t)G.cnt[s], first + kChunk);
  for (int it = 0; it < kItems; ++it) {
    const int64_t p = first + (int64_t)it * kThreads + t;
    if (p < end) atomicAdd(&cnt[label_at(G, s, forced, labels, p)], 1u);
  }
  __syncthreads();
  if (t < kK) {
    const uint32_t nch = cbase[s + 1] - cbase[s];
    H[4 * (int64_t)cbase[s] + (int64_t)t * nch + kc] = cnt[t];
  }
}

// Stable partition of every node's points by child: ids_out[start + offset of
// the child's run + rank] = ids_in[p], ranks in position order (wavefront
// ballots over the label bits, then earlier waves of the round).
__global__ __launch_bounds__(kThreads) void scatter_kernel(Segs G, int64_t S,
                                                           const uint32_t* __restrict__ cbase,
                                                           const uint8_t* __restrict__ forced,
                                                           const uint8_t* __restrict__ labels,
                                                           const uint32_t* __restrict__ H,
                                                           const uint32_t* __restrict__ ids_in,
                                                           uint32_t* __restrict__ ids_out) {
  __shared__ uint32_t run[kK];
  __shared__ uint32_t wcnt[kWavesPerBlock][kK];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t s = chunk_segment(cbase, S, blockIdx.x);
  const uint32_t kc = blockIdx.x - cbase[s];
  const uint32_t nch = cbase[s + 1] - cbase[s];
  const int64_t hb = 4 * (int64_t)cbase[s];
  if (t < kK) run[t] = G.start[s] + H[hb + (int64_t)t * nch + kc] - H[hb];
  if (t < kWavesPerBlock * kK) (&wcnt[0][0])[t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t first = (int64_t)G.start[s] + (int64_t)kc * kChunk;
  const int64_t end = min((int64_t)G.start[s] + (int64_t)G.cnt[s], first + kChunk);
  for (int it = 0; it < kItems; ++it) {
    const int64_t p = first + (int64_t)it * kThreads + t;
    const bool v = p < end;
    const int l = v ? label_at(G, s, forced, labels, p) : 0;
    uint64_t same = __ballot(v);
    for (int b = 0; b < 2; ++b) {
      const uint64_t bb = __ballot(v && ((l >> b) & 1));
      same &= ((l >> b) & 1) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    if (v && rank == 0) wcnt[wave][l] = (uint32_t)__popcll(same);
    __syncthreads();
    if (v) {
      uint32_t pos = run[l] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][l];
      ids_out[pos] = ids_in[p];
    }
    __syncthreads();
    if (t < kK) {
      uint32_t add = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][t];
      run[t] += add;
    }
    __syncthreads();
    if (t < kWavesPerBlock * kK) (&wcnt[0][0])[t] = 0;
    __syncthreads();
  }
}

// Splits of 4 needed to bring n points down to leaves of at most 64.
__device__ inline int splits_to_leaves(uint32_t n) {
  int d = 0;
  for (uint64_t c = (uint64_t)kAnnLeaf; c < n; c *= kK) ++d;
  return d;
}

// For every stored node o (the nodes of this round listed under o form one run
// of the owner-sorted order okey / oidx; at most kFan of them): a node whose
// remaining splits are a multiple of 3 becomes a stored node (so that stored
// nodes sit three 4-means levels apart counted from the leaves, where a full
// node has 4^3 = 64 children); the others are absorbed, smallest first (ties by
// position), while o's frontier stays within kFan entries (a split replaces one
// entry by its non-empty children), and become stored nodes when it would not.
// frontier[o] counts the entries of o.
__global__ void decide_kernel(Segs G, int64_t S, const uint32_t* __restrict__ okey,
                              const uint32_t* __restrict__ oidx, const uint32_t* __restrict__ ccnt,
                              uint32_t* __restrict__ frontier, uint32_t* __restrict__ store_f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const uint32_t o = okey[i];
  if (i > 0 && okey[i - 1] == o) return;   // not the first of its run
  int n = 1;
  while (i + n < S && n < kFan && okey[i + n] == o) ++n;
  uint32_t seg[kFan], size[kFan];
  uint8_t order[kFan];
  for (int t = 0; t < n; ++t) {
    seg[t] = oidx[i + t];
    size[t] = G.cnt[seg[t]];
  }
  for (int t = 0; t < n; ++t) {
    int rank = 0;
    for (int u = 0; u < n; ++u)
      rank += (size[u] < size[t] || (size[u] == size[t] && seg[u] < seg[t])) ? 1 : 0;
    order[rank] = (uint8_t)t;
  }
  int budget = kFan - (int)frontier[o];
  for (int r = 0; r < n; ++r) {
    const int64_t s = seg[order[r]];
    int c = 0;
    for (int j = 0; j < kK; ++j) c += ccnt[s * kK + j] > 0 ? 1 : 0;
    if (splits_to_leaves(size[order[r]]) % 3 != 0 && c - 1 <= budget) {
      budget -= c - 1;
      store_f[s] = 0u;
    } else {
      store_f[s] = 1u;
    }
  }
  frontier[o] = (uint32_t)(kFan - budget);
}

// Frontier sizes of the nodes stored this round: their non-empty children.
__global__ void new_frontier_kernel(int64_t S, const uint32_t* __restrict__ ccnt,
                                    const uint32_t* __restrict__ store_f,
                                    const uint32_t* __restrict__ store_at, uint32_t node_base,
                                    uint32_t* __restrict__ frontier) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !store_f[s]) return;
  uint32_t c = 0;
  for (int j = 0; j < kK; ++j) c += ccnt[s * kK + j] > 0 ? 1u : 0u;
  frontier[node_base + store_at[s]] = c;
}

// Children of every split: leaves (at most 64 points) and the nodes of the next
// round, flagged for compaction.
__global__ void children_kernel(int64_t S, const uint32_t* __restrict__ ccnt,
                                uint32_t* __restrict__ leaf_f, uint32_t* __restrict__ act_f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * kK) return;
  const uint32_t n = ccnt[i];
  leaf_f[i] = (n > 0 && n <= (uint32_t)kAnnLeaf) ? 1u : 0u;
  act_f[i] = (n > (uint32_t)kAnnLeaf) ? 1u : 0u;
}

struct LeafRec {
  uint32_t start, cnt, owner, pad;
};

__global__ void compact_kernel(Segs G, int64_t S, const uint32_t* __restrict__ ccnt,
                               const float* __restrict__ cmean, const uint32_t* __restrict__ leaf_f,
                               const uint32_t* __restrict__ leaf_at,
                               const uint32_t* __restrict__ act_f,
                               const uint32_t* __restrict__ act_at,
                               const uint32_t* __restrict__ store_f,
                               const uint32_t* __restrict__ store_at, uint32_t node_base,
                               LeafRec* __restrict__ leaves, int64_t leaf_base, Segs N2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * kK) return;
  const int64_t s = i / kK;
  const int j = (int)(i % kK);
  uint32_t off = G.start[s];
  for (int jj = 0; jj < j; ++jj) off += ccnt[s * kK + jj];
  const uint32_t owner = store_f[s] ? node_base + store_at[s] : G.owner[s];
  const uint32_t n = ccnt[i];
  if (leaf_f[i]) leaves[leaf_base + leaf_at[i]] = LeafRec{off, n, owner, 0u};
  if (act_f[i]) {
    const uint32_t a = act_at[i];
    N2.start[a] = off;
    N2.cnt[a] = n;
    N2.owner[a] = owner;
    N2.k[a] = (int)min((uint32_t)kK, (n + (uint32_t)kAnnLeaf - 1) / (uint32_t)kAnnLeaf);
    for (int c = 0; c < 12; ++c) N2.mean[a * 12 + c] = cmean[i * 12 + c];
  }
}

// k seeds per node, spread along its current order.
__global__ void seed_kernel(const uint32_t* __restrict__ ids, const double* __restrict__ w64,
                            Segs G, int64_t S, float* __restrict__ cent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * kK) return;
  const int64_t s = i / kK;
  const int j = (int)(i % kK);
  const int k = G.k[s];
  const uint32_t n = G.cnt[s];
  const int jj = j < k ? j : 0;
  const int64_t p = (int64_t)G.start[s] + (int64_t)(((uint64_t)n * (2 * jj + 1)) / (2 * k));
  const int64_t id = ids[p];
  for (int c = 0; c < 12; ++c) cent[i * 12 + c] = (float)w64[12 * id + c];
}

// Covering radius of every stored node about its FP32 centroid (FP64
// distances; the bits of non-negative doubles order as integers) and its box
// in principal-axis coordinates (rounded outward; order-preserving keys).
// rad[s]: radius bits; blo[s][12], bhi[s][12]: box keys (start at all ones / zero).
__global__ __launch_bounds__(kThreads) void node_stats_kernel(const uint32_t* __restrict__ ids,
                                                              const double* __restrict__ w64,
                                                              Segs G, int64_t S,
                                                              const uint32_t* __restrict__ cbase,
                                                              const uint32_t* __restrict__ store_f,
                                                              Axes R,
                                                              unsigned long long* __restrict__ rad,
                                                              uint32_t* __restrict__ kblo,
                                                              uint32_t* __restrict__ kbhi) {
  const int t = threadIdx.x;
  const int64_t s = chunk_segment(cbase, S, blockIdx.x);
  if (!store_f[s]) return;   // only the nodes stored this round need their ball and box
  const uint32_t kc = blockIdx.x - cbase[s];
  const int64_t first = (int64_t)G.start[s] + (int64_t)kc * kChunk;
  const int64_t end = min((int64_t)G.start[s] + (int64_t)G.cnt[s], first + kChunk);
  double c[12];
  for (int a = 0; a < 12; ++a) c[a] = (double)G.mean[s * 12 + a];
  double r = 0.0;
  float blo[12], bhi[12];
  for (int a = 0; a < 12; ++a) {
    blo[a] = INFINITY;
    bhi[a] = -INFINITY;
  }
  for (int it = 0; it < kItems; ++it) {
    const int64_t p = first + (int64_t)it * kThreads + t;
    if (p >= end) break;
    const int64_t id = ids[p];
    double x[12], d = 0.0;
    for (int a = 0; a < 12; ++a) {
      x[a] = w64[12 * id + a];
      const double u = x[a] - c[a];
      d = fma(u, u, d);
    }
    r = fmax(r, sqrt(d));
    float lo[12], hi[12];
    rotate_out(R, x, lo, hi);
    for (int a = 0; a < 12; ++a) {
      blo[a] = fminf(blo[a], lo[a]);
      bhi[a] = fmaxf(bhi[a], hi[a]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    r = fmax(r, __shfl_xor(r, off));
    for (int a = 0; a < 12; ++a) {
      blo[a] = fminf(blo[a], __shfl_xor(blo[a], off));
      bhi[a] = fmaxf(bhi[a], __shfl_xor(bhi[a], off));
    }
  }
  if ((t & 63) == 0) {
    atomicMax(&rad[s], (unsigned long long)__double_as_longlong(r));
    for (int a = 0; a < 12; ++a) {
      if (blo[a] != INFINITY) atomicMin(&kblo[12 * s + a], fkey(blo[a]));
      if (bhi[a] != -INFINITY) atomicMax(&kbhi[12 * s + a], fkey(bhi[a]));
    }
  }
}

// Child records of the nodes stored this round: ball and box of the node's
// points, code 1 << 28 | node, listed under the node's owner.
__global__ void node_record_kernel(Segs G, int64_t S, const unsigned long long* __restrict__ rad,
                                   const uint32_t* __restrict__ kblo,
                                   const uint32_t* __restrict__ kbhi,
                                   const uint32_t* __restrict__ store_f,
                                   const uint32_t* __restrict__ store_at, uint32_t node_base,
                                   float* __restrict__ rec, uint32_t* __restrict__ rec_owner,
                                   int64_t rec_base) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !store_f[s]) return;
  const int64_t at = rec_base + store_at[s];
  float* r = rec + kKmtBuild * at;
  for (int a = 0; a < 12; ++a) {
    r[16 + a] = fkey_inv(kblo[12 * s + a]);
    r[28 + a] = fkey_inv(kbhi[12 * s + a]);
  }
  for (int c = 0; c < 12; ++c) r[c] = G.mean[s * 12 + c];
  const double rd = __longlong_as_double((long long)rad[s]);
  r[12] = __double2float_ru(rd * (1.0 + 1e-12));
  r[13] = __uint_as_float((1u << 28) | (node_base + store_at[s]));
  r[14] = 0.0f;
  r[15] = 0.0f;
  rec_owner[at] = G.owner[s];
}

__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return __shfl(v, 0);   // one value for every lane (the butterfly order differs per lane)
}

// One wavefront per leaf: compact leaf block (centre, L2 radius, FP16 scaled
// offsets in slots leaf * 64 + lane, empty slots +inf), slot maps, and the
// leaf's child record.
__global__ __launch_bounds__(256) void leaf_kernel(const uint32_t* __restrict__ ids,
                                                   const double* __restrict__ w64, Axes R,
                                                   const LeafRec* __restrict__ leaves,
                                                   int64_t n_leaf, float* __restrict__ meta,
                                                   _Float16* __restrict__ h16,
                                                   uint32_t* __restrict__ slot_pos,
                                                   uint32_t* __restrict__ pos_slot,
                                                   float* __restrict__ rec,
                                                   uint32_t* __restrict__ rec_owner,
                                                   int64_t rec_base) {
  const int lane = threadIdx.x & 63;
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (leaf >= n_leaf) return;
  const LeafRec L = leaves[leaf];
  const bool v = lane < (int)L.cnt;
  const int64_t slot = leaf * kAnnLeaf + lane;
  const int64_t id = v ? (int64_t)ids[L.start + lane] : 0;
  double x[12];
  for (int a = 0; a < 12; ++a) x[a] = v ? w64[12 * id + a] : 0.0;
  float c[12];
  for (int a = 0; a < 12; ++a) c[a] = (float)(wave_sum_d(x[a]) / (double)L.cnt);
  double d2 = 0.0;
  for (int a = 0; a < 12; ++a) {
    const double t = x[a] - (double)c[a];
    d2 = fma(t, t, d2);
  }
  double r = v ? sqrt(d2) : 0.0;
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off));
  float rf = __double2float_ru(r * (1.0 + 1e-12));
  rf = fmaxf(rf, 9.5367431640625e-07f);   // 2^-20: bounded scaled offsets for tiny leaves
  const double inv = 1.0 / (double)rf;
  for (int a = 0; a < 12; ++a)
    h16[12 * slot + a] = v ? (_Float16)((x[a] - (double)c[a]) * inv) : (_Float16)INFINITY;
  float blo[12], bhi[12];
  rotate_out(R, x, blo, bhi);
  for (int a = 0; a < 12; ++a) {
    if (!v) {
      blo[a] = INFINITY;
      bhi[a] = -INFINITY;
    }
    for (int off = 32; off > 0; off >>= 1) {
      blo[a] = fminf(blo[a], __shfl_xor(blo[a], off));
      bhi[a] = fmaxf(bhi[a], __shfl_xor(bhi[a], off));
    }
  }
  slot_pos[slot] = v ? (uint32_t)id : 0xFFFFFFFFu;
  if (v) pos_slot[id] = (uint32_t)slot;
  if (lane == 0) {
    float* m = meta + 16 * leaf;
    float* q = rec + kKmtBuild * (rec_base + leaf);
    for (int a = 0; a < 12; ++a) {
      m[a] = c[a];
      q[a] = c[a];
    }
    m[12] = rf;
    m[13] = (float)inv;
    m[14] = __uint_as_float(L.cnt);
    m[15] = 0.0f;
    q[12] = rf;
    q[13] = __uint_as_float((uint32_t)leaf);
    q[14] = 0.0f;
    q[15] = 0.0f;
    for (int a = 0; a < 12; ++a) {
      q[16 + a] = blo[a];
      q[28 + a] = bhi[a];
    }
    rec_owner[rec_base + leaf] = L.owner;
  }
}

__global__ void gather_records_kernel(const float* __restrict__ rec, const uint32_t* __restrict__ order,
                                      int64_t n, float* __restrict__ child) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kKmtBuild * n) return;
  child[i] = rec[kKmtBuild * (int64_t)order[i / kKmtBuild] + (i % kKmtBuild)];
}

// Box of each stored node: the union of its child records' boxes (exact in
// FP32: the children's bounds are already rounded outward).
__global__ void node_box_kernel(const float* __restrict__ child, const int2* __restrict__ node,
                                int64_t n_nodes, float* __restrict__ nbox) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_nodes) return;
  float lo[12], hi[12];
  for (int a = 0; a < 12; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  const int2 r = node[o];
  for (int64_t i = r.x; i < r.y; ++i) {
    const float* c = child + kKmtBuild * i;
    for (int a = 0; a < 12; ++a) {
      lo[a] = fminf(lo[a], c[16 + a]);
      hi[a] = fmaxf(hi[a], c[28 + a]);
    }
  }
  for (int a = 0; a < 12; ++a) {
    nbox[24 * o + a] = lo[a];
    nbox[24 * o + 12 + a] = hi[a];
  }
}

// Walk records: centre, radius and code as built; the box quantised to bytes
// inside the owner node's box (lo rounded down, hi up, in FP64 from the FP32
// bounds), read back with the owner's box and an outward decoding margin.
__global__ void compress_records_kernel(const float* __restrict__ child,
                                        const uint32_t* __restrict__ owner, int64_t n,
                                        const float* __restrict__ nbox, float* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* c = child + kKmtBuild * i;
  float* q = rec + kKmtRecord * i;
  for (int a = 0; a < 14; ++a) q[a] = c[a];
  const float* p = nbox + 24 * (int64_t)owner[i];
  uint8_t b[24];
  for (int a = 0; a < 12; ++a) {
    const double plo = p[a], ext = (double)p[12 + a] - plo;
    int ql = 0, qh = 255;
    if (ext > 0.0) {
      ql = (int)floor(((double)c[16 + a] - plo) / ext * 255.0);
      qh = (int)ceil(((double)c[28 + a] - plo) / ext * 255.0);
      ql = ql < 0 ? 0 : (ql > 255 ? 255 : ql);
      qh = qh < 0 ? 0 : (qh > 255 ? 255 : qh);
    }
    b[a] = (uint8_t)ql;
    b[12 + a] = (uint8_t)qh;
  }
  for (int w = 0; w < 6; ++w)
    q[14 + w] = __uint_as_float((uint32_t)b[4 * w] | ((uint32_t)b[4 * w + 1] << 8) |
                                ((uint32_t)b[4 * w + 2] << 16) | ((uint32_t)b[4 * w + 3] << 24));
}

// node[o] = (first record, end) of owner o's run in the owner-sorted records.
__global__ void node_range_kernel(const uint32_t* __restrict__ owner, int64_t n,
                                  int2* __restrict__ node) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t o = owner[i];
  if (i == 0 || owner[i - 1] != o) node[o].x = (int)i;
  if (i == n - 1 || owner[i + 1] != o) node[o].y = (int)(i + 1);
}

// Growable device array (contents kept).
dd_status grow(DevBuf& b, size_t bytes, hipStream_t st) {
  if (b.bytes >= bytes) return DD_OK;
  DevBuf n;
  DD_TRY(n.alloc(std::max(bytes, 2 * b.bytes)));
  if (b.bytes) DD_HIP(hipMemcpyAsync(n.p, b.p, b.bytes, hipMemcpyDeviceToDevice, st));
  DD_HIP(hipStreamSynchronize(st));
  std::swap(b.p, n.p);
  std::swap(b.bytes, n.bytes);
  return DD_OK;
}

struct SegBufs {
  DevBuf start, cnt, owner, mean, k;
  dd_status alloc(int64_t S) {
    const size_t n = (size_t)std::max<int64_t>(S, 1);
    DD_TRY(start.alloc(4 * n));
    DD_TRY(cnt.alloc(4 * n));
    DD_TRY(owner.alloc(4 * n));
    DD_TRY(mean.alloc(4 * 12 * n));
    DD_TRY(k.alloc(4 * n));
    return DD_OK;
  }
  Segs view() {
    return Segs{start.as<uint32_t>(), cnt.as<uint32_t>(), owner.as<uint32_t>(), mean.as<float>(),
                k.as<int>()};
  }
};

uint32_t read_u32(const uint32_t* p, hipStream_t st) {
  uint32_t v = 0;
  (void)hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  return v;
}

}  // namespace

dd_status build_kmeans_tree(Dataset& D, hipStream_t st) {
  const int64_t N = D.N;
  if (N > 0xFFFFFFFFll) return set_error(DD_ERR_TOO_LARGE, "k-means tree: N exceeds 2^32-1");
  // fixed-point scale of the centroid sums: |sum| <= N xmax 2^e < 2^62
  int e = 40;
  {
    const double m = (double)N * std::max(D.xmax, 1e-300);
    int ex = 0;
    std::frexp(std::ldexp(1.0, 62) / m, &ex);
    e = std::min(e, ex - 1);
  }
  const double fix = std::ldexp(1.0, e);
  Axes R;
  std::memcpy(R.V, D.V, sizeof(R.V));

  DevBuf ids[2], labels, leaves_b, recs, rec_owner, frontier;
  DD_TRY(ids[0].alloc(4 * (size_t)N));
  DD_TRY(ids[1].alloc(4 * (size_t)N));
  DD_TRY(labels.alloc((size_t)N));
  DD_TRY(iota_u32(ids[0].as<uint32_t>(), N, st));
  int cur = 0;
  int64_t n_leaf = 0, n_rec = 0, n_nodes = 1;

  SegBufs segs;
  int64_t S = 0;
  if (N <= kAnnLeaf) {
    DD_TRY(grow(leaves_b, sizeof(LeafRec), st));
    LeafRec r{0u, (uint32_t)N, 0u, 0u};
    DD_HIP(hipMemcpyAsync(leaves_b.p, &r, sizeof r, hipMemcpyHostToDevice, st));
    n_leaf = 1;
  } else {
    // the root (stored node 0) starts with itself as its one frontier entry
    S = 1;
    DD_TRY(segs.alloc(1));
    DD_TRY(grow(frontier, 4, st));
    const uint32_t one = 1;
    DD_HIP(hipMemcpyAsync(frontier.p, &one, 4, hipMemcpyHostToDevice, st));
    const uint32_t z = 0, n = (uint32_t)N;
    const int k = (int)std::min<int64_t>(kK, (N + kAnnLeaf - 1) / kAnnLeaf);
    DD_HIP(hipMemcpyAsync(segs.start.p, &z, 4, hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(segs.cnt.p, &n, 4, hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(segs.owner.p, &z, 4, hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(segs.k.p, &k, 4, hipMemcpyHostToDevice, st));
  }

  int round = 0;
  bool root_mean = true;
  while (S > 0) {
    if (round >= kMaxRounds) return set_error(DD_ERR_TOO_LARGE, "k-means tree too deep");
    Segs G = segs.view();
    // chunks of at most kChunk positions per node
    DevBuf cbase_b, cent_b, acc_b, ccnt_b, cmean_b, forced_b, rad_b;
    DD_TRY(cbase_b.alloc(4 * (size_t)(S + 1)));
    // first chunk of every node (ceil(cnt / kChunk) chunks each); entry S: total
    uint32_t n_chunks = 0;
    {
      std::vector<uint32_t> cnt((size_t)S);
      DD_HIP(hipMemcpyAsync(cnt.data(), G.cnt, 4 * (size_t)S, hipMemcpyDeviceToHost, st));
      DD_HIP(hipStreamSynchronize(st));
      std::vector<uint32_t> base((size_t)S + 1);
      uint64_t acc = 0;
      for (int64_t s = 0; s < S; ++s) {
        base[(size_t)s] = (uint32_t)acc;
        acc += (cnt[(size_t)s] + (uint64_t)kChunk - 1) / kChunk;
      }
      base[(size_t)S] = (uint32_t)acc;
      if (acc > 0x7FFFFFFFull) return set_error(DD_ERR_TOO_LARGE, "k-means tree: too many chunks");
      n_chunks = (uint32_t)acc;
      DD_HIP(hipMemcpyAsync(cbase_b.p, base.data(), 4 * ((size_t)S + 1), hipMemcpyHostToDevice, st));
      DD_HIP(hipStreamSynchronize(st));
    }
    const uint32_t* cbase = cbase_b.as<uint32_t>();
    DD_TRY(cent_b.alloc(4 * 12 * kK * (size_t)S));
    DD_TRY(acc_b.alloc(8 * kAcc * (size_t)S));
    DD_TRY(ccnt_b.alloc(4 * kK * (size_t)S));
    DD_TRY(cmean_b.alloc(4 * 12 * kK * (size_t)S));
    DD_TRY(forced_b.alloc((size_t)S));
    DD_HIP(hipMemsetAsync(acc_b.p, 0, acc_b.bytes, st));
    const uint32_t* ids_in = ids[cur].as<uint32_t>();
    const double* w64 = D.w64.as<double>();

    if (root_mean) {
      // centroid of all points: one pass with a single child
      root_mean = false;
      const int one = 1;
      DD_HIP(hipMemcpyAsync(G.k, &one, 4, hipMemcpyHostToDevice, st));
      DD_HIP(hipMemsetAsync(cent_b.p, 0, cent_b.bytes, st));
      hipLaunchKernelGGL(lloyd_kernel<false>, dim3(n_chunks), dim3(kThreads), 0, st, ids_in, w64,
                         G, S, cbase, cent_b.as<float>(), acc_b.as<unsigned long long>(),
                         labels.as<uint8_t>(), fix);
      hipLaunchKernelGGL(update_kernel<false>, dim3(1), dim3(256), 0, st, G, S,
                         acc_b.as<unsigned long long>(), cent_b.as<float>(), ccnt_b.as<uint32_t>(),
                         cmean_b.as<float>(), fix);
      DD_HIP(hipMemcpyAsync(G.mean, cent_b.p, 48, hipMemcpyDeviceToDevice, st));
      const int k = (int)std::min<int64_t>(kK, (N + kAnnLeaf - 1) / kAnnLeaf);
      DD_HIP(hipMemcpyAsync(G.k, &k, 4, hipMemcpyHostToDevice, st));
      DD_HIP(hipStreamSynchronize(st));
      DD_HIP(hipGetLastError());
    }

    // Lloyd iterations
    hipLaunchKernelGGL(seed_kernel, dim3(grid_of(S * kK, 256)), dim3(256), 0, st, ids_in, w64, G,
                       S, cent_b.as<float>());
    for (int it = 0; it < kLloyd; ++it) {
      hipLaunchKernelGGL(lloyd_kernel<false>, dim3(n_chunks), dim3(kThreads), 0, st, ids_in, w64,
                         G, S, cbase, cent_b.as<float>(), acc_b.as<unsigned long long>(),
                         labels.as<uint8_t>(), fix);
      hipLaunchKernelGGL(update_kernel<false>, dim3(grid_of(S * kK, 256)), dim3(256), 0, st, G, S,
                         acc_b.as<unsigned long long>(), cent_b.as<float>(), ccnt_b.as<uint32_t>(),
                         cmean_b.as<float>(), fix);
    }
    hipLaunchKernelGGL(lloyd_kernel<true>, dim3(n_chunks), dim3(kThreads), 0, st, ids_in, w64, G,
                       S, cbase, cent_b.as<float>(), acc_b.as<unsigned long long>(),
                       labels.as<uint8_t>(), fix);
    hipLaunchKernelGGL(update_kernel<true>, dim3(grid_of(S * kK, 256)), dim3(256), 0, st, G, S,
                       acc_b.as<unsigned long long>(), cent_b.as<float>(), ccnt_b.as<uint32_t>(),
                       cmean_b.as<float>(), fix);
    hipLaunchKernelGGL(balance_kernel, dim3(grid_of(S, 256)), dim3(256), 0, st, G, S,
                       ccnt_b.as<uint32_t>(), cmean_b.as<float>(), forced_b.as<uint8_t>());
    DD_HIP(hipGetLastError());

    // frontier budgets: which of this round's nodes become stored nodes
    DevBuf store_f, store_at;
    DD_TRY(store_f.alloc(4 * (size_t)S));
    DD_TRY(store_at.alloc(4 * (size_t)S));
    DD_HIP(hipMemsetAsync(store_f.p, 0, store_f.bytes, st));
    {
      DevBuf okey, oidx;
      DD_TRY(okey.alloc(4 * (size_t)S));
      DD_TRY(oidx.alloc(4 * (size_t)S));
      DD_HIP(hipMemcpyAsync(okey.p, G.owner, 4 * (size_t)S, hipMemcpyDeviceToDevice, st));
      DD_TRY(iota_u32(oidx.as<uint32_t>(), S, st));
      int obits = 1;
      while (obits < 32 && (1ll << obits) < n_nodes) ++obits;
      DD_TRY(radix_sort_pairs(okey.as<uint32_t>(), oidx.as<uint32_t>(), S, obits, st));
      hipLaunchKernelGGL(decide_kernel, dim3(grid_of(S, 256)), dim3(256), 0, st, G, S,
                         okey.as<uint32_t>(), oidx.as<uint32_t>(), ccnt_b.as<uint32_t>(),
                         frontier.as<uint32_t>(), store_f.as<uint32_t>());
      DD_HIP(hipGetLastError());
      DD_HIP(hipStreamSynchronize(st));
    }
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpyAsync(store_at.p, store_f.p, store_f.bytes, hipMemcpyDeviceToDevice, st));
    DD_TRY(exclusive_scan_u32(store_at.as<uint32_t>(), S, st));
    const int64_t n_store = (int64_t)read_u32(store_at.as<uint32_t>() + S - 1, st) +
                            (int64_t)read_u32(store_f.as<uint32_t>() + S - 1, st);
    const uint32_t node_base = (uint32_t)n_nodes;
    if (n_store > 0) {
      // their balls and boxes become child records of their owners
      DevBuf kblo, kbhi;
      DD_TRY(rad_b.alloc(8 * (size_t)S));
      DD_TRY(kblo.alloc(4 * 12 * (size_t)S));
      DD_TRY(kbhi.alloc(4 * 12 * (size_t)S));
      DD_HIP(hipMemsetAsync(rad_b.p, 0, rad_b.bytes, st));
      DD_HIP(hipMemsetAsync(kblo.p, 0xFF, kblo.bytes, st));
      DD_HIP(hipMemsetAsync(kbhi.p, 0, kbhi.bytes, st));
      hipLaunchKernelGGL(node_stats_kernel, dim3(n_chunks), dim3(kThreads), 0, st, ids_in, w64, G,
                         S, cbase, store_f.as<uint32_t>(), R, rad_b.as<unsigned long long>(),
                         kblo.as<uint32_t>(), kbhi.as<uint32_t>());
      DD_TRY(grow(recs, 4 * kKmtBuild * (size_t)(n_rec + n_store), st));
      DD_TRY(grow(rec_owner, 4 * (size_t)(n_rec + n_store), st));
      DD_TRY(grow(frontier, 4 * (size_t)(n_nodes + n_store), st));
      hipLaunchKernelGGL(node_record_kernel, dim3(grid_of(S, 256)), dim3(256), 0, st, G, S,
                         rad_b.as<unsigned long long>(), kblo.as<uint32_t>(), kbhi.as<uint32_t>(),
                         store_f.as<uint32_t>(),
                         store_at.as<uint32_t>(), node_base, recs.as<float>(),
                         rec_owner.as<uint32_t>(), n_rec);
      hipLaunchKernelGGL(new_frontier_kernel, dim3(grid_of(S, 256)), dim3(256), 0, st, S,
                         ccnt_b.as<uint32_t>(), store_f.as<uint32_t>(), store_at.as<uint32_t>(),
                         node_base, frontier.as<uint32_t>());
      DD_HIP(hipGetLastError());
      n_rec += n_store;
      n_nodes += n_store;
    }

    // stable partition of every node by child
    {
      DevBuf H;
      DD_TRY(H.alloc(4 * 4 * (size_t)n_chunks));
      hipLaunchKernelGGL(hist_kernel, dim3(n_chunks), dim3(kThreads), 0, st, G, S, cbase,
                         forced_b.as<uint8_t>(), labels.as<uint8_t>(), H.as<uint32_t>());
      DD_HIP(hipGetLastError());
      DD_TRY(exclusive_scan_u32(H.as<uint32_t>(), 4 * (int64_t)n_chunks, st));
      DD_HIP(hipMemcpyAsync(ids[1 - cur].p, ids[cur].p, 4 * (size_t)N, hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(scatter_kernel, dim3(n_chunks), dim3(kThreads), 0, st, G, S, cbase,
                         forced_b.as<uint8_t>(), labels.as<uint8_t>(), H.as<uint32_t>(), ids_in,
                         ids[1 - cur].as<uint32_t>());
      DD_HIP(hipGetLastError());
      cur = 1 - cur;
    }

    // leaves and next round's nodes
    DevBuf leaf_f, leaf_at, act_f, act_at;
    const int64_t SK = S * kK;
    DD_TRY(leaf_f.alloc(4 * (size_t)SK));
    DD_TRY(leaf_at.alloc(4 * (size_t)SK));
    DD_TRY(act_f.alloc(4 * (size_t)SK));
    DD_TRY(act_at.alloc(4 * (size_t)SK));
    hipLaunchKernelGGL(children_kernel, dim3(grid_of(SK, 256)), dim3(256), 0, st, S,
                       ccnt_b.as<uint32_t>(), leaf_f.as<uint32_t>(), act_f.as<uint32_t>());
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpyAsync(leaf_at.p, leaf_f.p, leaf_f.bytes, hipMemcpyDeviceToDevice, st));
    DD_HIP(hipMemcpyAsync(act_at.p, act_f.p, act_f.bytes, hipMemcpyDeviceToDevice, st));
    DD_TRY(exclusive_scan_u32(leaf_at.as<uint32_t>(), SK, st));
    DD_TRY(exclusive_scan_u32(act_at.as<uint32_t>(), SK, st));
    const int64_t new_leaves = (int64_t)read_u32(leaf_at.as<uint32_t>() + SK - 1, st) +
                               (int64_t)read_u32(leaf_f.as<uint32_t>() + SK - 1, st);
    const int64_t S2 = (int64_t)read_u32(act_at.as<uint32_t>() + SK - 1, st) +
                       (int64_t)read_u32(act_f.as<uint32_t>() + SK - 1, st);
    DD_TRY(grow(leaves_b, sizeof(LeafRec) * (size_t)(n_leaf + new_leaves), st));
    SegBufs next;
    DD_TRY(next.alloc(S2));
    hipLaunchKernelGGL(compact_kernel, dim3(grid_of(SK, 256)), dim3(256), 0, st, G, S,
                       ccnt_b.as<uint32_t>(), cmean_b.as<float>(), leaf_f.as<uint32_t>(),
                       leaf_at.as<uint32_t>(), act_f.as<uint32_t>(), act_at.as<uint32_t>(),
                       store_f.as<uint32_t>(), store_at.as<uint32_t>(), node_base,
                       leaves_b.as<LeafRec>(), n_leaf, next.view());
    DD_HIP(hipGetLastError());
    DD_HIP(hipStreamSynchronize(st));
    n_leaf += new_leaves;
    std::swap(segs.start.p, next.start.p);
    std::swap(segs.start.bytes, next.start.bytes);
    std::swap(segs.cnt.p, next.cnt.p);
    std::swap(segs.cnt.bytes, next.cnt.bytes);
    std::swap(segs.owner.p, next.owner.p);
    std::swap(segs.owner.bytes, next.owner.bytes);
    std::swap(segs.mean.p, next.mean.p);
    std::swap(segs.mean.bytes, next.mean.bytes);
    std::swap(segs.k.p, next.k.p);
    std::swap(segs.k.bytes, next.k.bytes);
    S = S2;
    ++round;
  }

  // leaves: compact blocks, slot maps, child records.  Slots are u32 and the
  // walk's codes hold 28-bit leaf and node numbers.
  if (n_leaf * kAnnLeaf > 0xFFFFFFFFll || n_leaf >= (1ll << 28) || n_nodes >= (1ll << 28))
    return set_error(DD_ERR_TOO_LARGE, "k-means tree: too many leaves or nodes");
  D.kmt_leaves = n_leaf;
  DD_TRY(D.kmt_meta.alloc(64 * (size_t)n_leaf));
  DD_TRY(D.kmt_h16.alloc(2 * 12 * kAnnLeaf * (size_t)n_leaf));
  DD_TRY(D.kmt_pos.alloc(4 * kAnnLeaf * (size_t)n_leaf));
  DD_TRY(D.kmt_slot.alloc(4 * (size_t)N));
  DD_TRY(grow(recs, 4 * kKmtBuild * (size_t)(n_rec + n_leaf), st));
  DD_TRY(grow(rec_owner, 4 * (size_t)(n_rec + n_leaf), st));
  hipLaunchKernelGGL(leaf_kernel, dim3(grid_of(n_leaf, 4)), dim3(256), 0, st,
                     ids[cur].as<uint32_t>(), D.w64.as<double>(), R, leaves_b.as<LeafRec>(), n_leaf,
                     D.kmt_meta.as<float>(), D.kmt_h16.as<_Float16>(), D.kmt_pos.as<uint32_t>(),
                     D.kmt_slot.as<uint32_t>(), recs.as<float>(), rec_owner.as<uint32_t>(), n_rec);
  DD_HIP(hipGetLastError());
  n_rec += n_leaf;

  // child records grouped by owner (stable), node ranges
  DevBuf order;
  DD_TRY(order.alloc(4 * (size_t)n_rec));
  DD_TRY(iota_u32(order.as<uint32_t>(), n_rec, st));
  int bits = 1;
  while (bits < 32 && (1ll << bits) < n_nodes) ++bits;
  DD_TRY(radix_sort_pairs(rec_owner.as<uint32_t>(), order.as<uint32_t>(), n_rec, bits, st));
  DevBuf full;
  DD_TRY(full.alloc(4 * kKmtBuild * (size_t)n_rec));
  hipLaunchKernelGGL(gather_records_kernel, dim3(grid_of(kKmtBuild * n_rec, 256)), dim3(256), 0, st,
                     recs.as<float>(), order.as<uint32_t>(), n_rec, full.as<float>());
  DD_TRY(D.kmt_node.alloc(8 * (size_t)n_nodes));
  DD_HIP(hipMemsetAsync(D.kmt_node.p, 0, D.kmt_node.bytes, st));
  hipLaunchKernelGGL(node_range_kernel, dim3(grid_of(n_rec, 256)), dim3(256), 0, st,
                     rec_owner.as<uint32_t>(), n_rec, D.kmt_node.as<int2>());
  DD_TRY(D.kmt_nbox.alloc(4 * 24 * (size_t)n_nodes));
  hipLaunchKernelGGL(node_box_kernel, dim3(grid_of(n_nodes, 256)), dim3(256), 0, st,
                     full.as<float>(), D.kmt_node.as<int2>(), n_nodes, D.kmt_nbox.as<float>());
  DD_TRY(D.kmt_child.alloc(4 * kKmtRecord * (size_t)n_rec));
  hipLaunchKernelGGL(compress_records_kernel, dim3(grid_of(n_rec, 256)), dim3(256), 0, st,
                     full.as<float>(), rec_owner.as<uint32_t>(), n_rec, D.kmt_nbox.as<float>(),
                     D.kmt_child.as<float>());
  DD_HIP(hipGetLastError());
  DD_HIP(hipStreamSynchronize(st));
  D.kmt_nodes = n_nodes;
  D.kmt_records = n_rec;
  D.kmt_rounds = round;
  return DD_OK;
}

}  // namespace dd
