// Projection kernels: launch interfaces (host side).
#pragma once
#include "dd_internal.h"

namespace dd {

// Whitened queries and per-query search state, produced by prepare_queries.
struct QueryPrep {
  double* qw = nullptr;     // [m][12] whitened queries (zero rows for invalid states)
  double* qn2 = nullptr;    // [m] |q|^2
  double* u64 = nullptr;    // [m] FP64-path initial bound on min d (warm start) or +inf
  float* u32 = nullptr;     // [m] sqrt-space initial bound (warm start) or +inf, in the
                            // scaled coordinates of the 16-bit scans in those modes
  int* invalid = nullptr;   // [m] 1 for non-finite states
  float* yq = nullptr;      // [m][12] queries on the principal axes of the dataset's trees
                            // (walk modes; written by launch_ann_walk)
};

// Candidate lists written by the scans: slot = (list position * S + split) * P + part.
struct CandBuf {
  float* lb = nullptr;      // [slots][K] lower bound of the candidate (scan's own units)
  uint32_t* j = nullptr;    // [slots][K] sorted data position
  int* count = nullptr;     // [slots] number of entries; bit 30 set = overflowed
  float* U = nullptr;       // [positions][S] upper bound of the minimum (scan's units)
  int K = 0, S = 0, P = 0;
};
constexpr int kOverflowBit = 1 << 30;

// Query list: either the identity over [0, m) (list == nullptr) or list[0..*count).
struct QueryList {
  const int* list = nullptr;
  const int* count = nullptr;   // device counter when list != nullptr
  int64_t m = 0;                // capacity / identity length
};

struct Outputs {
  int64_t* idx = nullptr;       // [m] original index
  double* dist = nullptr;       // [m] 1/2 d^2 or nullptr
};

// Whiten m states (or take them as already whitened), |q|^2, warm-start bounds
// (the sqrt-space one multiplied by u32_scale: the 16-bit scans' scale, else 1).
dd_status prepare_queries(const Dataset& D, const double* states, bool whitened, int64_t m,
                          const int64_t* warm, double u32_scale, QueryPrep& Q, hipStream_t st);

// FP64 MFMA scan (expanded form) over the list; fills cb (P = 4, d-space bounds).
dd_status launch_scan64(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len,
                        const CandBuf& cb, hipStream_t st);
// FP32 MFMA scan (expanded form, stored norms as the accumulator input) over the
// list; fills cb (P = 2, d-space bounds), like the FP64 scan.
dd_status launch_scan32(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len,
                        const CandBuf& cb, hipStream_t st);
// 16-bit MFMA scan over tile-centred data (sqrt-space bounds), in phases:
//   kBound    streaming pass: U_out[p][S] = split bounds (tiles visited with stride)
//   kMark     the same, also logging work items (query group, tile) that may hold
//             candidates under the running bound
//   kExtract  recompute the logged items and append every point whose lower bound
//             is <= the query's final bound Q->u32 to cb (slot p*2 + half, counts
//             claimed atomically; cb.count must start at zero)
struct WorkItem {
  uint32_t group;   // list position of the group's first query / 32
  uint32_t tile;
};
struct Scan16Call {
  enum Phase { kBound = 0, kMark = 1, kExtract = 2 };
  int phase = kBound;
  const QueryPrep* Q = nullptr;
  QueryList L;
  int64_t list_len_max = 0;
  int S = 1;
  int stride = 1;
  float* U_out = nullptr;
  WorkItem* items = nullptr;
  unsigned* n_items = nullptr;
  unsigned item_cap = 0;
  CandBuf cb;
};
dd_status launch_scan16(const Dataset& D, bool fp16, const Scan16Call& call, hipStream_t st);
// Merge candidate lists, rerank in FP64 direct form, write outputs; queries that
// overflowed (or found no candidate) are appended to fb_list / fb_count.  The
// bound is Uq[q] when given, else the minimum of cb.U over the splits.
dd_status launch_merge_rerank(const Dataset& D, const QueryPrep& Q, QueryList L,
                              int64_t list_len, const CandBuf& cb, const float* Uq, Outputs out,
                              int* fb_list, int* fb_count, unsigned long long* n_cand,
                              hipStream_t st);
// Plain FP64 direct-form scan with lexicographic (dist, original index) minimum,
// split over the data, followed by its merge.  The per-split partial results
// (list_len x splits, splits = choose_splits(list blocks, tiles, S)) go to
// part_d / part_o when both are given, else to stream-ordered allocations.
dd_status run_direct(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len, int S,
                     Outputs out, hipStream_t st, double* part_d = nullptr,
                     uint32_t* part_o = nullptr);

// Splits of a scan over the data (FP64 and direct scans): `requested` if > 0;
// with fewer than 64 query blocks one round of workgroups (512), otherwise
// about 2048; multiples of 8 give a grid that the scans can deal to the eight
// XCDs split by split.
int choose_splits(int64_t n_query_blocks, int64_t n_tiles, int requested);
// The splits run_direct takes for a list of list_len queries when S = 0.
int direct_splits(const Dataset& D, int64_t list_len);

// Queries per workgroup of the 16-bit pass (sixteen waves of two 32-query groups).
constexpr int kScan16Queries = 1024;

// Splits of the 16-bit pass: with fewer than 64 query blocks, one round of
// workgroups (256: one per CU), so that no second round waits on a short
// first one; otherwise about 1024 workgroups.  Multiples of 8 keep a split's
// workgroups on one XCD.
int choose_splits16(int64_t n_query_blocks, int64_t n_tiles, int requested);

// DD_ANN walk over the dataset's box tree (kmt: DD_KMEANS walk over its
// k-means tree); Q.yq must hold room for the rotated queries.
// k-means tree with radius factor fd) for the queries of L (one wavefront
// each): writes outputs, appends overflowed queries to fb_list / fb_count, adds
// (points visited, boxes tested, leaves visited, candidates reranked, leaf
// boxes tested, nodes expanded) to slot blockIdx % kCounterSlots of counters
// (kCounterStride u64 per slot).
// budget = max leaves per query, 0 = exact.
// With dist2 (exact walk only) the walk certifies the two nearest points and
// writes the second distance (1/2 d^2; -1 when the query went to the fallback).
// fd_q / budget_q (device, indexed by query, optional): per-query radius factor
// (k-means walk) and leaf budget in place of fd and budget.
dd_status launch_ann_walk(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t len_max,
                          const int64_t* warm, int budget, Outputs out, int* fb_list, int* fb_count,
                          unsigned long long* counters, double* dist2, hipStream_t st,
                          bool kmt = false, double fd = 1.0, const float* fd_q = nullptr,
                          const int* budget_q = nullptr);

// u32[q] = min(u32[q], min over the S split bounds U[p][S]).
dd_status launch_reduce_bounds(QueryList L, int64_t list_len_max, const float* U, int S, float* u32,
                               hipStream_t st);

// ---------------------------------------------------------------------------
// Device helpers shared by the scan translation units
// ---------------------------------------------------------------------------
constexpr float kRelUp = 1.0f + 9.5367431640625e-07f;   // 1 + 2^-20
constexpr float kRelDn = 1.0f - 9.5367431640625e-07f;   // 1 - 2^-20

// Candidate list append; a full list is compacted to the entries whose lower
// bound is still <= U before it is declared overflowed.
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


}  // namespace dd
