// Projection kernels: launch interfaces (host side).
#pragma once
#include "dd_internal.h"

namespace dd {

// Whitened queries and per-query search state, produced by prepare_queries.
struct QueryPrep {
  double* qw = nullptr;     // [m][12] whitened queries (zero rows for invalid states)
  double* qn2 = nullptr;    // [m] |q|^2
  double* u64 = nullptr;    // [m] FP64-path initial bound on min d (warm start) or +inf
  float* u32 = nullptr;     // [m] sqrt-space initial bound (warm start) or +inf
  int* invalid = nullptr;   // [m] 1 for non-finite states
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

dd_status prepare_queries(const Dataset& D, const double* states, int64_t m, const int64_t* warm,
                          QueryPrep& Q, hipStream_t st);

// FP64 MFMA scan (expanded form) over the list; fills cb (P = 4, d-space bounds).
dd_status launch_scan64(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len,
                        const CandBuf& cb, hipStream_t st);
// 16-bit MFMA scan over tile-centred data (P = 2, sqrt-space bounds).
dd_status launch_scan16(const Dataset& D, bool fp16, const QueryPrep& Q, QueryList L,
                        int64_t list_len, const CandBuf& cb, hipStream_t st);
// Merge candidate lists, rerank in FP64 direct form, write outputs; queries that
// overflowed (or found no candidate) are appended to fb_list / fb_count.
dd_status launch_merge_rerank(const Dataset& D, const QueryPrep& Q, QueryList L,
                              int64_t list_len, const CandBuf& cb, bool sqrt_space, Outputs out,
                              int* fb_list, int* fb_count, unsigned long long* n_cand,
                              hipStream_t st);
// Plain FP64 direct-form scan with lexicographic (dist, original index) minimum,
// split over the data, followed by its merge.
dd_status run_direct(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t list_len, int S,
                     Outputs out, hipStream_t st);
// Write idx -1 / dist NaN for invalid states.
dd_status launch_mark_invalid(const QueryPrep& Q, int64_t m, Outputs out, hipStream_t st);

int choose_splits(int64_t n_query_blocks, int64_t n_tiles, int requested);

}  // namespace dd
