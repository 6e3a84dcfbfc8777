// dd_project: dispatch of the projection P_D (Section 2) to the scan kernels.
#include <algorithm>
#include <memory>
#include <mutex>
#include <vector>

#include "pack16.h"
#include "scan.h"
#include "solve.h"

namespace dd {

namespace {

// Device scratch of one call, carved from one of the dataset's arenas (see
// ScratchArena); what does not fit is allocated stream-ordered and freed when
// the call ends.  With a caller's arena (`fixed`) the call carves from that
// block only and fails with DD_ERR_TOO_LARGE rather than allocate: the FP64
// and direct scans then take as many data splits as the block holds.
struct Scratch {
  const Dataset& D;
  hipStream_t st;
  std::unique_ptr<ScratchArena> a;
  ScratchArena* fixed = nullptr;
  size_t off = 0;    // bytes carved from the block
  size_t need = 0;   // bytes requested by the call
  std::vector<void*> extra;
  Scratch(const Dataset& d, hipStream_t s, ScratchArena* f = nullptr) : D(d), st(s), fixed(f) {}
  ScratchArena* arena() const { return fixed ? fixed : a.get(); }
  // bytes left in a caller's block; SIZE_MAX with the dataset's arenas
  size_t room() const { return fixed ? fixed->bytes - off : SIZE_MAX; }
  dd_status open() {
    if (fixed) {
      DD_HIP(hipStreamWaitEvent(st, fixed->done, 0));
      return DD_OK;
    }
    {
      std::lock_guard<std::mutex> lk(D.arena_mu);
      if (!D.arenas.empty()) {
        a = std::move(D.arenas.back());
        D.arenas.pop_back();
      }
    }
    if (a) {
      DD_HIP(hipStreamWaitEvent(st, a->done, 0));
      return DD_OK;
    }
    std::unique_ptr<ScratchArena> n(new ScratchArena);
    DD_HIP(hipEventCreateWithFlags(&n->done, hipEventDisableTiming));
    DD_HIP(hipHostMalloc((void**)&n->pinned, sizeof(uint32_t) * kArenaPinnedWords,
                         hipHostMallocDefault));
    a = std::move(n);
    return DD_OK;
  }
  // word i of the arena's pinned host memory
  uint32_t* host_word(int i) const { return arena()->pinned + i; }
  template <class T>
  dd_status get(T*& out, size_t n) {
    const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
    need += bytes;
    ScratchArena* ar = arena();
    if (ar->block && off + bytes <= ar->bytes) {
      out = reinterpret_cast<T*>(static_cast<char*>(ar->block) + off);
      off += bytes;
      return DD_OK;
    }
    if (fixed)
      return set_error(DD_ERR_TOO_LARGE, "projection scratch beyond the caller's reserve");
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, st);
    if (e != hipSuccess)
      return set_error(e == hipErrorOutOfMemory ? DD_ERR_OOM : DD_ERR_DEVICE,
                       std::string("hipMallocAsync: ") + hipGetErrorString(e));
    extra.push_back(p);
    out = static_cast<T*>(p);
    return DD_OK;
  }
  ~Scratch() {
    for (void* p : extra) (void)hipFreeAsync(p, st);
    if (fixed) {
      if (hipEventRecord(fixed->done, st) != hipSuccess) (void)hipStreamSynchronize(st);
      return;
    }
    if (!a) return;
    if (need > a->bytes && need <= kArenaKeepBytes) {
      // grow the block for the next call once the work queued on it is done
      const size_t grown = std::min(kArenaKeepBytes, ((need + need / 4) + ((1u << 20) - 1)) &
                                                         ~(size_t)((1u << 20) - 1));
      void* p = nullptr;
      const int64_t old = (int64_t)a->bytes;
      if (hipStreamSynchronize(st) != hipSuccess) {   // the arena is dropped
        std::lock_guard<std::mutex> lk(D.arena_mu);
        D.arena_bytes -= old;
        return;
      }
      if (a->block) (void)hipFree(a->block);
      a->block = nullptr;
      a->bytes = 0;
      if (hipMalloc(&p, grown) == hipSuccess) {
        a->block = p;
        a->bytes = grown;
      } else {
        (void)hipGetLastError();
      }
      std::lock_guard<std::mutex> lk(D.arena_mu);
      D.arena_bytes += (int64_t)a->bytes - old;
    }
    if (hipEventRecord(a->done, st) != hipSuccess) {
      (void)hipStreamSynchronize(st);
      std::lock_guard<std::mutex> lk(D.arena_mu);
      D.arena_bytes -= (int64_t)a->bytes;
      a.reset();
      return;
    }
    std::unique_ptr<ScratchArena> drop;   // freed after the lock is released
    std::lock_guard<std::mutex> lk(D.arena_mu);
    if ((int)D.arenas.size() < kArenaKeep) {
      D.arenas.push_back(std::move(a));
    } else {
      D.arena_bytes -= (int64_t)a->bytes;
      drop = std::move(a);   // its destructor waits for `done` before freeing
    }
  }
};

dd_status alloc_cands(Scratch& sc, int64_t positions, int S, int P, int K, CandBuf& cb) {
  cb.S = S;
  cb.P = P;
  cb.K = K;
  size_t slots = (size_t)positions * S * P;
  DD_TRY(sc.get(cb.lb, slots * K));
  DD_TRY(sc.get(cb.j, slots * K));
  DD_TRY(sc.get(cb.count, slots));
  DD_TRY(sc.get(cb.U, (size_t)positions * S));
  return DD_OK;
}

// Optional HIP events bracketing the main scan and the whole call.
struct Timing {
  bool on = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  dd_status init(hipStream_t st) {
    on = true;
    for (auto& e : ev) DD_HIP(hipEventCreate(&e));
    DD_HIP(hipEventRecord(ev[0], st));
    return DD_OK;
  }
  dd_status mark(int k, hipStream_t st) {
    if (on) DD_HIP(hipEventRecord(ev[k], st));
    return DD_OK;
  }
  ~Timing() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

struct Counters {
  int fb1;
  int fb2;
  unsigned long long cand;
};

// Bytes per (query, split) of the candidate lists of the FP64 scan (four lists
// of 16 entries, their counts, the split's bound) and of the FP32 scan (two
// lists), and per (query, split) of the direct scan's partial results.
constexpr size_t kCandBytes64 = 4 * 16 * (sizeof(float) + sizeof(uint32_t)) + 4 * sizeof(int) + sizeof(float);
constexpr size_t kCandBytes32 = 2 * 16 * (sizeof(float) + sizeof(uint32_t)) + 2 * sizeof(int) + sizeof(float);
constexpr size_t kDirectBytes = sizeof(double) + sizeof(uint32_t);
constexpr size_t kAlignSlack = 16 * 256;   // 256-byte alignment of up to 16 pieces

size_t aligned(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255; }

// Scratch of exact64 over a list of len queries with S scan splits and the
// direct fallback at one split (the least it needs).
size_t exact64_bytes(int64_t len, int S) {
  const size_t n = (size_t)len;
  return 2 * aligned(n * S * 4 * 16 * 4) + aligned(n * S * 4 * sizeof(int)) +
         aligned(n * S * sizeof(float)) + aligned(n * sizeof(int)) + aligned(n * sizeof(double)) +
         aligned(n * sizeof(uint32_t));
}

// The plain direct scan of list L2 (h queries), its per-split partial results
// carved from the call's scratch (from a caller's reserve with as many splits
// as the reserve holds).
dd_status direct_from(const Dataset& D, const QueryPrep& Q, QueryList L2, int64_t h, int splits,
                      Outputs out, Scratch& sc, hipStream_t st) {
  const size_t room = sc.room() > 1024 ? sc.room() - 1024 : 0;
  const int S0 = splits > 0 ? splits : direct_splits(D, h);
  const int S = (int)std::min<int64_t>(S0, (int64_t)(room / ((size_t)h * kDirectBytes)));
  if (S < 1) return set_error(DD_ERR_TOO_LARGE, "direct scan: the projection's reserve is too small");
  double* pd = nullptr;
  uint32_t* po = nullptr;
  DD_TRY(sc.get(pd, (size_t)h * S));
  DD_TRY(sc.get(po, (size_t)h * S));
  return run_direct(D, Q, L2, h, S, out, st, pd, po);
}

// FP64 MFMA scan over list L, merge, and the direct fallback for its overflow.
dd_status exact64(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t len_max, int splits,
                  Outputs out, Scratch& sc, int* d_counters, hipStream_t st, int64_t* n_fallback,
                  Timing* tm) {
  int64_t qblocks = (len_max + 255) / 256;
  int S = choose_splits(qblocks, D.n_pad64 / kTile64, splits);
  if (sc.room() != SIZE_MAX) {
    // a caller's reserve: as many splits as it holds beside the fallback list
    // and the direct scan's partial results at one split
    const size_t keep = kAlignSlack + (size_t)len_max * (sizeof(int) + kDirectBytes);
    const size_t room = sc.room() > keep ? sc.room() - keep : 0;
    S = (int)std::min<int64_t>(S, (int64_t)(room / ((size_t)len_max * kCandBytes64)));
    if (S < 1) return set_error(DD_ERR_TOO_LARGE, "FP64 scan: the projection's reserve is too small");
  }
  CandBuf cb;
  DD_TRY(alloc_cands(sc, len_max, S, 4, 16, cb));
  if (tm) DD_TRY(tm->mark(1, st));
  DD_TRY(launch_scan64(D, Q, L, len_max, cb, st));
  if (tm) DD_TRY(tm->mark(2, st));
  int* fb = nullptr;
  DD_TRY(sc.get(fb, (size_t)len_max));
  int* fb_count = d_counters + 1;
  // candidates are counted only for the statistics
  unsigned long long* n_cand =
      (tm && tm->on) ? reinterpret_cast<unsigned long long*>(d_counters + 2) : nullptr;
  DD_TRY(launch_merge_rerank(D, Q, L, len_max, cb, nullptr, out, fb, fb_count, n_cand, st));
  uint32_t* hw = sc.host_word(0);
  DD_HIP(hipMemcpyAsync(hw, fb_count, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  const int h = (int)*hw;
  if (n_fallback) *n_fallback += h;
  if (h > 0) {
    QueryList L2{fb, fb_count, h};
    DD_TRY(direct_from(D, Q, L2, h, 0, out, sc, st));
  }
  return DD_OK;
}

// FP32 MFMA scan over list L, merge and FP64 rerank; the queries whose lists
// overflowed (or that the scan leaves out) go to the FP64 MFMA scan.
dd_status mixed32(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t len_max, int splits,
                  Outputs out, Scratch& sc, int* d_counters, hipStream_t st, int64_t* n_fallback,
                  Timing* tm) {
  const int64_t qblocks = (len_max + 255) / 256;
  int S = choose_splits(qblocks, D.n_pad32 / kTile32, splits);
  if (sc.room() != SIZE_MAX) {
    // a caller's reserve: as many splits as it holds beside the fallback list
    // and the FP64 scan of every query at one split
    const size_t keep = kAlignSlack + aligned((size_t)len_max * sizeof(int)) + exact64_bytes(len_max, 1);
    const size_t room = sc.room() > keep ? sc.room() - keep : 0;
    S = (int)std::min<int64_t>(S, (int64_t)(room / ((size_t)len_max * kCandBytes32)));
    if (S < 1) return set_error(DD_ERR_TOO_LARGE, "FP32 scan: the projection's reserve is too small");
  }
  CandBuf cb;
  DD_TRY(alloc_cands(sc, len_max, S, 2, 16, cb));
  if (tm) DD_TRY(tm->mark(1, st));
  DD_TRY(launch_scan32(D, Q, L, len_max, cb, st));
  if (tm) DD_TRY(tm->mark(2, st));
  int* fb = nullptr;
  DD_TRY(sc.get(fb, (size_t)len_max));
  unsigned long long* n_cand =
      (tm && tm->on) ? reinterpret_cast<unsigned long long*>(d_counters + 2) : nullptr;
  DD_TRY(launch_merge_rerank(D, Q, L, len_max, cb, nullptr, out, fb, d_counters, n_cand, st));
  uint32_t* hw = sc.host_word(1);
  DD_HIP(hipMemcpyAsync(hw, d_counters, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  const int h = (int)*hw;
  if (n_fallback) *n_fallback += h;
  if (h > 0) {
    QueryList L1{fb, d_counters, h};
    DD_TRY(exact64(D, Q, L1, h, 0, out, sc, d_counters, st, nullptr, nullptr));
  }
  return DD_OK;
}

}  // namespace

}  // namespace dd

namespace dd {

dd_status project_impl_ex(const Dataset& D, const double* states_dev, bool whitened, int64_t m,
                          const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                          int64_t* idx_out_dev, double* dist_out_dev, double* dist2_out_dev,
                          hipStream_t st, const float* fd_q = nullptr,
                          const int* budget_q = nullptr, ScratchArena* fixed = nullptr);

dd_status project_impl(const Dataset& D, const double* states_dev, bool whitened, int64_t m,
                       const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                       int64_t* idx_out_dev, double* dist_out_dev, hipStream_t st) {
  return project_impl_ex(D, states_dev, whitened, m, warm_start_idx_dev, opts, idx_out_dev,
                         dist_out_dev, nullptr, st);
}

// Scratch bytes a projection of up to m_max queries in `mode` carves at most
// from a caller's reserve: its main path at the default splits (the largest
// over the batch sizes up to m_max, as the splits follow the number of query
// blocks), every fallback at one split.
size_t project_scratch_need(const Dataset& D, int mode, int64_t m_max) {
  constexpr int kNumCounters = 32 + 2 * kCounterStride * kCounterSlots;
  auto need = [&](int64_t m) {
    const size_t n = (size_t)std::max<int64_t>(m, 1);
    size_t b = aligned(n * 12 * sizeof(double)) + 2 * aligned(n * sizeof(double)) +
               2 * aligned(n * sizeof(int)) + aligned(kNumCounters * sizeof(int));
    if (mode == DD_DIRECT_FP64) {
      const int S = direct_splits(D, m);
      b += aligned(n * S * sizeof(double)) + aligned(n * S * sizeof(uint32_t));
    } else if (mode == DD_EXACT_FP64) {
      b += exact64_bytes(m, choose_splits((m + 255) / 256, D.n_pad64 / kTile64, 0));
    } else if (mode == DD_MIXED_FP32) {
      const int S = choose_splits((m + 255) / 256, D.n_pad32 / kTile32, 0);
      b += 2 * aligned(n * S * 2 * 16 * 4) + aligned(n * S * 2 * sizeof(int)) +
           aligned(n * S * sizeof(float)) + aligned(n * sizeof(int)) + exact64_bytes(m, 1);
    } else if (walk_mode(mode)) {
      b += aligned(n * sizeof(int)) + aligned(n * 12 * sizeof(double)) + exact64_bytes(m, 1);
    } else {
      const int S = choose_splits16((m + kScan16Queries - 1) / kScan16Queries, D.n_tiles, 0);
      const size_t cap = (size_t)std::min<int64_t>(std::max<int64_t>(32 * m, 1 << 20), 1 << 26);
      b += aligned(n * S * sizeof(float)) + aligned(cap * sizeof(WorkItem)) +
           2 * aligned(n * 2 * 32 * 4) + aligned(n * 2 * sizeof(int)) + aligned(n * sizeof(int)) +
           exact64_bytes(m, 1);
    }
    return b + kAlignSlack;
  };
  size_t best = need(m_max);
  for (int64_t m = 256; m < m_max; m += 256) best = std::max(best, need(m));
  return best;
}

// As project_impl, every temporary buffer carved from `arena` (a caller's
// reserve, see project_scratch_need) instead of the dataset's arenas.
dd_status project_reserved(const Dataset& D, const double* states_dev, bool whitened, int64_t m,
                           const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                           int64_t* idx_out_dev, double* dist_out_dev, ScratchArena* arena,
                           hipStream_t st) {
  if (!arena) return set_error(DD_ERR_ARG, "no reserve");
  return project_impl_ex(D, states_dev, whitened, m, warm_start_idx_dev, opts, idx_out_dev,
                         dist_out_dev, nullptr, st, nullptr, nullptr, arena);
}

// As project_impl; dist2_out_dev (exact DD_ANN only) receives the distance to
// the second nearest point, -1 where it is not certified; fd_q / budget_q
// (walk modes, device arrays over the m states) give each state its own
// radius factor and leaf budget; `fixed` (optional) is a caller's reserve that
// the call carves every temporary buffer from.
dd_status project_impl_ex(const Dataset& D, const double* states_dev, bool whitened, int64_t m,
                          const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                          int64_t* idx_out_dev, double* dist_out_dev, double* dist2_out_dev,
                          hipStream_t st, const float* fd_q, const int* budget_q,
                          ScratchArena* fixed) {
  if (m < 0 || m > 0x7FFFFFFFll) return set_error(DD_ERR_ARG, "m must be in [0, 2^31-1]");
  if (m == 0) return DD_OK;
  if (!states_dev || !idx_out_dev) return set_error(DD_ERR_ARG, "NULL states or idx_out");
  const int mode = opts ? opts->mode : DD_EXACT_FP64;
  const int splits = opts ? opts->splits : 0;
  if (splits < 0) return set_error(DD_ERR_ARG, "splits must be >= 0");
  const int budget = opts ? opts->ann_budget : 0;
  if (budget < 0) return set_error(DD_ERR_ARG, "ann_budget must be >= 0");
  if (opts && (opts->passes < 0 || opts->passes > 2))
    return set_error(DD_ERR_ARG, "passes must be 0, 1 or 2");
  const double discount = opts ? opts->ann_radius_discount : 0.0;
  if (!(discount >= 0.0 && discount <= 1.0))
    return set_error(DD_ERR_ARG, "ann_radius_discount must be in [0, 1]");
  const double fd = 1.0 - discount;
  if (discount > 0.0 && mode != DD_KMEANS)
    return set_error(DD_ERR_ARG, "ann_radius_discount applies to the k-means walk only");
  switch (mode) {
    case DD_EXACT_FP64:
    case DD_DIRECT_FP64:
      if (!(D.packs & DD_PACK_FP64)) return set_error(DD_ERR_UNSUPPORTED, "dataset has no FP64 pack");
      break;
    case DD_MIXED_FP32:
      if (!(D.packs & DD_PACK_FP32) || !(D.packs & DD_PACK_FP64))
        return set_error(DD_ERR_UNSUPPORTED, "FP32 mode needs the FP32 and FP64 packs");
      break;
    case DD_MIXED_BF16:
      if (!(D.packs & DD_PACK_BF16) || !(D.packs & DD_PACK_FP64))
        return set_error(DD_ERR_UNSUPPORTED, "BF16 mode needs the BF16 and FP64 packs");
      break;
    case DD_MIXED_FP16:
      if (!(D.packs & DD_PACK_FP16) || !(D.packs & DD_PACK_FP64))
        return set_error(DD_ERR_UNSUPPORTED, "FP16 mode needs the FP16 and FP64 packs");
      break;
    case DD_ANN:
      if (!(D.packs & DD_PACK_ANN)) return set_error(DD_ERR_UNSUPPORTED, "dataset has no ANN tree");
      break;
    case DD_KMEANS:
      if (!(D.packs & DD_PACK_KMEANS))
        return set_error(DD_ERR_UNSUPPORTED, "dataset has no k-means tree");
      break;
    default:
      return set_error(DD_ERR_UNSUPPORTED, "projection mode not available");
  }
  int cur_dev = -1;
  DD_HIP(hipGetDevice(&cur_dev));
  if (cur_dev != D.device) return set_error(DD_ERR_ARG, "dataset lives on another device");

  Scratch sc(D, st, fixed);
  DD_TRY(sc.open());
  Timing timing;
  if (opts && opts->stats) DD_TRY(timing.init(st));
  QueryPrep Q;
  DD_TRY(sc.get(Q.qw, (size_t)m * 12));
  DD_TRY(sc.get(Q.qn2, (size_t)m));
  DD_TRY(sc.get(Q.u64, (size_t)m));
  DD_TRY(sc.get(Q.u32, (size_t)m));
  DD_TRY(sc.get(Q.invalid, (size_t)m));
  // [0] fb1, [1] fb2, [2..3] candidates (u64), [4..5] slow tiles (u64),
  // [32..) ANN walk statistics (kCounterSlots slots of kCounterStride u64, each
  // slot on its own 128-byte line)
  constexpr int kNumCounters = 32 + 2 * kCounterStride * kCounterSlots;
  int* counters = nullptr;
  DD_TRY(sc.get(counters, kNumCounters));
  DD_HIP(hipMemsetAsync(counters, 0, kNumCounters * sizeof(int), st));
  const bool scan16 = (mode == DD_MIXED_BF16 || mode == DD_MIXED_FP16);
  DD_TRY(prepare_queries(D, states_dev, whitened, m, warm_start_idx_dev,
                         scan16 ? (double)D.sc16.s : 1.0, Q, st));
  Outputs out{idx_out_dev, dist_out_dev};
  QueryList all{nullptr, nullptr, m};
  int64_t n_fallback = 0;
  int64_t n_items_host = 0;
  unsigned long long* ann = nullptr;

  if (mode == DD_DIRECT_FP64) {
    DD_TRY(timing.mark(1, st));
    DD_TRY(direct_from(D, Q, all, m, splits, out, sc, st));
    DD_TRY(timing.mark(2, st));
  } else if (mode == DD_EXACT_FP64) {
    DD_TRY(exact64(D, Q, all, m, splits, out, sc, counters, st, &n_fallback, &timing));
  } else if (mode == DD_MIXED_FP32) {
    DD_TRY(mixed32(D, Q, all, m, splits, out, sc, counters, st, &n_fallback, &timing));
  } else if (walk_mode(mode)) {
    int* fb = nullptr;
    DD_TRY(sc.get(fb, (size_t)m));
    DD_TRY(sc.get(Q.yq, (size_t)m * 12));
    ann = reinterpret_cast<unsigned long long*>(counters + 32);
    DD_TRY(timing.mark(1, st));
    if (dist2_out_dev && (budget != 0 || fd < 1.0))
      return set_error(DD_ERR_ARG, "second distances need the exact walk");
    DD_TRY(launch_ann_walk(D, Q, all, m, warm_start_idx_dev, budget, out, fb, counters, ann,
                           dist2_out_dev, st, mode == DD_KMEANS, fd, fd_q, budget_q));
    DD_TRY(timing.mark(2, st));
    uint32_t* hw = sc.host_word(1);
    DD_HIP(hipMemcpyAsync(hw, counters, sizeof(int), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    const int h = (int)*hw;
    n_fallback += h;
    if (h > 0) {
      QueryList L1{fb, counters, h};
      DD_TRY(exact64(D, Q, L1, h, 0, out, sc, counters, st, nullptr, nullptr));
    }
  } else {
    const bool fp16 = (mode == DD_MIXED_FP16);
    const int64_t qblocks = (m + kScan16Queries - 1) / kScan16Queries;
    const int S = choose_splits16(qblocks, D.n_tiles, splits);
    Scan16Call c;
    c.Q = &Q;
    c.L = all;
    c.list_len_max = m;
    c.S = S;
    DD_TRY(sc.get(c.U_out, (size_t)m * S));
    unsigned* n_items = reinterpret_cast<unsigned*>(counters + 4);
    c.n_items = n_items;
    c.item_cap = (unsigned)std::min<int64_t>(std::max<int64_t>(32 * m, 1 << 20), 1 << 26);
    DD_TRY(sc.get(c.items, c.item_cap));
    CandBuf cb;
    cb.S = 1;
    cb.P = 2;
    cb.K = 32;
    DD_TRY(sc.get(cb.lb, (size_t)m * 2 * cb.K));
    DD_TRY(sc.get(cb.j, (size_t)m * 2 * cb.K));
    DD_TRY(sc.get(cb.count, (size_t)m * 2));
    DD_HIP(hipMemsetAsync(cb.count, 0, sizeof(int) * (size_t)m * 2, st));
    c.cb = cb;
    // Without a warm start the bound starts at +inf; a streaming pass over every
    // 64th tile seeds it, so the marking pass logs few stale work items (a
    // denser seeding pass costs more than the extra items it saves: at N = 2^27,
    // m = 65536 every 16th tile gives 299 ms per step, every 64th 289 ms).
    const int passes = (opts && opts->passes) ? opts->passes : (warm_start_idx_dev ? 1 : 2);
    if (passes >= 2) {
      c.phase = Scan16Call::kBound;
      c.stride = 64;
      DD_TRY(launch_scan16(D, fp16, c, st));
      DD_TRY(launch_reduce_bounds(all, m, c.U_out, S, Q.u32, st));
    }
    c.phase = Scan16Call::kMark;
    c.stride = 1;
    DD_TRY(timing.mark(1, st));   // the main scan: every (query, data point) pair
    DD_TRY(launch_scan16(D, fp16, c, st));
    DD_TRY(timing.mark(2, st));
    DD_TRY(launch_reduce_bounds(all, m, c.U_out, S, Q.u32, st));
    // every (query group, tile) pair is logged at most once: when that many
    // items fit the list and make a small grid, the extraction is launched for
    // all of them (its waves read the logged count and the rest exit) and the
    // count is not read back (no host round trip in small projections)
    const int64_t max_items = (m + 31) / 32 * D.n_tiles;
    const bool bounded = max_items <= std::min<int64_t>(c.item_cap, 1 << 16);
    uint32_t* nw = sc.host_word(2);
    unsigned ni = (unsigned)std::min<int64_t>(max_items, c.item_cap);
    if (!bounded) {
      DD_HIP(hipMemcpyAsync(nw, n_items, sizeof(unsigned), hipMemcpyDeviceToHost, st));
      DD_HIP(hipStreamSynchronize(st));
      ni = *nw;
    }
    if (!bounded && ni > c.item_cap) {
      // too many items were logged under the running bound: mark again under
      // the final bound, which logs only tiles holding certified candidates
      DD_HIP(hipMemsetAsync(n_items, 0, sizeof(unsigned), st));
      DD_TRY(launch_scan16(D, fp16, c, st));
      DD_HIP(hipMemcpyAsync(nw, n_items, sizeof(unsigned), hipMemcpyDeviceToHost, st));
      DD_HIP(hipStreamSynchronize(st));
      ni = *nw;
      if (ni > c.item_cap) return set_error(DD_ERR_TOO_LARGE, "16-bit scan work list overflow");
    }
    n_items_host = bounded ? -1 : (int64_t)ni;   // -1: read with the statistics
    c.phase = Scan16Call::kExtract;
    c.item_cap = ni;
    DD_TRY(launch_scan16(D, fp16, c, st));
    int* fb = nullptr;
    DD_TRY(sc.get(fb, (size_t)m));
    DD_TRY(launch_merge_rerank(
        D, Q, all, m, cb, Q.u32, out, fb, counters,
        timing.on ? reinterpret_cast<unsigned long long*>(counters + 2) : nullptr, st));
    uint32_t* hw = sc.host_word(1);
    DD_HIP(hipMemcpyAsync(hw, counters, sizeof(int), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    const int h = (int)*hw;
    n_fallback += h;
    if (h > 0) {
      QueryList L1{fb, counters, h};
      DD_TRY(exact64(D, Q, L1, h, 0, out, sc, counters, st, nullptr, nullptr));
    }
  }
  if (opts && opts->stats) {
    unsigned long long nc = 0;
    unsigned long long slots[kCounterStride * kCounterSlots] = {};
    unsigned long long a[6] = {0, 0, 0, 0, 0, 0};
    unsigned items = 0;
    DD_HIP(hipMemcpyAsync(&nc, counters + 2, sizeof(nc), hipMemcpyDeviceToHost, st));
    if (n_items_host < 0)
      DD_HIP(hipMemcpyAsync(&items, counters + 4, sizeof(items), hipMemcpyDeviceToHost, st));
    if (ann) DD_HIP(hipMemcpyAsync(slots, ann, sizeof(slots), hipMemcpyDeviceToHost, st));
    DD_TRY(timing.mark(3, st));
    DD_HIP(hipStreamSynchronize(st));
    for (int s = 0; s < kCounterSlots; ++s)
      for (int i = 0; i < 6; ++i) a[i] += slots[kCounterStride * s + i];
    nc += a[3];
    float scan_ms = 0.0f, total_ms = 0.0f;
    DD_HIP(hipEventElapsedTime(&scan_ms, timing.ev[1], timing.ev[2]));
    DD_HIP(hipEventElapsedTime(&total_ms, timing.ev[0], timing.ev[3]));
    opts->stats->candidates = (int64_t)nc;
    opts->stats->overflowed = n_fallback;
    opts->stats->visited = (int64_t)a[0];
    opts->stats->boxes = (int64_t)a[1];
    opts->stats->leaves = (int64_t)a[2];
    opts->stats->leaf_boxes = (int64_t)a[4];
    opts->stats->nodes = (int64_t)a[5];
    opts->stats->scan_ms = scan_ms;
    opts->stats->total_ms = total_ms;
    opts->stats->slow_tiles = n_items_host < 0 ? (int64_t)items : n_items_host;
  }
  return DD_OK;
}

dd_status project_whitened(const Dataset& D, const double* qw_dev, int64_t m,
                           const int64_t* warm_dev, int mode, int ann_budget, int64_t* idx_out,
                           double* dist_out, hipStream_t st, double* dist2_out, double fd,
                           int passes, const float* fd_q, const int* budget_q) {
  dd_project_opts o{};
  o.mode = mode;
  o.passes = passes;
  o.ann_budget = ann_budget;
  o.ann_radius_discount = 1.0 - fd;
  return project_impl_ex(D, qw_dev, true, m, warm_dev, &o, idx_out, dist_out, dist2_out, st, fd_q,
                         budget_q);
}

}  // namespace dd

extern "C" dd_status dd_project(const dd_dataset* ds, const double* states_dev, int64_t m,
                                const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                                int64_t* idx_out_dev, double* dist_out_dev, void* hip_stream) {
  if (!ds) return dd::set_error(DD_ERR_ARG, "dataset is NULL");
  return dd::project_impl(ds->d, states_dev, false, m, warm_start_idx_dev, opts, idx_out_dev,
                          dist_out_dev, static_cast<hipStream_t>(hip_stream));
}
