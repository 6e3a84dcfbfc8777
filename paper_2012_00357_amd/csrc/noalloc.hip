// dd_project_noalloc: the projection P_D of dd_project (Section 2) for callers
// that cannot allocate device memory (work captured into HIP graphs, serving
// loops, harnesses that forbid allocation).  Its temporary buffers come from one
// file-scope device array instead of the dataset's scratch arenas; it calls no
// allocating routine and reads nothing back to the host: the fallback scans are
// launched with grids sized for every query and read the length of their query
// list on the device.
#include <algorithm>
#include <mutex>
#include <string>

#include "pack16.h"
#include "scan.h"

namespace dd {

namespace {

// The scratch array: every call on a GPU uses that GPU's copy, which keeps the
// last call's contents (what must start at zero is cleared by each call).
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the scratch array on device dev (the current device),
// looked up once per device.  The array's name is a host-side stand-in, not a
// device address: host code uses only this pointer.
dd_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(DD_ERR_DEVICE, "device id out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(DD_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return DD_OK;
}

__global__ void zero_words_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Consecutive 256-byte aligned pieces of the scratch array.
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <class T>
  bool get(T*& out, size_t n) {
    const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
    if (off + bytes > kNoAllocBytes) return false;
    out = reinterpret_cast<T*>(base + off);
    off += bytes;
    return true;
  }
  size_t left() const { return kNoAllocBytes - off; }
};

// Bytes per (query, split) of the FP64 scan's candidate lists (four lists of
// 16 entries, counts, split bound) and of the direct scan's partial results.
constexpr size_t kBytesPerSplit = 4 * 16 * (sizeof(float) + sizeof(uint32_t)) + 4 * sizeof(int) +
                                  sizeof(float) + sizeof(double) + sizeof(uint32_t);

// FP64 MFMA scan of list L (at most m queries, its length read on the device),
// merge and FP64 rerank, then the plain direct scan of the queries whose lists
// overflowed (count at *fb_count, which must start at zero).
dd_status exact_from_scratch(const Dataset& D, const QueryPrep& Q, QueryList L, int64_t m,
                             Outputs out, Carve& c, int* fb_list, int* fb_count, hipStream_t st) {
  const int64_t qblocks = (m + 255) / 256;
  const int64_t tiles = D.n_pad64 / kTile64;
  // as many data splits as the scratch holds, up to dd_project's own choice
  const size_t room = c.left() > 4096 ? c.left() - 4096 : 0;   // 4096: alignment of six pieces
  const int64_t fit = (int64_t)(room / ((size_t)m * kBytesPerSplit));
  const int S = (int)std::min<int64_t>(choose_splits(qblocks, tiles, 0), fit);
  if (S < 1) return set_error(DD_ERR_TOO_LARGE, "dd_project_noalloc: scratch too small");
  CandBuf cb;
  cb.S = S;
  cb.P = 4;
  cb.K = 16;
  const size_t slots = (size_t)m * S * 4;
  double* pd = nullptr;
  uint32_t* po = nullptr;
  if (!c.get(cb.lb, slots * cb.K) || !c.get(cb.j, slots * cb.K) || !c.get(cb.count, slots) ||
      !c.get(cb.U, (size_t)m * S) || !c.get(pd, (size_t)m * S) || !c.get(po, (size_t)m * S))
    return set_error(DD_ERR_TOO_LARGE, "dd_project_noalloc: scratch too small");
  DD_TRY(launch_scan64(D, Q, L, m, cb, st));
  DD_TRY(launch_merge_rerank(D, Q, L, m, cb, nullptr, out, fb_list, fb_count, nullptr, st));
  const QueryList L2{fb_list, fb_count, m};
  return run_direct(D, Q, L2, m, S, out, st, pd, po);
}

}  // namespace

}  // namespace dd

extern "C" dd_status dd_project_noalloc(const dd_dataset* ds, const double* states_dev, int64_t m,
                                        const int64_t* warm_start_idx_dev,
                                        const dd_project_opts* opts, int64_t* idx_out_dev,
                                        double* dist_out_dev, void* hip_stream) {
  using namespace dd;
  if (!ds) return set_error(DD_ERR_ARG, "dataset is NULL");
  const Dataset& D = ds->d;
  if (m < 0) return set_error(DD_ERR_ARG, "m must be >= 0");
  if (m > DD_NOALLOC_MAX_QUERIES)
    return set_error(DD_ERR_TOO_LARGE, "dd_project_noalloc: m exceeds DD_NOALLOC_MAX_QUERIES");
  if (m == 0) return DD_OK;
  if (!states_dev || !idx_out_dev) return set_error(DD_ERR_ARG, "NULL states or idx_out");
  const int mode = opts ? opts->mode : DD_EXACT_FP64;
  const int budget = opts ? opts->ann_budget : 0;
  const double discount = opts ? opts->ann_radius_discount : 0.0;
  if (opts && opts->stats)
    return set_error(DD_ERR_ARG, "dd_project_noalloc keeps no statistics (stats must be NULL)");
  if (opts && (opts->splits < 0 || opts->passes < 0 || opts->passes > 2 || budget < 0))
    return set_error(DD_ERR_ARG, "splits, passes or ann_budget out of range");
  if (!(discount >= 0.0 && discount <= 1.0))
    return set_error(DD_ERR_ARG, "ann_radius_discount must be in [0, 1]");
  if (discount > 0.0 && mode != DD_KMEANS)
    return set_error(DD_ERR_ARG, "ann_radius_discount applies to the k-means walk only");
  if (mode == DD_EXACT_FP64) {
    if (budget != 0) return set_error(DD_ERR_ARG, "ann_budget applies to the walks only");
  } else if (mode == DD_ANN) {
    if (!(D.packs & DD_PACK_ANN)) return set_error(DD_ERR_UNSUPPORTED, "dataset has no ANN tree");
  } else if (mode == DD_KMEANS) {
    if (!(D.packs & DD_PACK_KMEANS))
      return set_error(DD_ERR_UNSUPPORTED, "dataset has no k-means tree");
  } else {
    return set_error(DD_ERR_UNSUPPORTED,
                     "dd_project_noalloc supports DD_EXACT_FP64, DD_ANN and DD_KMEANS");
  }
  int dev = -1;
  DD_HIP(hipGetDevice(&dev));
  if (dev != D.device) return set_error(DD_ERR_ARG, "dataset lives on another device");
  unsigned char* base = nullptr;
  DD_TRY(scratch_address(dev, &base));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);

  Carve c{base};
  QueryPrep Q;
  // [0] walk fallback count, [1] scan fallback count, [32..) walk statistics
  constexpr int kNumCounters = 32 + 2 * kCounterStride * kCounterSlots;
  int* counters = nullptr;
  int* fb1 = nullptr;
  int* fb2 = nullptr;
  if (!c.get(Q.qw, (size_t)m * 12) || !c.get(Q.qn2, (size_t)m) || !c.get(Q.u64, (size_t)m) ||
      !c.get(Q.u32, (size_t)m) || !c.get(Q.invalid, (size_t)m) || !c.get(counters, kNumCounters) ||
      !c.get(fb1, (size_t)m) || !c.get(fb2, (size_t)m))
    return set_error(DD_ERR_TOO_LARGE, "dd_project_noalloc: scratch too small");
  hipLaunchKernelGGL(zero_words_kernel, dim3((kNumCounters + 255) / 256), dim3(256), 0, st, counters,
                     kNumCounters);
  DD_HIP(hipGetLastError());
  DD_TRY(prepare_queries(D, states_dev, false, m, warm_start_idx_dev, 1.0, Q, st));
  const Outputs out{idx_out_dev, dist_out_dev};
  const QueryList all{nullptr, nullptr, m};
  if (mode == DD_EXACT_FP64)
    return exact_from_scratch(D, Q, all, m, out, c, fb2, counters + 1, st);
  if (!c.get(Q.yq, (size_t)m * 12))
    return set_error(DD_ERR_TOO_LARGE, "dd_project_noalloc: scratch too small");
  unsigned long long* walk_stats = reinterpret_cast<unsigned long long*>(counters + 32);
  DD_TRY(launch_ann_walk(D, Q, all, m, warm_start_idx_dev, budget, out, fb1, counters, walk_stats,
                         nullptr, st, mode == DD_KMEANS, 1.0 - discount));
  const QueryList L1{fb1, counters, m};
  return exact_from_scratch(D, Q, L1, m, out, c, fb2, counters + 1, st);
}
