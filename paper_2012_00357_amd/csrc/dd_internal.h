// Internal declarations shared by the libdd translation units (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "pack16.h"

namespace dd {

// ---------------------------------------------------------------------------
// Error handling
// ---------------------------------------------------------------------------
dd_status set_error(dd_status st, const std::string& msg);

#define DD_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::dd::set_error(e_ == hipErrorOutOfMemory ? DD_ERR_OOM : DD_ERR_DEVICE,      \
                             std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define DD_TRY(expr)                  \
  do {                                \
    dd_status s_ = (expr);            \
    if (s_ != DD_OK) return s_;       \
  } while (0)

// Device buffer owned by a host object; released in the destructor.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;   // false: a view into memory another DevBuf owns
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  dd_status alloc(size_t n);
  void view(void* ptr, size_t n) {
    release();
    p = ptr;
    bytes = n;
    owned = false;
  }
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// Small dense linear algebra on the host (6x6 / 12x12)
// ---------------------------------------------------------------------------
// Cholesky C = L L^T (row-major, lower); returns false if not SPD.
bool cholesky6(const double* C, double* L);
// Inverse of a lower-triangular 6x6 matrix (row-major).
void lower_inverse6(const double* L, double* Linv);
// Symmetric eigen-decomposition (cyclic Jacobi); eigenvalues descending,
// eigenvectors as columns of V (row-major n x n).
void sym_eigen(int n, const double* A, double* evals, double* V);

// ---------------------------------------------------------------------------
// Dataset
// ---------------------------------------------------------------------------
constexpr int kDim = 12;           // phase-space dimension 2M (M = 6 Voigt components)
constexpr int kKeyAxes = 6;        // principal axes used for the spatial order
constexpr int kAnnLeaf = 64;       // points per ANN leaf (one wavefront)
constexpr int kAnnFan = 64;        // children per ANN tree node (one wavefront)
constexpr int kCounterSlots = 32;  // ANN walk statistics: slots, each on its own 128-byte line
constexpr int kCounterStride = 16; // u64 per slot (8 used)
constexpr int kKmtRecord = 20;     // floats per k-means tree child record (80 B)

// projection modes that walk a tree (warm starts, budgets, skipping)
inline bool walk_mode(int mode) { return mode == DD_ANN || mode == DD_KMEANS; }
constexpr int kAnnMaxLevels = 6;   // 64^6 leaves exceed any N <= 2^31 - 1

// K^-1 of one mesh and Dirichlet pattern (P_C by a dense product), padded to
// n_pad rows and columns, row-major.
struct DenseInverse {
  int nx = 0, ny = 0, nz = 0;
  double hx = 0, hy = 0, hz = 0;
  std::vector<uint8_t> mask;
  int64_t n = 0, n_pad = 0;
  DevBuf inv;
};
constexpr int64_t kDenseMaxDof = 16384;               // meshes up to here use K^-1
constexpr int64_t kDenseCacheBytes = (int64_t)4 << 30;  // inverses kept per dataset

// Device scratch of the projection, reused from call to call.  A call takes an
// idle arena (or makes one), carves its buffers out of the arena's block and
// hands the arena back when it returns, recording `done` on its stream; the
// next call that takes the arena makes its own stream wait for `done`, so the
// reuse is stream-ordered on any stream.  Requests beyond the block are
// allocated stream-ordered and freed on return, and the block then grows (up
// to kArenaKeepBytes) so that a call of the same size fits next time.
struct ScratchArena {
  void* block = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;   // recorded on the last user's stream
  uint32_t* pinned = nullptr;  // kArenaPinnedWords of pinned host memory (small readbacks)
  ScratchArena() = default;
  ScratchArena(const ScratchArena&) = delete;
  ScratchArena& operator=(const ScratchArena&) = delete;
  ~ScratchArena();
};
constexpr size_t kArenaKeepBytes = (size_t)1 << 30;  // largest block an arena keeps
constexpr int kArenaKeep = 8;                         // idle arenas kept per dataset
constexpr int kArenaPinnedWords = 64;

struct Dataset {
  int device = 0;
  int64_t N = 0;
  uint32_t packs = 0;
  double C[36];
  double F[36];    // strain whitening F = L^T  (F^T F = C)
  double G[36];    // stress whitening G = L^-1 (G^T G = C^-1)
  // spatial order
  DevBuf perm;     // uint32 [N]: sorted position -> original index
  DevBuf iperm;    // uint32 [N]: original index -> sorted position
  // FP64 pack (sorted order), padded to n_pad64 rows
  int64_t n_pad64 = 0;
  DevBuf w64;      // double [n_pad64][12]
  DevBuf n64;      // double [n_pad64]  |x|^2 (padding rows: +inf)
  double xmax = 0; // max_j |x_j|
  // FP32 pack
  int64_t n_pad32 = 0;
  DevBuf w32;      // float [n_pad32][12]
  DevBuf n32;      // float [n_pad32] |x|^2 of the FP32 values (padding: +inf)
  double xmax32 = 0;
  // 16-bit packs (tile-centred), in coordinates scaled by sc16.s (a power of two)
  int tile = 256;
  int64_t n_tiles = 0;
  DevBuf centre;   // float [n_tiles][12] scaled tile centres
  DevBuf radius;   // float [n_tiles]  upper bound of |s x_j - c_T| over the tile
  Scale16 sc16{1.0f, 0.0f, {0}};   // scale and scaled data mean (far set per format)
  double span16 = 0.0;             // max_T |c_T - scaled mean|
  DevBuf wbf16;    // uint16 [n_tiles*tile][16]
  DevBuf wfp16;    // uint16 [n_tiles*tile][16]
  // principal axes of the whitened data (sample estimate): V[12*k + a] is
  // component k of axis a, axes by decreasing variance
  double V[kDim * kDim];
  DevBuf vrot;     // double [144]: V on the device (the walks rotate their queries with it)
  double mean[kDim];
  double lo[kKeyAxes], hi[kKeyAxes];
  // ANN box tree over the sorted order: level 0 boxes bound leaves of kAnnLeaf
  // consecutive points, level k+1 boxes bound kAnnFan boxes of level k; boxes
  // are float lo[12], hi[12] in principal-axis coordinates y = V^T x, rounded
  // outward.  The top stored level has at most kAnnFan boxes.
  DevBuf ann_box[kAnnMaxLevels];
  int64_t ann_n[kAnnMaxLevels] = {0};
  int ann_levels = 0;
  // compact leaves read by the walk, in principal-axis coordinates y = V^T x:
  // per leaf the FP32 centre c (mean of its points), radius r (max |y - c|,
  // rounded up, at least 2^-20) and its box quantised to 8 bits inside its
  // parent's box (rounded outward); per point the FP16 scaled offset (y - c) / r
  // (round to nearest)
  DevBuf ann_meta;   // float [n_leaf][16]: c[12], r, 1/r, 0, 0
  DevBuf ann_q0;     // uint8 [n_leaf][24]: lo[12], hi[12] in 1/255 of the parent box
  DevBuf ann_h16;    // uint16 [n_leaf*64][12]
  // k-means tree (DD_PACK_KMEANS): recursive 4-means, stored as a 64-ary cut,
  // each stored node with up to 64 child records (ball of the child's points:
  // FP32 centre c, radius >= max |x - c|; their box in principal-axis
  // coordinates, quantised to bytes inside the node's own box; code
  // (1 << 28 | node) or leaf); leaves of at most 64 points in padded 64-slot
  // blocks, compact as above
  int64_t kmt_nodes = 0, kmt_leaves = 0, kmt_records = 0;
  int kmt_rounds = 0;
  DevBuf kmt_node;   // int2 [nodes]: first child record, end of its records (node 0: root)
  DevBuf kmt_nbox;   // float [nodes][24]: box lo[12], hi[12] of the node's points (rounded outward)
  DevBuf kmt_child;  // float [records][kKmtRecord]: c[12], r, code (bits), box lo[12], hi[12] as
                     // bytes inside the owner node's box (lo rounded down, hi up)
  DevBuf kmt_meta;   // float [leaves][16]: c[12], r, 1/r, count (bits), 0
  DevBuf kmt_h16;    // uint16 [leaves*64][12]; empty slots +inf
  DevBuf kmt_pos;    // uint32 [leaves*64]: sorted position of each slot (empty: 0xFFFFFFFF)
  DevBuf kmt_slot;   // uint32 [N]: slot of each sorted position

  // inverses of K for dd_solve, most recently used first (see DenseInverse)
  mutable std::mutex cache_mu;
  mutable std::list<std::shared_ptr<DenseInverse>> pc_cache;
  // idle projection scratch arenas (see ScratchArena); arena_bytes counts the
  // blocks of idle and busy arenas
  mutable std::mutex arena_mu;
  mutable std::vector<std::unique_ptr<ScratchArena>> arenas;
  mutable int64_t arena_bytes = 0;

  int64_t device_bytes() const;
};

// Builds the k-means tree of DD_PACK_KMEANS over D's sorted FP64 pack.
dd_status build_kmeans_tree(Dataset& D, hipStream_t st);

}  // namespace dd

struct dd_dataset {
  dd::Dataset d;
};
