// Dataset creation: whitening (Section 3.2), spatial order, FP64 / FP32 /
// tile-centred 16-bit packs and the ANN box tree.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dd_internal.h"
#include "pack16.h"
#include "sort.h"

namespace dd {

struct Mat6x2 {
  double F[36];
  double G[36];
};

// Whitened row w = (F eps, G sig) of point i of a chunk; false if non-finite.
__device__ inline bool whiten_row(const double* __restrict__ strain,
                                  const double* __restrict__ stress, int64_t i, const Mat6x2& M,
                                  double w[12]) {
  double e[6], s[6];
  bool ok = true;
  for (int k = 0; k < 6; ++k) {
    e[k] = strain[6 * i + k];
    s[k] = stress[6 * i + k];
    ok = ok && isfinite(e[k]) && isfinite(s[k]);
  }
  for (int r = 0; r < 6; ++r) {
    double a = 0.0, b = 0.0;
    for (int c = 0; c < 6; ++c) {
      a = fma(M.F[6 * r + c], e[c], a);
      b = fma(M.G[6 * r + c], s[c], b);
    }
    w[r] = a;
    w[6 + r] = b;
  }
  return ok;
}

// Pass 1 over a chunk of rows first .. first+n-1: non-finite flag, max |w|
// (non-negative doubles order like their bit patterns) and the strided sample
// rows {s * stride : s < ns} used for the principal axes.
__global__ __launch_bounds__(256) void stats_kernel(const double* __restrict__ strain,
                                                    const double* __restrict__ stress, int64_t n,
                                                    int64_t first, Mat6x2 M, int64_t stride,
                                                    int64_t ns, double* __restrict__ samp,
                                                    int* __restrict__ bad,
                                                    unsigned long long* __restrict__ maxn) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double w[12];
    if (!whiten_row(strain, stress, i, M, w)) atomicOr(bad, 1);
    double s = 0.0;
    for (int k = 0; k < 12; ++k) s = fma(w[k], w[k], s);
    v = isfinite(s) ? sqrt(s) : 0.0;
    const int64_t g = first + i;
    if (g % stride == 0 && g / stride < ns)
      for (int k = 0; k < 12; ++k) samp[12 * (g / stride) + k] = w[k];
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(maxn, (unsigned long long)__double_as_longlong(red[0]));
}

struct KeyParams {
  double axes[kKeyAxes * kDim];
  double mean[kDim];
  double lo[kKeyAxes];
  double scale[kKeyAxes];
  int bits;
};

// Pass 2: Morton key of the point's cell in the principal-axis grid.
__global__ void key_kernel(const double* __restrict__ strain, const double* __restrict__ stress,
                           int64_t n, int64_t first, Mat6x2 M, KeyParams P,
                           uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[kDim];
  whiten_row(strain, stress, i, M, x);
  for (int k = 0; k < kDim; ++k) x[k] -= P.mean[k];
  const int maxc = (1 << P.bits) - 1;
  uint32_t key = 0;
  int q[kKeyAxes];
  for (int a = 0; a < kKeyAxes; ++a) {
    double p = 0.0;
    for (int k = 0; k < kDim; ++k) p = fma(P.axes[kDim * a + k], x[k], p);
    double c = floor((p - P.lo[a]) * P.scale[a]);
    q[a] = c < 0.0 ? 0 : (c > (double)maxc ? maxc : (int)c);
  }
  for (int b = 0; b < P.bits; ++b)
    for (int a = 0; a < kKeyAxes; ++a) key |= (uint32_t)((q[a] >> b) & 1) << (b * kKeyAxes + a);
  keys[first + i] = key;
}

__global__ void invert_perm_kernel(const uint32_t* __restrict__ perm, int64_t n,
                                   uint32_t* __restrict__ iperm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) iperm[perm[i]] = (uint32_t)i;
}

// Pass 3: each point's whitened row goes to its sorted position: the FP64 pack
// with |x|^2, and the FP32 pack (round to nearest) with the FP32-rounded
// squared norm of the stored values.
__global__ void scatter_kernel(const double* __restrict__ strain, const double* __restrict__ stress,
                               int64_t n, int64_t first, Mat6x2 M,
                               const uint32_t* __restrict__ iperm, double* __restrict__ w64,
                               double* __restrict__ n64, float* __restrict__ w32,
                               float* __restrict__ n32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double w[12];
  whiten_row(strain, stress, i, M, w);
  const int64_t p = iperm[first + i];
  if (w64) {
    double s = 0.0;
    for (int k = 0; k < 12; ++k) {
      w64[12 * p + k] = w[k];
      s = fma(w[k], w[k], s);
    }
    n64[p] = s;
  }
  if (w32) {
    double s = 0.0;
    for (int k = 0; k < 12; ++k) {
      const float v = (float)w[k];
      w32[12 * p + k] = v;
      s = fma((double)v, (double)v, s);
    }
    n32[p] = (float)s;
  }
}

// Padding rows [N, n_pad): zero with norm +inf (never a candidate).
template <class T>
__global__ void pad_kernel(int64_t N, int64_t n_pad, T* __restrict__ w, T* __restrict__ nrm) {
  const int64_t i = N + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  for (int k = 0; k < 12; ++k) w[12 * i + k] = T(0);
  nrm[i] = T(INFINITY);
}

// Per tile of the sorted FP64 pack: centre = mean of its points (rounded to
// FP32), radius = max distance of its points to that FP32 centre, rounded up.
// One block of 256 per tile.
__global__ __launch_bounds__(256) void tile_stats_kernel(const double* __restrict__ w, int64_t n,
                                                         int tile, float* __restrict__ centre,
                                                         float* __restrict__ radius) {
  __shared__ double red[256];
  __shared__ float cen[12];
  int64_t t = blockIdx.x;
  int64_t first = t * tile;
  int64_t last = min(first + (int64_t)tile, n);
  int cnt = (int)(last - first);
  for (int k = 0; k < 12; ++k) {
    double s = 0.0;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) s += w[12 * i + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) cen[k] = (float)(red[0] / (double)cnt);
    __syncthreads();
  }
  double r = 0.0;
  for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
    const double* x = w + 12 * i;
    double s = 0.0;
    for (int k = 0; k < 12; ++k) {
      double d = x[k] - (double)cen[k];
      s = fma(d, d, s);
    }
    r = fmax(r, sqrt(s));
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 12; ++k) centre[12 * t + k] = cen[k];
    // round up with a relative margin far above the rounding of the sums above
    radius[t] = __double2float_ru(red[0] * (1.0 + 1e-12) + 1e-30);
  }
}

// Tile centres and radii to the scaled coordinates of the 16-bit scans.  The
// scale is a power of two, so the products are exact for normal values; the
// radius keeps its absolute floor so that it still bounds the scaled offsets
// where they fall into the subnormal range.
__global__ void scale_tiles_kernel(int64_t n_tiles, float scale, float* __restrict__ centre,
                                   float* __restrict__ radius) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  for (int k = 0; k < 12; ++k) centre[12 * t + k] *= scale;
  radius[t] = radius[t] * scale + 1e-30f;
}

// 16-bit tile-centred pack: row j of tile T holds
//   (-2 x'_0 .. -2 x'_11, n_hi, n_mid, n_lo, 0),  x' = round16(s x_j - c_T),
//   n = |x'|^2 (exact in FP64) split into three 16-bit terms,
// with s the dataset's power-of-two scale and c_T the scaled tile centre.
// Padding rows (the tail of the last tile) repeat the last point, so that every
// score a scan forms is the distance to a real point; the extraction and the
// merge never report a row >= N.
template <class T16>
__global__ void pack16_kernel(const double* __restrict__ w, int64_t n, int64_t n_rows, int tile,
                              double scale, const float* __restrict__ centre,
                              uint16_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  uint16_t row[16];
  {
    const double* x = w + 12 * (i < n ? i : n - 1);   // row n - 1 lies in the last tile too
    const float* c = centre + 12 * (i / tile);
    double nn = 0.0;
    for (int k = 0; k < 12; ++k) {
      float xf = (float)(x[k] * scale - (double)c[k]);
      uint16_t b = T16::from_float(xf);
      double v = (double)T16::to_float(b);
      nn = fma(v, v, nn);
      row[k] = T16::from_float(-2.0f * T16::to_float(b));   // exact scaling by -2
    }
    uint16_t hi = T16::from_float((float)nn);
    double r1 = nn - (double)T16::to_float(hi);
    uint16_t mid = T16::from_float((float)r1);
    double r2 = r1 - (double)T16::to_float(mid);
    uint16_t lo = T16::from_float((float)r2);
    row[12] = hi;
    row[13] = mid;
    row[14] = lo;
    row[15] = 0;
  }
  uint4 a, b;
  a.x = row[0] | ((uint32_t)row[1] << 16);
  a.y = row[2] | ((uint32_t)row[3] << 16);
  a.z = row[4] | ((uint32_t)row[5] << 16);
  a.w = row[6] | ((uint32_t)row[7] << 16);
  b.x = row[8] | ((uint32_t)row[9] << 16);
  b.y = row[10] | ((uint32_t)row[11] << 16);
  b.z = row[12] | ((uint32_t)row[13] << 16);
  b.w = row[14] | ((uint32_t)row[15] << 16);
  uint4* o = reinterpret_cast<uint4*>(out + 16 * i);
  o[0] = a;
  o[1] = b;
}

// ---------------------------------------------------------------------------
// ANN box tree.  A box bounds its points in principal-axis coordinates y = V^T x
// (a rotation, so box distances are lower bounds of whitened distances); the
// FP64 coordinates are rounded outward to FP32.
// ---------------------------------------------------------------------------
struct Rot12 {
  double V[144];
};

__device__ inline double wave_min_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ inline double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// One wavefront per leaf of kAnnLeaf consecutive sorted points.
__global__ __launch_bounds__(256) void ann_leaf_box_kernel(const double* __restrict__ w64, int64_t N,
                                                           Rot12 R, int64_t n_leaf,
                                                           float* __restrict__ box) {
  const int lane = threadIdx.x & 63;
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (leaf >= n_leaf) return;
  const int64_t i = leaf * kAnnLeaf + lane;
  const bool v = i < N;
  double x[12];
  for (int k = 0; k < 12; ++k) x[k] = v ? w64[12 * i + k] : 0.0;
  float* b = box + 24 * leaf;
  for (int a = 0; a < 12; ++a) {
    double y = 0.0;
    for (int k = 0; k < 12; ++k) y = fma(R.V[12 * k + a], x[k], y);
    const double lo = wave_min_d(v ? y : INFINITY);
    const double hi = wave_max_d(v ? y : -INFINITY);
    if (lane == 0) {
      b[a] = __double2float_rd(lo);
      b[12 + a] = __double2float_ru(hi);
    }
  }
}

// One wavefront per node: the box of its (up to) kAnnFan child boxes.
__global__ __launch_bounds__(256) void ann_node_box_kernel(const float* __restrict__ child,
                                                           int64_t n_child, int64_t n_node,
                                                           float* __restrict__ box) {
  const int lane = threadIdx.x & 63;
  const int64_t node = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (node >= n_node) return;
  const int64_t c = node * kAnnFan + lane;
  const bool v = c < n_child;
  for (int a = 0; a < 12; ++a) {
    double lo = v ? (double)child[24 * c + a] : INFINITY;
    double hi = v ? (double)child[24 * c + 12 + a] : -INFINITY;
    lo = wave_min_d(lo);
    hi = wave_max_d(hi);
    if (lane == 0) {
      box[24 * node + a] = (float)lo;
      box[24 * node + 12 + a] = (float)hi;
    }
  }
}

// Compact leaf of the walk (one wavefront per leaf): centre, radius and the
// scaled FP16 offsets of its points, in principal-axis coordinates.
__global__ __launch_bounds__(256) void ann_leaf_pack_kernel(const double* __restrict__ w64,
                                                            int64_t N, Rot12 R, int64_t n_leaf,
                                                            float* __restrict__ meta,
                                                            _Float16* __restrict__ h16) {
  const int lane = threadIdx.x & 63;
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (leaf >= n_leaf) return;
  const int64_t i = leaf * kAnnLeaf + lane;
  const bool v = i < N;
  int cnt = __popcll(__ballot(v));
  // the point in principal-axis coordinates y = V^T x (the boxes' frame)
  double x[12];
  {
    double w[12];
    for (int k = 0; k < 12; ++k) w[k] = v ? w64[12 * i + k] : 0.0;
    for (int a = 0; a < 12; ++a) {
      double y = 0.0;
      for (int k = 0; k < 12; ++k) y = fma(R.V[12 * k + a], w[k], y);
      x[a] = y;
    }
  }
  float c[12];
  for (int k = 0; k < 12; ++k) {
    double sum = x[k];
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    sum = __shfl(sum, 0);   // one value for every lane (the butterfly order differs per lane)
    c[k] = (float)(sum / (double)cnt);
  }
  double d2 = 0.0;
  for (int k = 0; k < 12; ++k) {
    const double t = x[k] - (double)c[k];
    d2 = fma(t, t, d2);
  }
  double r = v ? sqrt(d2) : 0.0;
  r = wave_max_d(r);
  float rf = __double2float_ru(r * (1.0 + 1e-12));
  rf = fmaxf(rf, 9.5367431640625e-07f);   // 2^-20: bounded scaled offsets for tiny leaves
  const double inv = 1.0 / (double)rf;
  for (int k = 0; k < 12; ++k)
    h16[12 * i + k] = v ? (_Float16)((x[k] - (double)c[k]) * inv) : (_Float16)0.0f;
  if (lane == 0) {
    float* m = meta + 16 * leaf;
    for (int k = 0; k < 12; ++k) m[k] = c[k];
    m[12] = rf;
    m[13] = (float)inv;
    m[14] = 0.0f;
    m[15] = 0.0f;
  }
}

// Leaf boxes quantised inside their level-1 parent box: lo rounded down, hi up.
__global__ void ann_qbox_kernel(const float* __restrict__ box0, const float* __restrict__ box1,
                                int64_t n_leaf, uint8_t* __restrict__ q0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_leaf) return;
  const float* b = box0 + 24 * t;
  const float* p = box1 + 24 * (t / kAnnFan);
  for (int a = 0; a < 12; ++a) {
    const double plo = p[a], ext = (double)p[12 + a] - plo;
    int ql = 0, qh = 255;
    if (ext > 0.0) {
      ql = (int)floor(((double)b[a] - plo) / ext * 255.0);
      qh = (int)ceil(((double)b[12 + a] - plo) / ext * 255.0);
      ql = ql < 0 ? 0 : (ql > 255 ? 255 : ql);
      qh = qh < 0 ? 0 : (qh > 255 ? 255 : qh);
    }
    q0[24 * t + a] = (uint8_t)ql;
    q0[24 * t + 12 + a] = (uint8_t)qh;
  }
}

static unsigned grid_for(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// Chunked access to the caller's raw (strain, stress) rows.  Creation reads
// every row three times (statistics, keys, packs), a chunk at a time.
struct Source {
  int64_t chunk = 0;
  virtual ~Source() = default;
  // device pointers to rows first .. first+n-1 (n <= chunk), valid on st until
  // the next call
  virtual dd_status rows(int64_t first, int64_t n, const double** e, const double** s,
                         hipStream_t st) = 0;
};

struct MemSource : Source {
  const double* e;
  const double* s;
  MemSource(const double* e_, const double* s_, int64_t N) : e(e_), s(s_) { chunk = N; }
  dd_status rows(int64_t first, int64_t, const double** eo, const double** so, hipStream_t) override {
    *eo = e + 6 * first;
    *so = s + 6 * first;
    return DD_OK;
  }
};

// Host arrays, copied to the device chunk by chunk (each copy is ordered on the
// stream after the kernels that read the previous chunk).
struct HostSource : Source {
  const double* e;
  const double* s;
  DevBuf be, bs;
  HostSource(const double* e_, const double* s_, int64_t N) : e(e_), s(s_) {
    chunk = std::min<int64_t>(N, (int64_t)1 << 24);
  }
  dd_status init() {
    DD_TRY(be.alloc(sizeof(double) * 6 * (size_t)chunk));
    DD_TRY(bs.alloc(sizeof(double) * 6 * (size_t)chunk));
    return DD_OK;
  }
  dd_status rows(int64_t first, int64_t n, const double** eo, const double** so,
                 hipStream_t st) override {
    DD_HIP(hipMemcpyAsync(be.p, e + 6 * first, sizeof(double) * 6 * (size_t)n,
                          hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(bs.p, s + 6 * first, sizeof(double) * 6 * (size_t)n,
                          hipMemcpyHostToDevice, st));
    *eo = be.as<double>();
    *so = bs.as<double>();
    return DD_OK;
  }
};

struct FillSource : Source {
  dd_fill_fn fn;
  void* user;
  DevBuf be, bs;
  FillSource(dd_fill_fn f, void* u, int64_t N) : fn(f), user(u) {
    chunk = std::min<int64_t>(N, (int64_t)1 << 24);
  }
  dd_status init() {
    DD_TRY(be.alloc(sizeof(double) * 6 * (size_t)chunk));
    DD_TRY(bs.alloc(sizeof(double) * 6 * (size_t)chunk));
    return DD_OK;
  }
  dd_status rows(int64_t first, int64_t n, const double** eo, const double** so,
                 hipStream_t st) override {
    const int rc = fn(user, first, n, be.as<double>(), bs.as<double>(), st);
    if (rc != 0)
      return set_error(DD_ERR_ARG, "data producer returned " + std::to_string(rc) + " for rows " +
                                       std::to_string(first) + ".." + std::to_string(first + n - 1));
    DD_HIP(hipGetLastError());
    *eo = be.as<double>();
    *so = bs.as<double>();
    return DD_OK;
  }
};

// Scale of the 16-bit scans (see Scale16): the power of two s that brings the
// largest tile radius into [1, 2), bounded so that the scaled centres stay far
// inside the FP32 range; then the scaled mean of the data and, per format, the
// query radius around it inside which the centred query coordinates cannot
// overflow.  Scales the tile centres and radii in place.
static dd_status choose_scale16(Dataset& D, hipStream_t st) {
  std::vector<float> cen(12 * (size_t)D.n_tiles), rad((size_t)D.n_tiles);
  DD_HIP(hipMemcpyAsync(cen.data(), D.centre.p, sizeof(float) * cen.size(), hipMemcpyDeviceToHost, st));
  DD_HIP(hipMemcpyAsync(rad.data(), D.radius.p, sizeof(float) * rad.size(), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  double rmax = 0.0, cmax = 0.0;
  for (float r : rad) rmax = std::max(rmax, (double)r);
  for (float c : cen) cmax = std::max(cmax, std::fabs((double)c));
  int k = -(int)std::floor(std::log2(std::max(rmax, 1e-300)));
  k = std::max(-100, std::min(k, 100));
  while (k > -100 && std::ldexp(std::max(cmax, rmax), k) > 0x1p100) --k;
  const double s = std::ldexp(1.0, k);
  D.sc16.s = (float)s;
  double span = 0.0;
  for (int k2 = 0; k2 < 12; ++k2) D.sc16.mean[k2] = (float)(D.mean[k2] * s);
  for (int64_t t = 0; t < D.n_tiles; ++t) {
    double a = 0.0;
    for (int k2 = 0; k2 < 12; ++k2) {
      const double d = (double)cen[12 * t + k2] * s - (double)D.sc16.mean[k2];
      a += d * d;
    }
    span = std::max(span, std::sqrt(a));
  }
  D.span16 = span * (1.0 + 1e-6);
  hipLaunchKernelGGL(scale_tiles_kernel, dim3(grid_for(D.n_tiles)), dim3(256), 0, st, D.n_tiles,
                     (float)s, D.centre.as<float>(), D.radius.as<float>());
  DD_HIP(hipGetLastError());
  return DD_OK;
}

static dd_status create_impl(Source& src, int64_t N, const double* C, const dd_dataset_opts* opts,
                             hipStream_t st, Dataset& D) {
  uint32_t packs = (opts && opts->packs) ? opts->packs : DD_PACK_DEFAULT;
  int tile = (opts && opts->tile) ? opts->tile : 2048;
  if (tile != 128 && tile != 256 && tile != 512 && tile != 1024 && tile != 2048)
    return set_error(DD_ERR_ARG, "tile must be 128, 256, 512, 1024 or 2048");
  if (opts && (opts->flags & ~DD_DATASET_HOST_INPUT))
    return set_error(DD_ERR_ARG, "dd_dataset_opts.flags: unknown bits");
  if (packs & ~(DD_PACK_FP64 | DD_PACK_FP32 | DD_PACK_BF16 | DD_PACK_FP16 | DD_PACK_ANN |
                DD_PACK_KMEANS))
    return set_error(DD_ERR_ARG, "unknown pack bits");
  // every dataset holds the FP64 pack: the trees and the 16-bit packs are built
  // from it, and the FP64 rerank, the fallback scans and dd_solve read it
  packs |= DD_PACK_FP64;
  D.N = N;
  D.packs = packs;
  D.tile = tile;
  DD_HIP(hipGetDevice(&D.device));

  // metric: symmetric positive definite, whitening factors from its Cholesky factor
  double cnorm = 0.0, asym = 0.0;
  for (int i = 0; i < 36; ++i) {
    if (!std::isfinite(C[i])) return set_error(DD_ERR_ARG, "metric C has a non-finite entry");
    cnorm = std::max(cnorm, std::fabs(C[i]));
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) asym = std::max(asym, std::fabs(C[6 * i + j] - C[6 * j + i]));
  if (asym > 1e-12 * cnorm) return set_error(DD_ERR_NOT_SPD, "metric C is not symmetric");
  double L[36], Li[36];
  if (!cholesky6(C, L)) return set_error(DD_ERR_NOT_SPD, "metric C is not positive definite");
  lower_inverse6(L, Li);
  std::memcpy(D.C, C, sizeof(D.C));
  Mat6x2 M;
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      M.F[6 * r + c] = L[6 * c + r];  // F = L^T
      M.G[6 * r + c] = Li[6 * r + c]; // G = L^-1
    }
  std::memcpy(D.F, M.F, sizeof(D.F));
  std::memcpy(D.G, M.G, sizeof(D.G));
  const int64_t CH = src.chunk;

  // 1. statistics pass: finiteness, max |x|, strided sample of whitened rows
  const int64_t ns = std::min<int64_t>(N, 65536);
  const int64_t stride = std::max<int64_t>(1, N / ns);
  DevBuf dsamp, flag, mx;
  DD_TRY(dsamp.alloc(sizeof(double) * 12 * (size_t)ns));
  DD_TRY(flag.alloc(sizeof(int)));
  DD_TRY(mx.alloc(sizeof(unsigned long long)));
  DD_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  DD_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned long long), st));
  for (int64_t f = 0; f < N; f += CH) {
    const int64_t n = std::min(CH, N - f);
    const double *e, *s;
    DD_TRY(src.rows(f, n, &e, &s, st));
    hipLaunchKernelGGL(stats_kernel, dim3(grid_for(n)), dim3(256), 0, st, e, s, n, f, M, stride, ns,
                       dsamp.as<double>(), flag.as<int>(), mx.as<unsigned long long>());
    DD_HIP(hipGetLastError());
  }
  int bad = 0;
  unsigned long long bitsx = 0;
  DD_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  DD_HIP(hipMemcpyAsync(&bitsx, mx.p, sizeof(bitsx), hipMemcpyDeviceToHost, st));
  std::vector<double> samp(12 * (size_t)ns);
  DD_HIP(hipMemcpyAsync(samp.data(), dsamp.p, sizeof(double) * samp.size(), hipMemcpyDeviceToHost, st));
  DD_HIP(hipStreamSynchronize(st));
  if (bad) return set_error(DD_ERR_ARG, "data set contains non-finite strain or stress values");
  std::memcpy(&D.xmax, &bitsx, sizeof(D.xmax));

  // 2. principal axes of the sample (host, 12x12 eigenproblem)
  KeyParams P;
  {
    double mean[12] = {0};
    for (int64_t s = 0; s < ns; ++s)
      for (int k = 0; k < 12; ++k) mean[k] += samp[12 * s + k];
    for (int k = 0; k < 12; ++k) mean[k] /= (double)ns;
    double cov[144] = {0};
    for (int64_t s = 0; s < ns; ++s)
      for (int a = 0; a < 12; ++a)
        for (int b = 0; b < 12; ++b)
          cov[12 * a + b] += (samp[12 * s + a] - mean[a]) * (samp[12 * s + b] - mean[b]);
    double ev[12];
    sym_eigen(12, cov, ev, D.V);
    DD_TRY(D.vrot.alloc(sizeof(D.V)));
    DD_HIP(hipMemcpyAsync(D.vrot.p, D.V, sizeof(D.V), hipMemcpyHostToDevice, st));
    for (int a = 0; a < kKeyAxes; ++a)
      for (int k = 0; k < 12; ++k) P.axes[kDim * a + k] = D.V[12 * k + a];
    for (int k = 0; k < 12; ++k) P.mean[k] = mean[k];
    for (int a = 0; a < kKeyAxes; ++a) {
      double lo = INFINITY, hi = -INFINITY;
      for (int64_t s = 0; s < ns; ++s) {
        double p = 0.0;
        for (int k = 0; k < 12; ++k) p += P.axes[kDim * a + k] * (samp[12 * s + k] - mean[k]);
        lo = std::min(lo, p);
        hi = std::max(hi, p);
      }
      double span = std::max(hi - lo, 1e-300);
      lo -= 0.01 * span;
      hi += 0.01 * span;
      P.lo[a] = lo;
      P.scale[a] = 1.0 / (hi - lo);
      D.lo[a] = lo;
      D.hi[a] = hi;
    }
    std::memcpy(D.mean, P.mean, sizeof(D.mean));
  }
  // cell resolution: 2^bits cells per axis, 6 axes -> 6*bits key bits
  const int bits = 5;
  P.bits = bits;
  for (int a = 0; a < kKeyAxes; ++a) P.scale[a] *= (double)(1 << bits);
  dsamp.release();

  // 3. keys pass, stable sort -> permutation and its inverse
  {
    DevBuf keys;
    DD_TRY(keys.alloc(sizeof(uint32_t) * (size_t)N));
    DD_TRY(D.perm.alloc(sizeof(uint32_t) * (size_t)N));
    for (int64_t f = 0; f < N; f += CH) {
      const int64_t n = std::min(CH, N - f);
      const double *e, *s;
      DD_TRY(src.rows(f, n, &e, &s, st));
      hipLaunchKernelGGL(key_kernel, dim3(grid_for(n)), dim3(256), 0, st, e, s, n, f, M, P,
                         keys.as<uint32_t>());
      DD_HIP(hipGetLastError());
    }
    DD_TRY(iota_u32(D.perm.as<uint32_t>(), N, st));
    DD_TRY(radix_sort_pairs(keys.as<uint32_t>(), D.perm.as<uint32_t>(), N, kKeyAxes * bits, st));
  }
  DD_TRY(D.iperm.alloc(sizeof(uint32_t) * (size_t)N));
  hipLaunchKernelGGL(invert_perm_kernel, dim3(grid_for(N)), dim3(256), 0, st,
                     D.perm.as<uint32_t>(), N, D.iperm.as<uint32_t>());
  DD_HIP(hipGetLastError());

  // 4. packs pass: rows scattered to their sorted positions
  if (packs & DD_PACK_FP64) {
    D.n_pad64 = (N + kTile64 - 1) / kTile64 * kTile64;
    DD_TRY(D.w64.alloc(sizeof(double) * 12 * (size_t)D.n_pad64));
    DD_TRY(D.n64.alloc(sizeof(double) * (size_t)D.n_pad64));
  }
  if (packs & DD_PACK_FP32) {
    D.n_pad32 = (N + kTile32 - 1) / kTile32 * kTile32;
    DD_TRY(D.w32.alloc(sizeof(float) * 12 * (size_t)D.n_pad32));
    DD_TRY(D.n32.alloc(sizeof(float) * (size_t)D.n_pad32));
    D.xmax32 = D.xmax * (1.0 + 1e-6);
  }
  for (int64_t f = 0; f < N; f += CH) {
    const int64_t n = std::min(CH, N - f);
    const double *e, *s;
    DD_TRY(src.rows(f, n, &e, &s, st));
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(n)), dim3(256), 0, st, e, s, n, f, M,
                       D.iperm.as<uint32_t>(), D.w64.as<double>(), D.n64.as<double>(),
                       D.w32.as<float>(), D.n32.as<float>());
    DD_HIP(hipGetLastError());
  }
  if (D.n_pad64 > N) {
    hipLaunchKernelGGL(pad_kernel<double>, dim3(grid_for(D.n_pad64 - N)), dim3(256), 0, st, N,
                       D.n_pad64, D.w64.as<double>(), D.n64.as<double>());
    DD_HIP(hipGetLastError());
  }
  if (D.n_pad32 > N) {
    hipLaunchKernelGGL(pad_kernel<float>, dim3(grid_for(D.n_pad32 - N)), dim3(256), 0, st, N,
                       D.n_pad32, D.w32.as<float>(), D.n32.as<float>());
    DD_HIP(hipGetLastError());
  }

  // 5. tile-centred 16-bit packs, from the sorted FP64 pack
  if (packs & (DD_PACK_BF16 | DD_PACK_FP16)) {
    D.n_tiles = (N + tile - 1) / tile;
    int64_t rows = D.n_tiles * tile;
    DD_TRY(D.centre.alloc(sizeof(float) * 12 * (size_t)D.n_tiles));
    DD_TRY(D.radius.alloc(sizeof(float) * (size_t)D.n_tiles));
    hipLaunchKernelGGL(tile_stats_kernel, dim3((unsigned)D.n_tiles), dim3(256), 0, st,
                       D.w64.as<double>(), N, tile, D.centre.as<float>(), D.radius.as<float>());
    DD_HIP(hipGetLastError());
    DD_TRY(choose_scale16(D, st));
    if (packs & DD_PACK_BF16) {
      DD_TRY(D.wbf16.alloc(sizeof(uint16_t) * 16 * (size_t)rows));
      hipLaunchKernelGGL(pack16_kernel<Bf16>, dim3(grid_for(rows)), dim3(256), 0, st,
                         D.w64.as<double>(), N, rows, tile, (double)D.sc16.s, D.centre.as<float>(),
                         D.wbf16.as<uint16_t>());
      DD_HIP(hipGetLastError());
    }
    if (packs & DD_PACK_FP16) {
      DD_TRY(D.wfp16.alloc(sizeof(uint16_t) * 16 * (size_t)rows));
      hipLaunchKernelGGL(pack16_kernel<Fp16>, dim3(grid_for(rows)), dim3(256), 0, st,
                         D.w64.as<double>(), N, rows, tile, (double)D.sc16.s, D.centre.as<float>(),
                         D.wfp16.as<uint16_t>());
      DD_HIP(hipGetLastError());
    }
  }

  // 6. ANN box tree over the sorted order
  if (packs & DD_PACK_ANN) {
    Rot12 R;
    std::memcpy(R.V, D.V, sizeof(R.V));
    int64_t n = (N + kAnnLeaf - 1) / kAnnLeaf;
    int l = 0;
    DD_TRY(D.ann_box[0].alloc(sizeof(float) * 24 * (size_t)n));
    D.ann_n[0] = n;
    hipLaunchKernelGGL(ann_leaf_box_kernel, dim3(grid_for(n, 4)), dim3(256), 0, st,
                       D.w64.as<double>(), N, R, n, D.ann_box[0].as<float>());
    DD_HIP(hipGetLastError());
    while (n > kAnnFan) {
      const int64_t m = (n + kAnnFan - 1) / kAnnFan;
      if (l + 1 >= kAnnMaxLevels) return set_error(DD_ERR_TOO_LARGE, "ANN tree too deep");
      DD_TRY(D.ann_box[l + 1].alloc(sizeof(float) * 24 * (size_t)m));
      hipLaunchKernelGGL(ann_node_box_kernel, dim3(grid_for(m, 4)), dim3(256), 0, st,
                         D.ann_box[l].as<float>(), n, m, D.ann_box[l + 1].as<float>());
      DD_HIP(hipGetLastError());
      ++l;
      D.ann_n[l] = m;
      n = m;
    }
    D.ann_levels = l + 1;
    const int64_t nl = D.ann_n[0];
    DD_TRY(D.ann_meta.alloc(sizeof(float) * 16 * (size_t)nl));
    DD_TRY(D.ann_h16.alloc(sizeof(uint16_t) * 12 * (size_t)(nl * kAnnLeaf)));
    hipLaunchKernelGGL(ann_leaf_pack_kernel, dim3(grid_for(nl, 4)), dim3(256), 0, st,
                       D.w64.as<double>(), N, R, nl, D.ann_meta.as<float>(),
                       D.ann_h16.as<_Float16>());
    DD_HIP(hipGetLastError());
    if (D.ann_levels >= 2) {
      DD_TRY(D.ann_q0.alloc(24 * (size_t)nl));
      hipLaunchKernelGGL(ann_qbox_kernel, dim3(grid_for(nl)), dim3(256), 0, st,
                         D.ann_box[0].as<float>(), D.ann_box[1].as<float>(), nl,
                         D.ann_q0.as<uint8_t>());
      DD_HIP(hipGetLastError());
      // the walk reads leaf boxes only in quantised form from here on
      DD_HIP(hipStreamSynchronize(st));
      D.ann_box[0].release();
    }
  }

  // 7. k-means tree over the sorted order
  if (packs & DD_PACK_KMEANS) DD_TRY(build_kmeans_tree(D, st));
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

}  // namespace dd

static dd_status finish_create(dd::Source& src, int64_t N, const double* C,
                               const dd_dataset_opts* opts, void* hip_stream, dd_dataset** out) {
  dd_dataset* ds = new (std::nothrow) dd_dataset();
  if (!ds) return dd::set_error(DD_ERR_OOM, "host allocation failed");
  dd_status st = dd::create_impl(src, N, C, opts, static_cast<hipStream_t>(hip_stream), ds->d);
  if (st != DD_OK) {
    delete ds;
    return st;
  }
  *out = ds;
  return DD_OK;
}

extern "C" dd_status dd_dataset_create(const double* strain, const double* stress, int64_t N,
                                       const double* C, const dd_dataset_opts* opts,
                                       void* hip_stream, dd_dataset** out) {
  if (!out) return dd::set_error(DD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!strain || !stress || !C) return dd::set_error(DD_ERR_ARG, "NULL input pointer");
  if (N < 1 || N > 0x7FFFFFFFll) return dd::set_error(DD_ERR_ARG, "N must be in [1, 2^31-1]");
  if (opts && (opts->flags & DD_DATASET_HOST_INPUT)) {
    dd::HostSource src(strain, stress, N);
    dd_status s = src.init();
    if (s != DD_OK) return s;
    return finish_create(src, N, C, opts, hip_stream, out);
  }
  dd::MemSource src(strain, stress, N);
  return finish_create(src, N, C, opts, hip_stream, out);
}

extern "C" dd_status dd_dataset_create_streamed(int64_t N, const double* C, dd_fill_fn fill,
                                                void* user, const dd_dataset_opts* opts,
                                                void* hip_stream, dd_dataset** out) {
  if (!out) return dd::set_error(DD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!fill || !C) return dd::set_error(DD_ERR_ARG, "NULL producer or metric");
  if (N < 1 || N > 0x7FFFFFFFll) return dd::set_error(DD_ERR_ARG, "N must be in [1, 2^31-1]");
  dd::FillSource src(fill, user, N);
  dd_status s = src.init();
  if (s != DD_OK) return s;
  return finish_create(src, N, C, opts, hip_stream, out);
}

extern "C" dd_status dd_dataset_destroy(dd_dataset* ds) {
  delete ds;
  return DD_OK;
}

extern "C" dd_status dd_dataset_info(const dd_dataset* ds, int64_t* n_points, int64_t* device_bytes) {
  if (!ds) return dd::set_error(DD_ERR_ARG, "dataset is NULL");
  if (n_points) *n_points = ds->d.N;
  if (device_bytes) *device_bytes = ds->d.device_bytes();
  return DD_OK;
}

extern "C" dd_status dd_dataset_index_info(const dd_dataset* ds, dd_index_info* info) {
  if (!ds || !info) return dd::set_error(DD_ERR_ARG, "dataset or info is NULL");
  const dd::Dataset& D = ds->d;
  info->ann_levels = D.ann_levels;
  info->kmeans_levels = D.kmt_rounds;
  info->ann_leaves = D.ann_levels > 0 ? D.ann_n[0] : 0;
  info->kmeans_nodes = D.kmt_nodes;
  info->kmeans_leaves = D.kmt_leaves;
  info->kmeans_records = D.kmt_records;
  return DD_OK;
}
