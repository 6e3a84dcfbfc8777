// Stable LSD radix sort of (uint32 key, uint32 value) pairs on the device.
//
// Each pass handles one 8-bit digit: per-block digit histograms (digit-major,
// so that one exclusive scan gives every (digit, block) output offset), then a
// stable scatter in which every block ranks its items in index order using
// wavefront ballots (lanes with equal digits are found by intersecting the
// per-bit ballot masks).  No atomics touch the output order, so the sort is
// deterministic.
#include "dd_internal.h"
#include "sort.h"

namespace dd {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                      // rounds per block
constexpr int kSortChunk = kSortThreads * kSortItems;
constexpr int kWaves = kSortThreads / 64;

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                                  int64_t n, int shift,
                                                                  uint32_t* __restrict__ hist,
                                                                  int64_t n_blocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_blocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan in three levels: per-block scan with block sums, scan of the
// block sums (single block, looping), add-back.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  int t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint32_t a = (t >= off) ? tmp[t - off] : 0u;
    __syncthreads();
    tmp[t] += a;
    __syncthreads();
  }
  uint32_t incl = tmp[t];
  *total = tmp[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(uint32_t* __restrict__ a,
                                                                   int64_t n,
                                                                   uint32_t* __restrict__ sums) {
  __shared__ uint32_t tmp[kScanThreads];
  int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? a[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t off = block_exclusive_scan(s, tmp, &total);
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) a[base + i] = off;
    off += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint32_t* __restrict__ sums,
                                                                 int64_t n) {
  __shared__ uint32_t tmp[kScanThreads];
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += kScanThreads) {
    int64_t i = base + threadIdx.x;
    uint32_t v = (i < n) ? sums[i] : 0u;
    uint32_t total;
    uint32_t off = block_exclusive_scan(v, tmp, &total);
    if (i < n) sums[i] = off + carry;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(uint32_t* __restrict__ a, int64_t n,
                                                                const uint32_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t add = sums[blockIdx.x];
  for (int i = threadIdx.x; i < kScanChunk; i += kScanThreads)
    if (base + i < n) a[base + i] += add;
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, int64_t n, int shift,
    const uint32_t* __restrict__ offsets, int64_t n_blocks, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t run[256];           // running output position per digit
  __shared__ uint32_t wcnt[kWaves][256];  // per-wave digit counts of the current round
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  run[t] = offsets[(int64_t)t * n_blocks + blockIdx.x];
  for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + (int64_t)r * kSortThreads + t;
    bool valid = i < n;
    uint32_t key = valid ? keys_in[i] : 0u;
    uint32_t val = valid ? vals_in[i] : 0u;
    uint32_t dig = (key >> shift) & 0xFFu;
    uint64_t same = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot(valid && ((dig >> b) & 1u));
      same &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(same & lt_mask);
    if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kWaves; ++w) {
      add += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

__global__ void iota_kernel(uint32_t* __restrict__ v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}

dd_status exclusive_scan_u32(uint32_t* a, int64_t n, hipStream_t st) {
  int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  DevBuf sums;
  DD_TRY(sums.alloc(sizeof(uint32_t) * (size_t)(nb > 0 ? nb : 1)));
  hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, n,
                     sums.as<uint32_t>());
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, st, sums.as<uint32_t>(), nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, n,
                     sums.as<uint32_t>());
  DD_HIP(hipGetLastError());
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

dd_status radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits,
                           hipStream_t st) {
  if (n <= 1) return DD_OK;
  if (n > 0xFFFFFFFFll) return set_error(DD_ERR_TOO_LARGE, "radix sort: n exceeds 2^32-1");
  int64_t n_blocks = (n + kSortChunk - 1) / kSortChunk;
  DevBuf k2, v2, hist;
  DD_TRY(k2.alloc(sizeof(uint32_t) * (size_t)n));
  DD_TRY(v2.alloc(sizeof(uint32_t) * (size_t)n));
  DD_TRY(hist.alloc(sizeof(uint32_t) * 256 * (size_t)n_blocks));
  uint32_t *ka = keys, *va = vals, *kb = k2.as<uint32_t>(), *vb = v2.as<uint32_t>();
  int passes = (key_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)n_blocks), dim3(kSortThreads), 0, st, ka,
                       n, shift, hist.as<uint32_t>(), n_blocks);
    DD_HIP(hipGetLastError());
    DD_TRY(exclusive_scan_u32(hist.as<uint32_t>(), 256 * n_blocks, st));
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)n_blocks), dim3(kSortThreads), 0, st,
                       ka, va, n, shift, hist.as<uint32_t>(), n_blocks, kb, vb);
    DD_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    DD_HIP(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
    DD_HIP(hipMemcpyAsync(vals, va, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
  }
  DD_HIP(hipStreamSynchronize(st));
  return DD_OK;
}

dd_status iota_u32(uint32_t* v, int64_t n, hipStream_t st) {
  if (n <= 0) return DD_OK;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, n);
  DD_HIP(hipGetLastError());
  return DD_OK;
}

}  // namespace dd
