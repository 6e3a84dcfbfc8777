// Device sort / scan helpers (stable LSD radix sort of uint32 pairs).
#pragma once
#include "dd_internal.h"

namespace dd {
// Sorts (keys, vals) in place by the low key_bits bits of keys, stably.  Synchronises st.
dd_status radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int key_bits, hipStream_t st);
// In-place exclusive prefix sum of n uint32 values.  Synchronises st.
dd_status exclusive_scan_u32(uint32_t* a, int64_t n, hipStream_t st);
// v[i] = i.
dd_status iota_u32(uint32_t* v, int64_t n, hipStream_t st);
}  // namespace dd
