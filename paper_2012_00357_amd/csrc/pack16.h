// 16-bit element formats of the tile-centred packs and shared scan constants.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dd {

// Rows per LDS tile of the FP64 and FP32 scans (padding granularity of those packs).
constexpr int kTile64 = 256;
constexpr int kTile32 = 256;

// Coordinates of the 16-bit scans: the whitened data, tile centres, radii and
// queries multiplied by a per-dataset power of two s, chosen so that the
// largest tile radius lies in [1, 2).  The scaling is exact (no rounding), so
// the certified bounds hold unchanged in the scaled units, and it keeps |x'|^2
// inside the FP16 range whatever the units of the data (Pa or MPa).  A query
// is scanned only while |s q - mean| < far (else its candidate list stays
// empty and the FP64 fallback answers it): with far = limit - max_T |c_T - mean|
// every centred query coordinate stays below the limit, far below the largest
// finite value of the format.
struct Scale16 {
  float s;          // power of two
  float far;        // <= 0: no query is scanned in this format
  float mean[12];   // scaled mean of the data
};
constexpr float kFarLimitFp16 = 16384.0f;
constexpr float kFarLimitBf16 = 1.0e30f;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4_t;

// bfloat16: round to nearest even from FP32 (finite inputs).
struct Bf16 {
  // unit roundoff of the conversion double -> float -> bf16 (both round to nearest)
  static constexpr float kUnit = 0.00390625f * (1.0f + 3.0517578125e-05f);
  static constexpr float kAbs = 0.0f;          // no subnormal range at our magnitudes
  __host__ __device__ static inline uint16_t from_float(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  }
  __host__ __device__ static inline float to_float(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
  }
};

// IEEE half: round to nearest even from FP32.
struct Fp16 {
  static constexpr float kUnit = 0.00048828125f + 5.9604645e-08f;
  static constexpr float kAbs = 2.9802322e-08f;  // half of the smallest subnormal step
  __host__ __device__ static inline uint16_t from_float(float f) {
    return __builtin_bit_cast(uint16_t, (_Float16)f);
  }
  __host__ __device__ static inline float to_float(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
  }
};

}  // namespace dd
