// Diagnostic: one wavefront multiplies small host matrices with the matrix
// instructions the scans use, loading operands and storing results with the
// lane layouts the scans assume.  A correct layout reproduces A x B exactly.
#include "pack16.h"
#include "dd_internal.h"

namespace dd {

template <class T16, class Vec>
__global__ void mfma32_probe(const float* A, const float* B, float* D, int use_f16) {
  const int l = threadIdx.x;
  uint16_t a[8], b[8];
  for (int i = 0; i < 8; ++i) {
    a[i] = T16::from_float(A[(l % 32) * 16 + 8 * (l / 32) + i]);
    b[i] = T16::from_float(B[(8 * (l / 32) + i) * 32 + (l % 32)]);
  }
  uint4 pa, pb;
  pa.x = a[0] | ((uint32_t)a[1] << 16); pa.y = a[2] | ((uint32_t)a[3] << 16);
  pa.z = a[4] | ((uint32_t)a[5] << 16); pa.w = a[6] | ((uint32_t)a[7] << 16);
  pb.x = b[0] | ((uint32_t)b[1] << 16); pb.y = b[2] | ((uint32_t)b[3] << 16);
  pb.z = b[4] | ((uint32_t)b[5] << 16); pb.w = b[6] | ((uint32_t)b[7] << 16);
  f32x16_t acc = {};
  if (use_f16)
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, pa),
                                                 __builtin_bit_cast(f16x8_t, pb), acc, 0, 0, 0);
  else
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, pa),
                                                  __builtin_bit_cast(bf16x8_t, pb), acc, 0, 0, 0);
  for (int i = 0; i < 16; ++i) D[(8 * (i / 4) + 4 * (l / 32) + (i % 4)) * 32 + (l % 32)] = acc[i];
}

__global__ void mfma64_probe(const double* A, const double* B, double* D) {
  const int l = threadIdx.x;
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(l % 16) * 4 + l / 16], B[(l / 16) * 16 + (l % 16)],
                                              acc, 0, 0, 0);
  for (int i = 0; i < 4; ++i) D[((l / 16) + 4 * i) * 16 + (l % 16)] = acc[i];
}

// FP32 32x32x2 with an accumulator input in the output layout: C[i][j] = i.
__global__ void mfma32f_probe(const float* A, const float* B, float* D) {
  const int l = threadIdx.x;
  f32x16_t c;
  for (int i = 0; i < 16; ++i) c[i] = (float)(8 * (i / 4) + 4 * (l / 32) + (i % 4));
  f32x16_t acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[(l % 32) * 2 + l / 32],
                                                      B[(l / 32) * 32 + (l % 32)], c, 0, 0, 0);
  for (int i = 0; i < 16; ++i) D[(8 * (i / 4) + 4 * (l / 32) + (i % 4)) * 32 + (l % 32)] = acc[i];
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

// Round 512 FP32 values with the packed conversions the scans use for their
// query operands (v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32) and widen them back.
__global__ void cvt_probe(const float* in, float* out, int use_f16) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    float a = in[2 * i], b = in[2 * i + 1];
    if (use_f16) {
      f16x2_t v = {(_Float16)a, (_Float16)b};
      out[2 * i] = (float)v[0];
      out[2 * i + 1] = (float)v[1];
    } else {
      bf16x2_t v = {(__bf16)a, (__bf16)b};
      out[2 * i] = (float)v[0];
      out[2 * i + 1] = (float)v[1];
    }
  }
}

}  // namespace dd

extern "C" dd_status dd_selftest_mfma(int kind, const double* A, const double* B, double* D) {
  using namespace dd;
  if (!A || !D || kind < 0 || kind > 5 || ((kind < 3 || kind == 5) && !B))
    return set_error(DD_ERR_ARG, "selftest arguments");
  if (kind == 5) {
    float Af[64], Bf[64], Df[1024];
    for (int i = 0; i < 64; ++i) { Af[i] = (float)A[i]; Bf[i] = (float)B[i]; }
    DevBuf a, b, d;
    DD_TRY(a.alloc(sizeof(Af))); DD_TRY(b.alloc(sizeof(Bf))); DD_TRY(d.alloc(sizeof(Df)));
    DD_HIP(hipMemcpy(a.p, Af, sizeof(Af), hipMemcpyHostToDevice));
    DD_HIP(hipMemcpy(b.p, Bf, sizeof(Bf), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(mfma32f_probe, dim3(1), dim3(64), 0, 0, a.as<float>(), b.as<float>(), d.as<float>());
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpy(Df, d.p, sizeof(Df), hipMemcpyDeviceToHost));
    for (int i = 0; i < 1024; ++i) D[i] = Df[i];
    return DD_OK;
  }
  if (kind >= 3) {
    float in[512], outv[512];
    for (int i = 0; i < 512; ++i) in[i] = (float)A[i];
    DevBuf a, d;
    DD_TRY(a.alloc(sizeof(in))); DD_TRY(d.alloc(sizeof(outv)));
    DD_HIP(hipMemcpy(a.p, in, sizeof(in), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(cvt_probe, dim3(1), dim3(256), 0, 0, a.as<float>(), d.as<float>(), kind == 4);
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpy(outv, d.p, sizeof(outv), hipMemcpyDeviceToHost));
    for (int i = 0; i < 512; ++i) D[i] = outv[i];
    return DD_OK;
  }
  if (kind == 2) {
    DevBuf a, b, d;
    DD_TRY(a.alloc(64 * 8)); DD_TRY(b.alloc(64 * 8)); DD_TRY(d.alloc(256 * 8));
    DD_HIP(hipMemcpy(a.p, A, 64 * 8, hipMemcpyHostToDevice));
    DD_HIP(hipMemcpy(b.p, B, 64 * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(mfma64_probe, dim3(1), dim3(64), 0, 0, a.as<double>(), b.as<double>(), d.as<double>());
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemcpy(D, d.p, 256 * 8, hipMemcpyDeviceToHost));
    return DD_OK;
  }
  float Af[32 * 16], Bf[16 * 32], Df[32 * 32];
  for (int i = 0; i < 512; ++i) { Af[i] = (float)A[i]; Bf[i] = (float)B[i]; }
  DevBuf a, b, d;
  DD_TRY(a.alloc(sizeof(Af))); DD_TRY(b.alloc(sizeof(Bf))); DD_TRY(d.alloc(sizeof(Df)));
  DD_HIP(hipMemcpy(a.p, Af, sizeof(Af), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(b.p, Bf, sizeof(Bf), hipMemcpyHostToDevice));
  if (kind == 0)
    hipLaunchKernelGGL((mfma32_probe<Bf16, bf16x8_t>), dim3(1), dim3(64), 0, 0, a.as<float>(), b.as<float>(), d.as<float>(), 0);
  else
    hipLaunchKernelGGL((mfma32_probe<Fp16, f16x8_t>), dim3(1), dim3(64), 0, 0, a.as<float>(), b.as<float>(), d.as<float>(), 1);
  DD_HIP(hipGetLastError());
  DD_HIP(hipMemcpy(Df, d.p, sizeof(Df), hipMemcpyDeviceToHost));
  for (int i = 0; i < 1024; ++i) D[i] = Df[i];
  return DD_OK;
}
