// GPU twin of the seeded data-point recipe: the same gen_core.h compiled for
// the device, so a point generated here has the same bits as the host
// generator's point with the same (seed, item).  Input generation only.
//
// ddsynth_dev_fill has the producer signature of dd_dataset_create_streamed:
// it writes points first .. first+count-1 into device arrays strain[count][6],
// stress[count][6], stream-ordered on hip_stream; `user` points to a host
// DdsPointParams.
#include <hip/hip_runtime.h>

#include "gen_core.h"

struct DdsPointParams {
  uint64_t seed;
  double eps_amp;
  double S0[36];
  double noise_std;
};

__global__ void dds_points_kernel(DdsPointParams P, int64_t first, int64_t n,
                                  double* __restrict__ strain, double* __restrict__ stress) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double se[6], ss[6];
  dds_point(P.seed, (uint64_t)(first + i), P.eps_amp, P.S0, P.noise_std, se, ss);
  for (int k = 0; k < 6; ++k) {
    strain[6 * i + k] = se[k];
    stress[6 * i + k] = ss[k];
  }
}

extern "C" int ddsynth_dev_fill(void* user, int64_t first, int64_t count, double* strain,
                                double* stress, void* hip_stream) {
  if (!user || count < 0 || first < 0 || (count > 0 && (!strain || !stress))) return 1;
  if (count == 0) return 0;
  const DdsPointParams* P = static_cast<const DdsPointParams*>(user);
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(dds_points_kernel, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), *P, first, count, strain, stress);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int ddsynth_dev_params_bytes(void) { return (int)sizeof(DdsPointParams); }

// The paper's example (nonlinear law, no noise); `user` points to a host
// DdsNonlinearParams.
struct DdsNonlinearParams {
  uint64_t seed;
  double eps_amp;
  double E;
  double alpha;
};

__global__ void dds_points_nonlinear_kernel(DdsNonlinearParams P, int64_t first, int64_t n,
                                            double* __restrict__ strain,
                                            double* __restrict__ stress) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double se[6], ss[6];
  dds_point_nonlinear(P.seed, (uint64_t)(first + i), P.eps_amp, P.E, P.alpha, se, ss);
  for (int k = 0; k < 6; ++k) {
    strain[6 * i + k] = se[k];
    stress[6 * i + k] = ss[k];
  }
}

extern "C" int ddsynth_dev_fill_nonlinear(void* user, int64_t first, int64_t count, double* strain,
                                          double* stress, void* hip_stream) {
  if (!user || count < 0 || first < 0 || (count > 0 && (!strain || !stress))) return 1;
  if (count == 0) return 0;
  const DdsNonlinearParams* P = static_cast<const DdsNonlinearParams*>(user);
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(dds_points_nonlinear_kernel, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), *P, first, count, strain, stress);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}
