/*
 * Seeded synthetic inputs for the data-driven (DD) projection workloads.
 *
 * This file holds input generation only: a counter-based random number
 * generator and the recipes that turn its output into material data points,
 * query states and random initial assignments.  It contains none of the DD
 * method's arithmetic (no metric, no projection, no finite elements); both the
 * CPU oracle and the GPU library consume the arrays it writes.
 *
 * The generator (Philox4x32-10), the uniform and Gaussian transforms and the
 * data-point recipe live in gen_core.h, shared with the GPU generator
 * (gen_dev.hip) so that both write the same bits for the same item.
 */
#include "gen_core.h"

/* Raw block: out[4] for (item, stream) under seed. */
void ddsynth_philox(uint64_t seed, uint64_t item, uint32_t stream, uint32_t out[4]) {
  dds_block(seed, item, stream, out);
}

void ddsynth_philox_many(uint64_t seed, uint32_t stream, const uint64_t* items,
                         int64_t n, uint32_t* out /* [n][4] */) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) dds_block(seed, items[i], stream, out + 4 * i);
}

/* Standard normals from the shared Box-Muller (exported for the tests). */
void ddsynth_box_muller(const double* ua, const double* ub, int64_t n, double* z /* [n][2] */) {
  for (int64_t i = 0; i < n; ++i) dds_box_muller(ua[i], ub[i], &z[2 * i], &z[2 * i + 1]);
}

/* log and (cos, sin)(2 pi u) of the shared core (exported for the tests). */
void ddsynth_elementary(const double* x, int64_t n, double* out /* [n][3] */) {
  for (int64_t i = 0; i < n; ++i) {
    out[3 * i] = dds_log(x[i]);
    dds_cos_sin_2pi(x[i], &out[3 * i + 1], &out[3 * i + 2]);
  }
}

/*
 * Material data points: strain components uniform in [-eps_amp, eps_amp]
 * (streams 0..3), stress = S0 * strain + noise_std * N(0,1) (streams 4..7),
 * S0 a 6x6 row-major stiffness supplied by the caller.
 * Writes strain[n][6], stress[n][6] for items first .. first+n-1.
 */
void ddsynth_points(uint64_t seed, int64_t first, int64_t n, double eps_amp,
                    const double* S0, double noise_std, double* strain, double* stress) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    dds_point(seed, (uint64_t)(first + i), eps_amp, S0, noise_std, strain + 6 * i, stress + 6 * i);
}

/* Data points of the paper's example (nonlinear law, no noise), items first .. first+n-1. */
void ddsynth_points_nonlinear(uint64_t seed, int64_t first, int64_t n, double eps_amp, double E,
                              double a, double* strain, double* stress) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    dds_point_nonlinear(seed, (uint64_t)(first + i), eps_amp, E, a, strain + 6 * i, stress + 6 * i);
}

/* The nonlinear reference law applied to given strains (exported for the tests). */
void ddsynth_nonlinear_stress(const double* strain, int64_t n, double E, double a, double* stress) {
  for (int64_t i = 0; i < n; ++i) dds_nonlinear_stress(strain + 6 * i, E, a, stress + 6 * i);
}

/*
 * Query states: base point j uniform over [0, n_data) (stream 16), then
 * strain + eps_std * N(0,1) and stress + sig_std * N(0,1) (streams 18..23).
 * Reads the data arrays (for the base point), writes q_strain/q_stress [m][6]
 * and base[m].
 */
void ddsynth_queries(uint64_t seed, int64_t m, const double* strain, const double* stress,
                     int64_t n_data, double eps_std, double sig_std, double* q_strain,
                     double* q_stress, int64_t* base) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t a[4];
    dds_block(seed, (uint64_t)i, 16u, a);
    double u = dds_u53(a[0], a[1]);
    int64_t j = (int64_t)(u * (double)n_data);
    if (j >= n_data) j = n_data - 1;
    base[i] = j;
    double ua[4], ub[4], uc[4];
    dds_uniforms4(seed, (uint64_t)i, 18u, ua);
    dds_uniforms4(seed, (uint64_t)i, 20u, ub);
    dds_uniforms4(seed, (uint64_t)i, 22u, uc);
    double z[12];
    dds_box_muller(ua[0], ua[1], &z[0], &z[1]);
    dds_box_muller(ua[2], ua[3], &z[2], &z[3]);
    dds_box_muller(ub[0], ub[1], &z[4], &z[5]);
    dds_box_muller(ub[2], ub[3], &z[6], &z[7]);
    dds_box_muller(uc[0], uc[1], &z[8], &z[9]);
    dds_box_muller(uc[2], uc[3], &z[10], &z[11]);
    for (int k = 0; k < 6; ++k) {
      q_strain[6 * i + k] = strain[6 * j + k] + eps_std * z[k];
      q_stress[6 * i + k] = stress[6 * j + k] + sig_std * z[6 + k];
    }
  }
}

/*
 * Query states around generated data points, for data sets too large to hold
 * on the host: the base point j (stream 16) is regenerated from the data-point
 * recipe (data_seed, item j), then perturbed as in ddsynth_queries.
 */
void ddsynth_queries_gen(uint64_t seed, int64_t m, uint64_t data_seed, int64_t n_data,
                         double eps_amp, const double* S0, double noise_std, double eps_std,
                         double sig_std, double* q_strain, double* q_stress, int64_t* base) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t a[4];
    dds_block(seed, (uint64_t)i, 16u, a);
    double u = dds_u53(a[0], a[1]);
    int64_t j = (int64_t)(u * (double)n_data);
    if (j >= n_data) j = n_data - 1;
    base[i] = j;
    double e[6], s[6];
    dds_point(data_seed, (uint64_t)j, eps_amp, S0, noise_std, e, s);
    double ua[4], ub[4], uc[4];
    dds_uniforms4(seed, (uint64_t)i, 18u, ua);
    dds_uniforms4(seed, (uint64_t)i, 20u, ub);
    dds_uniforms4(seed, (uint64_t)i, 22u, uc);
    double z[12];
    dds_box_muller(ua[0], ua[1], &z[0], &z[1]);
    dds_box_muller(ua[2], ua[3], &z[2], &z[3]);
    dds_box_muller(ub[0], ub[1], &z[4], &z[5]);
    dds_box_muller(ub[2], ub[3], &z[6], &z[7]);
    dds_box_muller(uc[0], uc[1], &z[8], &z[9]);
    dds_box_muller(uc[2], uc[3], &z[10], &z[11]);
    for (int k = 0; k < 6; ++k) {
      q_strain[6 * i + k] = e[k] + eps_std * z[k];
      q_stress[6 * i + k] = s[k] + sig_std * z[6 + k];
    }
  }
}

/* Uniform indices over [0, n_data) for items 0..n-1 (stream 32). */
void ddsynth_indices(uint64_t seed, int64_t n, int64_t n_data, int64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t a[4];
    dds_block(seed, (uint64_t)i, 32u, a);
    double u = dds_u53(a[0], a[1]);
    int64_t j = (int64_t)(u * (double)n_data);
    if (j >= n_data) j = n_data - 1;
    out[i] = j;
  }
}

/* Uniform doubles in [lo, hi) for items 0..n-1 (stream 40). */
void ddsynth_uniform(uint64_t seed, int64_t n, double lo, double hi, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t a[4];
    dds_block(seed, (uint64_t)i, 40u, a);
    out[i] = lo + (hi - lo) * dds_u53(a[0], a[1]);
  }
}
