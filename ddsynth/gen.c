/*
 * Seeded synthetic inputs for the data-driven (DD) projection workloads.
 *
 * This file holds input generation only: a counter-based random number
 * generator and the recipes that turn its output into material data points,
 * query states and random initial assignments.  It contains none of the DD
 * method's arithmetic (no metric, no projection, no finite elements); both the
 * CPU oracle and the GPU library consume the arrays it writes.
 *
 * Generator: Philox4x32 with 10 rounds, written from its published definition
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): per round the two odd counter words are combined with the high/low
 * halves of 32x32->64 products by the multipliers 0xD2511F53 and 0xCD9E8D57,
 * and the key is bumped by the Weyl constants 0x9E3779B9 / 0xBB67AE85.
 *
 * Counter layout used by every recipe: (item index low word, item index high
 * word, stream id, 0); key = (seed low word, seed high word).  A recipe reads
 * one or more streams per item, so any item can be generated independently.
 *
 * Uniform doubles use 53 bits from two 32-bit words; Gaussians use Box-Muller
 * with the C library's log, sqrt, cos and sin.
 */
#include <math.h>
#include <stdint.h>

static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Raw block: out[4] for (item, stream) under seed. */
void ddsynth_philox(uint64_t seed, uint64_t item, uint32_t stream, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)item, (uint32_t)(item >> 32), stream, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  philox4x32_10(ctr, key, out);
}

void ddsynth_philox_many(uint64_t seed, uint32_t stream, const uint64_t* items,
                         int64_t n, uint32_t* out /* [n][4] */) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) ddsynth_philox(seed, items[i], stream, out + 4 * i);
}

static inline double u53(uint32_t a, uint32_t b) {
  /* (a >> 5) supplies the top 27 bits, (b >> 6) the low 26 bits: [0, 1). */
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Four uniforms in [0,1) from two Philox blocks of one (item, stream pair). */
static void uniforms4(uint64_t seed, uint64_t item, uint32_t stream, double u[4]) {
  uint32_t a[4], b[4];
  ddsynth_philox(seed, item, stream, a);
  ddsynth_philox(seed, item, stream + 1u, b);
  u[0] = u53(a[0], a[1]);
  u[1] = u53(a[2], a[3]);
  u[2] = u53(b[0], b[1]);
  u[3] = u53(b[2], b[3]);
}

/* Two standard normals by Box-Muller from two uniforms; 1-u keeps log finite. */
static void box_muller(double ua, double ub, double* z0, double* z1) {
  const double two_pi = 6.283185307179586476925286766559;
  double r = sqrt(-2.0 * log(1.0 - ua));
  double th = two_pi * ub;
  *z0 = r * cos(th);
  *z1 = r * sin(th);
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
  for (int64_t i = 0; i < n; ++i) {
    uint64_t item = (uint64_t)(first + i);
    double ua[4], ub[4], uc[4], ud[4];
    uniforms4(seed, item, 0u, ua);
    uniforms4(seed, item, 2u, ub);
    uniforms4(seed, item, 4u, uc);
    uniforms4(seed, item, 6u, ud);
    double e[6] = {ua[0], ua[1], ua[2], ua[3], ub[0], ub[1]};
    for (int k = 0; k < 6; ++k) e[k] = -eps_amp + 2.0 * eps_amp * e[k];
    double z[6];
    box_muller(uc[0], uc[1], &z[0], &z[1]);
    box_muller(uc[2], uc[3], &z[2], &z[3]);
    box_muller(ud[0], ud[1], &z[4], &z[5]);
    double* se = strain + 6 * i;
    double* ss = stress + 6 * i;
    for (int k = 0; k < 6; ++k) se[k] = e[k];
    for (int r = 0; r < 6; ++r) {
      double acc = 0.0;
      for (int c = 0; c < 6; ++c) acc += S0[6 * r + c] * e[c];
      ss[r] = acc + noise_std * z[r];
    }
  }
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
    ddsynth_philox(seed, (uint64_t)i, 16u, a);
    double u = u53(a[0], a[1]);
    int64_t j = (int64_t)(u * (double)n_data);
    if (j >= n_data) j = n_data - 1;
    base[i] = j;
    double ua[4], ub[4], uc[4];
    uniforms4(seed, (uint64_t)i, 18u, ua);
    uniforms4(seed, (uint64_t)i, 20u, ub);
    uniforms4(seed, (uint64_t)i, 22u, uc);
    double z[12];
    box_muller(ua[0], ua[1], &z[0], &z[1]);
    box_muller(ua[2], ua[3], &z[2], &z[3]);
    box_muller(ub[0], ub[1], &z[4], &z[5]);
    box_muller(ub[2], ub[3], &z[6], &z[7]);
    box_muller(uc[0], uc[1], &z[8], &z[9]);
    box_muller(uc[2], uc[3], &z[10], &z[11]);
    for (int k = 0; k < 6; ++k) {
      q_strain[6 * i + k] = strain[6 * j + k] + eps_std * z[k];
      q_stress[6 * i + k] = stress[6 * j + k] + sig_std * z[6 + k];
    }
  }
}

/* Uniform indices over [0, n_data) for items 0..n-1 (stream 32). */
void ddsynth_indices(uint64_t seed, int64_t n, int64_t n_data, int64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t a[4];
    ddsynth_philox(seed, (uint64_t)i, 32u, a);
    double u = u53(a[0], a[1]);
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
    ddsynth_philox(seed, (uint64_t)i, 40u, a);
    out[i] = lo + (hi - lo) * u53(a[0], a[1]);
  }
}
