/*
 * Core of the seeded input generator, compiled for the host (gcc, gen.c) and for
 * the GPU (hipcc, gen_dev.hip) from this one source so that both produce the
 * same bits.  Input generation only: nothing here computes the DD metric, a
 * projection or a finite-element quantity.
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
 * Uniform doubles use 53 bits from two 32-bit words.  Gaussians use Box-Muller
 * with a logarithm and a sine/cosine pair evaluated below from +, -, *, / and
 * sqrt only (all correctly rounded in IEEE binary64 on both compilers), with
 * floating-point contraction disabled, so host and device results agree bit
 * for bit.  Accuracy of these elementary functions is a few ulp, which is far
 * more than a noise generator needs.
 */
#ifndef DDSYNTH_GEN_CORE_H
#define DDSYNTH_GEN_CORE_H

#include <math.h>
#include <stdint.h>
#include <string.h>

#if defined(__HIPCC__)
#define DDS_FN static inline __host__ __device__
#else
#define DDS_FN static inline
#endif

#if defined(__clang__)
#pragma clang fp contract(off)
#endif

DDS_FN void dds_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
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
DDS_FN void dds_block(uint64_t seed, uint64_t item, uint32_t stream, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)item, (uint32_t)(item >> 32), stream, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  dds_philox4x32_10(ctr, key, out);
}

DDS_FN double dds_u53(uint32_t a, uint32_t b) {
  /* (a >> 5) supplies the top 27 bits, (b >> 6) the low 26 bits: [0, 1). */
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Four uniforms in [0,1) from two Philox blocks of one (item, stream pair). */
DDS_FN void dds_uniforms4(uint64_t seed, uint64_t item, uint32_t stream, double u[4]) {
  uint32_t a[4], b[4];
  dds_block(seed, item, stream, a);
  dds_block(seed, item, stream + 1u, b);
  u[0] = dds_u53(a[0], a[1]);
  u[1] = dds_u53(a[2], a[3]);
  u[2] = dds_u53(b[0], b[1]);
  u[3] = dds_u53(b[2], b[3]);
}

/* Natural logarithm of x in (0, 1]: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, by its odd series
 * through s^23 (next term < 2^-60), plus e log 2 in two parts. */
DDS_FN double dds_log(double x) {
  uint64_t bits;
  memcpy(&bits, &x, sizeof(bits));
  int e = (int)((bits >> 52) & 0x7FF) - 1023;
  bits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;   /* m in [1, 2) */
  double m;
  memcpy(&m, &bits, sizeof(m));
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 23.0;
  p = p * s2 + 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  const double logm = 2.0 * s + 2.0 * s * (s2 * p);
  const double ln2_hi = 6.93147180369123816490e-01;   /* 0x3FE62E42FEE00000 */
  const double ln2_lo = 1.90821492927058770002e-10;   /* 0x3DEA39EF35793C76 */
  return (double)e * ln2_hi + (logm + (double)e * ln2_lo);
}

/* cos(2 pi u), sin(2 pi u) for u in [0, 1): quarter-turn q = floor(4u), the
 * remainder r = 4u - q (both exact), reflected to phi in [0, pi/4], Taylor
 * series of sin and cos through degree 17 / 18 (error < 2^-60). */
DDS_FN void dds_cos_sin_2pi(double u, double* c_out, double* s_out) {
  const double t = 4.0 * u;
  int q = (int)t;
  double r = t - (double)q;
  const int refl = r > 0.5;
  if (refl) r = 1.0 - r;
  const double phi = 1.5707963267948966 * r;
  const double p2 = phi * phi;
  double sp = -1.0 / 355687428096000.0;                  /* -1/17! */
  sp = sp * p2 + 1.0 / 1307674368000.0;                  /*  1/15! */
  sp = sp * p2 - 1.0 / 6227020800.0;                     /* -1/13! */
  sp = sp * p2 + 1.0 / 39916800.0;                       /*  1/11! */
  sp = sp * p2 - 1.0 / 362880.0;                         /* -1/9!  */
  sp = sp * p2 + 1.0 / 5040.0;                           /*  1/7!  */
  sp = sp * p2 - 1.0 / 120.0;                            /* -1/5!  */
  sp = sp * p2 + 1.0 / 6.0;                              /*  1/3!  */
  const double sn = phi - phi * (p2 * sp);
  double cp = 1.0 / 6402373705728000.0;                  /*  1/18! */
  cp = cp * p2 - 1.0 / 20922789888000.0;                 /* -1/16! */
  cp = cp * p2 + 1.0 / 87178291200.0;                    /*  1/14! */
  cp = cp * p2 - 1.0 / 479001600.0;                      /* -1/12! */
  cp = cp * p2 + 1.0 / 3628800.0;                        /*  1/10! */
  cp = cp * p2 - 1.0 / 40320.0;                          /* -1/8!  */
  cp = cp * p2 + 1.0 / 720.0;                            /*  1/6!  */
  cp = cp * p2 - 1.0 / 24.0;                             /* -1/4!  */
  cp = cp * p2 + 0.5;                                    /*  1/2!  */
  const double cs = 1.0 - p2 * cp;
  /* angle within the quarter turn: r (or its reflection 1 - r) */
  double c = refl ? sn : cs;
  double s = refl ? cs : sn;
  /* rotate by q quarter turns */
  switch (q & 3) {
    case 0: *c_out = c; *s_out = s; break;
    case 1: *c_out = -s; *s_out = c; break;
    case 2: *c_out = -c; *s_out = -s; break;
    default: *c_out = s; *s_out = -c; break;
  }
}

/* Two standard normals by Box-Muller from two uniforms; 1-u keeps log finite. */
DDS_FN void dds_box_muller(double ua, double ub, double* z0, double* z1) {
  const double r = sqrt(-2.0 * dds_log(1.0 - ua));
  double c, s;
  dds_cos_sin_2pi(ub, &c, &s);
  *z0 = r * c;
  *z1 = r * s;
}

/* One material data point (item = global index): strain uniform in
 * [-eps_amp, eps_amp] (streams 0..3), stress = S0 strain + noise_std N(0,1)
 * (streams 4..7), S0 a 6x6 row-major stiffness. */
DDS_FN void dds_point(uint64_t seed, uint64_t item, double eps_amp, const double* S0,
                      double noise_std, double* se, double* ss) {
  double ua[4], ub[4], uc[4], ud[4];
  dds_uniforms4(seed, item, 0u, ua);
  dds_uniforms4(seed, item, 2u, ub);
  dds_uniforms4(seed, item, 4u, uc);
  dds_uniforms4(seed, item, 6u, ud);
  double e[6] = {ua[0], ua[1], ua[2], ua[3], ub[0], ub[1]};
  for (int k = 0; k < 6; ++k) e[k] = -eps_amp + 2.0 * eps_amp * e[k];
  double z[6];
  dds_box_muller(uc[0], uc[1], &z[0], &z[1]);
  dds_box_muller(uc[2], uc[3], &z[2], &z[3]);
  dds_box_muller(ud[0], ud[1], &z[4], &z[5]);
  for (int k = 0; k < 6; ++k) se[k] = e[k];
  for (int r = 0; r < 6; ++r) {
    double acc = 0.0;
    for (int c = 0; c < 6; ++c) acc += S0[6 * r + c] * e[c];
    ss[r] = acc + noise_std * z[r];
  }
}

/* Stress of the nonlinear isotropic reference law of the paper's example
 * (Section 3): sig = E (eps + a eps^3 + 0.5 (tr eps + a (tr eps)^3) I) with the
 * tensor strain eps (off-diagonal = half the engineering shear) and eps^3 its
 * matrix cube; Voigt order (11, 22, 33, 23, 13, 12). */
DDS_FN void dds_nonlinear_stress(const double* e, double E, double a, double* s) {
  double m[3][3];
  m[0][0] = e[0]; m[1][1] = e[1]; m[2][2] = e[2];
  m[1][2] = m[2][1] = 0.5 * e[3];
  m[0][2] = m[2][0] = 0.5 * e[4];
  m[0][1] = m[1][0] = 0.5 * e[5];
  double m2[3][3], m3[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += m[i][k] * m[k][j];
      m2[i][j] = acc;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += m2[i][k] * m[k][j];
      m3[i][j] = acc;
    }
  const double tr = m[0][0] + m[1][1] + m[2][2];
  const double vol = 0.5 * (tr + a * tr * tr * tr);
  double t[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[i][j] = E * (m[i][j] + a * m3[i][j] + (i == j ? vol : 0.0));
  s[0] = t[0][0]; s[1] = t[1][1]; s[2] = t[2][2];
  s[3] = t[1][2]; s[4] = t[0][2]; s[5] = t[0][1];
}

/* One data point of the paper's example: the 6 Voigt strain components uniform
 * in [-eps_amp, eps_amp] (streams 48..51), the stress from the nonlinear law
 * (no noise). */
DDS_FN void dds_point_nonlinear(uint64_t seed, uint64_t item, double eps_amp, double E, double a,
                                double* se, double* ss) {
  double ua[4], ub[4];
  dds_uniforms4(seed, item, 48u, ua);
  dds_uniforms4(seed, item, 50u, ub);
  const double u[6] = {ua[0], ua[1], ua[2], ua[3], ub[0], ub[1]};
  for (int k = 0; k < 6; ++k) se[k] = -eps_amp + 2.0 * eps_amp * u[k];
  dds_nonlinear_stress(se, E, a, ss);
}

#endif /* DDSYNTH_GEN_CORE_H */
