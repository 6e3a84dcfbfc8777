/*
 * Oracle for the data projection P_D: plain brute-force nearest neighbour in
 * FP64.  Test infrastructure only (called by tests, the smoke check and the
 * CPU baseline of the benchmark); the GPU library never links or calls it.
 *
 * For each query state y = (eps, sig) the oracle visits every data point
 * z_j = (eps'_j, sig'_j), j = 0 .. N-1, in index order and evaluates the local
 * distance of the paper's metric (Section 2, eq. "distmetric"), taken with the
 * factor 1/2 of the global distance (Section 2, the weighted sum over
 * integration points):
 *
 *     dist_j = 1/2 (eps - eps'_j) . C (eps - eps'_j)
 *            + 1/2 (sig - sig'_j) . C^-1 (sig - sig'_j)
 *
 * A strictly smaller distance replaces the current best, so ties go to the
 * lowest index (linear search, Section 1).  The second smallest value of the
 * distance multiset is returned as well (equal to the best when the best is
 * attained twice) so that callers can audit near ties.
 *
 * Two evaluation forms:
 *   raw       the 6x6 quadratic forms above with C and C^-1 as given,
 *   whitened  1/2 |q - x_j|^2 on 12-component points that the caller mapped
 *             with (C^1/2 eps, C^-1/2 sig) (Section 3.2), for timing.
 * Every sum runs in index order; build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

typedef struct {
  double best, second;
  int64_t idx;
} nn_state;

static inline void nn_visit(nn_state* s, double d, int64_t j) {
  if (d < s->best) {
    s->second = s->best;
    s->best = d;
    s->idx = j;
  } else if (d < s->second) {
    s->second = d;
  }
}

/* Merge b (covering higher indices) into a (covering lower indices). */
static inline void nn_merge(nn_state* a, const nn_state* b) {
  if (b->idx < 0) return;
  if (a->idx < 0) { *a = *b; return; }
  if (b->best < a->best) {
    double s = a->best < b->second ? a->best : b->second;
    a->best = b->best;
    a->idx = b->idx;
    a->second = s;
  } else {
    /* a keeps the best (on equality the lower index, from a) */
    double s = a->second < b->best ? a->second : b->best;
    a->second = s;
  }
}

static inline double quad6(const double* M, const double* v) {
  double acc = 0.0;
  for (int r = 0; r < 6; ++r) {
    double t = 0.0;
    for (int c = 0; c < 6; ++c) t += M[6 * r + c] * v[c];
    acc += v[r] * t;
  }
  return acc;
}

static inline double dist_raw(const double* C, const double* Ci, const double* qe,
                              const double* qs, const double* de, const double* ds) {
  double e[6], s[6];
  for (int k = 0; k < 6; ++k) {
    e[k] = qe[k] - de[k];
    s[k] = qs[k] - ds[k];
  }
  return 0.5 * quad6(C, e) + 0.5 * quad6(Ci, s);
}

static inline double dist_white(const double* q, const double* x) {
  double acc = 0.0;
  for (int k = 0; k < 12; ++k) {
    double t = q[k] - x[k];
    acc += t * t;
  }
  return 0.5 * acc;
}

static void finish(const nn_state* s, int64_t q, int64_t* idx, double* dist, double* second) {
  idx[q] = s->idx;
  dist[q] = s->best;
  if (second) second[q] = s->second;
}

/* Raw-metric brute force.  data_eps/data_sig [N][6], q_eps/q_sig [m][6]. */
void oracle_pd_raw(const double* data_eps, const double* data_sig, int64_t N,
                   const double* C, const double* Cinv, const double* q_eps,
                   const double* q_sig, int64_t m, int64_t* idx, double* dist,
                   double* second) {
  if (m >= 4 * omp_get_max_threads()) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < m; ++q) {
      nn_state s = {INFINITY, INFINITY, -1};
      for (int64_t j = 0; j < N; ++j)
        nn_visit(&s, dist_raw(C, Cinv, q_eps + 6 * q, q_sig + 6 * q, data_eps + 6 * j,
                              data_sig + 6 * j), j);
      finish(&s, q, idx, dist, second);
    }
    return;
  }
  /* few queries: split the data range, merge in index order */
  int nt = omp_get_max_threads();
  for (int64_t q = 0; q < m; ++q) {
    nn_state part[256];
    int used = nt < 256 ? nt : 256;
#pragma omp parallel num_threads(used)
    {
      int t = omp_get_thread_num();
      int64_t lo = N * t / used, hi = N * (t + 1) / used;
      nn_state s = {INFINITY, INFINITY, -1};
      for (int64_t j = lo; j < hi; ++j)
        nn_visit(&s, dist_raw(C, Cinv, q_eps + 6 * q, q_sig + 6 * q, data_eps + 6 * j,
                              data_sig + 6 * j), j);
      part[t] = s;
    }
    nn_state s = {INFINITY, INFINITY, -1};
    for (int t = 0; t < used; ++t) nn_merge(&s, &part[t]);
    finish(&s, q, idx, dist, second);
  }
}

/* Whitened brute force.  data [N][12] (float64), queries [m][12]. */
void oracle_pd_white(const double* data, int64_t N, const double* qw, int64_t m,
                     int64_t* idx, double* dist, double* second) {
  if (m >= 4 * omp_get_max_threads()) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < m; ++q) {
      nn_state s = {INFINITY, INFINITY, -1};
      for (int64_t j = 0; j < N; ++j) nn_visit(&s, dist_white(qw + 12 * q, data + 12 * j), j);
      finish(&s, q, idx, dist, second);
    }
    return;
  }
  int nt = omp_get_max_threads();
  for (int64_t q = 0; q < m; ++q) {
    nn_state part[256];
    int used = nt < 256 ? nt : 256;
#pragma omp parallel num_threads(used)
    {
      int t = omp_get_thread_num();
      int64_t lo = N * t / used, hi = N * (t + 1) / used;
      nn_state s = {INFINITY, INFINITY, -1};
      for (int64_t j = lo; j < hi; ++j) nn_visit(&s, dist_white(qw + 12 * q, data + 12 * j), j);
      part[t] = s;
    }
    nn_state s = {INFINITY, INFINITY, -1};
    for (int t = 0; t < used; ++t) nn_merge(&s, &part[t]);
    finish(&s, q, idx, dist, second);
  }
}

/* Whitened brute force over single-precision stored points (promoted exactly). */
void oracle_pd_white_f32data(const float* data, int64_t N, const double* qw, int64_t m,
                             int64_t* idx, double* dist, double* second) {
  int nt = omp_get_max_threads();
  for (int64_t q = 0; q < m; ++q) {
    nn_state part[256];
    int used = nt < 256 ? nt : 256;
#pragma omp parallel num_threads(used)
    {
      int t = omp_get_thread_num();
      int64_t lo = N * t / used, hi = N * (t + 1) / used;
      nn_state s = {INFINITY, INFINITY, -1};
      const double* qq = qw + 12 * q;
      for (int64_t j = lo; j < hi; ++j) {
        const float* x = data + 12 * j;
        double acc = 0.0;
        for (int k = 0; k < 12; ++k) {
          double d = qq[k] - (double)x[k];
          acc += d * d;
        }
        nn_visit(&s, 0.5 * acc, j);
      }
      part[t] = s;
    }
    nn_state s = {INFINITY, INFINITY, -1};
    for (int t = 0; t < used; ++t) nn_merge(&s, &part[t]);
    finish(&s, q, idx, dist, second);
  }
}

/* Raw-metric distances of m (query, data point) pairs, for global distances. */
void oracle_pair_dist_raw(const double* a_eps, const double* a_sig, const double* b_eps,
                          const double* b_sig, int64_t m, const double* C,
                          const double* Cinv, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    out[i] = dist_raw(C, Cinv, a_eps + 6 * i, a_sig + 6 * i, b_eps + 6 * i, b_sig + 6 * i);
}

int oracle_threads(void) { return omp_get_max_threads(); }
