// Host utilities: error reporting, device buffers, small dense linear algebra.
#include <cmath>
#include <cstring>

#include "dd_internal.h"

namespace dd {

static thread_local std::string g_last_error;

dd_status set_error(dd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

dd_status DevBuf::alloc(size_t n) {
  release();
  owned = true;
  if (n == 0) return DD_OK;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    return set_error(e == hipErrorOutOfMemory ? DD_ERR_OOM : DD_ERR_DEVICE,
                     std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e));
  }
  bytes = n;
  return DD_OK;
}

void DevBuf::release() {
  if (p && owned) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  owned = true;
}

ScratchArena::~ScratchArena() {
  // the last user's work on the block must end before the block is freed
  if (done) (void)hipEventSynchronize(done);
  if (block) (void)hipFree(block);
  if (pinned) (void)hipHostFree(pinned);
  if (done) (void)hipEventDestroy(done);
}

bool cholesky6(const double* C, double* L) {
  std::memset(L, 0, 36 * sizeof(double));
  for (int j = 0; j < 6; ++j) {
    double s = C[6 * j + j];
    for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    double d = std::sqrt(s);
    L[6 * j + j] = d;
    for (int i = j + 1; i < 6; ++i) {
      double t = C[6 * i + j];
      for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
      L[6 * i + j] = t / d;
    }
  }
  return true;
}

void lower_inverse6(const double* L, double* X) {
  // Forward substitution column by column: L X = I.
  std::memset(X, 0, 36 * sizeof(double));
  for (int c = 0; c < 6; ++c) {
    for (int i = 0; i < 6; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[6 * i + k] * X[6 * k + c];
      X[6 * i + c] = s / L[6 * i + i];
    }
  }
}

void sym_eigen(int n, const double* A_in, double* evals, double* V) {
  // Cyclic Jacobi rotations on a copy of A (n <= 16).
  double A[256];
  for (int i = 0; i < n * n; ++i) A[i] = A_in[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[n * i + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? diag : off) += A[n * i + j] * A[n * i + j];
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[n * p + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[n * p + p], aqq = A[n * q + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[n * k + p], akq = A[n * k + q];
          A[n * k + p] = c * akp - s * akq;
          A[n * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[n * p + k], aqk = A[n * q + k];
          A[n * p + k] = c * apk - s * aqk;
          A[n * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[n * k + p], vkq = V[n * k + q];
          V[n * k + p] = c * vkp - s * vkq;
          V[n * k + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  // sort descending (selection sort on eigenvalues, permuting columns)
  for (int i = 0; i < n; ++i) evals[i] = A[n * i + i];
  for (int i = 0; i < n; ++i) {
    int best = i;
    for (int j = i + 1; j < n; ++j)
      if (evals[j] > evals[best]) best = j;
    if (best != i) {
      double t = evals[i];
      evals[i] = evals[best];
      evals[best] = t;
      for (int k = 0; k < n; ++k) {
        double v = V[n * k + i];
        V[n * k + i] = V[n * k + best];
        V[n * k + best] = v;
      }
    }
  }
}

int64_t Dataset::device_bytes() const {
  int64_t b = (int64_t)(perm.bytes + iperm.bytes + w64.bytes + n64.bytes + w32.bytes + n32.bytes +
                        centre.bytes + radius.bytes + wbf16.bytes + wfp16.bytes);
  for (int l = 0; l < kAnnMaxLevels; ++l) b += (int64_t)ann_box[l].bytes;
  b += (int64_t)(ann_meta.bytes + ann_q0.bytes + ann_h16.bytes);
  b += (int64_t)(kmt_node.bytes + kmt_nbox.bytes + kmt_child.bytes + kmt_meta.bytes + kmt_h16.bytes +
                 kmt_pos.bytes + kmt_slot.bytes);
  std::lock_guard<std::mutex> lk(arena_mu);
  return b + arena_bytes;
}

}  // namespace dd

extern "C" const char* dd_last_error(void) { return dd::g_last_error.c_str(); }
extern "C" const char* dd_version(void) { return "libdd 0.1 (gfx950)"; }
