// DD fixed-point solver (host side) and the whitened-query projection it uses.
#pragma once
#include "dd_internal.h"

namespace dd {

// Structured hexahedral mesh of the box [0,lx] x [0,ly] x [0,lz]: node (i,j,k)
// has id i + (nx+1)(j + (ny+1)k), DOF 3 node + component; element (ex,ey,ez)
// has id ex + nx(ey + ny ez); material point 8 element + Gauss point, Gauss
// point a + 2(b + 2c) at -+1/sqrt(3).
struct FEMesh {
  int nx = 0, ny = 0, nz = 0;
  double hx = 0, hy = 0, hz = 0, w = 0;
  int64_t n_nodes = 0, n_dof = 0, n_el = 0, n_mp = 0;
  double B[8][6 * 24];   // strain-displacement operators (Voigt, engineering shear)
  void init(const dd_mesh& m);
  int64_t node(int i, int j, int k) const;
};

// P_D of whitened states (already in the dataset's coordinates).
// dist2_out (exact walks only): distance to the second nearest point, -1
// where not certified.
// fd: radius factor of the k-means walk's ball test (1 = exact).
// passes: as dd_project_opts.passes (0 = the default for the warm start given).
// fd_q / budget_q (walk modes, device arrays over the m states, optional): a
// radius factor and a leaf budget per state in place of fd and ann_budget.
dd_status project_whitened(const Dataset& D, const double* qw_dev, int64_t m,
                           const int64_t* warm_dev, int mode, int ann_budget, int64_t* idx_out,
                           double* dist_out, hipStream_t st, double* dist2_out = nullptr,
                           double fd = 1.0, int passes = 0, const float* fd_q = nullptr,
                           const int* budget_q = nullptr);

// K^-1 for the mesh and Dirichlet pattern, formed on st from the CSR matrix on
// first use and cached on the dataset.
dd_status dense_inverse_for(const Dataset& ds, const FEMesh& M, const uint8_t* mask,
                            const int32_t* rowptr, const int32_t* col, const double* val,
                            std::shared_ptr<DenseInverse>& out, hipStream_t st);
// The cached K^-1 for the mesh and Dirichlet pattern, or null.
std::shared_ptr<DenseInverse> dense_inverse_cached(const Dataset& ds, const FEMesh& M,
                                                   const uint8_t* mask);
// x[0..n) = K^-1 b[0..n), x[n..2n) = K^-1 b[n..2n).
dd_status dense_apply(const DenseInverse& D, const double* b, double* x, hipStream_t st);

class DDSolver {
 public:
  DDSolver() = default;
  DDSolver(const DDSolver&) = delete;
  DDSolver& operator=(const DDSolver&) = delete;
  ~DDSolver();
  dd_status setup(const Dataset& D, const dd_mesh& mesh, const uint8_t* mask, const double* force,
                  const dd_solve_opts* opts, hipStream_t st);
  dd_status set_assignment(const int64_t* idx_host);
  dd_status constraint_projection();
  dd_status cg_solve();
  dd_status run(int max_iter, dd_solve_result* res);
  // u, final association and the raw state of the last P_C (host arrays, any
  // may be NULL); synchronises st
  dd_status fetch_results(double* u, int64_t* idx, double* eps, double* sig);

  // Non-blocking stepping of one DD iteration, for callers that interleave many
  // solves (the server).  Every call only enqueues work on st; completion is
  // observed with hipEventQuery on the named event.
  dd_status async_init();        // pinned host mirrors and events
  dd_status pc_begin();          // gather z*, right-hand sides, CG start
  dd_status cg_batch();          // kCgPoll CG iterations, then the CG state -> host (ev_cg)
  bool cg_finished() const;      // after ev_cg: both systems converged or cg_max_iter reached
  dd_status pc_end();            // CG statistics, admissible state y (ev_ready)
  dd_status scalars_begin();     // after P_D: iteration scalars -> host (ev_scal)
  // after ev_scal: (d_half, d_full, changed, bad flag); swaps in the new association
  void scalars_end(double sc[3], int* bad);
  static int64_t footprint_bytes(const dd_mesh& mesh);
  // Device bytes of the K^-1 that setup() uses for the mesh (0: the mesh is
  // solved by CG), whether the dataset already caches it for the Dirichlet
  // pattern, and its formation ahead of setup() (a no-op when cached or when
  // the mesh is solved by CG; synchronises st).
  static int64_t inverse_bytes(const dd_mesh& mesh);
  static bool inverse_cached(const Dataset& D, const dd_mesh& mesh, const uint8_t* mask);
  static dd_status prepare_inverse(const Dataset& D, const dd_mesh& mesh, const uint8_t* mask,
                                   hipStream_t st);
  hipEvent_t ev_cg = nullptr, ev_ready = nullptr, ev_scal = nullptr;
  char* h_pin = nullptr;
  int cg_it = 0;

  FEMesh M;
  const Dataset* ds = nullptr;
  hipStream_t st = nullptr;
  int mode = DD_EXACT_FP64;
  int ann_budget = 0;
  int ann_ramp = 0;
  double ann_fd = 1.0;   // final radius factor of the k-means walk (1 = exact)
  // leaves per projection at DD iteration it (1-based); 0 = exact
  int budget_at(int it) const {
    if (!walk_mode(mode) || ann_budget <= 0) return 0;
    if (ann_ramp <= 0) return ann_budget;
    return it <= ann_ramp ? ann_budget * it : 0;
  }
  // radius factor of the k-means walk at DD iteration it: the linear ramp to
  // the final factor over the first ann_ramp iterations, then the final one
  // (iteration 1 uses f_d = 0, iteration ann_ramp the final factor)
  double fd_at(int it) const {
    if (mode != DD_KMEANS || ann_fd >= 1.0) return 1.0;
    if (ann_ramp <= 1 || it >= ann_ramp) return ann_fd;
    return ann_fd * (double)(it - 1) / (double)(ann_ramp - 1);
  }
  // iteration it projects approximately
  bool approximate_at(int it) const { return budget_at(it) > 0 || fd_at(it) < 1.0; }
  // accuracy that also depends on the distances (DD_SOLVE_LOCAL_ACCURACY): per
  // material point, from its latest local distance and the latest global one
  bool local_on = false;
  double last_full = INFINITY;     // D_full of the latest iteration
  DevBuf d_fdq, d_budq;            // per-point radius factor and leaf budget
  // associations the previous iteration changed (-1 before the first)
  int64_t last_changed = -1;
  // passes of the 16-bit scans at iteration it: the bound-seeding pass runs
  // beside the warm start while that start is stale (the first iteration, or
  // after an iteration that changed nearly every association); 0 = warm start
  // alone
  int scan_passes(int it) const {
    if (mode != DD_MIXED_BF16 && mode != DD_MIXED_FP16) return 0;
    return (it == 1 || last_changed < 0 || 10 * last_changed > 9 * M.n_mp) ? 2 : 0;
  }
  double cg_tol = 1e-13;
  int cg_max_iter = 20000;
  int64_t nnz = 0;
  double L[36], Lt[36];
  DevBuf d_rowptr, d_col, d_val, d_dinv, d_mask, d_f, d_b, d_x, d_work;
  DevBuf d_idx, d_idx_new, d_dist, d_zw, d_zc, d_yw, d_scal, d_cgstat;
  DevBuf d_part, d_cgstate;
  DevBuf d_uD, d_lift;   // prescribed displacements and K_fd u_D (empty: homogeneous)
  DevBuf arena;   // one allocation holding every buffer above
  // skipping of unmoved material points (exact walks): reference state, half
  // gap, compacted list and its projection buffers
  bool skip_on = false;
  DevBuf d_qref, d_gap, d_list, d_cnt, d_qc, d_wc, d_ic, d_dc, d_d2c;
  int64_t skipped_total = 0;
  dd_status project_step(int it);   // P_D of the current states into d_idx_new / d_dist
  bool use_graph = true;
  std::shared_ptr<DenseInverse> dense;   // set: P_C is a product with K^-1
  hipGraphExec_t cg_graph = nullptr;
  int cg_last_iters[2] = {0, 0};
  double cg_last_res[2] = {0.0, 0.0};
};

}  // namespace dd
