/*
 * dd.h — C ABI of libdd, the MI355X (gfx950) library for the nearest-neighbour
 * projection at the heart of model-free data-driven (DD) solid mechanics.
 *
 * Problem statement (Eggersmann, Stainier, Ortiz, Reese, "Efficient data
 * structures for model-free data-driven computational mechanics", Section 2):
 * a material data set D = {(eps'_j, sig'_j)}, j = 0..N-1, of 12-component
 * phase-space points (6 Voigt strains, 6 stresses); a constant symmetric
 * positive definite metric C (6x6); for each admissible state y = (eps, sig)
 * the projection P_D returns the data point minimising the local distance of
 * eq. "distmetric",
 *
 *     dist = 1/2 (eps - eps').C(eps - eps') + 1/2 (sig - sig').C^-1(sig - sig'),
 *
 * (the factor 1/2 is the one of the global distance d^2 = sum_e 1/2 w_e d_e^2,
 * so that sum_e w_e dist_e is the paper's global squared distance).  The DD
 * solver alternates P_D with the constraint-set projection P_C (eqs. "KuE",
 * "KeS") until the association stops changing.
 *
 * Conventions shared by every entry point
 *   Layout     states, strains and stresses are row-major float64; a state is
 *              (eps11, eps22, eps33, gamma23, gamma13, gamma12,
 *               sig11, sig22, sig33, sig23, sig13, sig12), engineering shear
 *              strains.  C is row-major 6x6 in the same Voigt order.
 *   Memory     array arguments named *_dev are DEVICE pointers on the current
 *              HIP device; small parameter arrays (C, options) are host memory.
 *              Inputs are borrowed for the duration of the call; outputs are
 *              caller-allocated.  A dataset owns the device memory it creates
 *              until dd_dataset_destroy.
 *   Streams    hip_stream is a hipStream_t (NULL = default stream).  Calls are
 *              stream-ordered: device outputs are valid once that stream has
 *              completed the work.  dd_dataset_create and dd_solve synchronise
 *              the stream before returning; dd_project does not.
 *   Indices    int64 at the ABI, always in the caller's original data order.
 *   Ties       equal distances resolve to the lowest original index.
 *   Errors     status codes only; dd_last_error() gives a thread-local message
 *              for the last non-OK status of the calling thread.
 *   Threads    a dataset is immutable after creation; concurrent dd_project
 *              calls on different streams are safe.
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dd_status {
  DD_OK = 0,
  DD_ERR_ARG = 1,            /* invalid argument (sizes, pointers, options, non-finite C) */
  DD_ERR_NOT_SPD = 2,        /* metric C not symmetric positive definite */
  DD_ERR_OOM = 3,            /* device allocation failed */
  DD_ERR_DEVICE = 4,         /* a HIP runtime call failed */
  DD_ERR_NOT_CONVERGED = 5,  /* dd_solve hit max_iter (results are still written) */
  DD_ERR_TOO_LARGE = 6,      /* request exceeds a documented capacity */
  DD_ERR_CANCELLED = 7,      /* serving request cancelled */
  DD_ERR_UNSUPPORTED = 8,    /* the dataset lacks the pack a mode needs */
  DD_ERR_TIMEOUT = 9         /* serving wait timed out */
} dd_status;

/* Projection algorithms (dd_project_opts.mode). */
typedef enum dd_mode {
  /* FP64 MFMA scan of the whole data set in whitened coordinates (expanded
   * form), candidates inside a proven FP64 error margin reranked in the direct
   * FP64 form.  Exact (indices of the FP64 nearest neighbour). */
  DD_EXACT_FP64 = 0,
  /* FP32 MFMA scan of the whole data set (pack DD_PACK_FP32, expanded form
   * with the stored FP32 norms), every candidate inside the proven FP32 error
   * margin a = 2^-18 (|q| + max|x|)^2 reranked in the direct FP64 form; queries
   * whose candidate lists overflow are rescanned in FP64.  Exact. */
  DD_MIXED_FP32 = 1,
  /* BF16 MFMA scan with FP32 accumulation on tile-centred coordinates, every
   * candidate inside the proven BF16 error margin reranked in FP64; queries
   * whose candidate list overflows are rescanned in FP64.  Exact. */
  DD_MIXED_BF16 = 2,
  /* Warm-started walk over a 64-ary tree of principal-axis boxes (dataset
   * pack DD_PACK_ANN), visiting subtrees nearest-box-first and pruning every
   * box whose distance bound exceeds the best certified distance so far; FP32
   * distances with a proven error margin, FP64 rerank.  With ann_budget = 0 the
   * walk ends only when every box is pruned, and the result is exact; with a
   * budget it stops after that many leaves (64 points each) and is approximate
   * (never worse than the warm-start point). */
  DD_ANN = 3,
  /* Plain FP64 direct-form scan (VALU), the simplest exact kernel. */
  DD_DIRECT_FP64 = 4,
  /* As DD_MIXED_BF16 with IEEE half precision instead of bfloat16. */
  DD_MIXED_FP16 = 5,
  /* Warm-started walk over the k-means tree of Section 4 (recursive 4-means,
   * pack DD_PACK_KMEANS): every stored node holds up to 64 children (up to
   * three 4-means levels), each with the ball (centroid, radius) of its points
   * and their box in principal-axis coordinates; a child is pruned when
   * |q - c| - f_d r (with f_d = 1 also its box distance) exceeds the best
   * certified distance so far.  Same certified FP32 arithmetic, FP64 rerank,
   * budget and warm-start rules as DD_ANN; exact with ann_budget = 0 and
   * f_d = 1 (ann_radius_discount = 0), approximate otherwise.  Siblings are
   * visited nearest centre first (so a budget keeps the leaves nearest the
   * query's path of centres).  With f_d < 1 the walk is the search of
   * Section 4.2: a child is entered while |q - c| - f_d r is below the best
   * distance the walk has found itself (the first descent reaches a leaf
   * whatever the warm start); the warm-start point stays a candidate, so the
   * answer is never farther than it. */
  DD_KMEANS = 6
} dd_mode;

/* Packs a dataset can hold (dd_dataset_opts.packs bit mask). */
#define DD_PACK_FP64 0x1u   /* whitened FP64 [N][12] + norms: DD_EXACT_FP64, DD_DIRECT_FP64, the
                               rerank and fallback of every mode; every dataset holds it */
#define DD_PACK_FP32 0x2u   /* whitened FP32 [N][12] + norms: DD_MIXED_FP32 */
#define DD_PACK_BF16 0x4u   /* tile-centred BF16 [N][16] + tile centres/radii: DD_MIXED_BF16 */
#define DD_PACK_FP16 0x8u   /* tile-centred FP16 [N][16]: DD_MIXED_FP16 */
#define DD_PACK_ANN 0x10u   /* box tree over the sorted order, compact leaves (implies FP64): DD_ANN */
#define DD_PACK_KMEANS 0x20u /* k-means tree, compact leaves (implies FP64): DD_KMEANS */
#define DD_PACK_DEFAULT (DD_PACK_FP64 | DD_PACK_BF16)

typedef struct dd_dataset dd_dataset;

typedef struct dd_dataset_opts {
  uint32_t packs;      /* DD_PACK_* mask; 0 = DD_PACK_DEFAULT */
  int32_t tile;        /* points per centring tile of the 16-bit packs: 128, 256, 512, 1024 or
                          2048; 0 = 2048 */
  uint32_t flags;      /* DD_DATASET_* bits; other bits are DD_ERR_ARG */
} dd_dataset_opts;
/* dd_dataset_create: strain and stress are HOST arrays; they are copied to the
 * device in chunks of up to 2^24 points (over PCIe, on hip_stream). */
#define DD_DATASET_HOST_INPUT 0x1u

/* Per-call statistics (optional output of dd_project). */
typedef struct dd_project_stats {
  int64_t candidates;       /* candidates reranked in FP64 (mixed modes) */
  int64_t overflowed;       /* queries rescanned by the FP64 fallback */
  int64_t visited;          /* data points visited (DD_ANN, DD_KMEANS) */
  double scan_ms;           /* device time of the main scan kernel, the one pass over every
                               (query, data point) pair (HIP events on the call's stream) */
  double total_ms;          /* device time from the first to the last kernel of the call */
  int64_t slow_tiles;       /* 16-bit scans: (32-query group, tile) items recomputed for candidates */
  int64_t boxes;            /* DD_ANN: tree boxes tested; DD_KMEANS: child balls tested */
  int64_t leaves;           /* DD_ANN, DD_KMEANS: leaves (blocks of up to 64 points) visited */
  int64_t leaf_boxes;       /* DD_ANN: of the boxes tested, leaf boxes (read quantised, 24 bytes;
                               the others are 96-byte FP32 boxes); DD_KMEANS: of the balls
                               tested, leaf balls */
  int64_t nodes;            /* DD_KMEANS: stored nodes expanded (each reads its 96-byte box, in
                               which its children's boxes are quantised); DD_ANN: 0 */
} dd_project_stats;

typedef struct dd_project_opts {
  int32_t mode;             /* dd_mode; default DD_EXACT_FP64 */
  int32_t splits;           /* data splits per query block; 0 = automatic */
  int32_t ann_budget;       /* DD_ANN, DD_KMEANS: max leaves visited per query;
                               0 = unlimited (exact) */
  int32_t passes;           /* 16-bit modes: 1 = marking pass only, 2 = a bound-seeding pass over
                               every 64th tile first; 0 = automatic (2 without a warm start);
                               any other value is DD_ERR_ARG */
  dd_project_stats* stats;  /* optional host pointer; filling it synchronises the stream */
  double ann_radius_discount;  /* DD_KMEANS: 1 - f_d in [0, 1], the part of a child's radius
                                  the ball test |q - c| - f_d r leaves out (Section 4.2):
                                  0 = exact (f_d = 1), 1 = centres only (f_d = 0);
                                  > 0 with another mode is DD_ERR_ARG */
} dd_project_opts;

/*
 * Create a dataset from N material data points (Section 2: D = {(eps'_j,
 * sig'_j)}) and the metric C (eq. "distmetric").
 *   strain, stress   float64 [N][6] each (borrowed): DEVICE arrays, or HOST
 *                    arrays with opts->flags & DD_DATASET_HOST_INPUT
 *   N                1 <= N <= 2^31 - 1
 *   C                host float64 [36], symmetric positive definite
 *   opts             NULL for defaults
 * Whitens every point to (C^1/2 eps, C^-1/2 sig) (Section 3.2; C^1/2 = L^T of
 * the Cholesky factor C = L L^T), orders the points spatially (principal-axis
 * cell keys, stable radix sort) and builds the requested packs.
 * Errors: DD_ERR_ARG (null pointers, N out of range, unknown flags, non-finite
 * C or data), DD_ERR_NOT_SPD, DD_ERR_OOM, DD_ERR_DEVICE.  Synchronises
 * hip_stream.
 */
dd_status dd_dataset_create(const double* strain, const double* stress, int64_t N,
                            const double* C, const dd_dataset_opts* opts, void* hip_stream,
                            dd_dataset** out);

/*
 * Producer of data points for dd_dataset_create_streamed: write points
 * first .. first+count-1 into the library's device arrays strain_dev[count][6]
 * and stress_dev[count][6], stream-ordered on hip_stream (the library's
 * stream; the producer must not synchronise other streams against it).  Must
 * return 0 on success and write the same values every time it is asked for a
 * point: creation reads the data set three times, in chunks of up to 2^24
 * points.  A non-zero return aborts creation with DD_ERR_ARG.
 */
typedef int (*dd_fill_fn)(void* user, int64_t first, int64_t count, double* strain_dev,
                          double* stress_dev, void* hip_stream);

/*
 * As dd_dataset_create for a data set too large to hold in raw form next to
 * its packs (Section 3 scales N to 10^9): the points come from `fill` in
 * chunks, so only the packs and a chunk of raw data are ever resident.  The
 * resulting dataset is identical to dd_dataset_create's on the same points.
 * Errors: as dd_dataset_create; DD_ERR_ARG if fill fails.
 */
dd_status dd_dataset_create_streamed(int64_t N, const double* C, dd_fill_fn fill, void* user,
                                     const dd_dataset_opts* opts, void* hip_stream,
                                     dd_dataset** out);

/* Release a dataset's device memory (NULL is a no-op). */
dd_status dd_dataset_destroy(dd_dataset* ds);

/* Number of points, and bytes of device memory the dataset holds: its packs and
   trees plus the projection scratch it keeps between calls (at most 8 idle
   blocks of at most 1 GiB, released by dd_dataset_destroy).  The K^-1 cache of
   dd_solve is not counted. */
dd_status dd_dataset_info(const dd_dataset* ds, int64_t* n_points, int64_t* device_bytes);

/* Shape of a dataset's search trees (zeros for a tree it does not hold). */
typedef struct dd_index_info {
  int32_t ann_levels;       /* box tree levels (level 0: leaves of 64 consecutive points) */
  int32_t kmeans_levels;    /* 4-means levels of the k-means tree (depth of its deepest leaf) */
  int64_t ann_leaves;       /* box tree leaves */
  int64_t kmeans_nodes;     /* stored k-means tree nodes (every third 4-means level) */
  int64_t kmeans_leaves;    /* k-means tree leaves (at most 64 points each) */
  int64_t kmeans_records;   /* child records (balls) of the stored nodes */
} dd_index_info;
dd_status dd_dataset_index_info(const dd_dataset* ds, dd_index_info* info);

/*
 * P_D (Section 2): for each of m states find the data point nearest under the
 * metric, ties to the lowest original index.
 *   states_dev          device float64 [m][12]
 *   warm_start_idx_dev  device int64 [m] or NULL: a previous association used
 *                       to seed the search bound (any valid index is allowed;
 *                       results do not depend on it in the exact modes)
 *   idx_out_dev         device int64 [m]: original index of the nearest point
 *   dist_out_dev        device float64 [m] or NULL: the local distance
 *                       1/2 d_e^2 of that point, evaluated in FP64
 * m = 0 is a no-op.  A non-finite state yields idx -1 and dist NaN.
 * Errors: DD_ERR_ARG, DD_ERR_UNSUPPORTED (mode needs a pack the dataset lacks),
 * DD_ERR_OOM, DD_ERR_DEVICE.  Asynchronous on hip_stream unless opts->stats.
 */
dd_status dd_project(const dd_dataset* ds, const double* states_dev, int64_t m,
                     const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                     int64_t* idx_out_dev, double* dist_out_dev, void* hip_stream);

/*
 * dd_project without device allocation, for callers that cannot allocate
 * (work captured into HIP graphs, tight serving loops, harnesses that forbid
 * allocation).  Arguments, layouts, results and errors as dd_project, with
 * these differences:
 *   mode        DD_EXACT_FP64, DD_ANN or DD_KMEANS (others: DD_ERR_UNSUPPORTED)
 *   m           at most DD_NOALLOC_MAX_QUERIES (else DD_ERR_TOO_LARGE)
 *   opts->stats must be NULL (DD_ERR_ARG); opts->splits and opts->passes are
 *               ignored (the FP64 scan uses as many data splits as the scratch
 *               holds)
 * The call's temporary buffers live in one 64 MiB device array of the library
 * (each GPU the library runs on holds its own copy until the process ends);
 * the call allocates nothing, device or host, and does not synchronise
 * hip_stream: it only enqueues kernels.  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.
 */
#define DD_NOALLOC_MAX_QUERIES 65536
dd_status dd_project_noalloc(const dd_dataset* ds, const double* states_dev, int64_t m,
                             const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                             int64_t* idx_out_dev, double* dist_out_dev, void* hip_stream);

/*
 * Diagnostic: multiply small HOST matrices with one wavefront of the matrix
 * instructions the scans use, with the operand/result lane layouts the scans
 * assume (so a correct layout reproduces the plain product A B exactly for
 * small-integer inputs).
 *   kind 0: bf16 32x32x16 (A [32][16], B [16][32], D [32][32]), FP32 accumulate
 *   kind 1: fp16 32x32x16 (same shapes)
 *   kind 2: fp64 16x16x4  (A [16][4], B [4][16], D [16][16])
 *   kind 3: round A[512] (taken as FP32) to bf16 with the packed conversion of
 *           the query operands and widen back into D[512] (B unused)
 *   kind 4: the same for IEEE half
 *   kind 5: fp32 32x32x2 (A [32][2], B [2][32], D [32][32]) with the accumulator
 *           input C[i][j] = i (the role of the FP32 scan's row norms): D = A B + C
 * Arrays are row-major float64 host memory; D is written.  Synchronous.
 */
dd_status dd_selftest_mfma(int kind, const double* A, const double* B, double* D);

/* Structured hexahedral mesh of the box [0,lx] x [0,ly] x [0,lz] with
 * nx x ny x nz trilinear elements and 2x2x2 Gauss points.
 *   node (i,j,k)      id i + (nx+1)(j + (ny+1)k), DOF = 3 id + component (x,y,z)
 *   element (ex,ey,ez) id ex + nx(ey + ny ez)
 *   material point    8 element + Gauss point a + 2(b + 2c), abscissae -+1/sqrt(3)
 *   weight w_e        (lx/nx)(ly/ny)(lz/nz)/8, the integration-point volume
 * (the "volumes associated with the integration points" of Section 2). */
typedef struct dd_mesh {
  int32_t nx, ny, nz;
  double lx, ly, lz;
} dd_mesh;

typedef struct dd_solve_opts {
  int32_t max_iter;      /* 0 = 500 */
  int32_t mode;          /* projection mode (dd_mode), default DD_EXACT_FP64 */
  int32_t cg_max_iter;   /* 0 = 20000 */
  int32_t flags;         /* DD_SOLVE_NO_GRAPH: launch the CG kernels one by one; DD_SOLVE_CG,
                            DD_SOLVE_SKIP, DD_SOLVE_LOCAL_ACCURACY (below) */
  double cg_tol;         /* relative residual of the two P_C solves; 0 = 1e-13 */
  int32_t ann_budget;    /* DD_ANN, DD_KMEANS: leaves per projection (0 = exact walk) */
  int32_t ann_ramp;      /* DD_ANN, DD_KMEANS: > 0 = accuracy schedule.  With a budget,
                            iteration i <= ann_ramp uses ann_budget * i leaves and later
                            iterations walk exactly; with ann_radius_discount > 0 see there
                            (the paper's search accuracy growing over the iterations,
                            Section 4.5) */
  const double* dirichlet_values;  /* host [ndof] or NULL: prescribed displacements at the
                                      Dirichlet DOFs (e.g. the rotated face of Section 3's
                                      example); eta stays homogeneous there */
  double ann_radius_discount;      /* DD_KMEANS: 1 - f_d^f in [0, 1], the final radius factor of
                                      the ball test (0 = exact); with ann_ramp > 1, iteration
                                      i <= ann_ramp uses f_d = f_d^f (i - 1) / (ann_ramp - 1),
                                      from 0 up to f_d^f (the paper's linear ramp of Section
                                      4.5), later ones f_d^f; > 0 with another mode is
                                      DD_ERR_ARG */
} dd_solve_opts;
#define DD_SOLVE_NO_GRAPH 0x1
/* P_C by CG even for meshes of at most 16384 DOFs, where dd_solve otherwise
 * forms K^-1 once (blocked Gauss-Jordan on the GPU, about 0.4 s at 16384),
 * keeps it on the dataset for that mesh and Dirichlet pattern (at most 4 GiB
 * of inverses per dataset, least recently used dropped first) and applies it
 * as one product per P_C. */
#define DD_SOLVE_CG 0x2
/* Exact DD_ANN and DD_KMEANS solves: skip the projection of material points whose state
 * moved less than half the certified gap between their nearest and second
 * nearest data points since that gap was measured (the association cannot
 * change, by the triangle inequality: the paper's criterion for unmoved
 * queries).  The walk then certifies two neighbours; results are unchanged. */
#define DD_SOLVE_SKIP 0x4
/* Approximate DD_ANN and DD_KMEANS solves (a budget or f_d < 1): the accuracy of
 * each material point's search also depends on the distances (Section 4: the
 * accuracy parameter as a function of the global distance, the local distance
 * and the iteration).  From the second iteration on, with rho = d_e / dbar
 * (d_e the point's distance to its association after the previous projection,
 * dbar = D_full / sum of the weights), a point at least as far from the data
 * as the mean keeps the schedule's f_d and leaf budget, a nearer one gets
 * f_d + (1 - f_d)(1 - rho) and budget * ceil(1 / rho) leaves (at most 16 times
 * the budget): points closing in on the data search more accurately. */
#define DD_SOLVE_LOCAL_ACCURACY 0x8

/* Results of dd_solve; every array is HOST memory provided by the caller and
 * may be NULL when not wanted. */
typedef struct dd_solve_result {
  double* u;                /* [ndof] displacement of the last P_C */
  int64_t* idx;             /* [n_mp] final association (original data indices) */
  double* eps;              /* [n_mp][6] strain of the last P_C (raw Voigt) */
  double* sig;              /* [n_mp][6] stress of the last P_C */
  double* d_half;           /* [history_capacity] sum_e w_e dist(y_i, z_i) */
  double* d_full;           /* [history_capacity] sum_e w_e dist(y_i, z_{i+1}) */
  int64_t* changed;         /* [history_capacity] #associations changed by P_D */
  int64_t* history;         /* [history_capacity+1][n_mp] idx_0 (init), idx_1, ... */
  int32_t history_capacity; /* entries available in the four arrays above */
  int32_t iterations;       /* out: DD iterations performed */
  int32_t converged;        /* out: 1 if the association stopped changing */
  int32_t stop_reason;      /* out: 0 max_iter reached, 1 association unchanged, 2 distance
                               no longer decreasing (approximate projection only) */
  int64_t cg_iterations;    /* out: total CG iterations (both systems) */
  double cg_max_residual;   /* out: largest final relative CG residual */
  double elapsed_ms;        /* out: host wall time of the loop */
  int64_t skipped;          /* out: projections skipped as unmoved (exact DD_ANN, DD_KMEANS) */
  double project_ms;        /* out: GPU time of the P_D steps (HIP events around each), the
                               paper's search time; dd_server_wait writes 0 (its projections
                               serve many solves at once) */
} dd_solve_result;

/*
 * DD fixed-point loop (Section 2): starting from the association init_idx,
 * repeat  y_i = P_C(z_i)  (eqs. "KuE", "KeS": K u = E, K eta = S with
 * K = A_e{w B^T C B} assembled once, E = A_e{w B^T C eps*},
 * S = f - A_e{w B^T sig*}, eps = B u, sig = sig* + C B eta), then
 * z_{i+1} = P_D(y_i), until no association changes (the stopping rule for
 * exact projections).  With an approximate projection (a walk with a budget
 * or f_d < 1) the loop also stops when sum_e w_e dist(y_i, z_{i+1}) no longer
 * decreases, since the alternating-minimisation descent no longer holds
 * (Section 4.1); with an accuracy schedule (ann_ramp) both stopping rules wait
 * until the schedule has ended.  Each projection is warm-started from the
 * current association; the 16-bit scans also run their bound-seeding pass
 * (passes = 2) at the first iteration and after an iteration that changed
 * more than 90 % of the associations, where that start is stale.
 *   mesh            structured box mesh (see dd_mesh)
 *   dirichlet_mask  host uint8 [ndof]: 1 = homogeneous Dirichlet DOF (u = eta = 0)
 *   nodal_force     host float64 [ndof]: consistent nodal forces f
 *   init_idx        host int64 [n_mp]: initial association (e.g. random)
 *   opts            NULL for defaults; result NULL or host arrays to fill
 * Errors: DD_ERR_ARG, DD_ERR_UNSUPPORTED (no FP64 pack), DD_ERR_TOO_LARGE,
 * DD_ERR_OOM, DD_ERR_DEVICE; DD_ERR_NOT_CONVERGED after max_iter (results are
 * still written).  Synchronises hip_stream.
 */
dd_status dd_solve(const dd_dataset* ds, const dd_mesh* mesh, const uint8_t* dirichlet_mask,
                   const double* nodal_force, const int64_t* init_idx, const dd_solve_opts* opts,
                   dd_solve_result* result, void* hip_stream);

/*
 * Serving: DD solves of different meshes against one resident dataset, their
 * projections batched across solves (continuous batching).  A server runs two
 * host threads: a scheduler that admits queued solves in arrival order while
 * their device footprint fits the budget and advances every admitted solve on
 * its own HIP stream, and a projection thread that runs one P_D batch at a
 * time over the admissible states of every solve that is ready (a large mesh
 * may span several batches).  Each solve computes exactly what dd_solve
 * computes, so its result is the same alone and in any mix.
 */
typedef struct dd_server dd_server;

typedef struct dd_server_opts {
  int32_t mode;          /* dd_mode of every projection (the dataset must hold its pack) */
  int32_t max_active;    /* solves admitted at once; 0 = 64 */
  int32_t max_batch;     /* queries per projection batch; 0 = 65536 */
  int32_t max_queue;     /* submitted, not yet admitted solves; 0 = 4096 */
  int32_t ann_budget;    /* DD_ANN, DD_KMEANS budget (0 = exact walk) */
  int32_t reserved;      /* must be 0 */
} dd_server_opts;

typedef struct dd_solve_request {
  dd_mesh mesh;                   /* as for dd_solve */
  const uint8_t* dirichlet_mask;  /* host [ndof]; copied by dd_server_submit */
  const double* nodal_force;      /* host [ndof]; copied */
  const int64_t* init_idx;        /* host [n_mp]; copied */
  int32_t max_iter;               /* 0 = 500 */
  int32_t reserved;               /* must be 0 */
  double deadline_s;              /* > 0: cancelled when still running this long after submit */
} dd_solve_request;

typedef struct dd_server_statistics {
  int64_t submitted, completed, failed, rejected, cancelled;
  int64_t active, queued;           /* admitted solves now; submitted, not yet admitted */
  int64_t batches, queries;         /* projection batches run; material points projected */
  int64_t peak_active, peak_bytes;  /* most solves admitted at once; most bytes charged at once
                                       (reserve, admitted solves, K^-1 inverses) */
  int64_t budget_bytes;             /* the admission budget */
  double proj_p50_ms, proj_p99_ms;  /* per projection: a solve's state ready -> association back */
  double solve_p50_ms, solve_p99_ms;  /* per solve: submit -> result ready */
  double queue_p50_ms, queue_p99_ms;  /* per solve: submit -> admission */
  double queries_per_s;             /* queries / elapsed_s */
  double elapsed_s;                 /* since the first submit */
  int64_t reserve_bytes;            /* the server's fixed reserve (batch buffers and the
                                       scratch of a full projection batch), part of peak_bytes */
} dd_server_statistics;

/*
 * Create a server over ds (which must outlive it).  hbm_budget_bytes bounds the
 * server's device memory: a fixed reserve held from creation to destroy (the
 * batch buffers and the scratch of a projection of max_batch states, which the
 * batch projections carve every temporary buffer from, so they allocate
 * nothing), plus the summed footprint of admitted solves (their P_C buffers and
 * states), plus the K^-1 inverses the server forms (from admission of the solve
 * that needs one, and for as long as the dataset's cache keeps it); an inverse
 * is formed on a builder thread while the other solves go on, and a solve whose
 * inverse cannot fit next to it even on an idle server is run by CG (dd_solve's
 * DD_SOLVE_CG trajectory); 0 = half of the free device memory.  opts NULL =
 * BF16 projections, defaults above.  Errors: DD_ERR_ARG, DD_ERR_UNSUPPORTED
 * (mode without its pack), DD_ERR_TOO_LARGE (the reserve alone exceeds the
 * budget: lower max_batch), DD_ERR_OOM, DD_ERR_DEVICE.
 */
dd_status dd_server_create(const dd_dataset* ds, size_t hbm_budget_bytes,
                           const dd_server_opts* opts, dd_server** out);

/* Queue a solve (non-blocking; inputs are copied).  *ticket identifies it.
 * Errors: DD_ERR_ARG (invalid request, as dd_solve), DD_ERR_TOO_LARGE (its
 * footprint does not fit the budget beside the server's reserve, or the queue
 * is full: rejected). */
dd_status dd_server_submit(dd_server* srv, const dd_solve_request* req, uint64_t* ticket);

/* Wait for a solve: timeout_s < 0 waits without limit, 0 polls.  On completion
 * fills result (host arrays as for dd_solve; history is not recorded) and
 * releases the ticket; returns the solve's status (DD_OK, DD_ERR_NOT_CONVERGED,
 * DD_ERR_CANCELLED, or the error that stopped it; other solves are not
 * affected).  DD_ERR_TIMEOUT leaves the ticket valid; DD_ERR_ARG for an
 * unknown ticket. */
dd_status dd_server_wait(dd_server* srv, uint64_t ticket, dd_solve_result* result, double timeout_s);

/* Ask a queued or running solve to stop; its wait returns DD_ERR_CANCELLED. */
dd_status dd_server_cancel(dd_server* srv, uint64_t ticket);

/* Counters and latency percentiles since creation. */
dd_status dd_server_stats(const dd_server* srv, dd_server_statistics* stats);

/* Stop the threads; unfinished solves end as DD_ERR_CANCELLED (their tickets
 * become invalid). */
dd_status dd_server_destroy(dd_server* srv);

/*
 * The metric of the paper's example (Section 3): principal component analysis
 * of the data set -- the 12 components centred and scaled by their standard
 * deviations, the 6 leading principal vectors unscaled into the columns of
 * A = [A_eps; A_sig] -- and C = sym(A_sig A_eps^-1), the slope of the
 * principal subspace read as a stiffness (on data lying on sig = C0 eps it
 * returns C0).
 *   strain_dev, stress_dev  device float64 [N][6] (borrowed), N >= 12
 *   C_out                   host float64 [36], row-major
 * Errors: DD_ERR_ARG (N, pointers, a component with zero variance, a singular
 * A_eps), DD_ERR_NOT_SPD (sym(A_sig A_eps^-1) not positive definite),
 * DD_ERR_DEVICE.  Synchronises hip_stream.
 */
dd_status dd_metric_pca(const double* strain_dev, const double* stress_dev, int64_t N,
                        double* C_out, void* hip_stream);

/* Thread-local message for the calling thread's last non-OK status. */
const char* dd_last_error(void);

/* Library version string. */
const char* dd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
