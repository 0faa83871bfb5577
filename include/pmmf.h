/*
 * pmmf.h — C ABI of the MI355X (gfx950) pMMF library.
 *
 * Parallel Multiresolution Matrix Factorization (Kondor, Teneva & Mudrakarta, "Parallel MMF: a
 * Multiresolution Approach to Matrix Computation"): a symmetric A in R^{n x n} is factored as
 *     A ~ U^T H U,   U = Qbar_P ... Qbar_1                               (Sec. 2, Eq. 1 and Eq. 4)
 * where each stage Qbar_p is a product of Givens (k = 2) or 3-point (k = 3) rotations that is
 * block diagonal in that stage's clustering (Def. 1), and H is core-diagonal: a dense core on the
 * final active set plus the diagonal entries of the retired ("wavelet") indices.
 *
 * Conventions shared by every call:
 *   - All functions return int: MMF_OK (0) or a negative MMF_E* code; no C++ exception crosses
 *     the ABI.  mmf_last_error() returns a thread-local message for the last failure.
 *   - Pointers prefixed d_ are device pointers (HIP global memory on the current device); all
 *     other pointers are host pointers.  Inputs are borrowed for the duration of the call; outputs
 *     are caller-allocated.  Work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *   - Matrices are 0-based CSR: int64 row pointers [n+1], int32 column indices (strictly ascending
 *     within each row) and float32 values [nnz], both triangles present.  Dense blocks of vectors are row-major [n][ld] float32 with
 *     ld >= nrhs, so a rotation of indices (i, j) touches two contiguous rows.
 *   - Global indices (retired ids, core ids, rotation ids) are row numbers of A.
 *   - A handle is not safe for concurrent use on two streams.  Device faults surface as
 *     MMF_EDEVICE at the next synchronizing call.
 */
#ifndef PMMF_H
#define PMMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MMF_OK = 0,
  MMF_EINVAL = -1,      /* bad size, k, eta, core size or cluster bounds                        */
  MMF_ENOTSYM = -2,     /* MMF_CHECK_SYMMETRY was set and A is not exactly symmetric            */
  MMF_ENONFINITE = -3,  /* NaN or Inf in the input                                              */
  MMF_ENOMEM = -4,      /* device allocation failed                                            */
  MMF_EDEVICE = -5,     /* a HIP runtime error; its text is in mmf_last_error()                 */
  MMF_ESINGULAR = -6,   /* H cannot be inverted: a zero retired diagonal or a core that is not
                           positive definite                                                    */
  MMF_ESTATE = -7,      /* NULL or destroyed handle, or a call that does not fit its state     */
  MMF_ECAPACITY = -8    /* a fixed device capacity was exceeded (message names it)             */
};

/* flags */
#define MMF_CHECK_SYMMETRY   0x1u  /* verify A == A^T on the device before factoring            */
#define MMF_EVEN_CLUSTERS    0x2u  /* round every cluster size but the last down to even (tests) */
#define MMF_CUT_CLUSTERS     0x4u  /* data-driven clustering (Alg. 1 "cluster"): contiguous clusters
                                      with sizes in [cluster_min, cluster_max] whose boundaries
                                      separate the fewest entries of the stage's active matrix,
                                      chosen at the start of each stage; excludes
                                      MMF_EVEN_CLUSTERS                                          */
#define MMF_TWO_ELIMINATIONS 0x8u  /* k = 3 only: each rotation retires its two slots with the
                                      smallest off-diagonal norms (Sec. 2: a k-point rotation may
                                      set several wavelets), so a cluster retiring r_u indices
                                      takes ceil(r_u / 2) rotations; the log keeps one entry per
                                      retired index, a rotation's second retirement as the next
                                      entry on the same tuple with the identity block.  FP32 Gram
                                      form only (MMF_EINVAL with gram_mode 1 or k = 2)          */

/* Factorization parameters (Sec. 2, Alg. 1 and Alg. 2). */
typedef struct {
  int32_t  k;            /* rotation order: 2 (Givens) or 3 (3-point rotations), Sec. 2 item 1  */
  double   eta;          /* fraction of the active set retired per stage, in (0, 0.5] (Alg. 2's
                            "compression ratio"): stage p performs
                            t_p = min(|S| - core_size, floor(eta |S|)) rotations               */
  int64_t  core_size;    /* delta_L, size of the dense core of H, 1 <= core_size <= n            */
  int32_t  cluster_min;  /* lo, hi: random uneven cluster sizes in [lo, hi], hi >= 2 lo >= 4;   */
  int32_t  cluster_max;  /* (0, 0) = one cluster per stage (plain MMF).  Sec. 2.1 clustering     */
  uint64_t seed;         /* drives the random seed rows (Alg. 2) and the cluster sizes          */
  int32_t  gram_mode;    /* 0 = FP32 cluster Gram; 1 = Gram of the BF16-rounded column slab on
                            the matrix cores (FP32 accumulation) used to shortlist partners, the
                            pick and G[T,T] then taken from exact FP32 dots of the slab columns,
                            which every rotation right-rotates (Sec. 2.1 Gram, Alg. 2 scores)    */
  uint32_t flags;        /* MMF_* flags above                                                   */
} mmf_params;

typedef struct mmf_plan* mmf_handle;

typedef struct {
  int64_t n;             /* dimension of A                                                      */
  int64_t core_size;     /* delta_L                                                             */
  int32_t k;             /* rotation order                                                      */
  int32_t num_stages;    /* P                                                                   */
  int64_t num_rotations; /* n - delta_L (one index retired per rotation)                         */
  int64_t max_clusters;  /* largest number of clusters in any stage                             */
  double  loss;          /* exact residual ||A - U^T H U||_F^2 = 2 sum_e m_e, FP64 accumulation   */
  double  loss_literal;  /* sum over retirements of 2 off^2 (an upper bound of loss)            */
  double  fro2_a;        /* ||A||_F^2, FP64 accumulation                                        */
  double  fro2_h;        /* ||H||_F^2, FP64 accumulation; loss ~ fro2_a - fro2_h                */
  double  trace_a;       /* trace(A); trace(H) equals it up to rounding                         */
  double  trace_h;
  double  factor_ms;     /* device time of mmf_factor measured with HIP events                  */
} mmf_info;

typedef struct {
  int64_t size;          /* |S_{p-1}|: active indices at the start of the stage                 */
  int64_t rotations;     /* t_p                                                                 */
  int64_t clusters;      /* m_p                                                                 */
  int64_t nnz;           /* nonzeros of the stage's active matrix A_{p-1}[S_{p-1}, S_{p-1}]     */
  int64_t max_cluster;   /* largest cluster of the stage                                        */
  int32_t max_depth;     /* deepest chain of dependent rotations inside one cluster             */
  int32_t dense_gram;    /* 1 if the stage's Gram took a dense matrix-core form (FP32: fill >=
                            0.1 and at most 16384 active rows; BF16 mode: always), 0 for the
                            sparse row-merge form                                              */
  double  loss;          /* residual contributed by this stage's retirements (FP64)             */
  double  gram_ms;       /* device time of the cluster Gram / diagonal-block kernel             */
  double  find_ms;       /* device time of the greedy rotation search (all clusters, one launch) */
  double  rotate_ms;     /* device time of levelling, Qbar extraction and the two-sided rotation
                            with peeling                                                         */
  int64_t find_bytes;    /* algorithmic bytes of the greedy search: per rotation in a cluster of
                            c, the seed's Gram row, then k rows and k columns of the Gram and of
                            the diagonal block read and written: 4c + 16kc + 16kc = 4c (1 + 8k)  */
  int64_t bf16_long;     /* BF16 mode: steps with more than 64 shortlisted partners (rescored in
                            several rounds)                                                      */
  int64_t bf16_rescored; /* BF16 mode: candidates rescored with exact FP32 dots (all steps)       */
  double  gram_flops;    /* flops the stage's Gram kernel performs: the matrix-core tiles of the
                            dense and BF16 forms (upper triangle, padded), else as below          */
  double  gram_useful_flops; /* flops the cluster Grams need: 2 sum over rows and clusters of the
                            row's entry count in the cluster squared (Sec. 2.1 Gram on a sparse
                            slab)                                                               */
} mmf_stage_info;

/*
 * mmf_factor — Alg. 1 with Alg. 2 inside.  For each stage: cluster the active set, form every
 * cluster's Gram matrix and diagonal block, run the randomized greedy rotation search in each
 * cluster, rotate the active matrix from both sides with the stage's rotations, and peel the
 * retired rows and columns into H.  H's core is the final active block.
 *   n, nnz, d_rowptr, d_colind, d_val : A in CSR (device), exactly symmetric.
 *   p      : parameters (host, borrowed).
 *   out    : receives a new handle owning all device state of the factorization.
 * Synchronizes `stream` once per stage (to size the next stage's sparse storage) and at the end.
 * Errors: MMF_EINVAL, MMF_ENOTSYM, MMF_ENONFINITE, MMF_ENOMEM, MMF_EDEVICE, MMF_ECAPACITY.
 */
int mmf_factor(int64_t n, int64_t nnz, const int64_t* d_rowptr, const int32_t* d_colind,
               const float* d_val, const mmf_params* p, void* stream, mmf_handle* out);

/*
 * mmf_apply — matrix-free product Y = U^T H U X (Sec. 2.4): the stages' rotations in order, the
 * retired diagonal and the dense core of H, then the transposed rotations in reverse order.
 *   d_x : [n][ld] input (device, read only); d_y : [n][ld] output (device), may not alias d_x.
 * Asynchronous on `stream`.  Errors: MMF_ESTATE, MMF_EINVAL, MMF_ENOMEM, MMF_EDEVICE.
 */
int mmf_apply(mmf_handle h, const float* d_x, float* d_y, int64_t nrhs, int64_t ld, void* stream);

/*
 * mmf_apply_inverse — Y = U^T H^{-1} U X (Sec. 2.4, inversion): reciprocal retired diagonal and
 * the inverse of the core (an FP32 Cholesky factor computed on first use and kept).
 * Errors as mmf_apply, plus MMF_ESINGULAR.
 */
int mmf_apply_inverse(mmf_handle h, const float* d_x, float* d_y, int64_t nrhs, int64_t ld,
                      void* stream);

/*
 * mmf_apply_inverse_sqrt — Y = U^T H^{-1/2} U X = A~^{-1/2} X (the xi = 1/2 power of Sec. 4's
 * preconditioner A~^{-xi}, as used for split-symmetric preconditioning): reciprocal square roots
 * of the retired diagonal, and V diag(lambda^{-1/2}) V^T for the core from its FP64 symmetric
 * eigendecomposition (rocSOLVER dsyevd on first use, kept until the parameters change).
 * Errors as mmf_apply, plus MMF_ESINGULAR (a retired entry <= 0 or a core eigenvalue <= 0).
 */
int mmf_apply_inverse_sqrt(mmf_handle h, const float* d_x, float* d_y, int64_t nrhs, int64_t ld,
                           void* stream);

/*
 * mmf_backward — adjoint of Y = U^T H U X (from Eq. 1; the paper has no gradient) given Ybar:
 *   d_xbar      [n][ld]         = U^T H^T U Ybar
 *   d_hdiag_bar [n]             : sum over columns of (U Ybar)_e (U X)_e on retired e (0 on core)
 *   d_hcore_bar [core][core]    : (U Ybar)_core (U X)_core^T, row-major
 *   d_theta_bar                 : d<Ybar, Y>/d theta in the layout of mmf_param_ptrs, in the
 *                                 order of mmf_export: [num_rotations] Givens angles (k = 2) or
 *                                 [num_rotations][3] angles of the 3-point rotations (k = 3)
 * Any of the four outputs may be NULL to skip it.  Stage states are recomputed by undoing
 * rotations, not stored.  Asynchronous.  Errors: MMF_ESTATE, MMF_EINVAL, MMF_ENOMEM, MMF_EDEVICE.
 */
int mmf_backward(mmf_handle h, const float* d_x, const float* d_ybar, float* d_xbar,
                 float* d_hdiag_bar, float* d_hcore_bar, float* d_theta_bar, int64_t nrhs,
                 int64_t ld, void* stream);

/*
 * Captured products (batching of Sec. 2.3 / Table 1's many small operations into one launch):
 * mmf_graph_capture records one mmf_apply (inverse = 0), mmf_apply_inverse (inverse = 1) or
 * mmf_apply_inverse_sqrt (inverse = 2) from
 * d_x to d_y ([n][ld], device, fixed for the graph's life) as a HIP graph.  It first runs the
 * product eagerly on `stream` (so d_y holds the result and every size-dependent preparation is
 * done) and synchronizes it; the graph contains kernel nodes only and owns its own workspace.
 * mmf_graph_launch replays it on `stream` (asynchronous); it reads d_x and the handle's current
 * rotations and H, and writes d_y.  A graph of an inverse is refused (MMF_ESTATE) once theta or H
 * have changed (mmf_set_params, mmf_sync_angles), since it holds the core factor of capture time.
 * Launching after mmf_destroy of its factorization, or after mmf_graph_destroy, is MMF_ESTATE.
 * mmf_graph_destroy waits for the device and frees the graph.  Errors: MMF_EINVAL, MMF_ESTATE,
 * MMF_ESINGULAR (inverse), MMF_ENOMEM, MMF_EDEVICE.
 */
typedef struct mmf_graph_s* mmf_graph;
int mmf_graph_capture(mmf_handle h, int32_t inverse, const float* d_x, float* d_y, int64_t nrhs,
                      int64_t ld, void* stream, mmf_graph* out);
int mmf_graph_launch(mmf_graph g, void* stream);
int mmf_graph_destroy(mmf_graph g);

/* Summary of a finished factorization (host struct).  Errors: MMF_ESTATE. */
int mmf_get_info(mmf_handle h, mmf_info* out);

/* Per-stage summary, stage in [0, num_stages).  Errors: MMF_ESTATE, MMF_EINVAL. */
int mmf_get_stage_info(mmf_handle h, int32_t stage, mmf_stage_info* out);

/*
 * mmf_export — copy the factorization to caller-allocated host arrays (any may be NULL):
 *   rot_ids     int32 [num_rotations][k]   global ids, slot order (seed row first)
 *   rot_o       float [num_rotations][k][k] rotation block O: x[ids] <- O x[ids]
 *   rot_retired int32 [num_rotations]      global id eliminated by each rotation
 *   rot_margin  float [num_rotations]      smallest relative decision margin of the step
 *   hdiag       float [n]                  retired diagonal of H (0 on core indices)
 *   core_ids    int32 [core_size]          ascending global ids of the core
 *   hcore       float [core_size][core_size]
 * Rotations are ordered by stage, then cluster, then step.  Synchronizes the handle's stream.
 */
int mmf_export(mmf_handle h, int32_t* rot_ids, float* rot_o, int32_t* rot_retired,
               float* rot_margin, float* hdiag, int32_t* core_ids, float* hcore);

/*
 * mmf_import — build a handle for mmf_apply / mmf_apply_inverse / mmf_backward from a host-side
 * factorization in the mmf_export layout plus its stage geometry:
 *   n, k, core_size, num_stages
 *   stage_sizes    int64 [num_stages]      |S_{p-1}|
 *   stage_clusters int64 [num_stages]      m_p
 *   cluster_sizes  int64 [sum m_p]         sizes of the contiguous clusters, stage by stage
 *   rotation arrays as in mmf_export (rot_margin may be NULL), hdiag, core_ids, hcore.
 * The active set of each stage is derived from the retirements.  Errors: MMF_EINVAL, MMF_ENOMEM,
 * MMF_EDEVICE.
 */
int mmf_import(int64_t n, int32_t k, int64_t core_size, int32_t num_stages,
               const int64_t* stage_sizes, const int64_t* stage_clusters,
               const int64_t* cluster_sizes, const int32_t* rot_ids, const float* rot_o,
               const int32_t* rot_retired, const float* hdiag, const int32_t* core_ids,
               const float* hcore, void* stream, mmf_handle* out);

/*
 * mmf_param_ptrs — device pointers to the handle-owned parameters used by apply and backward:
 *   theta   k = 2: [num_rotations] Givens angles, O_t = [[cos, -sin], [sin, cos]];
 *           k = 3: [num_rotations][3] angles w_t with O_t = expm(w_0 G_01 + w_1 G_02 + w_2 G_12) O0_t,
 *           G_pq = E_qp - E_pq the generator of the (p, q) plane of the rotation's slots and O0_t
 *           the rotation the search found (w = 0 after mmf_factor and mmf_import; the paper
 *           gives angles only for Givens rotations, this extends them to its k-point rotations);
 *   hdiag [n], hcore [core][core].
 * They may be updated in place (e.g. by an optimizer); after changing theta call
 * mmf_sync_angles so the rotations use the new angles.  Errors: MMF_ESTATE.
 */
int mmf_param_ptrs(mmf_handle h, float** theta, float** hdiag, float** hcore);

/* Recompute every rotation from theta (k = 2: (cos, sin); k = 3: expm(W(w_t)) O0_t by Rodrigues'
 * formula in FP64), on `stream`.  Also drops the cached core factor used by mmf_apply_inverse.
 * Errors: MMF_ESTATE, MMF_EDEVICE. */
int mmf_sync_angles(mmf_handle h, void* stream);

/*
 * mmf_get_params — copy the handle's parameters into caller device buffers, on `stream` (the
 * layouts of mmf_param_ptrs: theta [R] or [R][3], hdiag [n], hcore [core][core]); any may be NULL.
 * Errors: MMF_ESTATE, MMF_EDEVICE.
 */
int mmf_get_params(mmf_handle h, float* d_theta, float* d_hdiag, float* d_hcore, void* stream);

/*
 * mmf_set_params — copy new parameters from caller device buffers into the handle, on `stream`:
 *   d_theta (layout of mmf_param_ptrs), d_hdiag [n], d_hcore [core][core]; any may be NULL.
 * Recomputes the rotations from theta when it is given and drops the cached core factor.
 * Used by gradient refinement of the angles (the parameters of y = U^T H U x).
 * Errors: MMF_ESTATE, MMF_EDEVICE.
 */
int mmf_set_params(mmf_handle h, const float* d_theta, const float* d_hdiag, const float* d_hcore,
                   void* stream);

/* Result of mmf_pcg. */
typedef struct {
  int32_t iterations;        /* inner PCG iterations (all columns advance together)            */
  int32_t refinements;       /* FP64 residual corrections performed                            */
  int32_t converged;         /* columns with ||b_j - A x_j|| / ||b_j|| <= tol                  */
  int32_t pad;
  double  max_rel_residual;  /* max over columns of the FP64 relative residual at return        */
  double  solve_ms;          /* device time of the solve                                       */
} mmf_pcg_info;

/*
 * mmf_pcg — solve A X = B by conjugate gradients preconditioned with the factorization's inverse
 * A~^{-1} = U^T H^{-1} U (Sec. 4: pMMF as a preconditioner), all columns in lockstep.  Inner
 * iterations run in FP32 (CSR SpMM, mmf_apply_inverse, per-column dot products accumulated in FP64)
 * on A d = r / ||r|| until every active column's residual drops by `inner_reduction`; an outer loop
 * recomputes r = B - A X in FP64 and adds the correction to the FP64 solution, until
 * ||b_j - A x_j|| / ||b_j|| <= tol for every column or max_iter inner iterations in total.
 *   h       : factorization of (an approximation of) A, dimension n
 *   A       : CSR (device), the matrix of the system (the one that was factored)
 *   d_b     : [n][nrhs] float32 right-hand sides (device);  d_x : [n][nrhs] float64 solution (device)
 * The preconditioner product is captured once per call as a graph (mmf_graph_capture) and replayed.
 * Synchronizes `stream` once per inner iteration.  Errors: MMF_EINVAL, MMF_ESTATE, MMF_ENOMEM,
 * MMF_ESINGULAR (H not invertible), MMF_EDEVICE.
 */
int mmf_pcg(mmf_handle h, int64_t n, const int64_t* d_rowptr, const int32_t* d_colind,
            const float* d_val, const float* d_b, double* d_x, int64_t nrhs, double tol,
            int32_t max_iter, double inner_reduction, void* stream, mmf_pcg_info* out);

/*
 * mmf_pcg_split — the same solve in the split-symmetric form of Sec. 4: the inner iterations run
 * plain CG on the symmetric (M^{-1/2} A M^{-1/2}) y = M^{-1/2} r with M^{-1/2} = A~^{-1/2}
 * (mmf_apply_inverse_sqrt, two applications per iteration, both replayed as captured graphs) and
 * set d = M^{-1/2} y; the inner loop stops once every active column's ||M^{-1/2} (r - A d)|| has
 * dropped by `inner_reduction`, and the outer FP64 correction is as in mmf_pcg.  Requires H
 * positive definite (MMF_ESINGULAR otherwise).  Arguments, result and errors as mmf_pcg.
 */
int mmf_pcg_split(mmf_handle h, int64_t n, const int64_t* d_rowptr, const int32_t* d_colind,
                  const float* d_val, const float* d_b, double* d_x, int64_t nrhs, double tol,
                  int32_t max_iter, double inner_reduction, void* stream, mmf_pcg_info* out);

/*
 * mmf_spmm — Y = A X for a CSR matrix (device) and row-major [n][ld] blocks X, Y (device, no
 * aliasing).  The product that the factorization approximates (Sec. 2.4 uses A~ v in its place);
 * angle refinement contrasts it with mmf_apply on random probes, ||A x - A~ x||^2 being an
 * unbiased estimate of the objective ||A - A~||_F^2 of Eq. 1 for x ~ N(0, I).
 * One wave per row, one lane per column; each row's nonzeros are summed in ascending order.
 * Asynchronous on `stream`.  Errors: MMF_EINVAL, MMF_EDEVICE.
 */
int mmf_spmm(int64_t n, const int64_t* d_rowptr, const int32_t* d_colind, const float* d_val,
             const float* d_x, float* d_y, int64_t nrhs, int64_t ld, void* stream);

/*
 * mmf_apply_noalloc — y = A~ x exactly as mmf_apply computes it, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid it):
 * it calls no hipMalloc, hipFree or allocating library routine.  The two blocks of compacted
 * vectors the sweeps pass between stages live in one fixed 64 MiB array of the library's device
 * code (each device keeps its own copy until the process ends): 2 |S_1| nrhs floats must fit in
 * 2^24, |S_1| the number of indices active after the first stage (MMF_ECAPACITY otherwise).
 * The array keeps the last call's contents (every call overwrites what it reads); calls that
 * overlap on one device race on it, so serialize them (one stream, or events).
 * The handle's sweep plan must exist: it is built by the first mmf_apply, mmf_apply_inverse or
 * mmf_graph_capture on the handle (MMF_ESTATE before that).  Arguments, layout and errors as
 * mmf_apply otherwise.  Asynchronous on `stream`.
 */
int mmf_apply_noalloc(mmf_handle h, const float* d_x, float* d_y, int64_t nrhs, int64_t ld,
                      void* stream);

/*
 * mmf_set_tail_rows — how the products (mmf_apply, mmf_apply_inverse, mmf_apply_inverse_sqrt,
 * mmf_apply_noalloc and graphs captured afterwards) run the last stages of U and U^T (Sec. 2.4):
 * the trailing stages whose first active set has at most `rows` rows, all of whose rotation
 * components have at most 32 rows, and whose rows and programs fit one workgroup's LDS, run as
 * one launch per direction that keeps each column's active rows on chip between stages (at most
 * 16 stages and 8192 rows; fewer than two such stages: none).  `rows` caps the threshold the
 * library itself takes (the fastest of 0, 2048, 4096 and 8192 when autotuning is on, else 4096);
 * rows = 0 runs every stage as its own launch.  The default cap is 8192.  Results are the same
 * either way (same arithmetic, same order).  Errors: MMF_ESTATE (bad handle), MMF_EINVAL (rows < 0).
 */
int mmf_set_tail_rows(mmf_handle h, int64_t rows);

/* Free the handle and all device memory it owns (synchronizes its stream). */
int mmf_destroy(mmf_handle h);

/* Device memory of every later allocation of the library (handles, workspaces, PCG buffers):
 *   alloc(bytes, stream, ctx) returns device memory for use on `stream` (NULL on failure, reported
 *   as MMF_ENOMEM); release(ptr, stream, ctx) takes back a block with the stream it was allocated
 *   for.  The library waits for the device before it releases a block (as hipFree does), so an
 *   allocator that reuses memory in stream order (e.g. a caching allocator) never hands out memory
 *   still in use on another stream.  Blocks keep the allocator that produced them: a later call
 *   does not change how existing blocks are released.  Both NULL restores the default allocator
 *   (hipMalloc with released blocks kept for reuse, see mmf_trim).
 *   Process-wide; set it before creating handles that should use it.
 *   Errors: MMF_EINVAL when exactly one of alloc and release is NULL. */
int mmf_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                      void (*release)(void* ptr, void* stream, void* ctx), void* ctx);

/* Free the device blocks that the default allocator keeps for reuse (waits for the device).
 * Without a caller's allocator the library allocates with hipMalloc and keeps each released
 * block, up to 64 GiB per process: a later allocation of at most its size (and at least half of
 * it) on the same device takes it back, at once on the stream that released it, on another stream
 * after a device synchronization.  Handles and buffers in use are not affected.  Always MMF_OK. */
int mmf_trim(void);

/* Thread-local text of the last error reported on this thread ("" if none). */
const char* mmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMMF_H */
