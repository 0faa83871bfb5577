// Kernels of the pMMF factorization (Alg. 1 with Alg. 2 inside), gfx950.
//
// Every stage works on the active matrix A_{p-1}[S_{p-1}, S_{p-1}] in CSR over "positions":
// position q is the q-th smallest global index still active at the start of the stage.  The
// stage's clusters are contiguous position ranges [off_u, off_u + c_u).
#pragma once

#include "common.h"

namespace pmmf {

// row stride of a cluster's c x c (G, D) array: even, so every row starts 16-byte aligned and a
// pair of adjacent entries moves in one 16-byte access
__host__ __device__ inline int gd_stride(int c) { return c + (c & 1); }

struct FindArgs {
  int p;                     // stage number, 1-based (enters the seed-row hash)
  int k;                     // 2 or 3
  int elims = 1;             // indices retired per rotation (2 only with k = 3)
  uint64_t seed;
  const int32_t* order;      // launch slot -> cluster id (largest clusters first)
  const int32_t* off;        // [m+1] cluster offsets (positions)
  const int32_t* rcnt;       // [m] log entries (retired indices) of each cluster
  const int32_t* roff;       // [m+1] first stage-local rotation of each cluster
  const int64_t* gbase;      // [m] offset of each cluster's (G, D) array in the pool
  float2* GD;                // (Gram, diagonal block) pool, interleaved
  const int32_t* gid;        // [S] global id of each position
  int64_t rot0;              // global index of the stage's first rotation
  int32_t* rot_loc;          // [R][3] cluster-local ids, slot order
  int32_t* rot_gid;          // [R][3] global ids, slot order
  float* rot_o;              // [R][9] k x k block (row-major, leading dim 3)
  int32_t* rot_ret;          // [R] retired global id
  float* rot_margin;         // [R] smallest relative decision margin
  double* rot_lit;           // [R] 2 off^2 of the retired index (literal loss term)
  float* hdiag;              // [n] retired diagonal of H
  uint8_t* retflag;          // [S] 1 if the position retires in this stage
  int32_t* err;              // set to 1 if a cluster finds no partner (never expected)
  int32_t* rot_lvl = nullptr;  // [R] level of each rotation in its cluster's dependency order
                               // (1 + the latest level touching one of its indices), if wanted
  // BF16 form only: FP32 slabs (column-major, R_u rows per cluster) for exact rescoring, and
  // counters {steps with more than one rescoring round, candidates rescored}
  float* slab = nullptr;
  const int64_t* slab_off = nullptr;
  const int32_t* slab_rows = nullptr;
  unsigned long long* sl_stats = nullptr;
};

}  // namespace pmmf

// launchers (factor_kernels.hip)
namespace pmmf {
hipError_t launch_fill_cluster_of(const int32_t* off, int m, int S, int32_t* cl_of, hipStream_t s);
// sparse Gram of the active matrix (rp_nnz entries)
hipError_t launch_gram(int S, int64_t rp_nnz, const int64_t* rp, const int32_t* ci,
                       const float* cv, const int32_t* off, const int32_t* cl_of,
                       const int64_t* gbase, const int64_t* run_ptr, const int32_t* run_cl,
                       const int64_t* run_start, float2* GD, int cmax, hipStream_t s,
                       int wpb = 0, int form = -1);
// multiply-adds of the stage's cluster Grams (sum over rows and runs of the run length squared),
// added to *out
hipError_t launch_gram_work(int S, const int64_t* rp, const int64_t* run_ptr,
                            const int64_t* run_start, unsigned long long* out, hipStream_t s);
hipError_t launch_runs(int S, int fill, const int64_t* rp, const int32_t* ci,
                       const int32_t* cl_of, int32_t* nruns, const int64_t* run_ptr,
                       int32_t* run_cl, int64_t* run_start, hipStream_t s);
hipError_t launch_gram_dense(int S, const int64_t* rp, const int32_t* ci, const float* cv,
                             float* dense, const int32_t* off, int m, const int64_t* gbase,
                             float2* GD, int cmax, hipStream_t s);
hipError_t launch_find(const FindArgs& a, int m, int cmax, int nt, hipStream_t s);
hipError_t launch_find_bf16(const FindArgs& a, int m, int cmax, hipStream_t s);
hipError_t launch_slab_rows(int S, int m, const int64_t* rp, const int32_t* ci,
                            const int32_t* cl_of, int64_t W, uint32_t* bm, int32_t* pre,
                            int32_t* R, hipStream_t s);
hipError_t launch_gram_bf16(int S, int m, const int64_t* rp, const int32_t* ci, const float* cv,
                            const int32_t* off, const int32_t* cl_of, int64_t W,
                            const uint32_t* bm, const int32_t* pre, const int64_t* slab_off,
                            const int32_t* R, int64_t slab_elems, float* slab,
                            unsigned short* slab_bf, const int64_t* gbase, float2* GD,
                            int cmax, hipStream_t s);
size_t find_lds_bytes(int cmax);
// levels of the stage's rotations (from lvl_in when the search recorded them, else walked here),
// the level pointers and the sweep log in level order
hipError_t launch_levelize(int m, int k, const int32_t* off, const int32_t* rcnt,
                           const int32_t* roff, int64_t rot0, const int32_t* rot_loc,
                           const float* rot_o, const int32_t* lvl_in, int lvl_stride,
                           int32_t* lvl_ptr, int32_t* depth, int32_t* sw_loc, float* sw_o,
                           int32_t* sw_idx, float* theta, int cmax, hipStream_t s);
// the clusters' accumulated rotations from the levelized sweep log: column j of Qbar_u (row j of
// Qbar^T, rows ascending) into the c_u scratch slots at gbase[u] + j c_u of sci/scv, its count to
// cnt[j]; launch_qt_compact packs them into the CSR of Qbar^T with row pointers rp
hipError_t launch_qsparse(int m, int k, const int32_t* off, const int64_t* gbase,
                          const int32_t* lvl_ptr, int lvl_stride, const int32_t* depth,
                          const int32_t* sw_loc, const float* sw_o, int32_t* cnt, int32_t* sci,
                          float* scv, int cmax, hipStream_t s);
hipError_t launch_qt_compact(int S, const int32_t* off, const int32_t* cl_of,
                             const int64_t* gbase, const int32_t* sci, const float* scv,
                             const int64_t* rp, int32_t* qci, float* qcv, hipStream_t s);
// each row of a CSR (distinct columns) in ascending column order, out of place
hipError_t launch_sort_rows(int n, const int64_t* rp, const int32_t* ci, const float* cv,
                            int32_t* oci, float* ocv, hipStream_t s);
// W = M Qbar^T, run by run of M's run table (run_ptr, run_cl, run_start as built by launch_runs);
// with fill = 1 it also records where each run r of row x starts in W's staging row:
// wrs[run_ptr[x] + r]
hipError_t launch_right(int S, int fill, const int64_t* rp, const int32_t* ci, const float* cv,
                        const int32_t* off, const int64_t* run_ptr, const int32_t* run_cl,
                        const int64_t* run_start, const int64_t* qrp, const int32_t* qci,
                        const float* qcv, int32_t* cnt, const int64_t* orp, int32_t* oci,
                        float* ocv, int64_t* wrs, int cmax, hipStream_t s);
// A_p = Qbar W with peeling; W's rows are runs as recorded by launch_right (run table run_ptr,
// run_cl of M, starts wrs)
hipError_t launch_left(int S, int fill, const int64_t* qrp, const int32_t* qci, const float* qcv,
                       const int64_t* wrp, const int32_t* wcnt, const int32_t* wci,
                       const float* wcv, const int64_t* run_ptr, const int32_t* run_cl,
                       const int64_t* wrs,
                       const int32_t* off, const int32_t* cl_of, const int32_t* next,
                       int32_t* cnt, const int64_t* orp, int32_t* oci, float* ocv,
                       double* loss_row, int32_t* overflow, int cmax, hipStream_t s);
hipError_t launch_bound_right(int S, const int64_t* rp, const int32_t* ci, const int64_t* qrp,
                              int64_t cap, int32_t* ub, hipStream_t s);
hipError_t launch_bound_left(int S, const int64_t* qrp, const int32_t* qci, const int32_t* wcnt,
                             const int32_t* next, int64_t cap, int32_t* ub, hipStream_t s);
hipError_t launch_compact_rows(int64_t n, const int64_t* sb, const int32_t* cnt,
                               const int32_t* sci, const float* scv, const int64_t* rp,
                               int32_t* ci, float* cv, hipStream_t s);
hipError_t launch_next_positions(int S, const uint8_t* retflag, const int64_t* scan,
                                 const int32_t* gid, int32_t* next, int32_t* gid_new,
                                 hipStream_t s);
hipError_t launch_keep_flags(int S, const uint8_t* retflag, int32_t* keep, hipStream_t s);
hipError_t launch_scan(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// boundary cut counts of the active matrix (data-driven clustering): d (S + 2 ints) is scratch,
// w (S + 2 int64) receives at w[b + 1] the number of entries (i, j), i < j, with i < b <= j
hipError_t launch_cut_counts(int S, const int64_t* rp, const int32_t* ci, int32_t* d, int64_t* w,
                             int64_t* tmp, hipStream_t s);
// CSR transpose of an n x n matrix (rows of the result in arbitrary entry order): cnt (n ints) and
// cursor (n int64) are scratch, tmp as for launch_scan; trp receives n + 1 row pointers
hipError_t launch_csr_transpose(int n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                                const float* cv, int32_t* cnt, int64_t* trp, int64_t* tmp,
                                int64_t* cursor, int32_t* tci, float* tcv, hipStream_t s);
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_sum_double(const double* in, int64_t n, double* out, hipStream_t s);
hipError_t launch_csr_stats(int64_t n, const int64_t* rp, const int32_t* ci, const float* cv,
                            int check_sym, double* fro2_trace, int32_t* flags, hipStream_t s);
hipError_t launch_core_dense(int S, const int64_t* rp, const int32_t* ci, const float* cv,
                             float* hcore, hipStream_t s);
hipError_t launch_h_stats(int64_t n, const float* hdiag, int64_t core, const float* hcore,
                          double* out, hipStream_t s);
hipError_t launch_copy_csr(int64_t n, const int64_t* rp, const int32_t* ci, const float* cv,
                           int64_t* orp, int32_t* oci, float* ocv, hipStream_t s);
hipError_t launch_iota(int32_t* a, int64_t n, hipStream_t s);
}  // namespace pmmf
