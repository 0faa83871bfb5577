// Matrix-free sweeps over the factorization's stages and the small dense core kernels.
#pragma once

#include "common.h"

namespace pmmf {

// One stage of the factorization as the sweeps see it.
struct SweepStage {
  int m;                     // clusters
  int k;                     // rotation order
  int cmax;                  // largest cluster
  int rmax;                  // most rotations in one cluster
  int lvl_stride;            // row stride of lvl_ptr
  const int32_t* off;        // [m+1] cluster offsets (positions of S_{p-1})
  const int32_t* lvl_ptr;    // [m][lvl_stride] stage-local index where each level starts
  const int32_t* depth;      // [m] number of levels
  const int32_t* sw_loc;     // [t][k] cluster-local ids, level order
  const float* sw_o;         // [t][k*k] rotation blocks, level order
  const int32_t* next;       // [S] next-stage position, or -(gid + 1) if the row retires here
  const int32_t* gid;        // [S] global id of each position
  const int32_t* sw_idx;     // [t] canonical index of each sweep-log rotation
  int64_t rot_base;          // canonical index of the stage's first rotation
  const int32_t* clist;      // clusters to process (NULL: all m); grid.x = number of entries
};

// The same stage split into "units": whole connected components of the rotation graph (rows
// linked by a rotation), packed up to UNIT_MAX rows.  A unit's rotations touch only its rows, so
// one wave applies them in order to a 64-column slice held in its registers, with no barrier.
// Every unit has UNIT_MAX row slots and UNIT_MAX rotation slots (a unit of c rows carries at most
// c - 1 rotations, one retirement each), so a wave reads its whole description in one step.
constexpr int UNIT_MAX = 32;
struct UnitStage {
  int nu;                    // units
  int k;
  const int2* cnt;           // [nu] {rows, rotations}
  const int4* slot;          // [nu][UNIT_MAX] {position in S_{p-1}, next position or -(gid + 1),
                             //                 gid, 0}
  const int2* rot;           // [nu][UNIT_MAX] {unit-local slots, 5 bits each, slot a at bit 5a;
                             //                 canonical rotation index}
  const float* rot_o;        // canonical blocks [R][9], leading dimension 3
  int64_t rot_base;          // canonical index of the stage's first rotation
};

// The trailing stages, whose active sets are small, as one launch per direction.  A workgroup
// owns one column of the vector block and keeps that column of the whole active set in LDS from
// the first trailing stage to the core: each stage's rows sit in unit order (unit u's rows at
// consecutive slots), one thread walks one unit's rotations, and between stages the survivors
// move to their slots of the next stage.  A stage's program is one contiguous block of device
// memory, [nu + 1] {first slot, first rotation} per unit, then [t] unit-local slots (5 bits each,
// slot a at bit 5a), then [t][k*k] rotation blocks (each part 16-byte aligned); it is copied into
// LDS by direct-to-LDS loads while the stage before it is computed.
constexpr int TAIL_MAX_STAGES = 16;
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_J = 8;  // slots per thread: a trailing stage has at most TAIL_THREADS * TAIL_J rows
struct TailStage {
  int rows;           // |S_{p-1}|
  int t;              // rotations
  int nu;             // units
  int blob_bytes;     // size of the program block (a multiple of 16)
  int64_t blob_off;   // byte offset of the block in TailPlan::blob
  int64_t slot_off;   // offset of the stage's per-slot entries in trans, pos, gid
};
struct TailPlan {
  int nst = 0;        // trailing stages (0: none)
  int data_bytes = 0; // LDS bytes of the rows (first stage's rows, 16-byte aligned)
  int lds_bytes = 0;  // data_bytes + the largest pair of consecutive program blocks
  const uint8_t* blob = nullptr;
  const int32_t* trans = nullptr;  // per slot: >= 0 the slot in the next stage (last stage: the
                                   // position in the core's compact rows), < 0: -(gid + 1)
  const int32_t* pos = nullptr;    // per slot: position in S_{p-1}
  const int32_t* gid = nullptr;    // per slot: global id
  TailStage st[TAIL_MAX_STAGES];
};
// program block layout shared by the host that builds it and the kernels that read it
__host__ __device__ inline int tail_prog_off(int nu) { return 8 * (nu + 1); }
__host__ __device__ inline int tail_o_off(int nu, int t) {
  return (tail_prog_off(nu) + 4 * t + 15) & ~15;
}
__host__ __device__ inline int tail_blob_bytes(int nu, int t, int k) {
  return (tail_o_off(nu, t) + 4 * t * k * k + 15) & ~15;
}

struct FwdIO {
  const float* src[2];       // compact rows of S_{p-1}
  int64_t ld_src;
  float* dst_c[2];           // compact rows of S_p
  int64_t ld_c;
  float* dst_nat[2];         // natural rows (retired rows of this stage)
  int64_t ld_nat;
  int mode[2];               // retired rows: 0 copy, 1 times hdiag, 2 divided by hdiag,
                             // 3 divided by sqrt(hdiag)
  const float* hdiag;
  int64_t nrhs;
};

struct RevIO {
  const float* src_c[2];     // compact rows of S_p (survivors)
  int64_t ld_c;
  const float* src_nat[2];   // natural rows (this stage's retired rows)
  int64_t ld_nat;
  int mode[2];               // retired rows on load: 0 copy, 1 times hdiag
  const float* hdiag;
  float* dst_c[2];           // compact rows of S_{p-1} (NULL: do not write)
  int64_t ld_out;
  float* dst_nat[2];         // if set: write natural rows instead (first stage)
  int64_t ld_dnat;
  int64_t nrhs;
  float* theta_part;         // [theta_tiles][theta_stride] per-tile angle-gradient partials; a
  int64_t theta_stride;      // launch with fewer column tiles writes zeros into the rows past
  int theta_tiles;           // its own, so the buffer needs no clearing
};

size_t sweep_lds_bytes(int k, int W, int nv, int cmax, int rmax);
// trailing stages of U (from the compact rows io.src[v] to the core's compact rows io.dst_c[v],
// retired rows to io.dst_nat[v] scaled by io.mode[v]; v = 0, and v = 1 too if io.src[1] is set)
// and of U^T (from the core's rows
// io.src_c[0] and the retired rows io.src_nat[0], which are copied (mode 0 only), to the compact
// rows io.dst_c[0] of the first trailing stage or, if io.dst_nat[0] is set, to natural rows);
// one vector (U^T), grid = nrhs workgroups per vector
hipError_t launch_tail_fwd(int k, const TailPlan& tp, const FwdIO& io, hipStream_t s);
hipError_t launch_tail_rev(int k, const TailPlan& tp, const RevIO& io, hipStream_t s);
// the rotation blocks of the program blocks from the canonical blocks: entry e of the programs
// (canonical rotation idx[e]) at float offset dst[e] of the blob
hipError_t launch_tail_params(int64_t n, int k, const int32_t* idx, const int64_t* dst,
                              const float* rot_o, uint8_t* blob, hipStream_t s);
// wpb: waves (units) per workgroup, 1, 2 or 4
hipError_t launch_unit_fwd(const UnitStage& st, const FwdIO& io, int nv, int wpb, hipStream_t s);
// io2: a second, independent pass over the same stage in the same launch (same nrhs)
hipError_t launch_unit_rev(const UnitStage& st, const RevIO& io, int nv, bool theta, int wpb,
                           hipStream_t s, const RevIO* io2 = nullptr);
hipError_t launch_sweep_fwd(const SweepStage& st, const FwdIO& io, int W, int nv, hipStream_t s);
hipError_t launch_sweep_rev(const SweepStage& st, const RevIO& io, int W, int nv, bool theta,
                            hipStream_t s);
hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int ta, const float* B,
                       int ldb, int tb, float* C, int ldc, float beta, hipStream_t s);
// up to three independent products of launch_gemm's form in one launch
struct GemmArgs {
  int M, N, K;
  const float* A;
  int lda, ta;
  const float* B;
  int ldb, tb;
  float* C;
  int ldc;
  float beta;
};
hipError_t launch_gemm_batch(int n, const GemmArgs* args, hipStream_t s);
hipError_t launch_core_inverse(int n, float* work_L, float* work_X, float* out_inv,
                               int64_t nfull, const float* hdiag, const uint8_t* is_core,
                               int32_t* status, hipStream_t s);
hipError_t launch_check_hdiag_pos(int64_t n, const float* hdiag, const uint8_t* is_core,
                                  int32_t* status, hipStream_t s);
hipError_t launch_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s);
hipError_t launch_isqrt_assemble(int n, const double* V, const double* lam, float* out,
                                 int32_t* status, hipStream_t s);
hipError_t launch_rowdot(int64_t n, const float* a, const float* b, int64_t ld, int64_t nrhs,
                         const uint8_t* is_core, float* out, hipStream_t s);
hipError_t launch_theta_reduce(int t, int ntiles, int64_t stride, const float* pa,
                               const float* pb, int64_t rot_base, float* out, hipStream_t s);
hipError_t launch_gather_rows(int64_t rows, const float* src, int64_t lds, const int32_t* idx,
                              float* dst, int64_t ldd, int64_t ncol, int scatter, hipStream_t s);
hipError_t launch_sync_angles(int64_t R, const float* theta, float* rot_o, hipStream_t s);
hipError_t launch_sync_sweep(int t, const int32_t* sw_idx, const float* theta, float* sw_o,
                             hipStream_t s);
// 3-point rotations: O_t = expm(W(w_t)) O0_t, sweep-log copies, and the chain rule of d/dw
hipError_t launch_sync_rot3(int64_t R, const float* theta, const float* o0, float* rot_o,
                            hipStream_t s);
hipError_t launch_sync_sweep3(int t, const int32_t* sw_idx, const float* rot_o, float* sw_o,
                              hipStream_t s);
hipError_t launch_theta3_chain(int64_t R, const float* theta, float* g, hipStream_t s);

}  // namespace pmmf
