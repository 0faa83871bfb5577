// Matrix-free application of the factorization (Sec. 2.4) and its adjoint, gfx950.
//
// A block of vectors X [n][ld] goes through the stages one at a time.  In stage p a workgroup owns
// one cluster and a tile of W columns: it loads the cluster's c_u rows of the tile into LDS,
// applies the cluster's rotations level by level (rotations of one level touch disjoint rows, so
// each level is one parallel step), and writes the rows back: survivors to the next stage's compact
// buffer (ascending position order), retired rows to their natural place.  Every active row is
// read and written once per stage.
#include "sweep_kernels.h"

#include <algorithm>
#include <mutex>
#include <set>
#include <utility>

namespace pmmf {

// dynamic LDS of a sweep workgroup: tile[NV][cmax][W] floats, then the cluster's rotation ids
// [rmax][K] and k x k blocks [rmax][K*K]

__device__ inline int level_begin(const SweepStage& st, int u, int l) {
  return st.lvl_ptr[(size_t)u * st.lvl_stride + l];
}

// Load the cluster's rotations (ids and k x k blocks) into LDS.
template <int K>
__device__ inline void load_rotations(const SweepStage& st, int rb, int r, int* rid, float* rob) {
  for (int q = threadIdx.x; q < r * K; q += blockDim.x) rid[q] = st.sw_loc[(size_t)rb * K + q];
  for (int q = threadIdx.x; q < r * K * K; q += blockDim.x)
    rob[q] = st.sw_o[(size_t)rb * K * K + q];
}

// Apply one rotation (slot ids ids[], block o[]) to column w of every vector tile.
template <int K, int W, int NV, bool TRANS>
__device__ inline void rotate_cols(float* tile, int cstride, const int* ids, const float* o, int w) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float* t = tile + (size_t)v * cstride;
    float x[K];
#pragma unroll
    for (int a = 0; a < K; ++a) x[a] = t[ids[a] * W + w];
#pragma unroll
    for (int a = 0; a < K; ++a) {
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < K; ++b) s += (TRANS ? o[b * K + a] : o[a * K + b]) * x[b];
      t[ids[a] * W + w] = s;
    }
  }
}

// ------------------------------------------------------------------------------------------
// forward stage sweep: rows of S_{p-1} (compact, src) -> rotations in order -> survivors to
// dst_c (compact S_p), retired rows to dst_nat[gid] times the vector's scale mode
template <int K, int W, int NV>
__global__ void __launch_bounds__(256) k_sweep_fwd(SweepStage st, FwdIO io) {
  extern __shared__ float lds_f[];
  const int u = st.clist ? st.clist[blockIdx.x] : blockIdx.x;
  const int col0 = blockIdx.y * W;
  const int o = st.off[u];
  const int c = st.off[u + 1] - o;
  const int cstride = st.cmax * W;
  float* tile = lds_f;
  int* rid = reinterpret_cast<int*>(tile + (size_t)NV * cstride);
  const int rb = level_begin(st, u, 0);
  const int depth = st.depth[u];
  const int r = level_begin(st, u, depth) - rb;
  float* rob = reinterpret_cast<float*>(rid + st.rmax * K);
  load_rotations<K>(st, rb, r, rid, rob);
  for (int q = threadIdx.x; q < c * W; q += blockDim.x) {
    const int row = q / W, w = q % W;
    const int col = col0 + w;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float val = 0.f;
      if (col < io.nrhs) val = io.src[v][(size_t)(o + row) * io.ld_src + col];
      tile[(size_t)v * cstride + row * W + w] = val;
    }
  }
  __syncthreads();
  for (int l = 0; l < depth; ++l) {
    const int b0 = level_begin(st, u, l) - rb, b1 = level_begin(st, u, l + 1) - rb;
    for (int q = threadIdx.x; q < (b1 - b0) * W; q += blockDim.x) {
      const int rr = b0 + q / W, w = q % W;
      rotate_cols<K, W, NV, false>(tile, cstride, rid + rr * K, rob + rr * K * K, w);
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < c * W; q += blockDim.x) {
    const int row = q / W, w = q % W;
    const int col = col0 + w;
    if (col >= io.nrhs) continue;
    const int nx = st.next[o + row];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float val = tile[(size_t)v * cstride + row * W + w];
      if (nx >= 0) {
        io.dst_c[v][(size_t)nx * io.ld_c + col] = val;
      } else {
        const int g = -nx - 1;
        if (io.mode[v] == 1) val *= io.hdiag[g];
        else if (io.mode[v] == 2) val /= io.hdiag[g];
        else if (io.mode[v] == 3) val /= sqrtf(io.hdiag[g]);
        io.dst_nat[v][(size_t)g * io.ld_nat + col] = val;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// reverse stage sweep: rows of S_{p-1}: survivors from src_c (compact S_p), retired rows from
// src_nat[gid] (times hdiag if mode = 1) -> transposed rotations in reverse order -> dst_c
// (compact S_{p-1}) or, when dst_nat is set, natural order (first stage).  With THETA, vector 0
// is the state z and vector 1 the adjoint g, and before undoing rotation t the kernel adds
// sum_w <g[T], J z[T]> (J = [[0, -1], [1, 0]]) to the tile's partial angle gradient.
template <int K, int W, int NV, bool THETA>
__global__ void __launch_bounds__(256) k_sweep_rev(SweepStage st, RevIO io) {
  extern __shared__ float lds_f[];
  const int u = st.clist ? st.clist[blockIdx.x] : blockIdx.x;
  const int col0 = blockIdx.y * W;
  const int o = st.off[u];
  const int c = st.off[u + 1] - o;
  const int cstride = st.cmax * W;
  float* tile = lds_f;
  int* rid = reinterpret_cast<int*>(tile + (size_t)NV * cstride);
  const int rb = level_begin(st, u, 0);
  const int depth = st.depth[u];
  const int r = level_begin(st, u, depth) - rb;
  float* rob = reinterpret_cast<float*>(rid + st.rmax * K);
  load_rotations<K>(st, rb, r, rid, rob);
  for (int q = threadIdx.x; q < c * W; q += blockDim.x) {
    const int row = q / W, w = q % W;
    const int col = col0 + w;
    const int nx = st.next[o + row];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float val = 0.f;
      if (col < io.nrhs) {
        if (nx >= 0) {
          val = io.src_c[v][(size_t)nx * io.ld_c + col];
        } else {
          const int g = -nx - 1;
          val = io.src_nat[v][(size_t)g * io.ld_nat + col];
          if (io.mode[v] == 1) val *= io.hdiag[g];
        }
      }
      tile[(size_t)v * cstride + row * W + w] = val;
    }
  }
  __syncthreads();
  for (int l = depth - 1; l >= 0; --l) {
    const int b0 = level_begin(st, u, l) - rb, b1 = level_begin(st, u, l + 1) - rb;
    const int nwork = (b1 - b0) * W;
    const int nround = (nwork + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (int q = threadIdx.x; q < nround; q += blockDim.x) {
      const bool live = q < nwork;
      const int rr = b0 + (live ? q / W : 0), w = q % W;
      if constexpr (THETA) {
        // k = 3: one partial per plane (0,1), (0,2), (1,2) of the slots
        constexpr int NP = K == 3 ? 3 : 1;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const int pp = m == 2 ? 1 : 0, qq = m == 0 ? 1 : 2;
          float part = 0.f;
          if (live) {
            const int* ids = rid + rr * K;
            const float* z = tile;
            const float* g = tile + cstride;
            const float zi = z[ids[pp] * W + w], zj = z[ids[qq] * W + w];
            const float gi = g[ids[pp] * W + w], gj = g[ids[qq] * W + w];
            part = gj * zi - gi * zj;
          }
          // reduce over the W consecutive lanes holding one rotation's columns
#pragma unroll
          for (int ofs = W / 2; ofs > 0; ofs >>= 1) part += __shfl_xor(part, ofs, W);
          if (live && w == 0) {
            const size_t at = (size_t)(st.sw_idx[rr + rb] - st.rot_base) * NP + m;
            io.theta_part[(size_t)blockIdx.y * io.theta_stride + at] = part;
            if (blockIdx.y == gridDim.y - 1)
              for (int y = blockIdx.y + 1; y < io.theta_tiles; ++y)
                io.theta_part[(size_t)y * io.theta_stride + at] = 0.f;
          }
        }
      }
      if (live) rotate_cols<K, W, NV, true>(tile, cstride, rid + rr * K, rob + rr * K * K, w);
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < c * W; q += blockDim.x) {
    const int row = q / W, w = q % W;
    const int col = col0 + w;
    if (col >= io.nrhs) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float val = tile[(size_t)v * cstride + row * W + w];
      if (io.dst_nat[v]) {
        io.dst_nat[v][(size_t)st.gid[o + row] * io.ld_dnat + col] = val;
      } else if (io.dst_c[v]) {
        io.dst_c[v][(size_t)(o + row) * io.ld_out + col] = val;
      }
    }
  }
}

size_t sweep_lds_bytes(int k, int W, int nv, int cmax, int rmax) {
  return (size_t)nv * cmax * W * sizeof(float) + (size_t)rmax * k * sizeof(int) +
         (size_t)rmax * k * k * sizeof(float);
}

template <int K, int W, int NV>
static hipError_t fwd_dispatch(const SweepStage& st, const FwdIO& io, hipStream_t s) {
  const size_t lds = sweep_lds_bytes(K, W, NV, st.cmax, st.rmax);
  auto fn = k_sweep_fwd<K, W, NV>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid(st.m, (io.nrhs + W - 1) / W);  // st.m = number of listed clusters
  k_sweep_fwd<K, W, NV><<<grid, 256, lds, s>>>(st, io);
  return hipGetLastError();
}

template <int K, int W, int NV, bool TH>
static hipError_t rev_dispatch(const SweepStage& st, const RevIO& io, hipStream_t s) {
  const size_t lds = sweep_lds_bytes(K, W, NV, st.cmax, st.rmax);
  auto fn = k_sweep_rev<K, W, NV, TH>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid(st.m, (io.nrhs + W - 1) / W);
  k_sweep_rev<K, W, NV, TH><<<grid, 256, lds, s>>>(st, io);
  return hipGetLastError();
}

#define PMMF_W_SWITCH(W, CALL)                     \
  switch (W) {                                     \
    case 1: { constexpr int WW = 1; return CALL; } \
    case 2: { constexpr int WW = 2; return CALL; } \
    case 4: { constexpr int WW = 4; return CALL; } \
    case 8: { constexpr int WW = 8; return CALL; } \
    case 16: { constexpr int WW = 16; return CALL; } \
    case 32: { constexpr int WW = 32; return CALL; } \
    default: return hipErrorInvalidValue;         \
  }

hipError_t launch_sweep_fwd(const SweepStage& st, const FwdIO& io, int W, int nv, hipStream_t s) {
  if (st.m == 0) return hipSuccess;
  if (st.k == 2) {
    if (nv == 1) { PMMF_W_SWITCH(W, (fwd_dispatch<2, WW, 1>(st, io, s))) }
    PMMF_W_SWITCH(W, (fwd_dispatch<2, WW, 2>(st, io, s)))
  }
  if (nv == 1) { PMMF_W_SWITCH(W, (fwd_dispatch<3, WW, 1>(st, io, s))) }
  PMMF_W_SWITCH(W, (fwd_dispatch<3, WW, 2>(st, io, s)))
}

hipError_t launch_sweep_rev(const SweepStage& st, const RevIO& io, int W, int nv, bool theta,
                            hipStream_t s) {
  if (st.m == 0) return hipSuccess;
  if (st.k == 2) {
    if (theta) { PMMF_W_SWITCH(W, (rev_dispatch<2, WW, 2, true>(st, io, s))) }
    if (nv == 1) { PMMF_W_SWITCH(W, (rev_dispatch<2, WW, 1, false>(st, io, s))) }
    PMMF_W_SWITCH(W, (rev_dispatch<2, WW, 2, false>(st, io, s)))
  }
  if (theta) { PMMF_W_SWITCH(W, (rev_dispatch<3, WW, 2, true>(st, io, s))) }
  if (nv == 1) { PMMF_W_SWITCH(W, (rev_dispatch<3, WW, 1, false>(st, io, s))) }
  PMMF_W_SWITCH(W, (rev_dispatch<3, WW, 2, false>(st, io, s)))
}

// ------------------------------------------------------------------------------------------
// dense FP32 GEMM  C[M][N] = op(A)[M][K] * op(B)[K][N] (+ beta C), row-major, op = transpose if
// flagged.  The products here are small (a core of a few hundred to a few thousand rows against
// at most a few hundred vectors), so a workgroup takes one 16 x 16 output tile and its eight waves
// split K: K is cut into 16-deep blocks, wave w takes blocks w, w + 8, ..., and each block is four
// v_mfma_f32_16x16x4f32 (A operand: lane l holds A[l % 16][.], B operand B[.][l % 16]; lane group
// l / 16 takes k = 4 (l / 16) + s of the block in step s, the same k for both operands, so the sum
// runs over every k once).  Lanes read their operands straight from memory (the core and the
// vectors stay in L2), four blocks per wave at a time with the next four in flight (a K of 512
// is one round); the eight partial tiles are added in LDS in wave order, so the result does not
// depend on timing.
typedef float pmmf_f4 __attribute__((ext_vector_type(4)));
constexpr int GEMM_T = 16, GEMM_KB = 16, GEMM_WAVES = 8, GEMM_BPW = 4;
// VA / VB: the operand's k runs along its rows (A not transposed / B transposed) in 16-byte
// aligned rows with K a multiple of 4: a lane's four k of a block are one 16-byte load
struct GemmProb {
  int M, N, K;
  const float* A;
  int lda, ta;
  const float* B;
  int ldb, tb;
  float* C;
  int ldc;
  float beta;
  int va, vb;  // 16-byte operand loads (see gemm_tile)
};
struct GemmBatch {
  int n;
  GemmProb p[3];
};

template <bool VA, bool VB>
__device__ inline void gemm_tile(const GemmProb& g, int bx, int by) {
  __shared__ pmmf_f4 part[GEMM_WAVES - 1][PMMF_WAVE];
  const int M = g.M, N = g.N, K = g.K, lda = g.lda, ta = g.ta, ldb = g.ldb, tb = g.tb, ldc = g.ldc;
  const float* __restrict__ A = g.A;
  const float* __restrict__ B = g.B;
  float* __restrict__ C = g.C;
  const float beta = g.beta;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, grp = lane >> 4;
  const int m0 = by * GEMM_T, n0 = bx * GEMM_T;
  const bool mok = m0 + r < M, nok = n0 + r < N;
  const int64_t gm = min(m0 + r, M - 1), gn = min(n0 + r, N - 1);
  const int nb = (K + GEMM_KB - 1) / GEMM_KB;
  constexpr int PER_IT = GEMM_WAVES * GEMM_BPW;  // blocks per iteration of the whole workgroup
  const int nit = (nb + PER_IT - 1) / PER_IT;
  float fa0[GEMM_BPW][4], fb0[GEMM_BPW][4], fa1[GEMM_BPW][4], fb1[GEMM_BPW][4];
  // block it * PER_IT + j * GEMM_WAVES + w; addresses clamped into the matrices, values past the
  // edges replaced by zero after the load
  auto fetch = [&](int it, float (&xa)[GEMM_BPW][4], float (&xb)[GEMM_BPW][4]) {
#pragma unroll
    for (int j = 0; j < GEMM_BPW; ++j) {
      const int kb = (it * PER_IT + j * GEMM_WAVES + w) * GEMM_KB + 4 * grp;
      if constexpr (VA) {
        const pmmf_f4 a4 = *reinterpret_cast<const pmmf_f4*>(A + gm * lda + min(kb, K - 4));
        const bool ok = mok && kb < K;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) xa[j][s4] = ok ? a4[s4] : 0.f;
      }
      if constexpr (VB) {
        const pmmf_f4 b4 = *reinterpret_cast<const pmmf_f4*>(B + gn * ldb + min(kb, K - 4));
        const bool ok = nok && kb < K;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) xb[j][s4] = ok ? b4[s4] : 0.f;
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = kb + s4;
        const int64_t kc = min(k, K - 1);
        if constexpr (!VA) {
          const float va = ta ? A[kc * lda + gm] : A[gm * lda + kc];
          xa[j][s4] = (mok && k < K) ? va : 0.f;
        }
        if constexpr (!VB) {
          const float vb = tb ? B[gn * ldb + kc] : B[kc * ldb + gn];
          xb[j][s4] = (nok && k < K) ? vb : 0.f;
        }
      }
    }
  };
  pmmf_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  auto mult = [&](const float (&xa)[GEMM_BPW][4], const float (&xb)[GEMM_BPW][4]) {
#pragma unroll
    for (int j = 0; j < GEMM_BPW; ++j) {
#pragma unroll
      for (int s4 = 0; s4 < 4; s4 += 2) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[j][s4], xb[j][s4], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[j][s4 + 1], xb[j][s4 + 1], acc1, 0, 0, 0);
      }
    }
  };
  // two register sets used in turn: the next iteration's operands are in flight while the
  // current ones are multiplied
  if (nit > 0) fetch(0, fa0, fb0);
  for (int it = 0; it < nit; it += 2) {
    if (it + 1 < nit) fetch(it + 1, fa1, fb1);
    mult(fa0, fb0);
    if (it + 1 >= nit) break;
    if (it + 2 < nit) fetch(it + 2, fa0, fb0);
    mult(fa1, fb1);
  }
  pmmf_f4 acc = acc0 + acc1;
  if (w > 0) part[w - 1][lane] = acc;
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int q = 0; q < GEMM_WAVES - 1; ++q) acc += part[q][lane];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int cm = m0 + 4 * grp + i, cn = n0 + r;
    if (cm < M && cn < N) {
      float* cp = C + (size_t)cm * ldc + cn;
      *cp = beta == 0.f ? acc[i] : beta * *cp + acc[i];
    }
  }
}

template <bool VA, bool VB>
__global__ void __launch_bounds__(GEMM_WAVES * PMMF_WAVE) k_gemm(GemmProb g) {
  gemm_tile<VA, VB>(g, blockIdx.x, blockIdx.y);
}

// up to three independent products in one launch (blockIdx.z picks the product)
__global__ void __launch_bounds__(GEMM_WAVES * PMMF_WAVE) k_gemm_batch(GemmBatch b) {
  const GemmProb& g = b.p[blockIdx.z];
  if ((int)blockIdx.x * GEMM_T >= g.N || (int)blockIdx.y * GEMM_T >= g.M) return;
  if (g.va && g.vb) gemm_tile<true, true>(g, blockIdx.x, blockIdx.y);
  else if (g.va) gemm_tile<true, false>(g, blockIdx.x, blockIdx.y);
  else if (g.vb) gemm_tile<false, true>(g, blockIdx.x, blockIdx.y);
  else gemm_tile<false, false>(g, blockIdx.x, blockIdx.y);
}

static GemmProb gemm_prob(int M, int N, int K, const float* A, int lda, int ta, const float* B,
                          int ldb, int tb, float* C, int ldc, float beta) {
  auto rows16 = [&](const float* p, int ld) {
    return K % 4 == 0 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  };
  GemmProb g{M, N, K, A, lda, ta, B, ldb, tb, C, ldc, beta, 0, 0};
  g.va = !ta && rows16(A, lda);
  g.vb = tb && rows16(B, ldb);
  return g;
}

hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int ta, const float* B,
                       int ldb, int tb, float* C, int ldc, float beta, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 grid((N + GEMM_T - 1) / GEMM_T, (M + GEMM_T - 1) / GEMM_T);
  const GemmProb g = gemm_prob(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, beta);
  const int th = GEMM_WAVES * PMMF_WAVE;
  if (g.va && g.vb) k_gemm<true, true><<<grid, th, 0, s>>>(g);
  else if (g.va) k_gemm<true, false><<<grid, th, 0, s>>>(g);
  else if (g.vb) k_gemm<false, true><<<grid, th, 0, s>>>(g);
  else k_gemm<false, false><<<grid, th, 0, s>>>(g);
  return hipGetLastError();
}

hipError_t launch_gemm_batch(int n, const GemmArgs* args, hipStream_t s) {
  if (n < 1 || n > 3) return hipErrorInvalidValue;
  GemmBatch b{};
  b.n = n;
  int gx = 0, gy = 0;
  for (int q = 0; q < n; ++q) {
    const GemmArgs& a = args[q];
    b.p[q] = gemm_prob(a.M, a.N, a.K, a.A, a.lda, a.ta, a.B, a.ldb, a.tb, a.C, a.ldc, a.beta);
    gx = std::max(gx, (a.N + GEMM_T - 1) / GEMM_T);
    gy = std::max(gy, (a.M + GEMM_T - 1) / GEMM_T);
  }
  if (gx == 0 || gy == 0) return hipSuccess;
  k_gemm_batch<<<dim3(gx, gy, n), GEMM_WAVES * PMMF_WAVE, 0, s>>>(b);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// In-place Cholesky A = L L^T of a small SPD core (one workgroup, right-looking, lower triangle);
// status[0] = 1 if a pivot is not positive.
__global__ void __launch_bounds__(1024) k_cholesky(int n, float* __restrict__ A, int32_t* status) {
  __shared__ float piv;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const float d = A[(size_t)j * n + j];
      if (!(d > 0.f)) { status[0] = 1; piv = 0.f; }
      else { piv = sqrtf(d); A[(size_t)j * n + j] = piv; }
    }
    __syncthreads();
    if (piv == 0.f) return;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[(size_t)i * n + j] /= piv;
    __syncthreads();
    const int rem = n - j - 1;
    // trailing update of the lower triangle: A[i][l] -= L[i][j] L[l][j], j < l <= i
    for (int q = threadIdx.x; q < rem * rem; q += blockDim.x) {
      const int i = j + 1 + q / rem, l = j + 1 + q % rem;
      if (l <= i) A[(size_t)i * n + l] -= A[(size_t)i * n + j] * A[(size_t)l * n + j];
    }
    __syncthreads();
  }
}

// X = L^{-1} (lower triangular), one column per thread by forward substitution.
__global__ void k_tri_inverse(int n, const float* __restrict__ L, float* __restrict__ X) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < j; ++i) X[(size_t)i * n + j] = 0.f;
  for (int i = j; i < n; ++i) {
    float s = (i == j) ? 1.f : 0.f;
    for (int l = j; l < i; ++l) s -= L[(size_t)i * n + l] * X[(size_t)l * n + j];
    X[(size_t)i * n + j] = s / L[(size_t)i * n + i];
  }
}

__global__ void k_check_hdiag(int64_t n, const float* __restrict__ hdiag,
                              const uint8_t* __restrict__ is_core, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !is_core[i] && hdiag[i] == 0.f) atomicOr(status, 2);
}

hipError_t launch_core_inverse(int n, float* work_L, float* work_X, float* out_inv,
                               int64_t nfull, const float* hdiag, const uint8_t* is_core,
                               int32_t* status, hipStream_t s) {
  k_check_hdiag<<<(unsigned)((nfull + 255) / 256), 256, 0, s>>>(nfull, hdiag, is_core, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  k_cholesky<<<1, 1024, 0, s>>>(n, work_L, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_tri_inverse<<<(n + 63) / 64, 64, 0, s>>>(n, work_L, work_X);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // H^{-1} = L^{-T} L^{-1} = X^T X
  return launch_gemm(n, n, n, work_X, n, 1, work_X, n, 0, out_inv, n, 0.f, s);
}

// ------------------------------------------------------------------------------------------
// H^{-1/2}: the retired diagonal must be positive, and the core's inverse square root is
// V diag(lambda^{-1/2}) V^T from its FP64 eigendecomposition (eigenvectors in the columns of V,
// column-major as LAPACK leaves them); status bit 4: a retired entry <= 0, bit 8: an eigenvalue
// <= 0 (the core is not positive definite).
__global__ void k_check_hdiag_pos(int64_t n, const float* __restrict__ hdiag,
                                  const uint8_t* __restrict__ is_core, int32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !is_core[i] && !(hdiag[i] > 0.f)) atomicOr(status, 4);
}

__global__ void k_f32_to_f64(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_isqrt_assemble(int n, const double* __restrict__ V, const double* __restrict__ lam,
                                 float* __restrict__ out, int32_t* status) {
  // out[i][j] = sum_k V[k*n + i] lam_k^{-1/2} V[k*n + j]  (V column-major: column k at k*n)
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double l = lam[k];
    if (!(l > 0.0)) {
      if (i == 0 && j == 0) atomicOr(status, 8);
      continue;
    }
    acc += V[(size_t)k * n + i] * V[(size_t)k * n + j] / sqrt(l);
  }
  out[(size_t)i * n + j] = (float)acc;
}

hipError_t launch_check_hdiag_pos(int64_t n, const float* hdiag, const uint8_t* is_core,
                                  int32_t* status, hipStream_t s) {
  k_check_hdiag_pos<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, hdiag, is_core, status);
  return hipGetLastError();
}

hipError_t launch_f32_to_f64(int64_t n, const float* a, double* b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_f32_to_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, b);
  return hipGetLastError();
}

hipError_t launch_isqrt_assemble(int n, const double* V, const double* lam, float* out,
                                 int32_t* status, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  k_isqrt_assemble<<<grid, 256, 0, s>>>(n, V, lam, out, status);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// hdiag_bar[e] = sum_w b[e][w] a[e][w] on retired e (0 on the core); one wave per row
__global__ void k_rowdot(int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                         int64_t ld, int64_t nrhs, const uint8_t* __restrict__ is_core,
                         float* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (row >= n) return;
  float s = 0.f;
  if (!is_core[row])
    for (int64_t w = pmmf_lane(); w < nrhs; w += PMMF_WAVE) s += a[row * ld + w] * b[row * ld + w];
  s = pmmf_wave_sum_float(s);
  if (pmmf_lane() == 0) out[row] = s;
}
hipError_t launch_rowdot(int64_t n, const float* a, const float* b, int64_t ld, int64_t nrhs,
                         const uint8_t* is_core, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_rowdot<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, a, b, ld, nrhs, is_core, out);
  return hipGetLastError();
}

// theta_bar[rot_base + q] = sum over column tiles of (partA + partB)[tile][q]
__global__ void k_theta_reduce(int t, int ntiles, int64_t stride, const float* __restrict__ pa,
                               const float* __restrict__ pb, int64_t rot_base,
                               float* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= t) return;
  float s = 0.f;
  for (int y = 0; y < ntiles; ++y) s += pa[(size_t)y * stride + q] + pb[(size_t)y * stride + q];
  out[rot_base + q] = s;
}
hipError_t launch_theta_reduce(int t, int ntiles, int64_t stride, const float* pa,
                               const float* pb, int64_t rot_base, float* out, hipStream_t s) {
  if (t == 0) return hipSuccess;
  k_theta_reduce<<<(t + 255) / 256, 256, 0, s>>>(t, ntiles, stride, pa, pb, rot_base, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Unit sweeps: one wave per (unit, 64-column slice), lane = column.  The unit's description (row
// slots, rotation slots) is read in one step, every row segment is then requested at once into
// registers, the rotations are applied in order (MODE 0: O, forward) or in reverse with
// transposed blocks (MODE 1; MODE 2 also adds the angle-gradient partial sum_w <g[T], J z[T]> of
// each rotation before undoing it, vector 0 = z, vector 1 = g), and the rows are written back.
// Rotation parameters live in the lane of their slot and are broadcast with readlane; the rows
// are private to the wave (registers, or its own LDS tile), so no barrier is needed.
template <int K, int NV, int MODE>
__global__ void __launch_bounds__(256) k_unit_sweep(UnitStage st, FwdIO fio, RevIO rio0,
                                                    RevIO rio1, unsigned per_pass) {
  extern __shared__ float lds_f[];
  const int lane = pmmf_lane();
  const int wv = __builtin_amdgcn_readfirstlane(pmmf_wave());
  float* tile = lds_f + (size_t)wv * NV * UNIT_MAX * PMMF_WAVE;  // NV = 2 only
  // U^T sweeps may carry two independent passes over the same stage (the adjoint's two vector
  // pairs) in one launch: blocks [0, per_pass) take rio0, the rest rio1
  const bool second = MODE != 0 && blockIdx.x >= per_pass;
  const RevIO& rio = second ? rio1 : rio0;
  const unsigned bx = second ? blockIdx.x - per_pass : blockIdx.x;
  // one-dimensional grid, column tile fastest and consecutive blocks on one XCD: the tiles of a
  // unit run side by side in one L2, which fetches the unit's description once
  const int ntile = (int)(((MODE == 0 ? fio.nrhs : rio.nrhs) + PMMF_WAVE - 1) / PMMF_WAVE);
  const unsigned lb = (unsigned)pmmf_xcd_block((int)bx, (int)per_pass);
  const int ctile = (int)(lb % (unsigned)ntile);
  const int g = (int)(lb / (unsigned)ntile) * (blockDim.x / PMMF_WAVE) +
                __builtin_amdgcn_readfirstlane(pmmf_wave());
  if (g >= st.nu) return;
  const int64_t col = (int64_t)ctile * PMMF_WAVE + lane;
  const int64_t nrhs = MODE == 0 ? fio.nrhs : rio.nrhs;
  const bool cok = col < nrhs;
  const int2 cnt = st.cnt[g];
  const int ns = __builtin_amdgcn_readfirstlane(cnt.x);
  const int nr = __builtin_amdgcn_readfirstlane(cnt.y);
  int4 sl = make_int4(0, 0, 0, 0);
  int2 rt = make_int2(0, 0);
  if (lane < UNIT_MAX) {
    sl = st.slot[(int64_t)g * UNIT_MAX + lane];
    rt = st.rot[(int64_t)g * UNIT_MAX + lane];
  }
  // this lane's rotation block (slot = lane) and retired-row scale (row slot = lane)
  float om[K * K];
#pragma unroll
  for (int ab = 0; ab < K * K; ++ab)
    om[ab] = lane < nr ? st.rot_o[(int64_t)rt.y * 9 + (ab / K) * 3 + (ab % K)] : 0.f;
  float sc = 1.f;
  if (lane < ns && sl.y < 0) {
    if (MODE == 0 && fio.mode[0] + fio.mode[NV - 1] > 0) sc = fio.hdiag[-sl.y - 1];
    if (MODE != 0 && rio.mode[0] + rio.mode[NV - 1] > 0) sc = rio.hdiag[-sl.y - 1];
  }
  // requests for all rows, eight per uniform chunk; slots past ns repeat the last row and columns
  // past nrhs read the last column, so every address is valid and only the stores are masked
  const int64_t colc = cok ? col : nrhs - 1;
  float x[NV][UNIT_MAX];
#pragma unroll
  for (int c8 = 0; c8 < UNIT_MAX; c8 += 8) {
    if (c8 < ns) {
#pragma unroll
      for (int i = c8; i < c8 + 8; ++i) {
        const int li = min(i, ns - 1);
        const int pos = __builtin_amdgcn_readlane(sl.x, li);
        const int nx = __builtin_amdgcn_readlane(sl.y, li);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const float* src;
          if (MODE == 0) src = fio.src[v] + (int64_t)pos * fio.ld_src;
          else src = nx >= 0 ? rio.src_c[v] + (int64_t)nx * rio.ld_c
                             : rio.src_nat[v] + (int64_t)(-nx - 1) * rio.ld_nat;
          x[v][i] = src[colc];
        }
      }
    }
  }
  if (MODE != 0 && rio.mode[0] + rio.mode[NV - 1] > 0) {
#pragma unroll
    for (int i = 0; i < UNIT_MAX; ++i) {
      const float f = (i < ns && __builtin_amdgcn_readlane(sl.y, i) < 0) ? pmmf_readlane_f(sc, i)
                                                                           : 1.f;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (rio.mode[v] == 1) x[v][i] *= f;
    }
  }
  // one vector: the rows stay in registers (a rotation names its rows by wave-uniform slot
  // numbers, which index the register array directly with s_set_gpr_idx); two vectors: the rows
  // are parked in the wave's own LDS tile (64 indexed registers would go to scratch memory)
  if constexpr (NV > 1) {
#pragma unroll
    for (int c8 = 0; c8 < UNIT_MAX; c8 += 8) {
      if (c8 < ns) {
#pragma unroll
        for (int i = c8; i < c8 + 8; ++i)
#pragma unroll
          for (int v = 0; v < NV; ++v) tile[(v * UNIT_MAX + i) * PMMF_WAVE + lane] = x[v][i];
      }
    }
  }
  auto T = [&](int v, int i) -> float& {
    if constexpr (NV == 1) return x[v][i];
    else return tile[(v * UNIT_MAX + i) * PMMF_WAVE + lane];
  };
  if (MODE == 0) {
    for (int q = 0; q < nr; ++q) {
      const int locs = __builtin_amdgcn_readlane(rt.x, q);
      int id[K];
      float o[K * K];
#pragma unroll
      for (int a = 0; a < K; ++a) id[a] = (locs >> (5 * a)) & 31;
#pragma unroll
      for (int ab = 0; ab < K * K; ++ab) o[ab] = pmmf_readlane_f(om[ab], q);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        float y[K];
#pragma unroll
        for (int a = 0; a < K; ++a) y[a] = T(v, id[a]);
#pragma unroll
        for (int a = 0; a < K; ++a) {
          float acc = 0.f;
#pragma unroll
          for (int b = 0; b < K; ++b) acc += o[a * K + b] * y[b];
          T(v, id[a]) = acc;
        }
      }
    }
  } else {
    for (int q = nr - 1; q >= 0; --q) {
      const int locs = __builtin_amdgcn_readlane(rt.x, q);
      int id[K];
      float o[K * K];
#pragma unroll
      for (int a = 0; a < K; ++a) id[a] = (locs >> (5 * a)) & 31;
#pragma unroll
      for (int ab = 0; ab < K * K; ++ab) o[ab] = pmmf_readlane_f(om[ab], q);
      if constexpr (MODE == 2 && NV == 2) {
        // lanes past the last column hold a copy of it: they add nothing.  k = 3: one partial
        // per plane (0,1), (0,2), (1,2) of the slots, <g, G_pq z> = g_q z_p - g_p z_q
        constexpr int NP = K == 3 ? 3 : 1;
        const int64_t at = (int64_t)ctile * rio.theta_stride +
                           (int64_t)(__builtin_amdgcn_readlane(rt.y, q) - st.rot_base) * NP;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const int pp = m == 2 ? 1 : 0, qq = m == 0 ? 1 : 2;
          float part = cok ? T(1, id[qq]) * T(0, id[pp]) - T(1, id[pp]) * T(0, id[qq]) : 0.f;
          part = pmmf_wave_sum_dpp(part);
          if (lane == 0) {
            rio.theta_part[at + m] = part;
            if (ctile == ntile - 1)
              for (int y = ctile + 1; y < rio.theta_tiles; ++y)
                rio.theta_part[at + (int64_t)(y - ctile) * rio.theta_stride + m] = 0.f;
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        float y[K];
#pragma unroll
        for (int a = 0; a < K; ++a) y[a] = T(v, id[a]);
#pragma unroll
        for (int a = 0; a < K; ++a) {
          float acc = 0.f;
#pragma unroll
          for (int b = 0; b < K; ++b) acc += o[b * K + a] * y[b];
          T(v, id[a]) = acc;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < UNIT_MAX; ++i) {
    if (i >= ns) break;
    const int pos = __builtin_amdgcn_readlane(sl.x, i);
    const int nx = __builtin_amdgcn_readlane(sl.y, i);
    const int gd = __builtin_amdgcn_readlane(sl.z, i);
    const float f = pmmf_readlane_f(sc, i);
    if (!cok) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float val = T(v, i);
      if (MODE == 0) {
        if (nx >= 0) {
          fio.dst_c[v][(int64_t)nx * fio.ld_c + col] = val;
        } else {
          if (fio.mode[v] == 1) val *= f;
          else if (fio.mode[v] == 2) val /= f;
          else if (fio.mode[v] == 3) val /= sqrtf(f);
          fio.dst_nat[v][(int64_t)(-nx - 1) * fio.ld_nat + col] = val;
        }
      } else {
        if (rio.dst_nat[v]) rio.dst_nat[v][(int64_t)gd * rio.ld_dnat + col] = val;
        else if (rio.dst_c[v]) rio.dst_c[v][(int64_t)pos * rio.ld_out + col] = val;
      }
    }
  }
}

template <int K, int NV, int MODE>
static hipError_t unit_launch(const UnitStage& st, const FwdIO& fio, const RevIO& rio, int wpb,
                              hipStream_t s, const RevIO* rio2 = nullptr) {
  if (st.nu == 0) return hipSuccess;
  if (wpb != 1 && wpb != 2 && wpb != 4) return hipErrorInvalidValue;
  const size_t lds = NV == 1 ? 0 : (size_t)wpb * NV * UNIT_MAX * PMMF_WAVE * sizeof(float);
  const int64_t nrhs = MODE == 0 ? fio.nrhs : rio.nrhs;
  if (rio2 && rio2->nrhs != nrhs) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)((st.nu + wpb - 1) / wpb) * ((nrhs + PMMF_WAVE - 1) / PMMF_WAVE);
  if (blocks * (rio2 ? 2 : 1) > 0x7fffffff) return hipErrorInvalidValue;
  k_unit_sweep<K, NV, MODE><<<(unsigned)(blocks * (rio2 ? 2 : 1)), wpb * PMMF_WAVE, lds, s>>>(
      st, fio, rio, rio2 ? *rio2 : rio, (unsigned)blocks);
  return hipGetLastError();
}

hipError_t launch_unit_fwd(const UnitStage& st, const FwdIO& io, int nv, int wpb, hipStream_t s) {
  RevIO none{};
  if (st.k == 2)
    return nv == 1 ? unit_launch<2, 1, 0>(st, io, none, wpb, s)
                   : unit_launch<2, 2, 0>(st, io, none, wpb, s);
  return nv == 1 ? unit_launch<3, 1, 0>(st, io, none, wpb, s)
                 : unit_launch<3, 2, 0>(st, io, none, wpb, s);
}

hipError_t launch_unit_rev(const UnitStage& st, const RevIO& io, int nv, bool theta, int wpb,
                           hipStream_t s, const RevIO* io2) {
  FwdIO none{};
  if (st.k == 2) {
    if (theta) return unit_launch<2, 2, 2>(st, none, io, wpb, s, io2);
    return nv == 1 ? unit_launch<2, 1, 1>(st, none, io, wpb, s, io2)
                   : unit_launch<2, 2, 1>(st, none, io, wpb, s, io2);
  }
  if (theta) return unit_launch<3, 2, 2>(st, none, io, wpb, s, io2);
  return nv == 1 ? unit_launch<3, 1, 1>(st, none, io, wpb, s, io2)
                 : unit_launch<3, 2, 1>(st, none, io, wpb, s, io2);
}

// ------------------------------------------------------------------------------------------
// Trailing stages (TailPlan): one workgroup of TAIL_THREADS per column.  Thread tid owns the slots
// tid + j * TAIL_THREADS (j < TAIL_J) for the moves between stages, and unit tid (+ multiples of
// TAIL_THREADS) for the rotations.  Loads go out one stage ahead (the next program block straight
// into LDS, the next stage's slot table and the values it needs into registers), the current
// stage is computed from LDS meanwhile, and stores are issued at the start of the following
// stage, so the wait for the loads at the end of a stage does not also wait for fresh stores.
typedef __attribute__((address_space(3))) void* pmmf_lds_ptr;

// issue the copy of stage s's program block into LDS at dst (16 bytes per lane; the LDS address
// of a wave's request is the wave's first chunk, lanes follow at 16-byte steps)
__device__ inline void tail_copy_block(const TailPlan& tp, int s, unsigned char* dst) {
  const int nch = tp.st[s].blob_bytes >> 4;
  const unsigned char* src = tp.blob + tp.st[s].blob_off;
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < nch; c0 += TAIL_THREADS) {
    const int wfirst = __builtin_amdgcn_readfirstlane(c0 + (tid & ~(PMMF_WAVE - 1)));
    if (wfirst >= nch) break;
    const int c = c0 + tid;
    if (c < nch)
      __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)c * 16),
                                       (pmmf_lds_ptr)(dst + (size_t)wfirst * 16), 16, 0, 0);
  }
}

// stage s's program block: even stages right after the rows, odd stages at the end of the
// workgroup's LDS, so two consecutive blocks never overlap
__device__ inline unsigned char* tail_block(const TailPlan& tp, unsigned char* lds, int s) {
  return (s & 1) ? lds + tp.lds_bytes - tp.st[s].blob_bytes : lds + tp.data_bytes;
}

// wait for every outstanding vector memory operation (the direct-to-LDS copies included)
__device__ inline void tail_wait_mem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// the rotations of one stage: thread per unit, in order (forward: O) or reversed with transposed
// blocks (U^T), on the rows in LDS.  Same arithmetic as the unit sweep.
template <int K, bool REV>
__device__ inline void tail_rotate(const unsigned char* blk, int nu, int t, float* data) {
  const int2* units = reinterpret_cast<const int2*>(blk);
  const int* prog = reinterpret_cast<const int*>(blk + tail_prog_off(nu));
  const float* ob = reinterpret_cast<const float*>(blk + tail_o_off(nu, t));
  for (int u = threadIdx.x; u < nu; u += TAIL_THREADS) {
    const int2 a = units[u], b = units[u + 1];
    const int sb = a.x;
    const int n = b.y - a.y;
    for (int i = 0; i < n; ++i) {
      const int q = REV ? b.y - 1 - i : a.y + i;
      const int packed = prog[q];
      float o[K * K];
#pragma unroll
      for (int ab = 0; ab < K * K; ++ab) o[ab] = ob[(size_t)q * K * K + ab];
      int id[K];
      float y[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        id[c] = sb + ((packed >> (5 * c)) & 31);
        y[c] = data[id[c]];
      }
#pragma unroll
      for (int c = 0; c < K; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int d = 0; d < K; ++d) acc += (REV ? o[d * K + c] : o[c * K + d]) * y[d];
        data[id[c]] = acc;
      }
    }
  }
}

template <int K>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail_fwd(TailPlan tp, FwdIO io) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  float* data = reinterpret_cast<float*>(tail_lds);
  const int tid = threadIdx.x;
  // grid: nrhs workgroups per vector (io.src[1] set: two vectors, the second half of the grid)
  const int64_t lb = pmmf_xcd_block(blockIdx.x, gridDim.x);
  const int vsel = lb >= io.nrhs ? 1 : 0;
  const int64_t col = lb - vsel * io.nrhs;
  const float* __restrict__ src = vsel ? io.src[1] : io.src[0];
  float* __restrict__ dst_c = vsel ? io.dst_c[1] : io.dst_c[0];
  float* __restrict__ dst_nat = vsel ? io.dst_nat[1] : io.dst_nat[0];
  const int mode = vsel ? io.mode[1] : io.mode[0];
  const int nst = tp.nst;
  tail_copy_block(tp, 0, tail_block(tp, tail_lds, 0));
  int tc[TAIL_J], tn[TAIL_J], rg[TAIL_J];
  float v[TAIL_J], rv[TAIL_J];
  {
    const int rows = tp.st[0].rows;
    int ps[TAIL_J];
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const int i = min(tid + j * TAIL_THREADS, rows - 1);
      ps[j] = tp.pos[tp.st[0].slot_off + i];
      tc[j] = tp.trans[tp.st[0].slot_off + i];
    }
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) v[j] = src[(int64_t)ps[j] * io.ld_src + col];
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const int i = tid + j * TAIL_THREADS;
      if (i < rows) data[i] = v[j];
      rg[j] = -1;
      rv[j] = 0.f;
    }
  }
  tail_wait_mem();
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int rows = tp.st[s].rows;
    // retired rows of the previous stage
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j)
      if (rg[j] >= 0) dst_nat[(int64_t)rg[j] * io.ld_nat + col] = rv[j];
    if (s + 1 < nst) {
      tail_copy_block(tp, s + 1, tail_block(tp, tail_lds, s + 1));
      const int rn = tp.st[s + 1].rows;
#pragma unroll
      for (int j = 0; j < TAIL_J; ++j)
        tn[j] = tp.trans[tp.st[s + 1].slot_off + min(tid + j * TAIL_THREADS, rn - 1)];
    }
    float hd[TAIL_J];
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j)
      hd[j] = mode != 0 ? io.hdiag[tc[j] < 0 ? -tc[j] - 1 : 0] : 1.f;
    tail_rotate<K, false>(tail_block(tp, tail_lds, s), tp.st[s].nu, tp.st[s].t, data);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const int i = min(tid + j * TAIL_THREADS, rows - 1);
      v[j] = data[i];
    }
    __syncthreads();
    const bool last = s + 1 == nst;
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      rg[j] = -1;
      if (tid + j * TAIL_THREADS >= rows) continue;
      if (tc[j] >= 0) {
        if (!last) data[tc[j]] = v[j];
        else dst_c[(int64_t)tc[j] * io.ld_c + col] = v[j];
      } else {
        float val = v[j];
        if (mode == 1) val *= hd[j];
        else if (mode == 2) val /= hd[j];
        else if (mode == 3) val /= sqrtf(hd[j]);
        rv[j] = val;
        rg[j] = -tc[j] - 1;
      }
    }
    if (last) break;
    tail_wait_mem();
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) tc[j] = tn[j];
  }
#pragma unroll
  for (int j = 0; j < TAIL_J; ++j)
    if (rg[j] >= 0) dst_nat[(int64_t)rg[j] * io.ld_nat + col] = rv[j];
}

template <int K>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail_rev(TailPlan tp, RevIO io) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  float* data = reinterpret_cast<float*>(tail_lds);
  const int tid = threadIdx.x;
  const int64_t col = pmmf_xcd_block(blockIdx.x, gridDim.x);
  const int L = tp.nst - 1;
  tail_copy_block(tp, L, tail_block(tp, tail_lds, L));
  // tc: this stage's slot table, t1 / t2: the next two stages down; rv: the retired rows the
  // next stage down takes from natural order
  int tc[TAIL_J], t1[TAIL_J], t2[TAIL_J];
  float v[TAIL_J], rv[TAIL_J];
  {
    const int rows = tp.st[L].rows, r1 = tp.st[L - 1].rows;
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      tc[j] = tp.trans[tp.st[L].slot_off + min(tid + j * TAIL_THREADS, rows - 1)];
      t1[j] = tp.trans[tp.st[L - 1].slot_off + min(tid + j * TAIL_THREADS, r1 - 1)];
    }
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const float a = io.src_c[0][(int64_t)max(tc[j], 0) * io.ld_c + col];
      const float b = io.src_nat[0][(int64_t)(tc[j] < 0 ? -tc[j] - 1 : 0) * io.ld_nat + col];
      v[j] = tc[j] >= 0 ? a : b;
    }
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const int i = tid + j * TAIL_THREADS;
      if (i < rows) data[i] = v[j];
    }
  }
  tail_wait_mem();
  __syncthreads();
  for (int s = L; s >= 0; --s) {
    if (s > 0) {
      tail_copy_block(tp, s - 1, tail_block(tp, tail_lds, s - 1));
#pragma unroll
      for (int j = 0; j < TAIL_J; ++j)
        rv[j] = io.src_nat[0][(int64_t)(t1[j] < 0 ? -t1[j] - 1 : 0) * io.ld_nat + col];
      if (s > 1) {
        const int r2 = tp.st[s - 2].rows;
#pragma unroll
        for (int j = 0; j < TAIL_J; ++j)
          t2[j] = tp.trans[tp.st[s - 2].slot_off + min(tid + j * TAIL_THREADS, r2 - 1)];
      }
    } else {
      // output rows of the first trailing stage: positions of S_{p-1}, or global ids
      const int r0 = tp.st[0].rows;
      const int32_t* map = io.dst_nat[0] ? tp.gid : tp.pos;
#pragma unroll
      for (int j = 0; j < TAIL_J; ++j) t2[j] = map[tp.st[0].slot_off + min(tid + j * TAIL_THREADS, r0 - 1)];
    }
    tail_rotate<K, true>(tail_block(tp, tail_lds, s), tp.st[s].nu, tp.st[s].t, data);
    __syncthreads();
    if (s == 0) break;
    const int rn = tp.st[s - 1].rows;
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const float a = data[max(t1[j], 0)];
      v[j] = t1[j] >= 0 ? a : rv[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      const int i = tid + j * TAIL_THREADS;
      if (i < rn) data[i] = v[j];
    }
    tail_wait_mem();
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TAIL_J; ++j) {
      tc[j] = t1[j];
      t1[j] = t2[j];
    }
  }
  const int r0 = tp.st[0].rows;
  float* out = io.dst_nat[0] ? io.dst_nat[0] : io.dst_c[0];
  const int64_t ldo = io.dst_nat[0] ? io.ld_dnat : io.ld_out;
#pragma unroll
  for (int j = 0; j < TAIL_J; ++j) {
    const int i = tid + j * TAIL_THREADS;
    if (i < r0) out[(int64_t)t2[j] * ldo + col] = data[i];
  }
}

// the kernel's dynamic LDS limit raised to the device's per-workgroup maximum, once per kernel
// and device (the plans never ask for more than that)
template <class F>
static hipError_t tail_lds_limit(F* kernel) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;  // (kernel, device)
  int dev = 0, cap = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  const auto key = std::make_pair((const void*)kernel, dev);
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(key)) return hipSuccess;
  err = hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (err == hipSuccess)
    err = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
  if (err == hipSuccess) done.insert(key);
  return err;
}
template <int K>
static hipError_t tail_launch_fwd(const TailPlan& tp, const FwdIO& io, hipStream_t s) {
  const hipError_t e = tail_lds_limit(k_tail_fwd<K>);
  if (e != hipSuccess) return e;
  k_tail_fwd<K><<<(unsigned)(io.nrhs * (io.src[1] ? 2 : 1)), TAIL_THREADS, tp.lds_bytes, s>>>(
      tp, io);
  return hipGetLastError();
}
template <int K>
static hipError_t tail_launch_rev(const TailPlan& tp, const RevIO& io, hipStream_t s) {
  const hipError_t e = tail_lds_limit(k_tail_rev<K>);
  if (e != hipSuccess) return e;
  k_tail_rev<K><<<(unsigned)io.nrhs, TAIL_THREADS, tp.lds_bytes, s>>>(tp, io);
  return hipGetLastError();
}

hipError_t launch_tail_fwd(int k, const TailPlan& tp, const FwdIO& io, hipStream_t s) {
  if (io.nrhs == 0 || tp.nst == 0) return hipSuccess;
  if (tp.nst < 2 || tp.nst > TAIL_MAX_STAGES || tp.st[0].rows > TAIL_THREADS * TAIL_J)
    return hipErrorInvalidValue;
  return k == 2 ? tail_launch_fwd<2>(tp, io, s) : tail_launch_fwd<3>(tp, io, s);
}
hipError_t launch_tail_rev(int k, const TailPlan& tp, const RevIO& io, hipStream_t s) {
  if (io.nrhs == 0 || tp.nst == 0) return hipSuccess;
  if (tp.nst < 2 || tp.nst > TAIL_MAX_STAGES || tp.st[0].rows > TAIL_THREADS * TAIL_J ||
      io.mode[0] != 0)
    return hipErrorInvalidValue;
  return k == 2 ? tail_launch_rev<2>(tp, io, s) : tail_launch_rev<3>(tp, io, s);
}

__global__ void k_tail_params(int64_t n, int k, const int32_t* __restrict__ idx,
                              const int64_t* __restrict__ dst, const float* __restrict__ rot_o,
                              float* __restrict__ blob) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t r = idx[e], d = dst[e];
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) blob[d + a * k + b] = rot_o[r * 9 + a * 3 + b];
}
hipError_t launch_tail_params(int64_t n, int k, const int32_t* idx, const int64_t* dst,
                              const float* rot_o, uint8_t* blob, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_tail_params<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, k, idx, dst, rot_o,
                                                          reinterpret_cast<float*>(blob));
  return hipGetLastError();
}

// core rows: compact buffer of the final active set -> natural rows of the core ids
__global__ void k_gather_rows(int64_t rows, const float* __restrict__ src, int64_t lds,
                              const int32_t* __restrict__ idx, float* __restrict__ dst,
                              int64_t ldd, int64_t ncol, int scatter) {
  const int64_t r = blockIdx.x;
  const int64_t gi = idx[r];
  for (int64_t w = threadIdx.x; w < ncol; w += blockDim.x) {
    if (scatter) dst[gi * ldd + w] = src[r * lds + w];
    else dst[r * ldd + w] = src[gi * lds + w];
  }
}
hipError_t launch_gather_rows(int64_t rows, const float* src, int64_t lds, const int32_t* idx,
                              float* dst, int64_t ldd, int64_t ncol, int scatter, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  k_gather_rows<<<(unsigned)rows, 256, 0, s>>>(rows, src, lds, idx, dst, ldd, ncol, scatter);
  return hipGetLastError();
}

// (cos, sin) of every Givens rotation from its angle, in the canonical and the sweep logs
__global__ void k_sync_angles(int64_t R, const float* __restrict__ theta, float* __restrict__ rot_o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R) return;
  float s, c;
  sincosf(theta[i], &s, &c);
  rot_o[i * 9 + 0] = c;
  rot_o[i * 9 + 1] = -s;
  rot_o[i * 9 + 3] = s;
  rot_o[i * 9 + 4] = c;
}
__global__ void k_sync_sweep(int t, const int32_t* __restrict__ sw_idx,
                             const float* __restrict__ theta, float* __restrict__ sw_o) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= t) return;
  float s, c;
  sincosf(theta[sw_idx[q]], &s, &c);
  sw_o[(size_t)q * 4 + 0] = c;
  sw_o[(size_t)q * 4 + 1] = -s;
  sw_o[(size_t)q * 4 + 2] = s;
  sw_o[(size_t)q * 4 + 3] = c;
}
hipError_t launch_sync_angles(int64_t R, const float* theta, float* rot_o, hipStream_t s) {
  if (R == 0) return hipSuccess;
  k_sync_angles<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(R, theta, rot_o);
  return hipGetLastError();
}
hipError_t launch_sync_sweep(int t, const int32_t* sw_idx, const float* theta, float* sw_o,
                             hipStream_t s) {
  if (t == 0) return hipSuccess;
  k_sync_sweep<<<(t + 255) / 256, 256, 0, s>>>(t, sw_idx, theta, sw_o);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Angles of 3-point rotations: O_t = expm(W(w_t)) O0_t with W(w) = w_0 G_01 + w_1 G_02 + w_2 G_12
// and G_pq = E_qp - E_pq.  In axis form W(w) = hat(v), v = (w_2, -w_1, w_0) (hat(v) x = v x x), so
// expm follows Rodrigues' formula and the derivative of the exponential map is the left Jacobian
// J(v) = I + (1 - cos f)/f^2 hat(v) + (f - sin f)/f^3 hat(v)^2, f = |v|:
//     d expm(hat(v)) = hat(J(v) dv) expm(hat(v)).
// Both evaluated in FP64 (series near f = 0).
__device__ inline void so3_coeffs(double f2, double& a, double& b, double& c) {
  // a = sin f / f, b = (1 - cos f) / f^2, c = (f - sin f) / f^3
  if (f2 < 1e-8) {
    a = 1.0 - f2 / 6.0;
    b = 0.5 - f2 / 24.0;
    c = 1.0 / 6.0 - f2 / 120.0;
  } else {
    const double f = sqrt(f2);
    a = sin(f) / f;
    b = (1.0 - cos(f)) / f2;
    c = (f - sin(f)) / (f2 * f);
  }
}

__device__ inline void hat3(const double (&v)[3], double (&K)[3][3]) {
  K[0][0] = 0.0;   K[0][1] = -v[2]; K[0][2] = v[1];
  K[1][0] = v[2];  K[1][1] = 0.0;   K[1][2] = -v[0];
  K[2][0] = -v[1]; K[2][1] = v[0];  K[2][2] = 0.0;
}

// O_t = expm(W(w_t)) O0_t for every rotation (rot_o row-major [R][9])
__global__ void k_sync_rot3(int64_t R, const float* __restrict__ theta,
                            const float* __restrict__ o0, float* __restrict__ rot_o) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R) return;
  const double v[3] = {theta[3 * t + 2], -(double)theta[3 * t + 1], theta[3 * t + 0]};
  double K[3][3], E[3][3], a, b, c;
  hat3(v, K);
  so3_coeffs(v[0] * v[0] + v[1] * v[1] + v[2] * v[2], a, b, c);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double k2 = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) k2 += K[i][m] * K[m][j];
      E[i][j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * k2;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) acc += E[i][m] * (double)o0[t * 9 + m * 3 + j];
      rot_o[t * 9 + i * 3 + j] = (float)acc;
    }
}

// sweep-log blocks (k x k = 3 x 3 per entry) from the canonical blocks
__global__ void k_sync_sweep3(int t, const int32_t* __restrict__ sw_idx,
                              const float* __restrict__ rot_o, float* __restrict__ sw_o) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= t) return;
  const int64_t r = sw_idx[q];
#pragma unroll
  for (int ab = 0; ab < 9; ++ab) sw_o[(size_t)q * 9 + ab] = rot_o[r * 9 + ab];
}

// d/dw from the plane derivatives l (along exp(eps G_m) O_t): with P the map w -> v above (a
// signed permutation), dO = hat(J(v) P dw) O, so d/dw = P^T J(v)^T P l
__global__ void k_theta3_chain(int64_t R, const float* __restrict__ theta, float* __restrict__ g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R) return;
  const double v[3] = {theta[3 * t + 2], -(double)theta[3 * t + 1], theta[3 * t + 0]};
  double K[3][3], a, b, c;
  hat3(v, K);
  so3_coeffs(v[0] * v[0] + v[1] * v[1] + v[2] * v[2], a, b, c);
  // P l in axis form
  const double pl[3] = {g[3 * t + 2], -(double)g[3 * t + 1], g[3 * t + 0]};
  double y[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {  // y = J^T (P l), J = I + b K + c K^2
    double acc = pl[j];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double k2 = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) k2 += K[i][m] * K[m][j];
      acc += (b * K[i][j] + c * k2) * pl[i];
    }
    y[j] = acc;
  }
  // P^T y: w_0 <- v_z, w_1 <- -v_y, w_2 <- v_x
  g[3 * t + 0] = (float)y[2];
  g[3 * t + 1] = (float)-y[1];
  g[3 * t + 2] = (float)y[0];
}

hipError_t launch_sync_rot3(int64_t R, const float* theta, const float* o0, float* rot_o,
                            hipStream_t s) {
  if (R == 0) return hipSuccess;
  k_sync_rot3<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(R, theta, o0, rot_o);
  return hipGetLastError();
}
hipError_t launch_sync_sweep3(int t, const int32_t* sw_idx, const float* rot_o, float* sw_o,
                              hipStream_t s) {
  if (t == 0) return hipSuccess;
  k_sync_sweep3<<<(t + 255) / 256, 256, 0, s>>>(t, sw_idx, rot_o, sw_o);
  return hipGetLastError();
}
hipError_t launch_theta3_chain(int64_t R, const float* theta, float* g, hipStream_t s) {
  if (R == 0) return hipSuccess;
  k_theta3_chain<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(R, theta, g);
  return hipGetLastError();
}

}  // namespace pmmf
