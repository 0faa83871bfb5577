// Factorization kernels for pMMF on gfx950 (wave64).  See factor_kernels.h for the data layout.
#include "factor_kernels.h"

#include <algorithm>
#include <climits>

namespace pmmf {

// ------------------------------------------------------------------------------------------
// cluster of every position
__global__ void k_fill_cluster_of(const int32_t* __restrict__ off, int m, int S,
                                  int32_t* __restrict__ cl_of) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S) return;
  int lo = 0, hi = m - 1;  // last u with off[u] <= q
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= q) lo = mid; else hi = mid - 1;
  }
  cl_of[q] = lo;
}

hipError_t launch_fill_cluster_of(const int32_t* off, int m, int S, int32_t* cl_of, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_fill_cluster_of<<<(S + 255) / 256, 256, 0, s>>>(off, m, S, cl_of);
  return hipGetLastError();
}

__device__ inline int64_t lower_bound_i32(const int32_t* __restrict__ a, int64_t lo, int64_t hi,
                                          int32_t key) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------------------------------
// Cluster Gram, diagonal block and identity rotation accumulator (Sec. 2.1: G^u = A_Bu^T A_Bu).
// One wave per position a (row la of its cluster u).  Row la of G is
//     G[la, b] = sum_r M[a, r] * M[r, o_u + b],  b in [0, c_u)
// i.e. the inner products of column a with the cluster's columns over all active rows r (M is
// symmetric, so column a's entries are row a's).  The row is accumulated in LDS in ascending r
// (deterministic) and written densely, which also clears the previous stage's contents.
// Run table of the active matrix: for every row, the maximal runs of columns in one cluster
// (clusters are contiguous position ranges and columns ascend, so a row meets each cluster in at
// most one run), as (cluster, first entry) pairs in ascending cluster order.
__global__ void k_runs(int S, int fill, const int64_t* __restrict__ rp,
                       const int32_t* __restrict__ ci, const int32_t* __restrict__ cl_of,
                       int32_t* __restrict__ nruns, const int64_t* __restrict__ run_ptr,
                       int32_t* __restrict__ run_cl, int64_t* __restrict__ run_start) {
  const int r = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (r >= S) return;
  const int lane = pmmf_lane();
  const int64_t r0 = rp[r], r1 = rp[r + 1];
  int64_t out = fill ? run_ptr[r] : 0;
  int prev = -1;  // cluster of the entry before the current chunk
  for (int64_t t0 = r0; t0 < r1; t0 += PMMF_WAVE) {
    const int64_t t = t0 + lane;
    const int cl = t < r1 ? cl_of[ci[t]] : INT_MAX;
    int left = __shfl_up(cl, 1);
    if (lane == 0) left = prev;
    const bool head = t < r1 && cl != left;
    const uint64_t b = __ballot(head);
    if (fill && head) {
      const int64_t pos = out + pmmf_lanes_below(b);
      run_cl[pos] = cl;
      run_start[pos] = t;
    }
    out += __popcll(b);
    prev = __shfl(cl, PMMF_WAVE - 1);
  }
  if (!fill && lane == 0) nruns[r] = (int32_t)out;
}

hipError_t launch_runs(int S, int fill, const int64_t* rp, const int32_t* ci,
                       const int32_t* cl_of, int32_t* nruns, const int64_t* run_ptr,
                       int32_t* run_cl, int64_t* run_start, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_runs<<<(S + 3) / 4, 256, 0, s>>>(S, fill, rp, ci, cl_of, nruns, run_ptr, run_cl, run_start);
  return hipGetLastError();
}

// Useful work of the stage's cluster Grams: G^u = A[:, B_u]^T A[:, B_u] takes, from each row, the
// products of the row's entries in B_u with each other, |seg(row, u)|^2 multiply-adds per run.
// One thread per row sums them over its runs; one atomic add per wave.
__global__ void k_gram_work(int S, const int64_t* __restrict__ rp,
                            const int64_t* __restrict__ run_ptr,
                            const int64_t* __restrict__ run_start,
                            unsigned long long* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long w = 0;
  if (r < S) {
    const int64_t q0 = run_ptr[r], q1 = run_ptr[r + 1];
    for (int64_t q = q0; q < q1; ++q) {
      const int64_t len = (q + 1 < q1 ? run_start[q + 1] : rp[r + 1]) - run_start[q];
      w += (unsigned long long)(len * len);
    }
  }
  for (int d = PMMF_WAVE / 2; d > 0; d >>= 1) w += __shfl_xor(w, d);
  if (pmmf_lane() == 0 && w) atomicAdd(out, w);
}

hipError_t launch_gram_work(int S, const int64_t* rp, const int64_t* run_ptr,
                            const int64_t* run_start, unsigned long long* out, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_gram_work<<<(S + 255) / 256, 256, 0, s>>>(S, rp, run_ptr, run_start, out);
  return hipGetLastError();
}

// Up to GRAM_ITEM consecutive 64-entry chunks of one row segment: entries from off on (rem of
// them left in the segment) of the segment that starts at ci/cv index base, scaled by w.  All
// fields are wave-uniform (scalar registers).
struct GramItem {
  int64_t base;
  int off, rem;
  float w;
};
// One 64-entry chunk of a row segment (entries [off, off + rem) of the segment at base), for
// stages with short segments, where items of one segment would leave most of their chunks empty.
struct GramChunk {
  int64_t base;
  int off, rem;
  float w;
};
constexpr int GRAM_ITEM = 4;  // chunks whose loads are requested together
template <bool SEGMENT_ITEMS>
__global__ void __launch_bounds__(256) k_gram(int S, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci,
                                              const float* __restrict__ cv,
                                              const int32_t* __restrict__ off,
                                              const int32_t* __restrict__ cl_of,
                                              const int64_t* __restrict__ gbase,
                                              const int64_t* __restrict__ run_ptr,
                                              const int32_t* __restrict__ run_cl,
                                              const int64_t* __restrict__ run_start,
                                              float2* __restrict__ GD, int cmax) {
  extern __shared__ float lds_f[];
  const int wpb = blockDim.x / PMMF_WAVE;
  const int w = pmmf_wave(), lane = pmmf_lane();
  // cmax accumulator slots, then one spare slot per lane that takes the zero contributions of
  // lanes past a segment's end (so every lane adds unconditionally and no two lanes of one
  // chunk touch the same slot)
  float* acc = lds_f + (size_t)w * (cmax + PMMF_WAVE);
  // the positions of a cluster read the same row segments: keep them on one XCD (one L2)
  const int a = pmmf_xcd_block(blockIdx.x, gridDim.x) * wpb + w;
  if (a >= S) return;
  const int u = cl_of[a];
  const int o = off[u];
  const int c = off[u + 1] - o;
  const int la = a - o;
  for (int j = lane; j < c; j += PMMF_WAVE) acc[j] = 0.f;
  const int spare = cmax + lane;
  const int64_t a0 = rp[a], a1 = rp[a + 1];
  for (int64_t kb = a0; kb < a1; kb += PMMF_WAVE) {
    // each lane locates the cluster-u segment of one row r = ci[kb + lane]
    const int nb = (int)min<int64_t>(PMMF_WAVE, a1 - kb);
    int64_t lb = 0;
    int len = 0;
    float wr = 0.f;
    if (lane < nb) {
      // row r's run of columns in cluster u, from its run table (clusters ascending)
      const int r = ci[kb + lane];
      wr = cv[kb + lane];
      int64_t lo = run_ptr[r], hi = run_ptr[r + 1];
      const int64_t re = hi;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (run_cl[mid] < u) lo = mid + 1;
        else hi = mid;
      }
      if (lo < re && run_cl[lo] == u) {
        lb = run_start[lo];
        len = (int)((lo + 1 < re ? run_start[lo + 1] : rp[r + 1]) - lb);
      }
    }
    if constexpr (SEGMENT_ITEMS) {
      // Walk the non-empty segments in ascending r with a wave-uniform cursor, in items of up to
      // GRAM_ITEM consecutive chunks of one segment (the scalar work is per item); the loads of
      // the next item are requested before the current one is added.  The entries of one segment
      // hit distinct columns, so each column still sums in ascending r.
      uint64_t left = __ballot(len > 0);
      bool live = false;  // a segment is under the cursor
      int qn = 0, qoff = 0;
      int64_t qb = 0;
      float qw = 0.f;
      auto next_seg = [&]() {
        live = left != 0;
        const int l = live ? (int)__builtin_ctzll(left) : 0;
        left &= left - 1;
        qn = __builtin_amdgcn_readlane(len, l);
        qb = ((int64_t)__builtin_amdgcn_readlane((int)(lb >> 32), l) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)lb, l);
        qw = pmmf_readlane_f(wr, l);
        qoff = 0;
      };
      next_seg();
      // an exhausted cursor yields empty items at the last segment's start (a valid address)
      auto take = [&](GramItem& g) {
        g.base = qb;
        g.off = live ? qoff : 0;
        g.rem = live ? qn - qoff : 0;
        g.w = qw;
        qoff += GRAM_ITEM * PMMF_WAVE;
        if (live && qoff >= qn) next_seg();
      };
      auto load = [&](const GramItem& g, int* col, float* val) {
        const char* cp = reinterpret_cast<const char*>(ci + g.base);
        const char* vp = reinterpret_cast<const char*>(cv + g.base);
        const int last = max(g.rem - 1, 0);
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          // lanes past the end re-read the segment's last entry (an address inside it)
          const uint32_t eb = 4u * (uint32_t)(g.off + min(lane + t * PMMF_WAVE, last));
          col[t] = *reinterpret_cast<const int32_t*>(cp + eb);
          val[t] = *reinterpret_cast<const float*>(vp + eb);
        }
      };
      auto add = [&](const GramItem& g, const int* col, const float* val) {
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          const bool ok = lane + t * PMMF_WAVE < g.rem;
          acc[ok ? col[t] - o : spare] += ok ? g.w * val[t] : 0.f;
        }
      };
      // two register sets in turn, so that no loaded value is copied (a copy waits for its load)
      GramItem g0, g1;
      int c0[GRAM_ITEM], c1[GRAM_ITEM];
      float v0[GRAM_ITEM], v1[GRAM_ITEM];
      // a fixed, even number of items (the last ones may be empty): no exit test sits between a
      // load and the add that uses it
      const int nit = __builtin_amdgcn_readlane(
          pmmf_wave_incl_scan_dpp((len + GRAM_ITEM * PMMF_WAVE - 1) / (GRAM_ITEM * PMMF_WAVE)),
          PMMF_WAVE - 1);
      const int pairs = (nit + 1) / 2;
      take(g0);
      load(g0, c0, v0);
      for (int it = 0; it < pairs; ++it) {
        take(g1);
        load(g1, c1, v1);
        add(g0, c0, v0);
        take(g0);
        load(g0, c0, v0);
        add(g1, c1, v1);
      }
    } else {
      // Walk the chunks of the non-empty segments in ascending r with a wave-uniform cursor; the
      // loads of the next GRAM_ITEM chunks are requested before the current ones are added.  The
      // entries of one segment hit distinct columns, so each column still sums in ascending r.
      uint64_t left = __ballot(len > 0);
      bool live = false;  // a segment is under the cursor
      int qn = 0, qoff = 0;
      int64_t qb = 0;
      float qw = 0.f;
      auto next_seg = [&]() {
        live = left != 0;
        const int l = live ? (int)__builtin_ctzll(left) : 0;
        left &= left - 1;
        qn = __builtin_amdgcn_readlane(len, l);
        qb = ((int64_t)__builtin_amdgcn_readlane((int)(lb >> 32), l) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)lb, l);
        qw = pmmf_readlane_f(wr, l);
        qoff = 0;
      };
      next_seg();
      // an exhausted cursor yields empty chunks at the last segment's start (a valid address)
      auto take = [&](GramChunk& g) {
        g.base = qb;
        g.off = live ? qoff : 0;
        g.rem = live ? qn - qoff : 0;
        g.w = qw;
        qoff += PMMF_WAVE;
        if (live && qoff >= qn) next_seg();
      };
      auto load = [&](const GramChunk* g, int* col, float* val) {
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          // lanes past the end re-read an entry of the segment (an address inside it)
          const uint32_t eb = 4u * (uint32_t)(g[t].off + min(lane, max(g[t].rem - 1, 0)));
          col[t] = *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(ci + g[t].base) + eb);
          val[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(cv + g[t].base) + eb);
        }
      };
      auto add = [&](const GramChunk* g, const int* col, const float* val) {
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          const bool ok = lane < g[t].rem;
          acc[ok ? col[t] - o : spare] += ok ? g[t].w * val[t] : 0.f;
        }
      };
      // two register sets in turn, so that no loaded value is copied (a copy waits for its load)
      GramChunk g0[GRAM_ITEM], g1[GRAM_ITEM];
      int c0[GRAM_ITEM], c1[GRAM_ITEM];
      float v0[GRAM_ITEM], v1[GRAM_ITEM];
      // a fixed, even number of GRAM_ITEM-chunk items (the last ones may be empty): no exit test
      // sits between a load and the add that uses it
      const int nch = __builtin_amdgcn_readlane(pmmf_wave_incl_scan_dpp((len + PMMF_WAVE - 1) >> 6),
                                                PMMF_WAVE - 1);
      const int pairs = (nch + 2 * GRAM_ITEM - 1) / (2 * GRAM_ITEM);
  #pragma unroll
      for (int t = 0; t < GRAM_ITEM; ++t) take(g0[t]);
      load(g0, c0, v0);
      for (int it = 0; it < pairs; ++it) {
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) take(g1[t]);
        load(g1, c1, v1);
        add(g0, c0, v0);
  #pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) take(g0[t]);
        load(g0, c0, v0);
        add(g1, c1, v1);
      }
    }
  }
  // Gram halves of the interleaved (G, D) row, then the diagonal-block halves through the same
  // accumulator (the two store passes write disjoint words)
  const size_t base = (size_t)gbase[u] + (size_t)la * gd_stride(c);
  float* gd = reinterpret_cast<float*>(GD + base);
  for (int j = lane; j < c; j += PMMF_WAVE) {
    gd[2 * j] = acc[j];
    acc[j] = 0.f;
  }
  const int64_t lb = lower_bound_i32(ci, a0, a1, o);
  const int64_t ub = lower_bound_i32(ci, lb, a1, o + c);
  for (int64_t t = lb + lane; t < ub; t += PMMF_WAVE) acc[ci[t] - o] = cv[t];
  for (int j = lane; j < c; j += PMMF_WAVE) gd[2 * j + 1] = acc[j];
}

// ------------------------------------------------------------------------------------------
// Dense form of the cluster Gram for dense active matrices (late stages).  The active matrix is
// expanded to a row-major S x S array; cluster u's Gram G = A[:, B_u]^T A[:, B_u] is then a
// product of two column slices, computed in 32 x 32 tiles on v_mfma_f32_16x16x4f32 (one 16 x 16
// quarter per wave; A operand lane l holds (row l % 16, k = l / 16), B operand (k = l / 16,
// column l % 16), result row 4 (l / 16) + r, column l % 16 in register r).  Only tiles with
// ti <= tj are computed; each is stored at (ti, tj) and transposed at (tj, ti).  The diagonal
// block D is read from the same array (row i of the block = row o + i of A), Q starts at I.
__global__ void k_densify(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const float* __restrict__ cv, float* __restrict__ dense) {
  const int row = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (row >= S) return;
  for (int64_t t = rp[row] + pmmf_lane(); t < rp[row + 1]; t += PMMF_WAVE)
    dense[(size_t)row * S + ci[t]] = cv[t];
}

typedef float pmmf_gf4 __attribute__((ext_vector_type(4)));
constexpr int DG_T = 32, DG_K = 128, DG_PER = DG_T * DG_K / 256;
__global__ void __launch_bounds__(256) k_gram_dense(int S, const float* __restrict__ dense,
                                                    const int32_t* __restrict__ off,
                                                    const int64_t* __restrict__ gbase,
                                                    float2* __restrict__ GD, int ntmax) {
  __shared__ float As[DG_T][DG_K + 1];
  __shared__ float Bs[DG_K][DG_T + 1];
  const int u = blockIdx.y;
  const int o = off[u], c = off[u + 1] - o;
  const int nt = (c + DG_T - 1) / DG_T;
  // upper-triangle tile (ti, tj), ti <= tj, from the linear block index
  int t = blockIdx.x, ti = 0;
  while (ti < ntmax && t >= ntmax - ti) { t -= ntmax - ti; ++ti; }
  const int tj = ti + t;
  if (ti >= nt || tj >= nt) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
  const int ca = o + ti * DG_T, cb = o + tj * DG_T;  // first columns of the two slices
  const int lima = min(DG_T, c - ti * DG_T), limb = min(DG_T, c - tj * DG_T);
  float ra[DG_PER], rb[DG_PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int p = 0; p < DG_PER; ++p) {
      const int q = tid + p * 256;
      const int k = q / DG_T, m = q % DG_T;
      const bool okk = k0 + k < S;
      const size_t rowoff = (size_t)(k0 + k) * S;
      ra[p] = (okk && m < lima) ? dense[rowoff + ca + m] : 0.f;
      rb[p] = (okk && m < limb) ? dense[rowoff + cb + m] : 0.f;
    }
  };
  pmmf_gf4 acc = {0.f, 0.f, 0.f, 0.f};
  fetch(0);
  for (int k0 = 0; k0 < S; k0 += DG_K) {
#pragma unroll
    for (int p = 0; p < DG_PER; ++p) {
      const int q = tid + p * 256;
      const int k = q / DG_T, m = q % DG_T;
      As[m][k] = ra[p];
      Bs[k][m] = rb[p];
    }
    __syncthreads();
    if (k0 + DG_K < S) fetch(k0 + DG_K);
#pragma unroll 8
    for (int kk = 0; kk < DG_K; kk += 4) {
      const float av = As[wm + (lane & 15)][kk + (lane >> 4)];
      const float bv = Bs[kk + (lane >> 4)][wn + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const size_t base = (size_t)gbase[u];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * DG_T + wm + 4 * (lane >> 4) + r;
    const int j = tj * DG_T + wn + (lane & 15);
    if (i < c && j < c) {
      GD[base + (size_t)i * gd_stride(c) + j] =
          make_float2(acc[r], dense[(size_t)(o + i) * S + o + j]);
      if (ti != tj)
        GD[base + (size_t)j * gd_stride(c) + i] =
            make_float2(acc[r], dense[(size_t)(o + j) * S + o + i]);
    }
  }
}

hipError_t launch_gram_dense(int S, const int64_t* rp, const int32_t* ci, const float* cv,
                             float* dense, const int32_t* off, int m, const int64_t* gbase,
                             float2* GD, int cmax, hipStream_t s) {
  if (S == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(dense, 0, (size_t)S * S * sizeof(float), s);
  if (e != hipSuccess) return e;
  k_densify<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, cv, dense);
  const int ntmax = (cmax + DG_T - 1) / DG_T;
  dim3 grid((unsigned)(ntmax * (ntmax + 1) / 2), (unsigned)m);
  k_gram_dense<<<grid, 256, 0, s>>>(S, dense, off, gbase, GD, ntmax);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// BF16 form of the cluster Gram.  Cluster u's slab is S_u = A[R_u, B_u] with R_u the positions
// whose rows touch B_u (the union of the patterns of the rows of B_u, by symmetry); it is stored
// column-major (column j of the cluster contiguous over the R_u rows, in ascending position
// order), once in FP32 (kept for exact rescoring during the search and right-rotated with it) and
// once rounded to BF16 (nearest even).  G~ = bf16(S)^T bf16(S) is formed on
// v_mfma_f32_16x16x16bf16_1k with FP32 accumulation; its diagonal is then replaced by the exact
// FP32 column norms.  R_u is found with one bitmap of positions per cluster and a popcount prefix.
__device__ inline unsigned short pmmf_bf16_rne(float f) {
  const uint32_t b = __builtin_bit_cast(uint32_t, f);
  if ((b & 0x7f800000u) == 0x7f800000u) return (unsigned short)(b >> 16);  // inf / nan kept
  return (unsigned short)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__global__ void k_slab_mark(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const int32_t* __restrict__ cl_of, int64_t W,
                            uint32_t* __restrict__ bm) {
  const int a = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (a >= S) return;
  uint32_t* b = bm + (size_t)cl_of[a] * W;
  for (int64_t t = rp[a] + pmmf_lane(); t < rp[a + 1]; t += PMMF_WAVE) {
    const int r = ci[t];
    atomicOr(b + (r >> 5), 1u << (r & 31));
  }
}

// exclusive popcount prefix over each cluster's bitmap words; R[u] = the cluster's row count
__global__ void __launch_bounds__(256) k_slab_prefix(int64_t W, const uint32_t* __restrict__ bm,
                                                     int32_t* __restrict__ pre,
                                                     int32_t* __restrict__ R) {
  __shared__ int part[256];
  const int u = blockIdx.x, tid = threadIdx.x;
  const uint32_t* b = bm + (size_t)u * W;
  int32_t* pr = pre + (size_t)u * W;
  const int64_t per = (W + 255) / 256;
  const int64_t w0 = tid * per, w1 = min<int64_t>(W, w0 + per);
  int cnt = 0;
  for (int64_t w = w0; w < w1; ++w) cnt += __popc(b[w]);
  part[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - cnt;
  for (int64_t w = w0; w < w1; ++w) {
    pr[w] = run;
    run += __popc(b[w]);
  }
  if (tid == 255) R[u] = part[255];
}

__global__ void k_slab_fill(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const float* __restrict__ cv, const int32_t* __restrict__ off,
                            const int32_t* __restrict__ cl_of, int64_t W,
                            const uint32_t* __restrict__ bm, const int32_t* __restrict__ pre,
                            const int64_t* __restrict__ slab_off, const int32_t* __restrict__ R,
                            float* __restrict__ slab, unsigned short* __restrict__ slab_bf) {
  const int a = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (a >= S) return;
  const int u = cl_of[a];
  const int j = a - off[u];
  const uint32_t* b = bm + (size_t)u * W;
  const int32_t* pr = pre + (size_t)u * W;
  const size_t col = (size_t)slab_off[u] + (size_t)j * R[u];
  for (int64_t t = rp[a] + pmmf_lane(); t < rp[a + 1]; t += PMMF_WAVE) {
    const int r = ci[t];
    const int rho = pr[r >> 5] + __popc(b[r >> 5] & ((1u << (r & 31)) - 1u));
    slab[col + rho] = cv[t];
    slab_bf[col + rho] = pmmf_bf16_rne(cv[t]);
  }
}

typedef short pmmf_s4 __attribute__((ext_vector_type(4)));
constexpr int BG_T = 32, BG_K = 64;
__global__ void __launch_bounds__(256) k_gram_bf16(const unsigned short* __restrict__ slab_bf,
                                                   const int32_t* __restrict__ off,
                                                   const int64_t* __restrict__ gbase,
                                                   const int64_t* __restrict__ slab_off,
                                                   const int32_t* __restrict__ R,
                                                   float2* __restrict__ GD, int ntmax) {
  __shared__ unsigned short As[BG_T][BG_K + 4];
  __shared__ unsigned short Bs[BG_T][BG_K + 4];
  const int u = blockIdx.y;
  const int o = off[u], c = off[u + 1] - o;
  const int nt = (c + BG_T - 1) / BG_T;
  int t = blockIdx.x, ti = 0;
  while (ti < ntmax && t >= ntmax - ti) { t -= ntmax - ti; ++ti; }
  const int tj = ti + t;
  if (ti >= nt || tj >= nt) return;
  const int Ru = R[u];
  const unsigned short* Sb = slab_bf + slab_off[u];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
  pmmf_gf4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Ru; k0 += BG_K) {
    // 32 columns x 64 rows of each slice: thread -> (column, 8 consecutive rows)
    {
      const int cc = tid >> 3, kk = (tid & 7) * 8;
      const int ia = ti * BG_T + cc, ib = tj * BG_T + cc;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + kk + e;
        As[cc][kk + e] = (ia < c && k < Ru) ? Sb[(size_t)ia * Ru + k] : (unsigned short)0;
        Bs[cc][kk + e] = (ib < c && k < Ru) ? Sb[(size_t)ib * Ru + k] : (unsigned short)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BG_K; kk += 16) {
      pmmf_s4 av, bv;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        av[e] = (short)As[wm + (lane & 15)][kk + 4 * (lane >> 4) + e];
        bv[e] = (short)Bs[wn + (lane & 15)][kk + 4 * (lane >> 4) + e];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const size_t base = (size_t)gbase[u];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ti * BG_T + wm + 4 * (lane >> 4) + r;
    const int j = tj * BG_T + wn + (lane & 15);
    if (i < c && j < c) {
      GD[base + (size_t)i * gd_stride(c) + j] = make_float2(acc[r], 0.f);
      if (ti != tj) GD[base + (size_t)j * gd_stride(c) + i] = make_float2(acc[r], 0.f);
    }
  }
}

// diagonal block D (row a's entries inside its cluster) into the second halves, and the exact
// FP32 column norm ||S_j||^2 onto G~'s diagonal
__global__ void k_slab_finish(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const float* __restrict__ cv, const int32_t* __restrict__ off,
                              const int32_t* __restrict__ cl_of, const int64_t* __restrict__ gbase,
                              const int64_t* __restrict__ slab_off, const int32_t* __restrict__ R,
                              const float* __restrict__ slab, float2* __restrict__ GD) {
  const int a = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (a >= S) return;
  const int lane = pmmf_lane();
  const int u = cl_of[a];
  const int o = off[u], c = off[u + 1] - o, j = a - o;
  float* gd = reinterpret_cast<float*>(GD + (size_t)gbase[u] + (size_t)j * gd_stride(c));
  for (int64_t t = rp[a] + lane; t < rp[a + 1]; t += PMMF_WAVE) {
    const int col = ci[t];
    if (col >= o && col < o + c) gd[2 * (col - o) + 1] = cv[t];
  }
  const int Ru = R[u];
  const float* col = slab + slab_off[u] + (size_t)j * Ru;
  float acc = 0.f;
  for (int rho = lane; rho < Ru; rho += PMMF_WAVE) acc += col[rho] * col[rho];
  acc = pmmf_wave_sum_dpp(acc);
  if (lane == 0) gd[2 * j] = acc;
}

hipError_t launch_slab_rows(int S, int m, const int64_t* rp, const int32_t* ci,
                            const int32_t* cl_of, int64_t W, uint32_t* bm, int32_t* pre,
                            int32_t* R, hipStream_t s) {
  if (S == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(bm, 0, (size_t)m * W * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  k_slab_mark<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, cl_of, W, bm);
  k_slab_prefix<<<m, 256, 0, s>>>(W, bm, pre, R);
  return hipGetLastError();
}

hipError_t launch_gram_bf16(int S, int m, const int64_t* rp, const int32_t* ci, const float* cv,
                            const int32_t* off, const int32_t* cl_of, int64_t W,
                            const uint32_t* bm, const int32_t* pre, const int64_t* slab_off,
                            const int32_t* R, int64_t slab_elems, float* slab,
                            unsigned short* slab_bf, const int64_t* gbase, float2* GD,
                            int cmax, hipStream_t s) {
  if (S == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(slab, 0, (size_t)slab_elems * sizeof(float), s);
  if (e == hipSuccess) e = hipMemsetAsync(slab_bf, 0, (size_t)slab_elems * sizeof(unsigned short), s);
  if (e != hipSuccess) return e;
  k_slab_fill<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, cv, off, cl_of, W, bm, pre, slab_off, R, slab,
                                          slab_bf);
  const int ntmax = (cmax + BG_T - 1) / BG_T;
  dim3 grid((unsigned)(ntmax * (ntmax + 1) / 2), (unsigned)m);
  k_gram_bf16<<<grid, 256, 0, s>>>(slab_bf, off, gbase, slab_off, R, GD, ntmax);
  k_slab_finish<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, cv, off, cl_of, gbase, slab_off, R, slab, GD);
  return hipGetLastError();
}

hipError_t launch_gram(int S, int64_t rp_nnz, const int64_t* rp, const int32_t* ci,
                       const float* cv, const int32_t* off, const int32_t* cl_of,
                       const int64_t* gbase, const int64_t* run_ptr, const int32_t* run_cl,
                       const int64_t* run_start, float2* GD, int cmax, hipStream_t s, int wpb_cfg,
                       int form) {
  if (S == 0) return hipSuccess;
  int wpb = wpb_cfg > 0 ? wpb_cfg : 4;
  while (wpb > 1 && (size_t)wpb * (cmax + PMMF_WAVE) * 4 > 64 * 1024) wpb >>= 1;
  const size_t lds = (size_t)wpb * (cmax + PMMF_WAVE) * sizeof(float);
  // default: items of one segment once rows are long (their segments then span several chunks)
  const int64_t nnz = rp_nnz;
  const bool seg = form >= 0 ? form == 1 : nnz >= 128 * (int64_t)S;
  auto kern = seg ? k_gram<true> : k_gram<false>;
  kern<<<(S + wpb - 1) / wpb, wpb * PMMF_WAVE, lds, s>>>(S, rp, ci, cv, off, cl_of, gbase, run_ptr,
                                                         run_cl, run_start, GD, cmax);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// FP64 k x k rotations (Sec. 2.2: the rotation diagonalizes the k x k Gram block).

// 2x2 symmetric Schur decomposition (Golub & Van Loan Alg. 8.4.1) with |theta| <= pi/4.
// Returns O = [[c, -s], [s, c]] with O g O^T diagonal; O = I when the coupling is zero.
__device__ inline void rot2(double a, double b, double d, double& c, double& s, double& tau_abs) {
  if (b == 0.0) {
    c = 1.0; s = 0.0; tau_abs = 1e300;
    return;
  }
  const double tau = (d - a) / (2.0 * b);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  const double t = sg / (fabs(tau) + hypot(1.0, tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  tau_abs = fabs(tau);
}

// 3x3: cyclic Jacobi eigendecomposition, eigenvectors in descending eigenvalue order as rows,
// then the row permutation and signs maximizing trace(O) with O_rr >= 0 (lexicographically
// smallest permutation on ties).  Written with static indices only, so every array stays in
// registers.
// reciprocal and reciprocal square root: hardware estimates refined by two Newton steps each
// (within an ulp or two; the rotation is converged to the same fixed point either way)
__device__ inline double nr_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ inline double nr_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

__device__ inline void jacobi_pair(double (&A)[3][3], double (&V)[3][3], int p, int q, bool& rot) {
  const double apq = A[p][q];
  if (fabs(apq) <= 1e-18 * (fabs(A[p][p]) + fabs(A[q][q]))) {
    A[p][q] = A[q][p] = 0.0;
    return;
  }
  rot = true;
  const double tau = (A[q][q] - A[p][p]) * nr_rcp(2.0 * apq);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  const double r1 = fma(tau, tau, 1.0);
  const double t = sg * nr_rcp(fabs(tau) + r1 * nr_rsq(r1));
  const double c = nr_rsq(fma(t, t, 1.0));
  const double s = t * c;
  // A <- J^T A J with J = [[c, s], [-s, c]] on (p, q); V <- V J
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double arp = A[r][p], arq = A[r][q];
    A[r][p] = c * arp - s * arq;
    A[r][q] = s * arp + c * arq;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double apr = A[p][r], aqr = A[q][r];
    A[p][r] = c * apr - s * aqr;
    A[q][r] = s * apr + c * aqr;
  }
  A[p][q] = A[q][p] = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double vrp = V[r][p], vrq = V[r][q];
    V[r][p] = c * vrp - s * vrq;
    V[r][q] = s * vrp + c * vrq;
  }
}

// Arrangement of an eigendecomposition (eigenvalues e0..e2, eigenvectors the columns of V) as
// described above.
__device__ inline void arrange3(double e0, double e1, double e2, const double (&V)[3][3],
                                double (&O)[3][3], double& trace_margin, double& eig_margin) {
  // columns of V sorted by descending eigenvalue (three compare-swaps on scalars)
  double b00 = V[0][0], b01 = V[1][0], b02 = V[2][0];   // b0 = eigenvector of e0 (column 0)
  double b10 = V[0][1], b11 = V[1][1], b12 = V[2][1];
  double b20 = V[0][2], b21 = V[1][2], b22 = V[2][2];
#define PMMF_CSWAP(ex, ey, x0, x1, x2, y0, y1, y2)                              \
  if (ey > ex) {                                                               \
    double t_ = ex; ex = ey; ey = t_;                                          \
    t_ = x0; x0 = y0; y0 = t_; t_ = x1; x1 = y1; y1 = t_; t_ = x2; x2 = y2; y2 = t_; \
  }
  PMMF_CSWAP(e0, e1, b00, b01, b02, b10, b11, b12)
  PMMF_CSWAP(e0, e2, b00, b01, b02, b20, b21, b22)
  PMMF_CSWAP(e1, e2, b10, b11, b12, b20, b21, b22)
#undef PMMF_CSWAP
  const double emax = fmax(fabs(e0), fabs(e2));
  eig_margin = emax > 0.0 ? fmin(e0 - e1, e1 - e2) / emax : 0.0;
  const double b[3][3] = {{b00, b01, b02}, {b10, b11, b12}, {b20, b21, b22}};
  // traces of the six row permutations, in lexicographic order
  const double tr0 = fabs(b00) + fabs(b11) + fabs(b22);  // (0,1,2)
  const double tr1 = fabs(b00) + fabs(b21) + fabs(b12);  // (0,2,1)
  const double tr2 = fabs(b10) + fabs(b01) + fabs(b22);  // (1,0,2)
  const double tr3 = fabs(b10) + fabs(b21) + fabs(b02);  // (1,2,0)
  const double tr4 = fabs(b20) + fabs(b01) + fabs(b12);  // (2,0,1)
  const double tr5 = fabs(b20) + fabs(b11) + fabs(b02);  // (2,1,0)
  int best = 0;
  double bt = tr0, second = -1.0;
#define PMMF_PICK(trq, q)                        \
  if (trq > bt) { second = bt; bt = trq; best = q; } \
  else second = fmax(second, trq);
  PMMF_PICK(tr1, 1)
  PMMF_PICK(tr2, 2)
  PMMF_PICK(tr3, 3)
  PMMF_PICK(tr4, 4)
  PMMF_PICK(tr5, 5)
#undef PMMF_PICK
  trace_margin = bt > 0.0 ? (bt - second) / bt : 0.0;
  int p0, p1, p2;
  switch (best) {
    case 0: p0 = 0; p1 = 1; p2 = 2; break;
    case 1: p0 = 0; p1 = 2; p2 = 1; break;
    case 2: p0 = 1; p1 = 0; p2 = 2; break;
    case 3: p0 = 1; p1 = 2; p2 = 0; break;
    case 4: p0 = 2; p1 = 0; p2 = 1; break;
    default: p0 = 2; p1 = 1; p2 = 0; break;
  }
  // rows with static indices: select by comparing the permutation entries
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double r0 = p0 == 0 ? b[0][j] : (p0 == 1 ? b[1][j] : b[2][j]);
    const double r1 = p1 == 0 ? b[0][j] : (p1 == 1 ? b[1][j] : b[2][j]);
    const double r2 = p2 == 0 ? b[0][j] : (p2 == 1 ? b[1][j] : b[2][j]);
    O[0][j] = r0;
    O[1][j] = r1;
    O[2][j] = r2;
  }
  const double s0 = O[0][0] >= 0.0 ? 1.0 : -1.0;
  const double s1 = O[1][1] >= 0.0 ? 1.0 : -1.0;
  const double s2 = O[2][2] >= 0.0 ? 1.0 : -1.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    O[0][j] *= s0;
    O[1][j] *= s1;
    O[2][j] *= s2;
  }
}

// FP64 cyclic Jacobi sweeps on A (accumulated into V, A = V^T g V on entry), then the arrangement.
__device__ inline void rot3_finish(double (&A)[3][3], double (&V)[3][3], double (&O)[3][3],
                                   double& trace_margin, double& eig_margin) {
  for (int sweep = 0; sweep < 12; ++sweep) {
    bool rot = false;
    jacobi_pair(A, V, 0, 1, rot);
    jacobi_pair(A, V, 0, 2, rot);
    jacobi_pair(A, V, 1, 2, rot);
    if (!rot) break;
  }
  arrange3(A[0][0], A[1][1], A[2][2], V, O, trace_margin, eig_margin);
}

__device__ inline void rot3(const double (&g)[3][3], double (&O)[3][3], double& trace_margin,
                            double& eig_margin) {
  double A[3][3], V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { A[i][j] = g[i][j]; V[i][j] = (i == j) ? 1.0 : 0.0; }
  rot3_finish(A, V, O, trace_margin, eig_margin);
}

// FP32 cyclic Jacobi sweeps: the start of the FP64 eigendecomposition in k_find.  Off-diagonal
// pairs are rotated as 2-vectors, so their rounding is relative to their own size and the sweeps
// reach the FP32 threshold quadratically.
__device__ inline void jacobi_pair_f(float (&A)[3][3], float (&V)[3][3], int p, int q, bool& rot) {
  const float apq = A[p][q];
  // converged once the pivot is below FP32 resolution of the diagonal pair
  if (fabsf(apq) <= 1e-7f * (fabsf(A[p][p]) + fabsf(A[q][q]))) {
    A[p][q] = A[q][p] = 0.f;
    return;
  }
  rot = true;
  // t = tan(theta) = apq / (d + sign(d) sqrt(d^2 + apq^2)), d = (aqq - app) / 2 (the smaller
  // root of t^2 + 2 (d / apq) t - 1 = 0)
  const float d = 0.5f * (A[q][q] - A[p][p]);
  const float h2 = fmaf(d, d, apq * apq);
  const float den = fabsf(d) + h2 * __builtin_amdgcn_rsqf(h2);
  const float t = (d >= 0.f ? apq : -apq) * __builtin_amdgcn_rcpf(den);
  const float c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));
  const float s = t * c;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float arp = A[r][p], arq = A[r][q];
    A[r][p] = c * arp - s * arq;
    A[r][q] = s * arp + c * arq;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float apr = A[p][r], aqr = A[q][r];
    A[p][r] = c * apr - s * aqr;
    A[q][r] = s * apr + c * aqr;
  }
  A[p][q] = A[q][p] = 0.f;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float vrp = V[r][p], vrq = V[r][q];
    V[r][p] = c * vrp - s * vrq;
    V[r][q] = s * vrp + c * vrq;
  }
}

// The same FP64 eigendecomposition as rot3, started from FP32 sweeps: eigenvectors from FP32
// cyclic Jacobi, made orthonormal in FP64 by one Newton-Schulz step (V <- V (3I - V^T V) / 2, which
// squares the departure from orthogonality), then V^T g V formed in FP64 and finished by FP64
// Jacobi sweeps, which from off-diagonal entries at FP32 resolution converge in one or two
// sweeps instead of the four or five a start from the identity takes.
__device__ inline void rot3_polished(const double (&g)[3][3], double (&O)[3][3],
                                     double& trace_margin, double& eig_margin) {
  float Af[3][3], Vf[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { Af[i][j] = (float)g[i][j]; Vf[i][j] = (i == j) ? 1.f : 0.f; }
  for (int sweep = 0; sweep < 12; ++sweep) {
    bool rot = false;
    jacobi_pair_f(Af, Vf, 0, 1, rot);
    jacobi_pair_f(Af, Vf, 0, 2, rot);
    jacobi_pair_f(Af, Vf, 1, 2, rot);
    if (!rot) break;
  }
  double V0[3][3], P[3][3], V[3][3], W[3][3], A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V0[i][j] = (double)Vf[i][j];
  // P = (3I - V0^T V0) / 2, V = V0 P
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double vtv = V0[0][i] * V0[0][j] + V0[1][i] * V0[1][j] + V0[2][i] * V0[2][j];
      P[i][j] = (i == j ? 1.5 : 0.0) - 0.5 * vtv;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = V0[i][0] * P[0][j] + V0[i][1] * P[1][j] + V0[i][2] * P[2][j];
  // A = V^T g V
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) W[i][j] = g[i][0] * V[0][j] + g[i][1] * V[1][j] + g[i][2] * V[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = V[0][i] * W[0][j] + V[1][i] * W[1][j] + V[2][i] * W[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) A[i][j] = A[j][i] = 0.5 * (A[i][j] + A[j][i]);
  rot3_finish(A, V, O, trace_margin, eig_margin);
}

// FP32 cyclic Jacobi sweeps from the identity: eigenvectors of g to FP32 accuracy (columns of V)
__device__ inline void jacobi3_f(const double (&g)[3][3], float (&V)[3][3]) {
  float Af[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { Af[i][j] = (float)g[i][j]; V[i][j] = (i == j) ? 1.f : 0.f; }
  for (int sweep = 0; sweep < 12; ++sweep) {
    bool rot = false;
    jacobi_pair_f(Af, V, 0, 1, rot);
    jacobi_pair_f(Af, V, 0, 2, rot);
    jacobi_pair_f(Af, V, 1, 2, rot);
    if (!rot) break;
  }
}

// One step of the eigenvector refinement of Ogita and Aishima (Japan J. Indust. Appl. Math. 35,
// 2018) for a symmetric 3 x 3 g and approximate eigenvectors X (columns): with R = I - X^T X and
// S = X^T g X the eigenvalues are lam_i = S_ii / (1 - R_ii), and X <- X (I + F) with
// F_ii = R_ii / 2 and, for i != j, F_ij = (S_ij + lam_j R_ij) / (lam_j - lam_i), which is the
// first-order solution of (I + F)^T (I - R) (I + F) = I, (I + F)^T S (I + F) diagonal.  The error
// of X is squared (times |g| / gap).  Returns false, leaving X unchanged, when two eigenvalues
// lie within delta = 2 (|S - diag(lam)| + |g| |R|) (Frobenius norms), a cluster one step cannot
// separate; fmx = max |F_ij| over i != j, mingap = the smallest eigenvalue gap.
__device__ inline bool oa_step(const double (&g)[3][3], double (&X)[3][3], double (&lam)[3],
                               double& fmx, double& mingap) {
  double W[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) W[i][j] = g[i][0] * X[0][j] + g[i][1] * X[1][j] + g[i][2] * X[2][j];
  double S[3][3], R[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      S[i][j] = X[0][i] * W[0][j] + X[1][i] * W[1][j] + X[2][i] * W[2][j];
      R[i][j] = (i == j ? 1.0 : 0.0) - (X[0][i] * X[0][j] + X[1][i] * X[1][j] + X[2][i] * X[2][j]);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i) lam[i] = S[i][i] * nr_rcp(1.0 - R[i][i]);
  const double so = 2.0 * (S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2]) +
                    (S[0][0] - lam[0]) * (S[0][0] - lam[0]) +
                    (S[1][1] - lam[1]) * (S[1][1] - lam[1]) + (S[2][2] - lam[2]) * (S[2][2] - lam[2]);
  const double rr = 2.0 * (R[0][1] * R[0][1] + R[0][2] * R[0][2] + R[1][2] * R[1][2]) +
                    R[0][0] * R[0][0] + R[1][1] * R[1][1] + R[2][2] * R[2][2];
  double gg = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gg += g[i][j] * g[i][j];
  const double delta = 2.0 * (sqrt(so) + sqrt(gg * rr));
  const double d01 = lam[1] - lam[0], d02 = lam[2] - lam[0], d12 = lam[2] - lam[1];
  mingap = fmin(fabs(d01), fmin(fabs(d02), fabs(d12)));
  if (!(mingap > delta)) return false;
  const double r01 = nr_rcp(d01), r02 = nr_rcp(d02), r12 = nr_rcp(d12);
  double F[3][3];
  F[0][0] = 0.5 * R[0][0];
  F[1][1] = 0.5 * R[1][1];
  F[2][2] = 0.5 * R[2][2];
  F[0][1] = (S[0][1] + lam[1] * R[0][1]) * r01;
  F[1][0] = -(S[0][1] + lam[0] * R[0][1]) * r01;
  F[0][2] = (S[0][2] + lam[2] * R[0][2]) * r02;
  F[2][0] = -(S[0][2] + lam[0] * R[0][2]) * r02;
  F[1][2] = (S[1][2] + lam[2] * R[1][2]) * r12;
  F[2][1] = -(S[1][2] + lam[1] * R[1][2]) * r12;
  fmx = fmax(fmax(fmax(fabs(F[0][1]), fabs(F[1][0])), fmax(fabs(F[0][2]), fabs(F[2][0]))),
             fmax(fabs(F[1][2]), fabs(F[2][1])));
  double Xn[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Xn[i][j] = X[i][j] + (X[i][0] * F[0][j] + X[i][1] * F[1][j] + X[i][2] * F[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) X[i][j] = Xn[i][j];
  return true;
}

// FP64 eigendecomposition of a symmetric 3 x 3 g for the rotation (arranged as in rot3): FP32
// Jacobi sweeps, then FP64 refinement steps until the error left, about fmx^2 |g| / gap, is below
// 1e-12 (at most three steps; one or two from the FP32 start).  Eigenvalues closer than one step
// can separate are finished by FP64 Jacobi sweeps instead (rot3_polished).
__device__ inline void rot3_refined(const double (&g)[3][3], double (&O)[3][3],
                                    double& trace_margin, double& eig_margin) {
  float Vf[3][3];
  jacobi3_f(g, Vf);
  double X[3][3], lam[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) X[i][j] = (double)Vf[i][j];
  double gg = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gg += g[i][j] * g[i][j];
  const double gn = sqrt(gg);
  bool ok = false;
  for (int it = 0; it < 3; ++it) {
    double fm, mg;
    ok = oa_step(g, X, lam, fm, mg);
    if (!ok || fm * fm * gn <= 1e-12 * mg) break;
  }
  if (ok) {
    arrange3(lam[0], lam[1], lam[2], X, O, trace_margin, eig_margin);
    return;
  }
  rot3_polished(g, O, trace_margin, eig_margin);
}

// ------------------------------------------------------------------------------------------
// Randomized greedy rotation search inside one cluster (Alg. 2), one workgroup per cluster.
// rank-th, ..., (rank+N-1)-th set bits of the active bitmask in LDS (-1 where absent); called by
// one whole wave
template <int N>
__device__ inline void select_activeN(const uint32_t* mask, int nw, int rank, int (&out)[N]) {
  const int lane = pmmf_lane();
  const int wpl = (nw + PMMF_WAVE - 1) / PMMF_WAVE;
  const int w0 = lane * wpl;
  int cnt = 0;
  for (int t = 0; t < wpl; ++t) {
    const int wi = w0 + t;
    if (wi < nw) cnt += __popc(mask[wi]);
  }
  const int incl = pmmf_wave_incl_scan_dpp(cnt);
  int base = incl - cnt;
  int f[N];
#pragma unroll
  for (int d = 0; d < N; ++d) f[d] = -1;
  for (int t = 0; t < wpl; ++t) {
    const int wi = w0 + t;
    const uint32_t m = wi < nw ? mask[wi] : 0u;
    const int pc = __popc(m);
#pragma unroll
    for (int d = 0; d < N; ++d) {
      const int want = rank + d - base;
      if (want >= 0 && want < pc) f[d] = wi * 32 + pmmf_nth_bit(m, want);
    }
    base += pc;
  }
#pragma unroll
  for (int d = 0; d < N; ++d) {
    const uint64_t bb = __ballot(f[d] >= 0);
    out[d] = bb ? __shfl(f[d], __ffsll((unsigned long long)bb) - 1) : -1;
  }
}

__device__ inline int slot_of(int j, int t0, int t1, int t2) {
  return j == t0 ? 0 : (j == t1 ? 1 : (j == t2 ? 2 : -1));
}
// by value: a select between references would put the operands in memory
template <typename T>
__device__ inline T pick3(int a, T x0, T x1, T x2) {
  return a == 0 ? x0 : (a == 1 ? x1 : x2);
}
struct Cand {
  float s;
  int j;
};
__device__ inline bool better(const Cand& a, const Cand& b) {
  // bitwise, not short-circuit: straight-line compares and selects, no branches
  return (a.s > b.s) | ((a.s == b.s) & (a.j < b.j));
}
// top two of {b1, b2, o1, o2} (b1 before b2, o1 before o2), with scalar selects only
__device__ inline void merge2(Cand& b1, Cand& b2, Cand o1, Cand o2) {
  const bool o1_first = better(o1, b1);
  const bool b1_beats_o2 = better(b1, o2);
  const bool o1_beats_b2 = better(o1, b2);
  const float n2s = o1_first ? (b1_beats_o2 ? b1.s : o2.s) : (o1_beats_b2 ? o1.s : b2.s);
  const int n2j = o1_first ? (b1_beats_o2 ? b1.j : o2.j) : (o1_beats_b2 ? o1.j : b2.j);
  const float n1s = o1_first ? o1.s : b1.s;
  const int n1j = o1_first ? o1.j : b1.j;
  b1.s = n1s;
  b1.j = n1j;
  b2.s = n2s;
  b2.j = n2j;
}

// i-th set bit (0-based rank) of the active bitmask held in LDS; called by one whole wave.
__device__ inline int select_active(const uint32_t* mask, int nw, int rank) {
  const int lane = pmmf_lane();
  const int wpl = (nw + PMMF_WAVE - 1) / PMMF_WAVE;
  const int w0 = lane * wpl;
  int cnt = 0;
  for (int t = 0; t < wpl; ++t)
    if (w0 + t < nw) cnt += __popc(mask[w0 + t]);
  const int incl = pmmf_wave_incl_scan(cnt);
  int found = -1;
  int excl = incl - cnt;
  if (rank >= excl && rank < incl) {
    for (int t = 0; t < wpl; ++t) {
      uint32_t m = mask[w0 + t];
      const int pc = __popc(m);
      if (rank - excl < pc) {
        int rr = rank - excl;
        for (int q = 0; q < rr; ++q) m &= m - 1;
        found = (w0 + t) * 32 + (__ffs(m) - 1);
        break;
      }
      excl += pc;
    }
  }
  // exactly one lane found it
  uint64_t b = __ballot(found >= 0);
  const int src = __ffsll((unsigned long long)b) - 1;
  return __shfl(found, src);
}

// Top-2 (k = 3) or top-1 (k = 2) candidate of a wave through DPP row shifts (inclusive inside
// each row of 16 lanes, disjoint sets at every step) and the four row results read back with
// readlane.  Every lane must be active; all lanes return the same result.
template <int CTRL>
__device__ inline Cand dpp_cand(Cand v) {
  Cand o;
  o.s = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, -1.f),
                                                              __builtin_bit_cast(int, v.s), CTRL,
                                                              0xf, 0xf, false));
  o.j = __builtin_amdgcn_update_dpp(INT_MAX, v.j, CTRL, 0xf, 0xf, false);
  return o;
}
template <int K, int CTRL>
__device__ inline void top_step(Cand& b1, Cand& b2) {
  const Cand o1 = dpp_cand<CTRL>(b1);
  if (K == 3) {
    const Cand o2 = dpp_cand<CTRL>(b2);
    merge2(b1, b2, o1, o2);
  } else {
    const bool t = better(o1, b1);
    b1.s = t ? o1.s : b1.s;
    b1.j = t ? o1.j : b1.j;
  }
}
__device__ inline Cand readlane_cand(Cand v, int l) {
  return Cand{pmmf_readlane_f(v.s, l), __builtin_amdgcn_readlane(v.j, l)};
}
template <int K>
__device__ inline void wave_top(Cand& b1, Cand& b2) {
  top_step<K, 0x111>(b1, b2);
  top_step<K, 0x112>(b1, b2);
  top_step<K, 0x114>(b1, b2);
  top_step<K, 0x118>(b1, b2);
  Cand r1 = readlane_cand(b1, 15), r2 = readlane_cand(b2, 15);
#pragma unroll
  for (int rr = 1; rr < 4; ++rr) {
    const Cand o1 = readlane_cand(b1, 16 * rr + 15);
    if (K == 3) {
      merge2(r1, r2, o1, readlane_cand(b2, 16 * rr + 15));
    } else if (better(o1, r1)) {
      r1 = o1;
    }
  }
  b1 = r1;
  b2 = r2;
}

// new value of slot a of a rotated (G, D) pair: sum_b O[a][b] v[b], in one fixed order so that
// every thread that forms the same entry forms it bit-identically
template <int K>
__device__ inline float2 rot_entry(const float* o, int a, const float2* v) {
  float sg = 0.f, sd = 0.f;
#pragma unroll
  for (int b = 0; b < K; ++b) {
    sg = fmaf(o[a * 3 + b], v[b].x, sg);
    sd = fmaf(o[a * 3 + b], v[b].y, sd);
  }
  return make_float2(sg, sd);
}

// The cluster's state lives in HBM as a dense c x c array GD (Gram and diagonal block of the
// active matrix, interleaved so one 8-byte access moves both); the accumulated rotation Qbar is
// rebuilt from the log afterwards (k_qsparse).
// Each thread owns the columns j = tid + q NT (q < PER) and keeps its slice of the rows it needs
// in registers.  A step has two barriers:
//   A  after the partner argmax;
//   B  after the serial FP64 rotation on lane 0 (wave 1 meanwhile picks the two candidates for
//      the next seed from the active set before this step's retirement).
// After B every thread knows O, the retired slot and the next seed i'.  It requests row i' of GD
// before issuing this step's stores: entries of row i' outside the rotated columns T are not
// touched by this step, and the entries at T are re-formed from the pre-rotation rows kept in
// LDS (or, when i' is itself in T, the whole row is the one this thread just formed).  The next
// step's scoring therefore needs no third barrier; barrier A of the next step orders this step's
// stores before the partner rows are read.  The retirement is applied to the active mask one
// step late (the scoring also skips the previous retiree explicitly), so wave 1 can read a mask
// that nobody writes during the serial section.
// E = indices retired per rotation: a step's rotation retires its E slots with the smallest
// off-diagonal norms and writes E log entries, the later ones on the same tuple with the identity
// block.  Launched for two retirements per 3-point rotation (E = 2); one retirement per rotation
// runs k_search below.
// target of the column stores a step has none to make (the first step): written, never read, so the
// workgroups that share it may overwrite one another
__device__ float2 g_find_sink[4096];

template <int NT, int PER, int K, int E>
__global__ void __launch_bounds__(NT) k_find(FindArgs A, int cmax) {
  static_assert(NT >= 2 * PMMF_WAVE, "wave 1 selects the next seed");
  static_assert(E == 1 || (E == 2 && K == 3), "two eliminations need a 3-point rotation");
  extern __shared__ float lds_f[];
  float* gdiag = lds_f;
  float* ddiag = gdiag + cmax;
  float2* rowbuf = reinterpret_cast<float2*>(ddiag + cmax);  // seed rows (2 parities), partners
  int* lgid = reinterpret_cast<int*>(rowbuf + 4 * (size_t)cmax);
  uint32_t* mask = reinterpret_cast<uint32_t*>(lgid + cmax);
  float* gsq = reinterpret_cast<float*>(mask + (cmax + 31) / 32);  // sqrt(G_jj), for the scores
  constexpr int NW = NT / PMMF_WAVE;
  __shared__ Cand red1[NW], red2[NW];
  __shared__ int sh_i, sh_e, sh_e2, sh_c[E + 1], sh_k[2 * E + 1];
  __shared__ float sh_O[9], sh_gn[9], sh_dn[9], sh_mg[2], sh_de[2];
  __shared__ double sh_lit[2];

  const int tid = threadIdx.x;
  const int u = A.order[blockIdx.x];
  const int o = A.off[u];
  const int c = A.off[u + 1] - o;
  const int ld = gd_stride(c);  // row stride of the cluster's (G, D) array
  const int nent = A.rcnt[u];                 // log entries: indices the cluster retires
  const int r = (nent + E - 1) / E;           // rotations (steps)
  const int rb = A.roff[u];
  const int nw = (c + 31) / 32;
  constexpr int kk = K;
  float2* __restrict__ GD = A.GD + A.gbase[u];
  float2* R1 = rowbuf + 2 * (size_t)cmax;
  float2* R2 = rowbuf + 3 * (size_t)cmax;

  for (int j = tid; j < c; j += NT) {
    const float2 dg = GD[(size_t)j * ld + j];
    gdiag[j] = dg.x;
    gsq[j] = sqrtf(dg.x);
    ddiag[j] = dg.y;
    lgid[j] = A.gid[o + j];
  }
  for (int q = tid; q < nw; q += NT) {
    const int rem = c - q * 32;
    mask[q] = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
  }
  __syncthreads();
  if (tid < PMMF_WAVE && r > 0) {  // first seed row, uniform over the active set
    const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u, 0);
    const int i0 = select_active(mask, nw, (int)pmmf_mulhi(h, (uint64_t)c));
    if (tid == 0) sh_i = i0;
    if (r > 1) {  // the E + 1 candidates for the second seed (see the next-seed rule below)
      const uint64_t h1 = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u, 1);
      const int rank1 = (int)pmmf_mulhi(h1, (uint64_t)(c - E));
      int cs[E + 1];
      select_activeN<E + 1>(mask, nw, rank1, cs);
      if (tid == 0)
#pragma unroll
        for (int d = 0; d <= E; ++d) sh_c[d] = cs[d];
    }
  }
  __syncthreads();
  int i = r > 0 ? sh_i : 0;
  int e_prev = -1, e_prev2 = -1;
  // column stores of the previous step, issued during this step's rotation (see below): their
  // values, which of them are real, the T they belong to and that step's retiree, whose column
  // is dead and takes the lanes with nothing to store
  float2 cst[3][PER];
  uint64_t cmask = 0;
  int tq0 = -1, tq1 = -1, tq2 = -1, edead = 0;
  int jl[PER];  // this thread's columns, clamped into the cluster for address forming
  // candidates for the next seed (k = 2: their rows are loaded during this step's rotation)
  int cc[E + 1];
#pragma unroll
  for (int d = 0; d <= E; ++d) cc[d] = r > 1 ? sh_c[d] : 0;
  float2 c0r[PER], c1r[PER];
  float2 cur[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    jl[q] = min(j, c - 1);
    cur[q] = (r > 0 && j < c) ? GD[(size_t)i * ld + j] : make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < 3; ++a) cst[a][q] = make_float2(0.f, 0.f);
  }

  // scoring of a step's seed row (held in cur): written to R0 of that step's parity, partner
  // scores reduced per wave.  Called at the end of the previous step, so the wait for the seed
  // row's load is counted against the stores issued after it rather than a full drain.
  auto score_seed = [&](int sn) {
    float2* R0s = rowbuf + (size_t)(sn & 1) * cmax;
    // the seed's (G, D) row; partner scores |G_ij| / sqrt(G_jj) over the active set, top (k - 1),
    // lower j on ties
    Cand b1{-1.f, INT_MAX}, b2{-1.f, INT_MAX};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if (j < c) {
        R0s[j] = cur[q];
        const bool act = ((mask[j >> 5] >> (j & 31)) & 1u) && j != e_prev && j != e_prev2;
        if (act && j != i) {
          const float gq = gsq[j];  // > 0 exactly when G_jj > 0
          float sc = gq > 0.f ? fabsf(cur[q].x) / gq : 0.f;
          if (!(sc >= 0.f)) sc = 0.f;  // NaN from an overflowed Gram entry scores 0
          Cand cnd{sc, j};
          if (better(cnd, b1)) { b2 = b1; b1 = cnd; }
          else if (better(cnd, b2)) b2 = cnd;
        }
      }
    }
    wave_top<K>(b1, b2);
    if (pmmf_lane() == 0) { red1[pmmf_wave()] = b1; red2[pmmf_wave()] = b2; }
  };
  if (r > 0) score_seed(0);
  for (int s = 0; s < r; ++s) {
    float2* R0 = rowbuf + (size_t)(s & 1) * cmax;
    __syncthreads();  // A
    // every thread merges the per-wave winners
    Cand f1 = red1[0], f2 = red2[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      if (kk == 3) merge2(f1, f2, red1[q], red2[q]);
      else if (better(red1[q], f1)) f1 = red1[q];
    }
    if (f1.j >= c || (kk == 3 && f2.j >= c)) {  // impossible with >= k live indices
      if (tid == 0) atomicOr(A.err, 1);
      return;
    }
    const int t0 = i, t1 = f1.j, t2 = kk == 3 ? f2.j : -1;

    // The previous step's column stores (entries (j, T_{s-1}) of rows outside T_{s-1}) may still
    // be in flight: such an entry is read at its transpose (T_{s-1}[b], j), stored with the rows
    // T_{s-1} before barrier A and equal to it.  Everything older was stored before barrier B of
    // the previous step.
    const int st1 = slot_of(t1, tq0, tq1, tq2), st2 = kk == 3 ? slot_of(t2, tq0, tq1, tq2) : -1;
    // the (t1, t2) entries first (lane 0 needs them before anything else), then the partner rows
    float2 x12 = make_float2(0.f, 0.f), x21 = make_float2(0.f, 0.f);
    if (kk == 3 && tid < PMMF_WAVE) {
      x12 = GD[(size_t)t1 * ld + t2];
      x21 = GD[(size_t)t2 * ld + t1];
    }
    // the other waves' loads and stores queue behind these two in the compute unit's memory
    // pipeline (a barrier does not wait for loads in flight)
    if (kk == 3) __syncthreads();  // A'
    float2 p1[PER], p2[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      const int sj = slot_of(j, tq0, tq1, tq2);
      const uint32_t jq = (uint32_t)jl[q];
      p1[q] = GD[(sj >= 0 && st1 < 0) ? (uint32_t)(j * ld + t1) : (uint32_t)(t1 * ld) + jq];
      p2[q] = kk == 3 ? GD[(sj >= 0 && st2 < 0) ? (uint32_t)(j * ld + t2) : (uint32_t)(t2 * ld) + jq]
                      : make_float2(0.f, 0.f);
    }
    // the previous step's column stores, after this step's loads; a lane with no real entry
    // writes into the dead row of that step's retiree, contiguous across the wave (the first step
    // writes its zeros into the sink).  Branch-free, so a wait for the loads above does not wait
    // for these stores.
    float2* const cbase = s > 0 ? GD : g_find_sink;
    auto column_stores = [&]() {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
#pragma unroll
        for (int a = 0; a < K; ++a) {
          const int ta = a == 0 ? tq0 : (a == 1 ? tq1 : tq2);
          const bool real = (cmask >> (a * PER + q)) & 1ull;
          cbase[real ? (uint32_t)(j * ld + ta) : (uint32_t)(edead * ld + jl[q])] = cst[a][q];
        }
      }
    };
    // the rows of the two candidates for the next seed, read the same way (their entries at T
    // are re-formed after this step's rotation; one retirement per step only: with two the three
    // candidate rows would not fit in registers)
    if constexpr (E == 1) {
      const int sc0 = slot_of(cc[0], tq0, tq1, tq2), sc1 = slot_of(cc[1], tq0, tq1, tq2);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = tid + q * NT;
        const int sj = slot_of(j, tq0, tq1, tq2);
        const uint32_t jq = (uint32_t)jl[q];
        c0r[q] = GD[(sj >= 0 && sc0 < 0) ? (uint32_t)(j * ld + cc[0]) : (uint32_t)(cc[0] * ld) + jq];
        c1r[q] = GD[(sj >= 0 && sc1 < 0) ? (uint32_t)(j * ld + cc[1]) : (uint32_t)(cc[1] * ld) + jq];
      }
    }
    // the stores last: vector memory operations complete in issue order, so lane 0's wait for the
    // (t1, t2) entries does not wait for a store
    column_stores();

    if (tid == 0) {
      double g[3][3] = {}, d[3][3] = {}, O[3][3] = {};
      g[0][0] = gdiag[t0];
      d[0][0] = ddiag[t0];
      g[1][1] = gdiag[t1];
      d[1][1] = ddiag[t1];
      const float2 s01 = R0[t1];
      g[0][1] = g[1][0] = s01.x;
      d[0][1] = d[1][0] = s01.y;
      if (kk == 3) {
        g[2][2] = gdiag[t2];
        d[2][2] = ddiag[t2];
        const float2 s02 = R0[t2];
        g[0][2] = g[2][0] = s02.x;
        d[0][2] = d[2][0] = s02.y;
        // an entry whose column is in T_{s-1} and row is not may be stale: take its transpose
        const bool fresh12 = st1 >= 0 || st2 < 0, fresh21 = st2 >= 0 || st1 < 0;
        const float2 y12 = fresh12 ? x12 : x21, y21 = fresh21 ? x21 : x12;
        const double g12 = 0.5 * ((double)y12.x + (double)y21.x);
        const double d12 = 0.5 * ((double)y12.y + (double)y21.y);
        g[1][2] = g[2][1] = g12;
        d[1][2] = d[2][1] = d12;
      }
      double margin = 3.0e38;
      if (kk == 2) {
        double cc, ss, ta;
        rot2(g[0][0], g[0][1], g[1][1], cc, ss, ta);
        O[0][0] = cc; O[0][1] = -ss; O[1][0] = ss; O[1][1] = cc;
        margin = fmin(margin, ta);
      } else {
        double tm, em;
        rot3_polished(g, O, tm, em);
        margin = fmin(margin, fmin(tm, em));
      }
      // rotated k x k blocks: O g O^T and O d O^T
      double gn[3][3] = {}, dn[3][3] = {};
#pragma unroll
      for (int a = 0; a < kk; ++a)
#pragma unroll
        for (int b = 0; b < kk; ++b) {
          double sg = 0.0, sd = 0.0;
#pragma unroll
          for (int x = 0; x < kk; ++x) {
            double tg = 0.0, td = 0.0;
#pragma unroll
            for (int y = 0; y < kk; ++y) { tg += g[x][y] * O[b][y]; td += d[x][y] * O[b][y]; }
            sg += O[a][x] * tg;
            sd += O[a][x] * td;
          }
          gn[a][b] = sg;
          dn[a][b] = sd;
        }
      // eliminate the slot with the smallest off-diagonal norm (ties: later slot)
      const double f0 = fmax(0.0, gn[0][0] - dn[0][0] * dn[0][0]);
      const double f1v = fmax(0.0, gn[1][1] - dn[1][1] * dn[1][1]);
      const double f2v = kk == 3 ? fmax(0.0, gn[2][2] - dn[2][2] * dn[2][2]) : 1e300;
      int es = f1v <= f0 ? 1 : 0;
      double fmin_ = es == 1 ? f1v : f0;
      if (kk == 3 && f2v <= fmin_) { es = 2; fmin_ = f2v; }
      {
        // second smallest, for the (diagnostic) elimination margin
        const double hi01 = fmax(f0, f1v), lo01 = fmin(f0, f1v);
        const double lo2 = kk == 3 ? (f2v <= lo01 ? lo01 : fmin(hi01, f2v)) : hi01;
        const double lo1 = fmin(lo01, f2v);
        margin = fmin(margin, lo2 > 0.0 ? (lo2 - lo1) / lo2 : 0.0);
      }
      const int e = es == 0 ? t0 : (es == 1 ? t1 : t2);
      const double dee = es == 0 ? dn[0][0] : (es == 1 ? dn[1][1] : dn[2][2]);
      const double off2e = fmin_;
      // second elimination (E = 2): the smaller of the two remaining slots, ties to the later
      const int sa = es == 0 ? 1 : 0, sb = es == 2 ? 1 : 2;
      const double fa = sa == 0 ? f0 : f1v, fb = sb == 1 ? f1v : f2v;
      const int es2 = fb <= fa ? sb : sa;
      const int e2 = es2 == 0 ? t0 : (es2 == 1 ? t1 : t2);
      const double dee2 = es2 == 0 ? dn[0][0] : (es2 == 1 ? dn[1][1] : dn[2][2]);
      const double off2e2 = fmin(fa, fb);
      const double margin2 = fmax(fa, fb) > 0.0 ? fabs(fb - fa) / fmax(fa, fb) : 0.0;
      const bool second = E == 2 && E * s + 1 < nent;
      gdiag[t0] = (float)gn[0][0];
      ddiag[t0] = (float)dn[0][0];
      gdiag[t1] = (float)gn[1][1];
      ddiag[t1] = (float)dn[1][1];
      gsq[t0] = sqrtf((float)gn[0][0]);
      gsq[t1] = sqrtf((float)gn[1][1]);
      if (kk == 3) {
        gdiag[t2] = (float)gn[2][2];
        ddiag[t2] = (float)dn[2][2];
        gsq[t2] = sqrtf((float)gn[2][2]);
      }
      sh_e = e;
      sh_e2 = second ? e2 : -1;
#pragma unroll
      for (int a = 0; a < 9; ++a) { sh_O[a] = 0.f; sh_gn[a] = 0.f; sh_dn[a] = 0.f; }
#pragma unroll
      for (int a = 0; a < kk; ++a)
#pragma unroll
        for (int b = 0; b < kk; ++b) {
          sh_O[a * 3 + b] = (float)O[a][b];
          sh_gn[a * 3 + b] = (float)gn[a][b];
          sh_dn[a * 3 + b] = (float)dn[a][b];
        }
      // the rotation log is written by wave 1 after barrier B
      sh_mg[0] = (float)margin;
      sh_de[0] = (float)dee;
      sh_lit[0] = 2.0 * off2e;
      if (E == 2) {
        sh_mg[1] = (float)margin2;
        sh_de[1] = (float)dee2;
        sh_lit[1] = 2.0 * off2e2;
      }
    }
    if (tid >= PMMF_WAVE && tid < 2 * PMMF_WAVE && s + 2 < r) {
      // next-seed rule: the rank-th active index after a retirement e is the rank-th one before
      // it if that lies below e, else the (rank + 1)-th.  The seed of step s+2 is picked after
      // 2E more retirements (steps s and s+1), so the (rank + m)-th indices, m <= 2E, are taken
      // now; after this step E + 1 candidates for it remain, after the next step the seed.
      const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u,
                                    (uint64_t)(s + 2));
      int kn[2 * E + 1];
      select_activeN<2 * E + 1>(mask, nw, (int)pmmf_mulhi(h, (uint64_t)(c - E * (s + 2))), kn);
      if (tid == PMMF_WAVE)
#pragma unroll
        for (int d = 0; d <= 2 * E; ++d) sh_k[d] = kn[d];
    }
    // pre-rotation partner rows, for re-forming the next seed row's entries at T
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if (j < c) {
        R1[j] = p1[q];
        if (kk == 3) R2[j] = p2[q];
      }
    }
    __syncthreads();  // B

    float o_[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) o_[a] = sh_O[a];
    const int e = sh_e;
    const int e2 = E == 2 ? sh_e2 : -1;
    const bool more = s + 1 < r;
    // the next seed: the candidates with this step's retirements removed in turn
    int nxt = -1;
    if (E == 1) {
      nxt = more ? (cc[0] < e ? cc[0] : cc[1]) : -1;
    } else if (more) {
      const int m0 = cc[0] < e ? cc[0] : cc[1], m1 = cc[1] < e ? cc[1] : cc[E];
      nxt = m0 < e2 ? m0 : m1;
    }
    const int aslot = nxt == t0 ? 0 : (nxt == t1 ? 1 : ((kk == 3 && nxt == t2) ? 2 : -1));
    const int Tt[3] = {t0, t1, t2};
    if (tid < kk * kk) {
      const int a = tid / kk, b = tid % kk;
      GD[(size_t)Tt[a] * ld + Tt[b]] = make_float2(sh_gn[a * 3 + b], sh_dn[a * 3 + b]);
    }
    float2 nrow[PER];
    if constexpr (E == 1) {
#pragma unroll
      for (int q = 0; q < PER; ++q) nrow[q] = nxt == cc[0] ? c0r[q] : c1r[q];
    } else {
      const uint32_t nb = (uint32_t)((more && aslot < 0 ? nxt : 0) * ld);
#pragma unroll
      for (int q = 0; q < PER; ++q) nrow[q] = GD[nb + (uint32_t)jl[q]];
    }
    if (s + 2 < r) {  // candidates for the seed of step s+2
      int kn[2 * E + 1];
#pragma unroll
      for (int d = 0; d <= 2 * E; ++d) kn[d] = sh_k[d];
#pragma unroll
      for (int d = 0; d < 2 * E; ++d) kn[d] = kn[d] < e ? kn[d] : kn[d + 1];
      if (E == 2) {
#pragma unroll
        for (int d = 0; d < E + 1; ++d) kn[d] = kn[d] < e2 ? kn[d] : kn[d + 1];
      }
#pragma unroll
      for (int d = 0; d <= E; ++d) cc[d] = kn[d];
    }
    // pre-rotation values of rows T at column nxt (used when nxt is not in T)
    float2 vn[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    if (more && aslot < 0) {
      vn[0] = R0[nxt];
      vn[1] = R1[nxt];
      if (kk == 3) vn[2] = R2[nxt];
    }
    if (tid == 0) {
      mask[e >> 5] &= ~(1u << (e & 31));
      if (E == 2 && e2 >= 0) mask[e2 >> 5] &= ~(1u << (e2 & 31));
    }
    if (pmmf_wave() == 1) {  // rotation log, one entry per lane (stores only: nothing waits)
      const int l = pmmf_lane();
      const int64_t ridx = A.rot0 + rb + (int64_t)E * s;
      if (l < 9) A.rot_o[ridx * 9 + l] = sh_O[l];
      if (l < 3) {
        const int tl = l == 0 ? t0 : (l == 1 ? t1 : t2);
        A.rot_loc[ridx * 3 + l] = tl;
        A.rot_gid[ridx * 3 + l] = tl >= 0 ? lgid[tl] : -1;
      }
      if (l == 0) {
        A.rot_ret[ridx] = lgid[e];
        A.rot_margin[ridx] = sh_mg[0];
        A.rot_lit[ridx] = sh_lit[0];
        A.hdiag[lgid[e]] = sh_de[0];
        A.retflag[o + e] = 1;
      }
      if (E == 2 && e2 >= 0) {  // the same tuple with the identity block, retiring e2
        const int64_t r2 = ridx + 1;
        if (l < 9) A.rot_o[r2 * 9 + l] = (l % 4 == 0) ? 1.f : 0.f;
        if (l < 3) {
          const int tl = l == 0 ? t0 : (l == 1 ? t1 : t2);
          A.rot_loc[r2 * 3 + l] = tl;
          A.rot_gid[r2 * 3 + l] = lgid[tl];
        }
        if (l == 0) {
          A.rot_ret[r2] = lgid[e2];
          A.rot_margin[r2] = sh_mg[1];
          A.rot_lit[r2] = sh_lit[1];
          A.hdiag[lgid[e2]] = sh_de[1];
          A.retflag[o + e2] = 1;
        }
      }
    }

    // stores: GD <- O GD O^T on rows T now (the k x k block above; a column in T or beyond the
    // cluster writes into the dead column of this step's retiree, and a retired column's entry
    // is dead too), columns T during the next step's rotation
    cmask = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      const int bj = slot_of(j, t0, t1, t2);
      const bool in = j < c && bj < 0;
      const bool a_now = in && ((mask[j >> 5] >> (j & 31)) & 1u);
      const float2 v[3] = {cur[q], p1[q], p2[q]};
      float2 nv[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
#pragma unroll
      for (int a = 0; a < K; ++a) {
        nv[a] = rot_entry<K>(o_, a, v);
        GD[(uint32_t)(Tt[a] * ld) + (uint32_t)(in ? j : e)] = nv[a];
        cst[a][q] = nv[a];
        const uint32_t m = __float_as_uint(nv[a].x) | __float_as_uint(nv[a].y) |
                           __float_as_uint(v[a].x) | __float_as_uint(v[a].y);
        cmask |= (uint64_t)(a_now && (m << 1) != 0u) << (a * PER + q);
      }
      // the next seed row at column j
      if (more) {
        if (bj >= 0) {
          nrow[q] = aslot >= 0 ? make_float2(sh_gn[aslot * 3 + bj], sh_dn[aslot * 3 + bj])
                               : rot_entry<K>(o_, bj, vn);
        } else if (aslot >= 0) {
          nrow[q] = pick3(aslot, nv[0], nv[1], nv[2]);
        }
      }
    }
    tq0 = t0;
    tq1 = t1;
    tq2 = t2;
    edead = e;
#pragma unroll
    for (int q = 0; q < PER; ++q) cur[q] = nrow[q];
    e_prev = e;
    e_prev2 = e2;
    i = nxt;
    if (more) score_seed(s + 1);
  }
}

template <int NT, int PER, int K, int E>
static hipError_t find_launch(const FindArgs& a, int m, int cmax, size_t lds0, hipStream_t s) {
  const size_t lds = lds0 + (size_t)cmax * sizeof(float);  // + sqrt(G_jj)
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)&k_find<NT, PER, K, E>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_find<NT, PER, K, E><<<m, NT, lds, s>>>(a, cmax);
  return hipGetLastError();
}

template <int NT, int PER>
static hipError_t find_launch_k(const FindArgs& a, int m, int cmax, size_t lds, hipStream_t s) {
  if (a.k != 3 || a.elims != 2) return hipErrorInvalidValue;  // one retirement: k_search
  return find_launch<NT, PER, 3, 2>(a, m, cmax, lds, s);
}

// ------------------------------------------------------------------------------------------
// Greedy search with one retirement per rotation (Alg. 2), one workgroup per cluster, wave 0 a
// control wave and the other waves column waves.
//
// The control wave owns no columns: it fetches G_{t1 t2}, selects the seed candidates two steps
// ahead while that entry is in flight, computes the FP64 rotation on lane 0 and writes the log.
// Column thread x = tid - 64 owns the columns j = x + q (NT - 64), q < PER, and keeps its slices
// of the seed row, the partner rows and the two candidate rows of the next seed in registers.
// Step s (seed i, partners t1, t2 from the merged scores of row i):
//   after barrier A the column waves request the partner rows and the rows of the two candidates
//   for the next seed (one of them becomes the seed once the step's retiree is known), and store
//   the previous step's columns.  While lane 0 rotates they score both candidate rows over every
//   column outside T: those entries and G_jj are not changed by the rotation, and the retiree is
//   in T.
//   after barrier B the column waves rotate and store rows T and assemble the next seed row; the
//   control wave scores that row's entries at T, re-formed from the pre-rotation rows.  The next
//   merge takes the chosen candidate's per-wave winners and these three entries.  When the next
//   seed is itself in T its row is the one just formed, and it is scored in full.
// A column entry (j, t), t in T, is stored at the end of the next step's first half if it is not
// zero (a zero stays zero); until then that step's loads take its transpose from row t, which is
// stored before barrier A.
__device__ inline float inv_sqrt_pos(float g) { return g > 0.f ? 1.f / sqrtf(g) : 0.f; }
// partner score |G_xj| / sqrt(G_jj) from 1 / sqrt(G_jj); NaN (an overflowed entry) scores 0
__device__ inline float partner_score(float gxj, float rg) {
  const float sc = fabsf(gxj) * rg;
  return sc >= 0.f ? sc : 0.f;
}
template <int K>
__device__ inline void take(Cand& b1, Cand& b2, Cand c) {
  if (K == 3) {
    if (better(c, b1)) { b2 = b1; b1 = c; }
    else if (better(c, b2)) b2 = c;
  } else if (better(c, b1)) {
    b1 = c;
  }
}

template <int NT, int PER, int K>
__global__ void __launch_bounds__(NT) k_search(FindArgs A, int cmax) {
  static_assert(NT >= 2 * PMMF_WAVE, "a control wave and at least one column wave");
  constexpr int NW = NT / PMMF_WAVE;
  constexpr int NC = NT - PMMF_WAVE;  // column threads
  extern __shared__ float lds_f[];
  float2* rowbuf = reinterpret_cast<float2*>(lds_f);  // seed rows (2 parities), partner rows
  float* gdiag = reinterpret_cast<float*>(rowbuf + 4 * (size_t)cmax);
  float* ddiag = gdiag + cmax;
  float* rgs = ddiag + cmax;  // 1 / sqrt(G_jj), 0 where G_jj <= 0
  int* lgid = reinterpret_cast<int*>(rgs + cmax);
  uint32_t* mask = reinterpret_cast<uint32_t*>(lgid + cmax);
  // latest rotation level touching each index (16 bits: a stage has fewer than 65536 levels)
  unsigned short* lastlv = reinterpret_cast<unsigned short*>(mask + (cmax + 31) / 32);
  // per-wave winners [parity][0, 1: candidate rows, 2: full scoring][wave]; entries at T
  __shared__ Cand red1[2][3][NW], red2[2][3][NW], sh_tc[3];
  __shared__ int sh_i, sh_e, sh_c[2], sh_k[3];
  __shared__ float sh_O[9], sh_gn[9], sh_dn[9], sh_mg, sh_de;
  __shared__ double sh_lit;

  const int tid = threadIdx.x;
  const int wv = pmmf_wave(), lane = pmmf_lane();
  const int u = A.order[blockIdx.x];
  const int o = A.off[u];
  const int c = A.off[u + 1] - o;
  const int ld = gd_stride(c);  // row stride of the cluster's (G, D) array
  const int r = A.rcnt[u];      // rotations = retirements
  const int rb = A.roff[u];
  const int nw = (c + 31) / 32;
  float2* __restrict__ GD = A.GD + A.gbase[u];
  float2* R1 = rowbuf + 2 * (size_t)cmax;
  float2* R2 = rowbuf + 3 * (size_t)cmax;

  for (int j = tid; j < c; j += NT) {
    const float2 dg = GD[(size_t)j * ld + j];
    gdiag[j] = dg.x;
    ddiag[j] = dg.y;
    rgs[j] = inv_sqrt_pos(dg.x);
    lgid[j] = A.gid[o + j];
    lastlv[j] = 0;
  }
  for (int q = tid; q < nw; q += NT) {
    const int rem = c - q * 32;
    mask[q] = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
  }
  __syncthreads();
  if (wv == 0 && r > 0) {  // first seed row, uniform over the active set; candidates for the second
    const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u, 0);
    const int i0 = select_active(mask, nw, (int)pmmf_mulhi(h, (uint64_t)c));
    if (lane == 0) sh_i = i0;
    if (r > 1) {
      const uint64_t h1 = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u, 1);
      int cs[2];
      select_activeN<2>(mask, nw, (int)pmmf_mulhi(h1, (uint64_t)(c - 1)), cs);
      if (lane == 0) { sh_c[0] = cs[0]; sh_c[1] = cs[1]; }
    }
  }
  __syncthreads();

  // state of every wave: seed, the two candidates for the next seed, the previous T, and which
  // per-wave winners the next merge takes
  int i = r > 0 ? sh_i : 0;
  int cc0 = r > 1 ? sh_c[0] : 0, cc1 = r > 1 ? sh_c[1] : 0;
  int tq0 = -1, tq1 = -1, tq2 = -1;
  int sel = 2;
  // The control wave and the column waves run separate copies of the step loop (so that neither
  // holds the other's registers); both pass the same two barriers per step.  Parts both take:
  // the merge after barrier A (every thread forms the same partners) ...
  auto merge = [&](int par, Cand& f1, Cand& f2) {
    f1 = Cand{-1.f, INT_MAX};
    f2 = Cand{-1.f, INT_MAX};
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      if (K == 3) merge2(f1, f2, red1[par][sel][w], red2[par][sel][w]);
      else take<K>(f1, f2, red1[par][sel][w]);
    }
    if (sel < 2) {
#pragma unroll
      for (int a = 0; a < 3; ++a) take<K>(f1, f2, sh_tc[a]);
    }
  };
  // ... and after barrier B the retiree, the next seed, the candidates for the seed after it and
  // the pre-rotation entries of rows T at the next seed's column
  auto after_b = [&](int s, int t0, int t1, int t2, const float2* R0, float (&o_)[9], int& e,
                     int& nxt, int& aslot, int& nsel, float2 (&vn)[3]) {
    const bool more = s + 1 < r;
#pragma unroll
    for (int a = 0; a < 9; ++a) o_[a] = sh_O[a];
    e = sh_e;
    nxt = more ? (cc0 < e ? cc0 : cc1) : -1;
    aslot = nxt == t0 ? 0 : (nxt == t1 ? 1 : ((K == 3 && nxt == t2) ? 2 : -1));
    nsel = aslot >= 0 ? 2 : (nxt == cc0 ? 0 : 1);
    vn[0] = vn[1] = vn[2] = make_float2(0.f, 0.f);
    if (more && aslot < 0) {
      vn[0] = R0[nxt];
      vn[1] = R1[nxt];
      if (K == 3) vn[2] = R2[nxt];
    }
    if (s + 2 < r) {  // the candidates for the seed of step s+2, without this step's retiree
      const int k0 = sh_k[0], k1 = sh_k[1], k2 = sh_k[2];
      cc0 = k0 < e ? k0 : k1;
      cc1 = k1 < e ? k1 : k2;
    }
  };

  if (wv == 0) {
    // ---------------------------------------------------------------- control wave
    // G and D entries (t1, t2) and (t2, t1) of the next step, requested (or formed) after the
    // previous barrier B when that step's partners were known then
    bool pre = false;
    float2 x12 = make_float2(0.f, 0.f), x21 = make_float2(0.f, 0.f);
    for (int s = 0; s < r; ++s) {
      const int par = s & 1;
      const float2* R0 = rowbuf + (size_t)par * cmax;
      const bool more = s + 1 < r;
      __syncthreads();  // A
      Cand f1, f2;
      merge(par, f1, f2);
      if (f1.j >= c || (K == 3 && f2.j >= c)) {  // impossible with >= k live indices
        if (lane == 0) atomicOr(A.err, 1);
        return;
      }
      const int t0 = i, t1 = f1.j, t2 = K == 3 ? f2.j : -1;
      // an entry of a row outside T_{s-1} at a column in T_{s-1} may be stale until this step's
      // column stores land: its transpose is taken instead
      const int st1 = slot_of(t1, tq0, tq1, tq2), st2 = K == 3 ? slot_of(t2, tq0, tq1, tq2) : -1;
      if (K == 3 && !pre) {
        x12 = GD[(size_t)t1 * ld + t2];
        x21 = GD[(size_t)t2 * ld + t1];
      }
      if (lane == 0) {
        double g[3][3] = {}, d[3][3] = {}, O[3][3] = {};
        g[0][0] = gdiag[t0];
        d[0][0] = ddiag[t0];
        g[1][1] = gdiag[t1];
        d[1][1] = ddiag[t1];
        const float2 s01 = R0[t1];
        g[0][1] = g[1][0] = s01.x;
        d[0][1] = d[1][0] = s01.y;
        double margin = 3.0e38;
        if (K == 3) {
          g[2][2] = gdiag[t2];
          d[2][2] = ddiag[t2];
          const float2 s02 = R0[t2];
          g[0][2] = g[2][0] = s02.x;
          d[0][2] = d[2][0] = s02.y;
          const bool fresh12 = pre || st1 >= 0 || st2 < 0, fresh21 = pre || st2 >= 0 || st1 < 0;
          const float2 y12 = fresh12 ? x12 : x21, y21 = fresh21 ? x21 : x12;
          const double g12 = 0.5 * ((double)y12.x + (double)y21.x);
          const double d12 = 0.5 * ((double)y12.y + (double)y21.y);
          g[1][2] = g[2][1] = g12;
          d[1][2] = d[2][1] = d12;
          double tm, em;
          rot3_refined(g, O, tm, em);
          margin = fmin(tm, em);
        } else {
          double cs, sn, ta;
          rot2(g[0][0], g[0][1], g[1][1], cs, sn, ta);
          O[0][0] = cs; O[0][1] = -sn; O[1][0] = sn; O[1][1] = cs;
          margin = ta;
        }
        // rotated k x k blocks O g O^T and O d O^T
        double gn[3][3] = {}, dn[3][3] = {};
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
          for (int b = 0; b < K; ++b) {
            double sg = 0.0, sd = 0.0;
#pragma unroll
            for (int x = 0; x < K; ++x) {
              double tg = 0.0, td = 0.0;
#pragma unroll
              for (int y = 0; y < K; ++y) { tg += g[x][y] * O[b][y]; td += d[x][y] * O[b][y]; }
              sg += O[a][x] * tg;
              sd += O[a][x] * td;
            }
            gn[a][b] = sg;
            dn[a][b] = sd;
          }
        // eliminate the slot with the smallest off-diagonal norm (ties: later slot)
        const double f0 = fmax(0.0, gn[0][0] - dn[0][0] * dn[0][0]);
        const double fv1 = fmax(0.0, gn[1][1] - dn[1][1] * dn[1][1]);
        const double fv2 = K == 3 ? fmax(0.0, gn[2][2] - dn[2][2] * dn[2][2]) : 1e300;
        int es = fv1 <= f0 ? 1 : 0;
        double fm = es == 1 ? fv1 : f0;
        if (K == 3 && fv2 <= fm) { es = 2; fm = fv2; }
        {  // second smallest, for the (diagnostic) elimination margin
          const double hi01 = fmax(f0, fv1), lo01 = fmin(f0, fv1);
          const double lo2 = K == 3 ? (fv2 <= lo01 ? lo01 : fmin(hi01, fv2)) : hi01;
          const double lo1 = fmin(lo01, fv2);
          margin = fmin(margin, lo2 > 0.0 ? (lo2 - lo1) / lo2 : 0.0);
        }
        const int e = es == 0 ? t0 : (es == 1 ? t1 : t2);
        const int ta[3] = {t0, t1, t2};
#pragma unroll
        for (int a = 0; a < K; ++a) {
          gdiag[ta[a]] = (float)gn[a][a];
          ddiag[ta[a]] = (float)dn[a][a];
          rgs[ta[a]] = inv_sqrt_pos((float)gn[a][a]);
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) { sh_O[a] = 0.f; sh_gn[a] = 0.f; sh_dn[a] = 0.f; }
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
          for (int b = 0; b < K; ++b) {
            sh_O[a * 3 + b] = (float)O[a][b];
            sh_gn[a * 3 + b] = (float)gn[a][b];
            sh_dn[a * 3 + b] = (float)dn[a][b];
          }
        sh_e = e;
        sh_mg = (float)margin;
        sh_de = (float)(es == 0 ? dn[0][0] : (es == 1 ? dn[1][1] : dn[2][2]));
        sh_lit = 2.0 * fm;
      }
      __syncthreads();  // B

      float o_[9];
      float2 vn[3];
      int e, nxt, aslot, nsel;
      after_b(s, t0, t1, t2, R0, o_, e, nxt, aslot, nsel, vn);
      const int Tt[3] = {t0, t1, t2};
      {  // the next seed row's entries at T (a column of T other than the retiree), lane a
        Cand tc{-1.f, INT_MAX};
#pragma unroll
        for (int a = 0; a < K; ++a)
          if (lane == a && more && aslot < 0 && Tt[a] != e)
            tc = Cand{partner_score(rot_entry<K>(o_, a, vn).x, rgs[Tt[a]]), Tt[a]};
        if (lane < 3) sh_tc[lane] = tc;
      }
      // The next step's partners are known now unless its seed is in T (it is then scored in
      // full by the column waves): merge as after barrier A and request G_{t1 t2} at once, so
      // its latency passes during the column waves' half of the step.  An entry in a row or
      // column of this step's T is formed from the pre-rotation rows instead (its stores are
      // pending); every other entry is current.
      pre = false;
      if (K == 3 && more && nsel < 2) {
        const int sv = sel;
        sel = nsel;
        Cand g1, g2;
        merge(par ^ 1, g1, g2);
        sel = sv;
        const int n1 = g1.j, n2 = g2.j;
        if (n1 < c && n2 < c) {
          pre = true;
          const int a1 = slot_of(n1, t0, t1, t2), a2 = slot_of(n2, t0, t1, t2);
          if (a1 < 0 && a2 < 0) {
            x12 = GD[(size_t)n1 * ld + n2];
            x21 = GD[(size_t)n2 * ld + n1];
          } else if (a1 >= 0 && a2 >= 0) {
            x12 = make_float2(sh_gn[a1 * 3 + a2], sh_dn[a1 * 3 + a2]);
            x21 = make_float2(sh_gn[a2 * 3 + a1], sh_dn[a2 * 3 + a1]);
          } else {
            const int a = a1 >= 0 ? a1 : a2, x = a1 >= 0 ? n2 : n1;
            const float2 v[3] = {R0[x], R1[x], R2[x]};
            x12 = x21 = pick3(a, rot_entry<K>(o_, 0, v), rot_entry<K>(o_, 1, v),
                              rot_entry<K>(o_, 2, v));
          }
        }
      }
      if (lane == 0) {
        mask[e >> 5] &= ~(1u << (e & 31));
        // the rotation's level: one past the latest level touching its indices
        const int lv = 1 + max(max((int)lastlv[t0], (int)lastlv[t1]), K == 3 ? (int)lastlv[t2] : 0);
        lastlv[t0] = (unsigned short)lv;
        lastlv[t1] = (unsigned short)lv;
        if (K == 3) lastlv[t2] = (unsigned short)lv;
        if (A.rot_lvl) A.rot_lvl[A.rot0 + rb + s] = lv;
      }
      // the rotated k x k block and the rotation log, lane by lane; lanes past the last entry
      // repeat it, so the stores need no branch and the wait for the entries above counts them
      // exactly
      {
        const int kb = min(lane, K * K - 1), ka = kb / K, kc = kb % K;
        GD[(size_t)pick3(ka, t0, t1, t2) * ld + pick3(kc, t0, t1, t2)] =
            make_float2(sh_gn[ka * 3 + kc], sh_dn[ka * 3 + kc]);
        const int64_t ridx = A.rot0 + rb + s;
        const int l9 = min(lane, 8), l3 = min(lane, 2);
        A.rot_o[ridx * 9 + l9] = sh_O[l9];
        const int tl = l3 < K ? pick3(l3, t0, t1, t2) : -1;
        A.rot_loc[ridx * 3 + l3] = tl;
        A.rot_gid[ridx * 3 + l3] = tl >= 0 ? lgid[tl] : -1;
        A.rot_ret[ridx] = lgid[e];
        A.rot_margin[ridx] = sh_mg;
        A.rot_lit[ridx] = sh_lit;
        A.hdiag[lgid[e]] = sh_de;
        A.retflag[o + e] = 1;
      }
      tq0 = t0;
      tq1 = t1;
      tq2 = t2;
      i = nxt;
      sel = nsel;
    }
    return;
  }

  // ------------------------------------------------------------------ column waves
  // At equal priority wave 4 reaches barrier B last in nearly every step, ~2.5k cycles after the
  // other waves (per-wave timestamps), as a wave sharing a SIMD with the control wave's FP64
  // rotation arithmetic would; at a higher issue priority it no longer does, and the step
  // shortens by ~2% (the control wave then arrives last).
  if (wv == 4) __builtin_amdgcn_s_setprio(2);
  const int ct = tid - PMMF_WAVE;
  int jl[PER];           // own columns clamped into the cluster, for address forming
  float rg[PER];         // 1 / sqrt(G_jj) of the own columns
  uint32_t act = 0;      // bit q: own column q active
  float2 cur[PER], c0r[PER], c1r[PER], p1[PER], p2[PER];
  float2 cst[3][PER];    // column stores of the previous step
  uint64_t cmask = 0;    // which of them are real
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = ct + q * NC;
    const bool in = j < c;
    jl[q] = min(j, c - 1);
    act |= (uint32_t)in << q;
    rg[q] = in ? rgs[j] : 0.f;
    cur[q] = (in && r > 0) ? GD[(size_t)i * ld + j] : make_float2(0.f, 0.f);
    c0r[q] = c1r[q] = p1[q] = p2[q] = make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < 3; ++a) cst[a][q] = make_float2(0.f, 0.f);
  }
  // full scoring of the seed row held in cur (seed x; ex is skipped too) into slot 2 of parity par
  auto score_full = [&](int par, int x, int ex) {
    Cand b1{-1.f, INT_MAX}, b2{-1.f, INT_MAX};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
      if (((act >> q) & 1u) && j != x && j != ex)
        take<K>(b1, b2, Cand{partner_score(cur[q].x, rg[q]), j});
    }
    wave_top<K>(b1, b2);
    if (lane == 0) { red1[par][2][wv] = b1; red2[par][2][wv] = b2; }
  };
  if (r > 0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
      if (j < c) rowbuf[j] = cur[q];
    }
    score_full(0, i, -1);
  }

  for (int s = 0; s < r; ++s) {
    const int par = s & 1;
    const float2* R0 = rowbuf + (size_t)par * cmax;
    const bool more = s + 1 < r;
    __syncthreads();  // A
    Cand f1, f2;
    merge(par, f1, f2);
    if (f1.j >= c || (K == 3 && f2.j >= c)) return;  // reported by the control wave
    const int t0 = i, t1 = f1.j, t2 = K == 3 ? f2.j : -1;
    const int st1 = slot_of(t1, tq0, tq1, tq2), st2 = K == 3 ? slot_of(t2, tq0, tq1, tq2) : -1;
    if (wv == NW - 1 && s + 2 < r) {
      // next-seed rule: the rank-th active index after a retirement e is the rank-th one before
      // it if that lies below e, else the (rank + 1)-th.  The seed of step s+2 follows two more
      // retirements (steps s and s+1), so the rank-th to (rank + 2)-th indices are taken now;
      // after this step two candidates remain, after the next one the seed.  Taken by the last
      // column wave (among the first to reach barrier B), off the control wave's chain.
      const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u,
                                    (uint64_t)(s + 2));
      int kn[3];
      select_activeN<3>(mask, nw, (int)pmmf_mulhi(h, (uint64_t)(c - (s + 2))), kn);
      if (lane == 0) { sh_k[0] = kn[0]; sh_k[1] = kn[1]; sh_k[2] = kn[2]; }
    }
    // the next seed is cc0 if cc0 lies below this step's retiree e (one of T), else cc1: only the
    // rows that can be chosen are fetched and scored
    const int tmin = K == 3 ? min(t0, min(t1, t2)) : min(t0, t1);
    const int tmax = K == 3 ? max(t0, max(t1, t2)) : max(t0, t1);
    const bool need0 = more && cc0 < tmax, need1 = more && cc0 >= tmin;

    // partner rows (pre-rotation), then the candidate rows of the next seed, read the same way
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
      const int sj = slot_of(j, tq0, tq1, tq2);
      const uint32_t jq = (uint32_t)jl[q];
      p1[q] = GD[(sj >= 0 && st1 < 0) ? (uint32_t)(j * ld + t1) : (uint32_t)(t1 * ld) + jq];
      if (K == 3)
        p2[q] = GD[(sj >= 0 && st2 < 0) ? (uint32_t)(j * ld + t2) : (uint32_t)(t2 * ld) + jq];
    }
    if (need0) {
      const int sc0 = slot_of(cc0, tq0, tq1, tq2);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = ct + q * NC;
        const int sj = slot_of(j, tq0, tq1, tq2);
        c0r[q] = GD[(sj >= 0 && sc0 < 0) ? (uint32_t)(j * ld + cc0) : (uint32_t)(cc0 * ld + jl[q])];
      }
    }
    if (need1) {
      const int sc1 = slot_of(cc1, tq0, tq1, tq2);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = ct + q * NC;
        const int sj = slot_of(j, tq0, tq1, tq2);
        c1r[q] = GD[(sj >= 0 && sc1 < 0) ? (uint32_t)(j * ld + cc1) : (uint32_t)(cc1 * ld + jl[q])];
      }
    }
    // pre-rotation partner rows, for re-forming the next seed row's entries at T
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
      if (j < c) {
        R1[j] = p1[q];
        if (K == 3) R2[j] = p2[q];
      }
    }
    // the candidate rows that can become the next seed, scored outside T (for the merge of
    // step s+1)
    if (need0 || need1) {
      Cand a1{-1.f, INT_MAX}, a2{-1.f, INT_MAX}, b1{-1.f, INT_MAX}, b2{-1.f, INT_MAX};
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = ct + q * NC;
        const bool ok = ((act >> q) & 1u) && slot_of(j, t0, t1, t2) < 0;
        if (need0 && ok && j != cc0) take<K>(a1, a2, Cand{partner_score(c0r[q].x, rg[q]), j});
        if (need1 && ok && j != cc1) take<K>(b1, b2, Cand{partner_score(c1r[q].x, rg[q]), j});
      }
      const int np = par ^ 1;
      if (need0) {
        wave_top<K>(a1, a2);
        if (lane == 0) { red1[np][0][wv] = a1; red2[np][0][wv] = a2; }
      }
      if (need1) {
        wave_top<K>(b1, b2);
        if (lane == 0) { red1[np][1][wv] = b1; red2[np][1][wv] = b2; }
      }
    }
    // the previous step's column stores (the entries that are not zero), last: nothing before
    // barrier B waits for them, and the loads above take the transposes of these entries
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
#pragma unroll
      for (int a = 0; a < K; ++a) {
        const int ta = a == 0 ? tq0 : (a == 1 ? tq1 : tq2);
        if ((cmask >> (a * PER + q)) & 1ull) GD[(uint32_t)(j * ld + ta)] = cst[a][q];
      }
    }
    __syncthreads();  // B

    float o_[9];
    float2 vn[3];
    int e, nxt, aslot, nsel;
    after_b(s, t0, t1, t2, R0, o_, e, nxt, aslot, nsel, vn);
    const int Tt[3] = {t0, t1, t2};
    float2 nrow[PER];
    cmask = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = ct + q * NC;
      const int bj = slot_of(j, t0, t1, t2);
      if (bj >= 0) rg[q] = rgs[j];                  // new G_jj of a column in T
      if (j == e) act &= ~(1u << q);                // this step's retiree
      nrow[q] = nsel == 0 ? c0r[q] : c1r[q];
      const bool in = j < c && bj < 0;
      const bool a_now = in && ((act >> q) & 1u);
      const float2 v[3] = {cur[q], p1[q], p2[q]};
      // rows T: O applied to the pre-rotation rows (a column in T or beyond the cluster writes
      // into the dead column of the retiree; a retired column's entry is dead too)
      float2 nv[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
#pragma unroll
      for (int a = 0; a < K; ++a) {
        nv[a] = rot_entry<K>(o_, a, v);
        GD[(uint32_t)(Tt[a] * ld) + (uint32_t)(in ? j : e)] = nv[a];
        cst[a][q] = nv[a];
        const uint32_t m = __float_as_uint(nv[a].x) | __float_as_uint(nv[a].y) |
                           __float_as_uint(v[a].x) | __float_as_uint(v[a].y);
        cmask |= (uint64_t)(a_now && (m << 1) != 0u) << (a * PER + q);
      }
      // the next seed row at column j
      if (more) {
        if (bj >= 0) {
          nrow[q] = aslot >= 0 ? make_float2(sh_gn[aslot * 3 + bj], sh_dn[aslot * 3 + bj])
                               : pick3(bj, rot_entry<K>(o_, 0, vn), rot_entry<K>(o_, 1, vn),
                                       rot_entry<K>(o_, 2, vn));
        } else if (aslot >= 0) {
          nrow[q] = pick3(aslot, nv[0], nv[1], nv[2]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) cur[q] = nrow[q];
    if (more) {
      float2* R0n = rowbuf + (size_t)(par ^ 1) * cmax;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = ct + q * NC;
        if (j < c) R0n[j] = cur[q];
      }
      if (nsel == 2) score_full(par ^ 1, nxt, e);
    }
    tq0 = t0;
    tq1 = t1;
    tq2 = t2;
    i = nxt;
    sel = nsel;
  }
}

template <int NT, int PER, int K>
static hipError_t search_launch(const FindArgs& a, int m, int cmax, hipStream_t s) {
  const size_t lds = find_lds_bytes(cmax) + (size_t)cmax * (sizeof(float) + sizeof(unsigned short));
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)&k_search<NT, PER, K>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_search<NT, PER, K><<<m, NT, lds, s>>>(a, cmax);
  return hipGetLastError();
}
template <int PER>
static hipError_t search_launch_k(const FindArgs& a, int m, int cmax, hipStream_t s) {
  return a.k == 3 ? search_launch<512, PER, 3>(a, m, cmax, s)
                  : search_launch<512, PER, 2>(a, m, cmax, s);
}

// ------------------------------------------------------------------------------------------
// Greedy search on the BF16 Gram (Alg. 2 with the scores shortlisted from G~ and decided exactly).
// Same layout and step as k_find, with G~ in the first halves of the (G, D) pool; per step:
//   1. approximate top-(k-1) scores from the seed's G~ row;
//   2. shortlist, in ascending index order, every active j whose approximate score is within
//      2 e of the (k-1)-th best, e = BF16_SAFETY (2^-7 + R 2^-24) sqrt(G_ii) bounding the score
//      error (|G~_ij - G_ij| <= (2 u_bf16 + R u_f32) ||S_i|| ||S_j||, Cauchy-Schwarz);
//   3. exact FP32 dots of the seed's slab column with each shortlisted column decide the pick
//      (ties to the lower index), and the exact (t1, t2) dot completes G[T, T];
//   4. rotation, elimination and updates as in k_find, with G~ updated like G and the slab
//      columns T right-rotated (S[:, T] <- S[:, T] O^T) so later dots stay exact.
// Every shortlisted candidate is rescored (in rounds of BF16_LIST), so the pick is the exact one;
// steps whose shortlist needed more than one round are counted.
constexpr float BF16_SAFETY = 2.f;
constexpr int BF16_LIST = 64;

__device__ inline float slab_dot(const float* __restrict__ a, const float* __restrict__ b, int R,
                                 int lane) {
  float acc = 0.f;
  for (int r0 = 0; r0 < R; r0 += 4 * PMMF_WAVE) {
    float x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + q * PMMF_WAVE + lane;
      x[q] = r < R ? a[r] : 0.f;
      y[q] = r < R ? b[r] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fmaf(x[q], y[q], acc);
  }
  return pmmf_wave_sum_dpp(acc);
}

template <int PER, int K>
__global__ void __launch_bounds__(256) k_find_bf16(FindArgs A, int cmax) {
  constexpr int NT = 256, NW = NT / PMMF_WAVE;
  extern __shared__ float lds_f[];
  float* gdiag = lds_f;
  float* ddiag = gdiag + cmax;
  float2* rowbuf = reinterpret_cast<float2*>(ddiag + cmax);
  int* lgid = reinterpret_cast<int*>(rowbuf + 4 * (size_t)cmax);
  uint32_t* mask = reinterpret_cast<uint32_t*>(lgid + cmax);
  __shared__ Cand red1[NW], red2[NW];
  __shared__ int sh_i, sh_e, sh_c0, sh_c1, sh_t1, sh_t2;
  __shared__ float sh_O[9], sh_gn[9], sh_dn[9];
  __shared__ int qcount[PER][NW];
  __shared__ int list_j[BF16_LIST];
  __shared__ float list_dot[BF16_LIST];

  const int tid = threadIdx.x, lane = pmmf_lane(), wv = pmmf_wave();
  const int u = A.order[blockIdx.x];
  const int o = A.off[u];
  const int c = A.off[u + 1] - o;
  const int ld = gd_stride(c);  // row stride of the cluster's (G, D) array
  const int r = A.rcnt[u];
  const int rb = A.roff[u];
  const int nw = (c + 31) / 32;
  constexpr int kk = K;
  float2* __restrict__ GD = A.GD + A.gbase[u];
  const int Ru = A.slab_rows[u];
  float* __restrict__ SL = A.slab + A.slab_off[u];
  float2* R1 = rowbuf + 2 * (size_t)cmax;
  float2* R2 = rowbuf + 3 * (size_t)cmax;
  const float gamma = BF16_SAFETY * (0.0078125f + (float)Ru * 5.9604645e-8f);

  for (int j = tid; j < c; j += NT) {
    const float2 dg = GD[(size_t)j * ld + j];
    gdiag[j] = dg.x;
    ddiag[j] = dg.y;
    lgid[j] = A.gid[o + j];
  }
  for (int q = tid; q < nw; q += NT) {
    const int rem = c - q * 32;
    mask[q] = rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
  }
  __syncthreads();
  if (tid < PMMF_WAVE && r > 0) {
    const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u, 0);
    const int i0 = select_active(mask, nw, (int)pmmf_mulhi(h, (uint64_t)c));
    if (tid == 0) sh_i = i0;
  }
  __syncthreads();
  int i = r > 0 ? sh_i : 0;
  int e_prev = -1;
  float2 cur[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    cur[q] = (r > 0 && j < c) ? GD[(size_t)i * ld + j] : make_float2(0.f, 0.f);
  }
  unsigned long long n_cut = 0, n_scored = 0;

  for (int s = 0; s < r; ++s) {
    float2* R0 = rowbuf + (size_t)(s & 1) * cmax;
    // 1. approximate scores
    float sc[PER];
    Cand b1{-1.f, INT_MAX}, b2{-1.f, INT_MAX};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      sc[q] = -1.f;
      if (j < c) {
        R0[j] = cur[q];
        const bool act = ((mask[j >> 5] >> (j & 31)) & 1u) && j != e_prev;
        if (act && j != i) {
          const float gd = gdiag[j];
          float v = gd > 0.f ? fabsf(cur[q].x) / sqrtf(gd) : 0.f;
          if (!(v >= 0.f)) v = 0.f;
          sc[q] = v;
          Cand cnd{v, j};
          if (better(cnd, b1)) { b2 = b1; b1 = cnd; }
          else if (better(cnd, b2)) b2 = cnd;
        }
      }
    }
    for (int ofs = PMMF_WAVE / 2; ofs > 0; ofs >>= 1) {
      Cand o1{__shfl_xor(b1.s, ofs), __shfl_xor(b1.j, ofs)};
      if (kk == 3) {
        Cand o2{__shfl_xor(b2.s, ofs), __shfl_xor(b2.j, ofs)};
        merge2(b1, b2, o1, o2);
      } else if (better(o1, b1)) {
        b1 = o1;
      }
    }
    if (lane == 0) { red1[wv] = b1; red2[wv] = b2; }
    __syncthreads();  // A
    Cand f1 = red1[0], f2 = red2[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      if (kk == 3) merge2(f1, f2, red1[q], red2[q]);
      else if (better(red1[q], f1)) f1 = red1[q];
    }
    if (f1.j >= c || (kk == 3 && f2.j >= c)) {
      if (tid == 0) atomicOr(A.err, 1);
      return;
    }
    // 2. ordered shortlist: ballots per column slice, per-wave counts, offsets
    const float thr = (kk == 3 ? f2.s : f1.s) - 2.f * gamma * sqrtf(fmaxf(gdiag[i], 0.f));
    uint64_t ball[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      ball[q] = __ballot(sc[q] >= 0.f && sc[q] >= thr);
      if (lane == 0) qcount[q][wv] = __popcll(ball[q]);
    }
    __syncthreads();  // A2
    int total = 0, mypos[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      int before = 0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) {
        if (w2 == wv) before = total;
        total += qcount[q][w2];
      }
      mypos[q] = ((ball[q] >> lane) & 1ull) ? before + pmmf_lanes_below(ball[q]) : -1;
    }
    // 3. exact dots of the seed column with the shortlisted columns, in rounds of BF16_LIST
    //    candidates (ascending index), one wave per candidate
    const float* si = SL + (size_t)i * Ru;
    Cand x1{-1.f, INT_MAX}, x2{-1.f, INT_MAX};
    float d1 = 0.f, d2 = 0.f;
    for (int w0 = 0; w0 < total; w0 += BF16_LIST) {
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (mypos[q] >= w0 && mypos[q] < w0 + BF16_LIST) list_j[mypos[q] - w0] = tid + q * NT;
      const int nl = min(total - w0, BF16_LIST);
      __syncthreads();  // A3
      // four candidates per wave and pass: the seed column is read once for the four
      for (int c4 = 4 * wv; c4 < nl; c4 += 4 * NW) {
        const float* col[4];
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4)
          col[e4] = SL + (size_t)list_j[min(c4 + e4, nl - 1)] * Ru;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int r0 = 0; r0 < Ru; r0 += 2 * PMMF_WAVE) {
          float x[2], y[4][2];
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) {
            const int rr = r0 + h2 * PMMF_WAVE + lane;
            x[h2] = rr < Ru ? si[rr] : 0.f;
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) y[e4][h2] = rr < Ru ? col[e4][rr] : 0.f;
          }
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) acc[e4] = fmaf(x[h2], y[e4][h2], acc[e4]);
        }
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
          const float d = pmmf_wave_sum_dpp(acc[e4]);
          if (lane == 0 && c4 + e4 < nl) list_dot[c4 + e4] = d;
        }
      }
      __syncthreads();  // A4
      for (int ci = 0; ci < nl; ++ci) {
        const int j = list_j[ci];
        const float gd = gdiag[j];
        float v = gd > 0.f ? fabsf(list_dot[ci]) / sqrtf(gd) : 0.f;
        if (!(v >= 0.f)) v = 0.f;
        const Cand cnd{v, j};
        if (better(cnd, x1)) { x2 = x1; d2 = d1; x1 = cnd; d1 = list_dot[ci]; }
        else if (better(cnd, x2)) { x2 = cnd; d2 = list_dot[ci]; }
      }
      if (w0 + BF16_LIST < total) __syncthreads();  // the next round reuses the list
    }
    if (x1.j >= c || (kk == 3 && x2.j >= c)) {
      if (tid == 0) atomicOr(A.err, 1);
      return;
    }
    if (tid == 0) {
      n_cut += total > BF16_LIST ? 1 : 0;
      n_scored += total;
    }
    const int t0 = i, t1 = x1.j, t2 = kk == 3 ? x2.j : -1;
    // partner rows of G~ and D
    float2 p1[PER], p2[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      p1[q] = p2[q] = make_float2(0.f, 0.f);
      if (j < c) {
        p1[q] = GD[(size_t)t1 * ld + j];
        if (kk == 3) p2[q] = GD[(size_t)t2 * ld + j];
      }
    }
    float g12 = 0.f;
    if (kk == 3 && wv == 0) g12 = slab_dot(SL + (size_t)t1 * Ru, SL + (size_t)t2 * Ru, Ru, lane);
    if (tid == 0) {
      double g[3][3] = {}, d[3][3] = {}, O[3][3] = {};
      g[0][0] = gdiag[t0];
      d[0][0] = ddiag[t0];
      g[1][1] = gdiag[t1];
      d[1][1] = ddiag[t1];
      g[0][1] = g[1][0] = d1;
      d[0][1] = d[1][0] = R0[t1].y;
      if (kk == 3) {
        g[2][2] = gdiag[t2];
        d[2][2] = ddiag[t2];
        g[0][2] = g[2][0] = d2;
        d[0][2] = d[2][0] = R0[t2].y;
        g[1][2] = g[2][1] = g12;
        const float2 a12 = GD[(size_t)t1 * ld + t2], a21 = GD[(size_t)t2 * ld + t1];
        d[1][2] = d[2][1] = 0.5 * ((double)a12.y + (double)a21.y);
      }
      double margin = 3.0e38;
      if (kk == 2) {
        double cc, ss, ta;
        rot2(g[0][0], g[0][1], g[1][1], cc, ss, ta);
        O[0][0] = cc; O[0][1] = -ss; O[1][0] = ss; O[1][1] = cc;
        margin = fmin(margin, ta);
      } else {
        double tm, em;
        rot3(g, O, tm, em);
        margin = fmin(margin, fmin(tm, em));
      }
      double gn[3][3] = {}, dn[3][3] = {};
#pragma unroll
      for (int a = 0; a < kk; ++a)
#pragma unroll
        for (int b = 0; b < kk; ++b) {
          double sg = 0.0, sd = 0.0;
#pragma unroll
          for (int x = 0; x < kk; ++x) {
            double tg = 0.0, td = 0.0;
#pragma unroll
            for (int y = 0; y < kk; ++y) { tg += g[x][y] * O[b][y]; td += d[x][y] * O[b][y]; }
            sg += O[a][x] * tg;
            sd += O[a][x] * td;
          }
          gn[a][b] = sg;
          dn[a][b] = sd;
        }
      const double f0 = fmax(0.0, gn[0][0] - dn[0][0] * dn[0][0]);
      const double f1v = fmax(0.0, gn[1][1] - dn[1][1] * dn[1][1]);
      const double f2v = kk == 3 ? fmax(0.0, gn[2][2] - dn[2][2] * dn[2][2]) : 1e300;
      int es = f1v <= f0 ? 1 : 0;
      double fmin_ = es == 1 ? f1v : f0;
      if (kk == 3 && f2v <= fmin_) { es = 2; fmin_ = f2v; }
      {
        const double hi01 = fmax(f0, f1v), lo01 = fmin(f0, f1v);
        const double lo2 = kk == 3 ? (f2v <= lo01 ? lo01 : fmin(hi01, f2v)) : hi01;
        const double lo1 = fmin(lo01, f2v);
        margin = fmin(margin, lo2 > 0.0 ? (lo2 - lo1) / lo2 : 0.0);
      }
      const int e = es == 0 ? t0 : (es == 1 ? t1 : t2);
      const double dee = es == 0 ? dn[0][0] : (es == 1 ? dn[1][1] : dn[2][2]);
      gdiag[t0] = (float)gn[0][0];
      ddiag[t0] = (float)dn[0][0];
      gdiag[t1] = (float)gn[1][1];
      ddiag[t1] = (float)dn[1][1];
      if (kk == 3) {
        gdiag[t2] = (float)gn[2][2];
        ddiag[t2] = (float)dn[2][2];
      }
      sh_e = e;
#pragma unroll
      for (int a = 0; a < 9; ++a) { sh_O[a] = 0.f; sh_gn[a] = 0.f; sh_dn[a] = 0.f; }
#pragma unroll
      for (int a = 0; a < kk; ++a)
#pragma unroll
        for (int b = 0; b < kk; ++b) {
          sh_O[a * 3 + b] = (float)O[a][b];
          sh_gn[a * 3 + b] = (float)gn[a][b];
          sh_dn[a * 3 + b] = (float)dn[a][b];
        }
      const int64_t ridx = A.rot0 + rb + s;
      A.rot_loc[ridx * 3 + 0] = t0;
      A.rot_loc[ridx * 3 + 1] = t1;
      A.rot_loc[ridx * 3 + 2] = kk == 3 ? t2 : -1;
      A.rot_gid[ridx * 3 + 0] = lgid[t0];
      A.rot_gid[ridx * 3 + 1] = lgid[t1];
      A.rot_gid[ridx * 3 + 2] = kk == 3 ? lgid[t2] : -1;
#pragma unroll
      for (int a = 0; a < 9; ++a) A.rot_o[ridx * 9 + a] = sh_O[a];
      A.rot_ret[ridx] = lgid[e];
      A.rot_margin[ridx] = (float)margin;
      A.rot_lit[ridx] = 2.0 * fmin_;
      A.hdiag[lgid[e]] = (float)dee;
      A.retflag[o + e] = 1;
    } else if (wv == 1 && s + 1 < r) {
      const uint64_t h = pmmf_hash4(A.seed, PMMF_TAG_SEED_ROW, (uint64_t)A.p, (uint64_t)u,
                                    (uint64_t)(s + 1));
      const int rank = (int)pmmf_mulhi(h, (uint64_t)(c - s - 1));
      const int c0 = select_active(mask, nw, rank);
      const int c1 = select_active(mask, nw, rank + 1);
      if (tid == PMMF_WAVE) { sh_c0 = c0; sh_c1 = c1; }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if (j < c) {
        R1[j] = p1[q];
        if (kk == 3) R2[j] = p2[q];
      }
    }
    __syncthreads();  // B

    float o_[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) o_[a] = sh_O[a];
    const int e = sh_e;
    const bool more = s + 1 < r;
    const int nxt = more ? (sh_c0 < e ? sh_c0 : sh_c1) : -1;
    const int aslot = nxt == t0 ? 0 : (nxt == t1 ? 1 : ((kk == 3 && nxt == t2) ? 2 : -1));
    float2 nrow[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      nrow[q] = make_float2(0.f, 0.f);
      if (more && aslot < 0 && j < c) nrow[q] = GD[(size_t)nxt * ld + j];
    }
    float2 vn[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    if (more && aslot < 0) {
      vn[0] = R0[nxt];
      vn[1] = R1[nxt];
      if (kk == 3) vn[2] = R2[nxt];
    }
    if (tid == 0) mask[e >> 5] &= ~(1u << (e & 31));
    const int Tt[3] = {t0, t1, t2};
    if (tid < kk * kk) {
      const int a = tid / kk, b = tid % kk;
      GD[(size_t)Tt[a] * ld + Tt[b]] = make_float2(sh_gn[a * 3 + b], sh_dn[a * 3 + b]);
    }
    // slab columns T right-rotated: S[:, T] <- S[:, T] O^T
    for (int rr = tid; rr < Ru; rr += NT) {
      float v[3] = {SL[(size_t)t0 * Ru + rr], SL[(size_t)t1 * Ru + rr],
                    kk == 3 ? SL[(size_t)t2 * Ru + rr] : 0.f};
#pragma unroll
      for (int a = 0; a < K; ++a) {
        float acc = 0.f;
#pragma unroll
        for (int b = 0; b < K; ++b) acc = fmaf(o_[a * 3 + b], v[b], acc);
        SL[(size_t)Tt[a] * Ru + rr] = acc;
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if (j >= c) continue;
      const int bj = j == t0 ? 0 : (j == t1 ? 1 : ((kk == 3 && j == t2) ? 2 : -1));
      if (bj >= 0) {
        if (more) {
          if (aslot >= 0) nrow[q] = make_float2(sh_gn[aslot * 3 + bj], sh_dn[aslot * 3 + bj]);
          else nrow[q] = rot_entry<K>(o_, bj, vn);
        }
        continue;
      }
      const bool a_now = (mask[j >> 5] >> (j & 31)) & 1u;
      if (!a_now) continue;
      const float2 v[3] = {cur[q], p1[q], p2[q]};
#pragma unroll
      for (int a = 0; a < K; ++a) {
        const float2 nv = rot_entry<K>(o_, a, v);
        GD[(size_t)Tt[a] * ld + j] = nv;
        if (nv.x != 0.f || nv.y != 0.f || v[a].x != 0.f || v[a].y != 0.f)
          GD[(size_t)j * ld + Tt[a]] = nv;
        if (a == aslot) nrow[q] = nv;
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) cur[q] = nrow[q];
    e_prev = e;
    i = nxt;
  }
  if (tid == 0 && r > 0) {
    atomicAdd(A.sl_stats + 0, n_cut);
    atomicAdd(A.sl_stats + 1, n_scored);
  }
}

template <int PER, int K>
static hipError_t find_bf16_launch(const FindArgs& a, int m, int cmax, size_t lds,
                                   hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)&k_find_bf16<PER, K>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_find_bf16<PER, K><<<m, 256, lds, s>>>(a, cmax);
  return hipGetLastError();
}

template <int PER>
static hipError_t find_bf16_launch_k(const FindArgs& a, int m, int cmax, size_t lds,
                                     hipStream_t s) {
  return a.k == 3 ? find_bf16_launch<PER, 3>(a, m, cmax, lds, s)
                  : find_bf16_launch<PER, 2>(a, m, cmax, lds, s);
}

hipError_t launch_find_bf16(const FindArgs& a, int m, int cmax, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const size_t lds = find_lds_bytes(cmax);
  if (cmax <= 256) return find_bf16_launch_k<1>(a, m, cmax, lds, s);
  if (cmax <= 512) return find_bf16_launch_k<2>(a, m, cmax, lds, s);
  if (cmax <= 1024) return find_bf16_launch_k<4>(a, m, cmax, lds, s);
  if (cmax <= 2048) return find_bf16_launch_k<8>(a, m, cmax, lds, s);
  if (cmax <= 3072) return find_bf16_launch_k<12>(a, m, cmax, lds, s);
  return hipErrorInvalidValue;
}

size_t find_lds_bytes(int cmax) {
  return (size_t)cmax * 2 * sizeof(float) + (size_t)cmax * 4 * sizeof(float2) +
         (size_t)cmax * sizeof(int) + (size_t)((cmax + 31) / 32) * 4;
}

hipError_t launch_find(const FindArgs& a, int m, int cmax, int nt, hipStream_t s) {
  if (m == 0) return hipSuccess;
  if (a.elims != 2) {  // one retirement per rotation: control wave + 7 column waves
    if (cmax <= 448) return search_launch_k<1>(a, m, cmax, s);
    if (cmax <= 896) return search_launch_k<2>(a, m, cmax, s);
    if (cmax <= 1344) return search_launch_k<3>(a, m, cmax, s);
    if (cmax <= 2240) return search_launch_k<5>(a, m, cmax, s);
    if (cmax <= 3072) return search_launch_k<7>(a, m, cmax, s);
    return hipErrorInvalidValue;
  }
  const size_t lds = find_lds_bytes(cmax);
  if (nt == 512) {
    if (cmax <= 512) return find_launch_k<512, 1>(a, m, cmax, lds, s);
    if (cmax <= 1024) return find_launch_k<512, 2>(a, m, cmax, lds, s);
    if (cmax <= 2048) return find_launch_k<512, 4>(a, m, cmax, lds, s);
    if (cmax <= 3072) return find_launch_k<512, 6>(a, m, cmax, lds, s);
  } else {
    if (cmax <= 256) return find_launch_k<256, 1>(a, m, cmax, lds, s);
    if (cmax <= 512) return find_launch_k<256, 2>(a, m, cmax, lds, s);
    if (cmax <= 1024) return find_launch_k<256, 4>(a, m, cmax, lds, s);
    if (cmax <= 2048) return find_launch_k<256, 8>(a, m, cmax, lds, s);
    if (cmax <= 3072) return find_launch_k<256, 12>(a, m, cmax, lds, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// Accumulated rotation of each cluster, Qbar_u = O_r ... O_1, rebuilt from the stage's sweep log:
// one workgroup per (cluster, 4-column slice) holds the slice of the identity in LDS and applies
// the rotations level by level (a level's rotations touch disjoint rows); x[T] <- O x[T] on each
// column of the slice.  Only the nonzeros leave the workgroup: column j of Qbar_u (row j of
// Qbar^T, rows ascending) goes to its own c_u slots of a scratch pool at gbase[u] + j c_u, with
// its count; k_qt_compact then packs the columns into the CSR of Qbar^T.
template <int K, int BQ_W, int NT>
__global__ void __launch_bounds__(NT) k_qsparse(const int32_t* __restrict__ off,
                                                 const int64_t* __restrict__ gbase,
                                                 const int32_t* __restrict__ lvl_ptr,
                                                 int lvl_stride, const int32_t* __restrict__ depth,
                                                 const int32_t* __restrict__ sw_loc,
                                                 const float* __restrict__ sw_o,
                                                 int32_t* __restrict__ cnt,
                                                 int32_t* __restrict__ sci,
                                                 float* __restrict__ scv) {
  extern __shared__ float tile[];  // [BQ_W][cs], then the cluster's level starts [depth + 1]
  constexpr int NWV = NT / PMMF_WAVE;
  __shared__ int part[NWV][BQ_W];
  const int u = blockIdx.y;
  const int o = off[u];
  const int c = off[u + 1] - o;
  const int col0 = blockIdx.x * BQ_W;
  if (col0 >= c) return;
  const int tid = threadIdx.x;
  // column-major slice with an odd column stride: the BQ_W columns of one row fall in distinct
  // banks, and the extraction below reads 64 consecutive rows of one column per instruction
  const int cs = c | 1;
  const int* lp = lvl_ptr + (size_t)u * lvl_stride;
  const int dep = depth[u];
  int* slp = reinterpret_cast<int*>(tile + (size_t)BQ_W * cs);
  for (int q = tid; q <= dep; q += NT) slp[q] = lp[q];
  for (int q = tid; q < BQ_W * cs; q += NT) {
    const int w = q / cs, row = q - w * cs;
    tile[q] = row == col0 + w ? 1.f : 0.f;
  }
  __syncthreads();
  // Thread tid takes items tid + i NT (i < QS_I) of each level (item = rotation x column); their
  // slots and blocks are loaded one level ahead into a second register set.  Items past QS_I NT
  // in a level (a level of more than QS_I NT / BQ_W rotations) load their rotation when they are
  // applied.  One item: more items per thread cost registers, and the kernel is bound by how many
  // workgroups are resident (rotate phase 22.6 ms with four items, 21.8 ms with one).
  constexpr int QS_I = 1;
  struct Items {
    int id[QS_I][K];
    float om[QS_I][K * K];
  };
  auto fetch = [&](int l, Items& it) {
    if (l >= dep) return;
    const int r0 = slp[l], n = (slp[l + 1] - r0) * BQ_W;
#pragma unroll
    for (int i = 0; i < QS_I; ++i) {
      const int q = min(tid + i * NT, max(n - 1, 0));
      const int rr = r0 + q / BQ_W;
#pragma unroll
      for (int a = 0; a < K; ++a) it.id[i][a] = sw_loc[(size_t)rr * K + a];
#pragma unroll
      for (int ab = 0; ab < K * K; ++ab) it.om[i][ab] = sw_o[(size_t)rr * K * K + ab];
    }
  };
  auto rotate = [&](int w, const int (&id)[K], const float* om) {
    float* col = tile + w * cs;
    float x[K];
#pragma unroll
    for (int a = 0; a < K; ++a) x[a] = col[id[a]];
#pragma unroll
    for (int a = 0; a < K; ++a) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < K; ++b) acc = fmaf(om[a * K + b], x[b], acc);
      col[id[a]] = acc;
    }
  };
  auto level = [&](int l, const Items& it) {
    const int r0 = slp[l], n = (slp[l + 1] - r0) * BQ_W;
#pragma unroll
    for (int i = 0; i < QS_I; ++i) {
      const int q = tid + i * NT;
      if (q < n) rotate(q % BQ_W, it.id[i], it.om[i]);
    }
    for (int q = tid + QS_I * NT; q < n; q += NT) {
      const int rr = r0 + q / BQ_W;
      int id[K];
#pragma unroll
      for (int a = 0; a < K; ++a) id[a] = sw_loc[(size_t)rr * K + a];
      rotate(q % BQ_W, id, sw_o + (size_t)rr * K * K);
    }
    __syncthreads();
  };
  Items ia, ib;
  fetch(0, ia);
  for (int l = 0; l < dep; l += 2) {
    fetch(l + 1, ib);
    level(l, ia);
    if (l + 1 >= dep) break;
    fetch(l + 2, ia);
    level(l + 1, ib);
  }
  // nonzeros of each column in ascending rows: wave v takes rows [v rw, (v + 1) rw) in 64-row
  // chunks; a ballot orders a chunk's nonzeros, the waves' counts (scanned in wave order) place
  // each wave's run
  const int wv = tid / PMMF_WAVE, lane = pmmf_lane();
  const int rw = ((c + NWV * PMMF_WAVE - 1) / (NWV * PMMF_WAVE)) * PMMF_WAVE;
  const int rb = min(c, wv * rw), re = min(c, rb + rw);
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int w = 0; w < BQ_W; ++w) {
    const float* col = tile + w * cs;
    int n = 0;
    for (int r = rb; r < re; r += PMMF_WAVE) {
      const int row = r + lane;
      n += __popcll(__ballot(row < re && col[min(row, c - 1)] != 0.f));
    }
    if (lane == 0) part[wv][w] = n;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < BQ_W; ++w) {
    if (col0 + w >= c) continue;
    int before = 0, total = 0;
#pragma unroll
    for (int v = 0; v < NWV; ++v) {
      before += v < wv ? part[v][w] : 0;
      total += part[v][w];
    }
    if (tid == 0) cnt[o + col0 + w] = total;
    const size_t cb = (size_t)gbase[u] + (size_t)(col0 + w) * c;
    const float* col = tile + w * cs;
    int pos = before;
    for (int r = rb; r < re; r += PMMF_WAVE) {
      const int row = r + lane;
      const float v = col[min(row, c - 1)];
      const bool nz = row < re && v != 0.f;
      const uint64_t bm = __ballot(nz);
      if (nz) {
        const int at = pos + __popcll(bm & below);
        sci[cb + at] = o + row;
        scv[cb + at] = v;
      }
      pos += __popcll(bm);
    }
  }
}

hipError_t launch_qsparse(int m, int k, const int32_t* off, const int64_t* gbase,
                          const int32_t* lvl_ptr, int lvl_stride, const int32_t* depth,
                          const int32_t* sw_loc, const float* sw_o, int32_t* cnt, int32_t* sci,
                          float* scv, int cmax, hipStream_t s) {
  if (m == 0) return hipSuccess;
  // 4-column slices, 256 threads: the fastest of 2, 4, 8 and 16 columns with 128, 256 and 512
  // threads on the 262k factor (each workgroup is bound by its chain of level barriers, so more
  // resident workgroups win until the extra copies of the rotation loads cost more)
  constexpr int bw = 4;
  const size_t lds = (size_t)(cmax | 1) * bw * sizeof(float) + (size_t)lvl_stride * sizeof(int);
  dim3 grid((unsigned)((cmax + bw - 1) / bw), (unsigned)m);
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    kern<<<grid, 256, lds, s>>>(off, gbase, lvl_ptr, lvl_stride, depth, sw_loc, sw_o, cnt, sci,
                                scv);
    return hipGetLastError();
  };
  return k == 3 ? go(&k_qsparse<3, bw, 256>) : go(&k_qsparse<2, bw, 256>);
}

// Packs the columns left by k_qsparse into the CSR of Qbar^T (row pointers rp from the scan of
// their counts): one wave per position j.
__global__ void k_qt_compact(int S, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ cl_of, const int64_t* __restrict__ gbase,
                             const int32_t* __restrict__ sci, const float* __restrict__ scv,
                             const int64_t* __restrict__ rp, int32_t* __restrict__ qci,
                             float* __restrict__ qcv) {
  const int j = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (j >= S) return;
  const int u = cl_of[j];
  const int o = off[u], c = off[u + 1] - o;
  const size_t cb = (size_t)gbase[u] + (size_t)(j - o) * c;
  const int64_t q0 = rp[j];
  const int n = (int)(rp[j + 1] - q0);
  for (int t = pmmf_lane(); t < n; t += PMMF_WAVE) {
    qci[q0 + t] = sci[cb + t];
    qcv[q0 + t] = scv[cb + t];
  }
}

hipError_t launch_qt_compact(int S, const int32_t* off, const int32_t* cl_of,
                             const int64_t* gbase, const int32_t* sci, const float* scv,
                             const int64_t* rp, int32_t* qci, float* qcv, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_qt_compact<<<(S + 3) / 4, 256, 0, s>>>(S, off, cl_of, gbase, sci, scv, rp, qci, qcv);
  return hipGetLastError();
}

// Rows of a CSR put in ascending column order (out of place): one wave per row, each entry's rank
// among its row's columns (distinct) is its place.
__global__ void k_sort_rows(int n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const float* __restrict__ cv, int32_t* __restrict__ oci,
                            float* __restrict__ ocv) {
  const int r = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (r >= n) return;
  const int lane = pmmf_lane();
  const int64_t base = rp[r];
  const int len = (int)(rp[r + 1] - base);
  for (int i0 = 0; i0 < len; i0 += PMMF_WAVE) {
    const int i = i0 + lane;
    const int key = i < len ? ci[base + i] : INT_MAX;
    const float val = i < len ? cv[base + i] : 0.f;
    int rank = 0;
    for (int j0 = 0; j0 < len; j0 += PMMF_WAVE) {
      const int kj = j0 + lane < len ? ci[base + j0 + lane] : INT_MAX;
      const int m = min(PMMF_WAVE, len - j0);
      for (int l = 0; l < m; ++l) rank += __shfl(kj, l) < key;
    }
    if (i < len) {
      oci[base + rank] = key;
      ocv[base + rank] = val;
    }
  }
}

hipError_t launch_sort_rows(int n, const int64_t* rp, const int32_t* ci, const float* cv,
                            int32_t* oci, float* ocv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_sort_rows<<<(n + 3) / 4, 256, 0, s>>>(n, rp, ci, cv, oci, ocv);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Levels of each cluster's rotation sequence: rotation s sits one level above the latest
// earlier rotation sharing an index with it.  Rotations of one level touch disjoint indices, so
// they commute and can be applied together.  Writes the stage's sweep log in level order.
__global__ void k_levelize(int k, const int32_t* __restrict__ off, const int32_t* __restrict__ rcnt,
                           const int32_t* __restrict__ roff, int64_t rot0,
                           const int32_t* __restrict__ rot_loc, const float* __restrict__ rot_o,
                           const int32_t* __restrict__ lvl_in, int lvl_stride,
                           int32_t* __restrict__ lvl_ptr,
                           int32_t* __restrict__ depth_out, int32_t* __restrict__ sw_loc,
                           float* __restrict__ sw_o, int32_t* __restrict__ sw_idx,
                           float* __restrict__ theta, int cmax) {
  extern __shared__ int lds_i[];
  int* last = lds_i;            // [cmax]  latest level touching each index
  int* lvl = last + cmax;       // [cmax]  level of each rotation, then its slot in level order
  int* start = lvl + cmax;      // [cmax + 2]
  int* ids = start + cmax + 2;  // [cmax][3] the cluster's rotation ids, staged from HBM
  __shared__ int sh_depth;
  const int u = blockIdx.x;
  const int c = off[u + 1] - off[u];
  const int r = rcnt[u];
  const int rb = roff[u];
  for (int j = threadIdx.x; j < c; j += blockDim.x) last[j] = 0;
  for (int j = threadIdx.x; j < c + 2; j += blockDim.x) start[j] = 0;
  // the cluster's rotation ids (and the recorded levels) staged in LDS, eight loads in flight per
  // thread at a time
  {
    const int32_t* src = rot_loc + (rot0 + rb) * 3;
    const int n3 = r * 3, bd = blockDim.x;
    for (int q0 = 0; q0 < n3; q0 += 8 * bd) {
      int v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = src[min(q0 + t * bd + (int)threadIdx.x, max(n3 - 1, 0))];
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (q0 + t * bd + (int)threadIdx.x < n3) ids[q0 + t * bd + threadIdx.x] = v[t];
    }
    if (lvl_in) {
      const int32_t* li = lvl_in + rot0 + rb;
      for (int q0 = 0; q0 < r; q0 += 8 * bd) {
        int v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = li[min(q0 + t * bd + (int)threadIdx.x, max(r - 1, 0))];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (q0 + t * bd + (int)threadIdx.x < r) lvl[q0 + t * bd + threadIdx.x] = v[t];
      }
    }
  }
  __syncthreads();
  // Wave 0 walks the rotations with wave-uniform control flow: a chunk of 64 rotations' indices is
  // held one per lane and read back by readlane, and the per-level counts and next free slots
  // live in one register indexed by level (lane l holds level l), so only the latest-level table
  // goes through LDS.  Clusters whose depth reaches 64 levels are redone by the serial walk below.
  bool fast = false;
  if (threadIdx.x < PMMF_WAVE) {
    const int lane = pmmf_lane();
    int cnt_v = 0, depth = 0;
    for (int s0 = 0; s0 < r; s0 += PMMF_WAVE) {
      const int sl = min(s0 + lane, r - 1);
      const int c0 = ids[sl * 3], c1 = ids[sl * 3 + 1], c2 = ids[sl * 3 + 2];
      const int n = min(PMMF_WAVE, r - s0);
      int lv = 0;
      if (lvl_in) {  // levels recorded by the search: one ballot per distinct level of the chunk
        lv = lane < n ? lvl[s0 + lane] : 0;
        uint64_t pend = __ballot(lane < n);
        while (pend) {
          const int L = __builtin_amdgcn_readlane(lv, (int)__builtin_ctzll(pend));
          const uint64_t m = __ballot(lane < n && lv == L);
          cnt_v += lane == L ? (int)__popcll(m) : 0;
          pend &= ~m;
        }
        depth = max(depth, pmmf_wave_max_int(lv));
      } else {
        for (int t = 0; t < n; ++t) {
          const int i0 = __builtin_amdgcn_readlane(c0, t), i1 = __builtin_amdgcn_readlane(c1, t),
                    i2 = __builtin_amdgcn_readlane(c2, t);
          int L = max(last[i0], last[i1]);
          if (i2 >= 0) L = max(L, last[i2]);
          L += 1;
          // every lane writes the same value at the same address, so each lane reads back its
          // own writes (no lane depends on another lane's LDS write)
          last[i0] = L;
          last[i1] = L;
          if (i2 >= 0) last[i2] = L;
          cnt_v += lane == L ? 1 : 0;
          lv = lane == t ? L : lv;
          depth = max(depth, L);
        }
      }
      if (lane < n) lvl[s0 + lane] = lv;
    }
    fast = depth < PMMF_WAVE;
    if (fast) {
      // exclusive prefix of the level counts (levels 1..depth in lanes 1..depth)
      const int incl = pmmf_wave_incl_scan_dpp(cnt_v);
      int start_v = incl - cnt_v;
      if (lane >= 1 && lane <= depth) lvl_ptr[(size_t)u * lvl_stride + (lane - 1)] = rb + start_v;
      if (lane == 0) {
        lvl_ptr[(size_t)u * lvl_stride + depth] = rb + r;
        depth_out[u] = depth;
        sh_depth = depth;
      }
      // slot of each rotation in level order (rotation order inside a level)
      // (one ballot per distinct level of a chunk: the chunk's rotations of level L take the next
      // slots of L in chunk order)
      const uint64_t below = (1ull << lane) - 1ull;
      for (int s0 = 0; s0 < r; s0 += PMMF_WAVE) {
        const int n = min(PMMF_WAVE, r - s0);
        const int lvv = lane < n ? lvl[s0 + lane] : 0;
        int slot = 0;
        uint64_t pend = __ballot(lane < n);
        while (pend) {
          const int L = __builtin_amdgcn_readlane(lvv, (int)__builtin_ctzll(pend));
          const uint64_t m = __ballot(lane < n && lvv == L);
          const int base = __builtin_amdgcn_readlane(start_v, L);
          if ((m >> lane) & 1ull) slot = base + (int)__popcll(m & below);
          start_v += lane == L ? (int)__popcll(m) : 0;
          pend &= ~m;
        }
        if (lane < n) lvl[s0 + lane] = slot;
      }
    } else {
      for (int j = lane; j < c; j += PMMF_WAVE) last[j] = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sh_depth = fast ? sh_depth : -1;
  __syncthreads();
  if (sh_depth < 0 && threadIdx.x == 0) {
    int depth = 0;
    for (int s = 0; s < r; ++s) {
      const int i0 = ids[s * 3], i1 = ids[s * 3 + 1], i2 = ids[s * 3 + 2];
      int L = max(last[i0], last[i1]);
      if (i2 >= 0) L = max(L, last[i2]);
      L += 1;
      last[i0] = L;
      last[i1] = L;
      if (i2 >= 0) last[i2] = L;
      lvl[s] = L;
      start[L] += 1;
      depth = max(depth, L);
    }
    int acc = 0;
    for (int l = 1; l <= depth; ++l) {
      const int cnt = start[l];
      start[l] = acc;
      lvl_ptr[(size_t)u * lvl_stride + (l - 1)] = rb + acc;
      acc += cnt;
    }
    lvl_ptr[(size_t)u * lvl_stride + depth] = rb + r;
    depth_out[u] = depth;
    for (int s = 0; s < r; ++s) lvl[s] = start[lvl[s]]++;   // slot of rotation s in level order
    sh_depth = depth;
  }
  __syncthreads();
  // write the sweep log in level order (all lanes)
  const int kk2 = k * k;
  for (int s = threadIdx.x; s < r; s += blockDim.x) {
    const int64_t ridx = rot0 + rb + s;
    const int pos = rb + lvl[s];
    float ob[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) ob[q] = rot_o[ridx * 9 + q];
    for (int a = 0; a < k; ++a) sw_loc[(size_t)pos * k + a] = ids[s * 3 + a];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) sw_o[(size_t)pos * kk2 + a * k + b] = ob[a * 3 + b];
    sw_idx[pos] = (int32_t)ridx;
    if (k == 2) theta[ridx] = (float)atan2((double)ob[3], (double)ob[0]);
  }
}

hipError_t launch_levelize(int m, int k, const int32_t* off, const int32_t* rcnt,
                           const int32_t* roff, int64_t rot0, const int32_t* rot_loc,
                           const float* rot_o, const int32_t* lvl_in, int lvl_stride,
                           int32_t* lvl_ptr, int32_t* depth, int32_t* sw_loc, float* sw_o,
                           int32_t* sw_idx, float* theta, int cmax, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const size_t lds = (size_t)(6 * cmax + 2) * sizeof(int);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_levelize,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_levelize<<<m, 256, lds, s>>>(k, off, rcnt, roff, rot0, rot_loc, rot_o, lvl_in, lvl_stride,
                                lvl_ptr, depth, sw_loc, sw_o, sw_idx, theta, cmax);
  return hipGetLastError();
}


// Transpose of a CSR matrix (n x n): column counts, then each entry placed at its column's next
// free slot.  Entries of one output row land in arbitrary order (k_sort_rows orders them).
__global__ void k_csr_col_count(int64_t nnz, const int32_t* __restrict__ ci,
                                int32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) atomicAdd(cnt + ci[t], 1);
}

__global__ void k_csr_transpose_fill(int n, const int64_t* __restrict__ rp,
                                     const int32_t* __restrict__ ci, const float* __restrict__ cv,
                                     unsigned long long* __restrict__ cursor,
                                     int32_t* __restrict__ tci, float* __restrict__ tcv) {
  const int a = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (a >= n) return;
  for (int64_t t = rp[a] + pmmf_lane(); t < rp[a + 1]; t += PMMF_WAVE) {
    const int64_t pos = (int64_t)atomicAdd(cursor + ci[t], 1ull);
    tci[pos] = a;
    tcv[pos] = cv[t];
  }
}

hipError_t launch_csr_transpose(int n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                                const float* cv, int32_t* cnt, int64_t* trp, int64_t* tmp,
                                int64_t* cursor, int32_t* tci, float* tcv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(cnt, 0, (size_t)n * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  if (nnz > 0) k_csr_col_count<<<(unsigned)((nnz + 255) / 256), 256, 0, s>>>(nnz, ci, cnt);
  e = launch_scan(cnt, trp, n, tmp, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(cursor, trp, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  k_csr_transpose_fill<<<(n + 3) / 4, 256, 0, s>>>(n, rp, ci, cv,
                                                   reinterpret_cast<unsigned long long*>(cursor),
                                                   tci, tcv);
  return hipGetLastError();
}

// Boundary cut counts of the active matrix for the data-driven clustering: boundary b (between
// positions b-1 and b) separates the entries (i, j), i < j, with i < b <= j.  Each such entry adds
// +1 at i + 1 and -1 at j + 1 of a difference array whose prefix sums are the counts (integer
// atomics: the counts are exact, whatever the order).
__global__ void k_cut_marks(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            int32_t* __restrict__ d) {
  const int i = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (i >= S) return;
  int n = 0;
  for (int64_t t = rp[i] + pmmf_lane(); t < rp[i + 1]; t += PMMF_WAVE) {
    const int j = ci[t];
    const bool up = j > i;
    n += __popcll(__ballot(up));
    if (up) atomicAdd(d + j + 1, -1);
  }
  if (pmmf_lane() == 0 && n > 0) atomicAdd(d + i + 1, n);
}

hipError_t launch_cut_counts(int S, const int64_t* rp, const int32_t* ci, int32_t* d, int64_t* w,
                             int64_t* tmp, hipStream_t s) {
  hipError_t e = hipMemsetAsync(d, 0, (size_t)(S + 2) * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  if (S > 0) k_cut_marks<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // exclusive scan over S + 1 slots: w[b + 1] = d[0] + ... + d[b], the count at boundary b
  return launch_scan(d, w, S + 1, tmp, s);
}


// ------------------------------------------------------------------------------------------
// Right rotation W = M Qbar^T (the column half of [[A_p]]_{u,v} = Qbar_u [[A_{p-1}]]_{u,v}
// Qbar_v^T in Alg. 1).  One wave per row x; the row's entries come in runs of one cluster v (the
// run table of M: starts and clusters), and each run is expanded through Qbar_v^T in a dense LDS
// accumulator of c_v slots, 64 entries at a time, list by list in ascending entry order (lanes of
// one chunk that meet at a column from different lists are combined by the LDS atomic add, in the
// hardware's fixed lane order; each position's list comes from the few lists that start in its
// chunk, read lane by lane).  Up to 64 runs' bounds are held one per lane, so the next block's
// entries are requested before the current block is expanded.  fill = 0 counts, fill = 1 writes.
constexpr int RIGHT_CH = 2;  // flat 64-entry chunks whose loads are requested together
__global__ void __launch_bounds__(256) k_right(int S, int fill, const int64_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci,
                                               const float* __restrict__ cv,
                                               const int32_t* __restrict__ off,
                                               const int64_t* __restrict__ run_ptr,
                                               const int32_t* __restrict__ run_cl,
                                               const int64_t* __restrict__ run_start,
                                               const int64_t* __restrict__ qrp,
                                               const int32_t* __restrict__ qci,
                                               const float* __restrict__ qcv,
                                               int32_t* __restrict__ cnt,
                                               const int64_t* __restrict__ orp,
                                               int32_t* __restrict__ oci,
                                               float* __restrict__ ocv,
                                               int64_t* __restrict__ wrs, int cmax) {
  extern __shared__ float lds_f[];
  const int wpb = blockDim.x / PMMF_WAVE;
  const int w = pmmf_wave(), lane = pmmf_lane();
  // cmax accumulator slots
  float* acc = lds_f + (size_t)w * cmax;
  const int x = pmmf_xcd_block(blockIdx.x, gridDim.x) * wpb + w;
  if (x >= S) return;
  for (int j = lane; j < cmax; j += PMMF_WAVE) acc[j] = 0.f;
  const int64_t r0 = rp[x];
  const int64_t end = rp[x + 1];
  const int64_t rr0 = run_ptr[x], rr1 = run_ptr[x + 1];
  int64_t cur = fill ? orp[x] : 0;
  for (int64_t rg = rr0; rg < rr1; rg += PMMF_WAVE) {
    // this group's runs, one per lane: entries [r0 + rb, r0 + re) of cluster offset rov
    const int nr = (int)min<int64_t>(PMMF_WAVE, rr1 - rg);
    int rb = 0, re = 0, rov = 0;
    if (lane < nr) {
      const int64_t g = rg + lane;
      rb = (int)(run_start[g] - r0);
      re = (int)((g + 1 < rr1 ? run_start[g + 1] : end) - r0);
      rov = off[run_cl[g]];
    }
    // the block cursor: run ri, block start kb (relative to r0); blocks are a run's consecutive
    // 64-entry pieces, in run order
    int ri = 0;
    int kb = __builtin_amdgcn_readlane(rb, 0);
    int ke = __builtin_amdgcn_readlane(re, 0);
    // the pending block's entries (lanes past its end repeat its last entry)
    int py = ci[r0 + kb + min(lane, ke - kb - 1)];
    float pm = cv[r0 + kb + min(lane, ke - kb - 1)];
    while (ri < nr) {
      const int ov = __builtin_amdgcn_readlane(rov, ri);
      // W's entries of this run (cluster v) start here
      if (fill && lane == 0) wrs[rg + ri] = cur;
      int bmin = INT_MAX, bmax = -1;
      bool more = true;
      while (more) {
        const int nb = min(PMMF_WAVE, ke - kb);
        const int y = py;
        const float mv = lane < nb ? pm : 0.f;
        const int64_t q0 = qrp[y];
        const int64_t q1 = qrp[y + 1];
        // step the cursor and request the next block's entries (the current one again at the
        // group's end: a valid address whose values are not used)
        more = kb + PMMF_WAVE < ke;
        int nkb, nke;
        if (more) {
          nkb = kb + PMMF_WAVE;
          nke = ke;
        } else if (ri + 1 < nr) {
          nkb = __builtin_amdgcn_readlane(rb, ri + 1);
          nke = __builtin_amdgcn_readlane(re, ri + 1);
        } else {
          nkb = kb;
          nke = ke;
        }
        py = ci[r0 + nkb + min(lane, nke - nkb - 1)];
        pm = cv[r0 + nkb + min(lane, nke - nkb - 1)];
        const int len = lane < nb ? (int)(q1 - q0) : 0;
        // The lists, in entry order, form one flat sequence of T entries (a list of ~10-20
        // entries would leave most of a 64-lane chunk idle); flat position f of list l is entry
        // q0_l + f - P_l.  Lanes of one chunk may hit the same column from different lists,
        // hence the LDS atomic add.
        const int incl = pmmf_wave_incl_scan_dpp(len);
        const int P = incl - len;
        const int T = __builtin_amdgcn_readlane(incl, PMMF_WAVE - 1);
        const int64_t lbase = q0 - P;
        // the list of the positions before this chunk's first list start: its entry base and
        // weight (wave-uniform)
        int64_t cbase = 0;
        float cw = 0.f;
        for (int f0 = 0; f0 < T; f0 += RIGHT_CH * PMMF_WAVE) {
          int cc[RIGHT_CH];
          float vv[RIGHT_CH], qv[RIGHT_CH];
          bool ok[RIGHT_CH];
#pragma unroll
          for (int h = 0; h < RIGHT_CH; ++h) {
            // the list of each flat position: the lists that start in this chunk, in list order
            // (a few per chunk), each take over the positions from their start on
            const int fb = f0 + h * PMMF_WAVE;
            const int f = fb + lane;
            const int rel = P - fb;
            uint64_t starts = __ballot(len > 0 && rel >= 0 && rel < PMMF_WAVE);
            int64_t eb = cbase;
            float wq = cw;
            while (starts) {
              const int l = (int)__builtin_ctzll(starts);
              starts &= starts - 1;
              const int pl = __builtin_amdgcn_readlane(P, l);
              cbase = ((int64_t)__builtin_amdgcn_readlane((int)(lbase >> 32), l) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)lbase, l);
              cw = pmmf_readlane_f(mv, l);
              const bool in = f >= pl;
              eb = in ? cbase : eb;
              wq = in ? cw : wq;
            }
            // a position past T loads the last list's last entry (a valid address) and adds
            // nothing; the loads of all RIGHT_CH chunks are in flight before the first add
            ok[h] = f < T;
            const int64_t e = eb + min(f, T - 1);
            cc[h] = qci[e];
            qv[h] = qcv[e];
            vv[h] = wq;
          }
#pragma unroll
          for (int h = 0; h < RIGHT_CH; ++h) {
            if (ok[h]) {
              const int b = cc[h] - ov;
              __hip_atomic_fetch_add(acc + b, vv[h] * qv[h], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
              bmin = min(bmin, b);
              bmax = max(bmax, b);
            }
          }
        }
        kb = nkb;
        ke = nke;
      }
      bmin = pmmf_wave_min_int(bmin);
      bmax = pmmf_wave_max_int(bmax);
      // the run's accumulated row segment, eight 64-column chunks per round
      for (int bb0 = bmin; bb0 <= bmax; bb0 += 8 * PMMF_WAVE) {
        float vals[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int j = bb0 + t * PMMF_WAVE + lane;
          vals[t] = 0.f;
          if (j <= bmax) {
            vals[t] = acc[j];
            acc[j] = 0.f;
          }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const uint64_t b = __ballot(vals[t] != 0.f);
          if (fill && vals[t] != 0.f) {
            const int64_t pos = cur + pmmf_lanes_below(b);
            oci[pos] = ov + bb0 + t * PMMF_WAVE + lane;
            ocv[pos] = vals[t];
          }
          cur += __popcll(b);
        }
      }
      ++ri;
    }
  }
  if (lane == 0) cnt[x] = (int32_t)(fill ? cur - orp[x] : cur);
}

hipError_t launch_right(int S, int fill, const int64_t* rp, const int32_t* ci, const float* cv,
                        const int32_t* off, const int64_t* run_ptr, const int32_t* run_cl,
                        const int64_t* run_start, const int64_t* qrp, const int32_t* qci,
                        const float* qcv, int32_t* cnt, const int64_t* orp, int32_t* oci,
                        float* ocv, int64_t* wrs, int cmax, hipStream_t s) {
  if (S == 0) return hipSuccess;
  // one wave (one row) per workgroup, as in launch_left: the LDS of a finished row is released
  // at once instead of waiting for the slowest row of its workgroup
  int wpb = 1;
  while (wpb > 1 && (size_t)wpb * cmax * 4 > 64 * 1024) wpb >>= 1;
  const size_t lds = (size_t)wpb * cmax * sizeof(float);
  k_right<<<(S + wpb - 1) / wpb, wpb * PMMF_WAVE, lds, s>>>(S, fill, rp, ci, cv, off, run_ptr,
                                                            run_cl, run_start, qrp, qci, qcv,
                                                            cnt, orp, oci, ocv, wrs, cmax);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Left rotation and peel: rows of A_p = Qbar W for every position a of the stage.  Row a merges
// the rows W_x, x in supp(Qbar_a) (all inside a's cluster), cluster run by cluster run through a
// dense LDS accumulator (lists in ascending x, deterministic).  A surviving row keeps only its
// surviving columns, renumbered to the next stage's positions; a retired row contributes
//     2 sum_{b survives} A_p[a,b]^2 + sum_{b retired, b != a} A_p[a,b]^2
// to the exact residual (FP64), which totals 2 sum_e m_e over the stage's retirements.
// Rows of up to LEFT_QSMALL lists run in k_left_seg; this kernel takes the few longer rows, up to
// LEFT_QMAX lists, with the lists' positions in an LDS list area.
constexpr int LEFT_QMAX = 512;
constexpr int LEFT_QSMALL = 2 * PMMF_WAVE;
constexpr int LEFT_PER_LIST = 28;  // LDS bytes per list: cur, end (int64), next column, its cluster, weight

template <int QCAP>
__global__ void __launch_bounds__(256) k_left(int S, int fill, const int64_t* __restrict__ qrp,
                                              const int32_t* __restrict__ qci,
                                              const float* __restrict__ qcv,
                                              const int64_t* __restrict__ wrp,
                                              const int32_t* __restrict__ wcnt,
                                              const int32_t* __restrict__ wci,
                                              const float* __restrict__ wcv,
                                              const int32_t* __restrict__ off,
                                              const int32_t* __restrict__ cl_of,
                                              const int32_t* __restrict__ next,
                                              int32_t* __restrict__ cnt,
                                              const int64_t* __restrict__ orp,
                                              int32_t* __restrict__ oci,
                                              float* __restrict__ ocv,
                                              double* __restrict__ loss_row,
                                              int32_t* __restrict__ overflow, int cmax) {
  extern __shared__ float lds_f[];
  const int wpb = blockDim.x / PMMF_WAVE;
  const int w = pmmf_wave(), lane = pmmf_lane();
  char* base = reinterpret_cast<char*>(lds_f) +
               (size_t)w * ((size_t)cmax * 4 + (size_t)QCAP * LEFT_PER_LIST);
  float* acc = reinterpret_cast<float*>(base);
  int64_t* cur = reinterpret_cast<int64_t*>(base + (size_t)cmax * 4);
  int64_t* en = cur + QCAP;
  int* ncol = reinterpret_cast<int*>(en + QCAP);   // column at cur, INT_MAX when done
  int* ncl = ncol + QCAP;                          // its cluster
  float* qv = reinterpret_cast<float*>(ncl + QCAP);
  // a cluster's positions read the same rows of W: keep them on one XCD
  const int a = pmmf_xcd_block(blockIdx.x, gridDim.x) * wpb + w;
  if (a >= S) return;
  const int64_t q0 = qrp[a];
  const int nq = (int)(qrp[a + 1] - q0);
  // each row belongs to exactly one of the two launches
  if (QCAP == LEFT_QSMALL ? nq > LEFT_QSMALL : nq <= LEFT_QSMALL) return;
  if (nq > LEFT_QMAX) {
    if (lane == 0) {
      atomicOr(overflow, 1);
      if (next[a] >= 0) cnt[next[a]] = 0;
      if (fill) loss_row[a] = 0.0;
    }
    return;
  }
  for (int j = lane; j < cmax; j += PMMF_WAVE) acc[j] = 0.f;
  for (int li = lane; li < nq; li += PMMF_WAVE) {
    const int x = qci[q0 + li];
    const int64_t c0 = wrp[x], c1 = wcnt ? c0 + wcnt[x] : wrp[x + 1];
    cur[li] = c0;
    en[li] = c1;
    qv[li] = qcv[q0 + li];
    const int col = c0 < c1 ? wci[c0] : INT_MAX;
    ncol[li] = col;
    ncl[li] = col < INT_MAX ? cl_of[col] : INT_MAX;
  }
  const int na = next[a];
  const bool surv = na >= 0;
  int64_t ocur = (fill && surv) ? orp[na] : 0;
  double loss = 0.0;
  while (true) {
    int vmin = INT_MAX;
    for (int li = lane; li < nq; li += PMMF_WAVE) vmin = min(vmin, ncl[li]);
    vmin = pmmf_wave_min_int(vmin);
    if (vmin == INT_MAX) break;
    const int ov = off[vmin];
    const int lim = off[vmin + 1];
    int bmin = INT_MAX, bmax = -1;
    // lists with entries in this cluster, in ascending list order (deterministic sums); the
    // first 64-entry chunk of up to eight of them is requested together
    for (int g0 = 0; g0 < nq; g0 += PMMF_WAVE) {
      uint64_t sel = __ballot(g0 + lane < nq && ncl[g0 + lane] == vmin);
      while (sel) {
        int ids[8];
        int64_t cu[8], ee[8];
        float qq[8], valv[8];
        int colv[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          ids[b] = -1;
          if (sel) {
            ids[b] = g0 + (__ffsll((unsigned long long)sel) - 1);
            sel &= sel - 1;
          }
          cu[b] = ids[b] >= 0 ? cur[ids[b]] : 0;
          ee[b] = ids[b] >= 0 ? en[ids[b]] : 0;
          qq[b] = ids[b] >= 0 ? qv[ids[b]] : 0.f;
          const int64_t idx = cu[b] + lane;
          colv[b] = idx < ee[b] ? wci[idx] : INT_MAX;
          valv[b] = idx < ee[b] ? wcv[idx] : 0.f;
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          if (ids[b] < 0) break;
          int64_t c_ = cu[b];
          const int64_t e_ = ee[b];
          int col = colv[b];
          float val = valv[b];
          while (true) {
            const bool in = col < lim;
            const int n = __popcll(__ballot(in));
            if (in) {
              const int bb = col - ov;
              acc[bb] += qq[b] * val;
              bmin = min(bmin, bb);
              bmax = max(bmax, bb);
            }
            c_ += n;
            if (n < PMMF_WAVE) {
              // the first lane past the run holds the list's next column
              const int nc = __shfl(col, n);
              if (lane == 0) ncol[ids[b]] = nc;
              break;
            }
            if (c_ >= e_) {
              if (lane == 0) ncol[ids[b]] = INT_MAX;
              break;
            }
            const int64_t idx = c_ + lane;
            col = idx < e_ ? wci[idx] : INT_MAX;
            val = idx < e_ ? wcv[idx] : 0.f;
          }
          if (lane == 0) {
            cur[ids[b]] = c_;
            ncl[ids[b]] = -1;  // refreshed below, for all advanced lists at once
          }
        }
      }
    }
    for (int li = lane; li < nq; li += PMMF_WAVE)
      if (ncl[li] == -1) ncl[li] = ncol[li] < INT_MAX ? cl_of[ncol[li]] : INT_MAX;
    bmin = pmmf_wave_min_int(bmin);
    bmax = pmmf_wave_max_int(bmax);
    // the cluster's accumulated run, eight 64-column chunks per round (their next positions are
    // requested together, only where the value is nonzero)
    for (int bb0 = bmin; bb0 <= bmax; bb0 += 8 * PMMF_WAVE) {
      float vv[8];
      int nxv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int j = bb0 + t * PMMF_WAVE + lane;
        vv[t] = 0.f;
        nxv[t] = -1;
        if (j <= bmax) {
          vv[t] = acc[j];
          acc[j] = 0.f;
          if (vv[t] != 0.f) nxv[t] = next[ov + j];
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (bb0 + t * PMMF_WAVE > bmax) break;
        const int colpos = ov + bb0 + t * PMMF_WAVE + lane;
        const float val = vv[t];
        if (surv) {
          const bool keep = val != 0.f && nxv[t] >= 0;
          const uint64_t b = __ballot(keep);
          if (fill && keep) {
            const int64_t pos = ocur + pmmf_lanes_below(b);
            oci[pos] = nxv[t];
            ocv[pos] = val;
          }
          ocur += __popcll(b);
        } else if (fill && val != 0.f && colpos != a) {
          const double v2 = (double)val * (double)val;
          loss += nxv[t] >= 0 ? 2.0 * v2 : v2;
        }
      }
    }
  }
  if (fill && !surv) {
    loss = pmmf_wave_sum_double(loss);
    if (lane == 0) loss_row[a] = loss;
  } else if (fill && lane == 0) {
    loss_row[a] = 0.0;
  }
  if (lane == 0 && surv) cnt[na] = (int32_t)(fill ? ocur - orp[na] : ocur);
}

// Left rotation for rows with at most 128 lists (nearly all rows): two lists per lane (lists l and
// l + 64), each list's position kept in registers as an index into its row's run table (W's rows
// have the runs of M's rows, one per cluster, in ascending cluster order, with their starts in W
// recorded by k_right).  Each
// round takes the smallest cluster v among the lists' current runs and walks the runs of v of the
// lists that have one, in list order, with a wave-uniform cursor in items of up to GRAM_ITEM
// consecutive 64-entry chunks of one run (the loads of the next item requested before the
// current one is added); a run's entries hit distinct columns, so every column sums in list
// order, as in k_left.  The cluster's accumulated run is then emitted as in k_left.
__global__ void __launch_bounds__(256) k_left_seg(int S, int fill, const int64_t* __restrict__ qrp,
                                                  const int32_t* __restrict__ qci,
                                                  const float* __restrict__ qcv,
                                                  const int64_t* __restrict__ wrp,
                                                  const int32_t* __restrict__ wcnt,
                                                  const int32_t* __restrict__ wci,
                                                  const float* __restrict__ wcv,
                                                  const int64_t* __restrict__ run_ptr,
                                                  const int32_t* __restrict__ run_cl,
                                                  const int64_t* __restrict__ wrs,
                                                  const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ next,
                                                  int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ orp,
                                                  int32_t* __restrict__ oci,
                                                  float* __restrict__ ocv,
                                                  double* __restrict__ loss_row, int cmax) {
  extern __shared__ float lds_f[];
  const int wpb = blockDim.x / PMMF_WAVE;
  const int w = pmmf_wave(), lane = pmmf_lane();
  // cmax accumulator slots, then one spare slot per lane for the zero contributions of lanes past
  // a run's end
  float* acc = lds_f + (size_t)w * (cmax + PMMF_WAVE);
  const int spare = cmax + lane;
  // a cluster's positions read the same rows of W: keep them on one XCD
  const int a = pmmf_xcd_block(blockIdx.x, gridDim.x) * wpb + w;
  if (a >= S) return;
  const int64_t q0 = qrp[a];
  const int nq = (int)(qrp[a + 1] - q0);
  constexpr int NS = 2;            // list slots per lane
  if (nq > NS * PMMF_WAVE) return;  // longer rows: k_left
  for (int j = lane; j < cmax; j += PMMF_WAVE) acc[j] = 0.f;
  // this lane's lists h = 0, 1 (list lane + 64 h): row x of W, weight Qbar[a, x], current run ri
  // of [ri, r1), its cluster and entries [rs, re)
  int64_t ri[2] = {0, 0}, r1[2] = {0, 0}, rs[2] = {0, 0}, re[2] = {0, 0}, wend[2] = {0, 0};
  int cl[2] = {INT_MAX, INT_MAX};
  float qv[2] = {0.f, 0.f};
#pragma unroll
  for (int h = 0; h < NS; ++h) {
    const int li = lane + h * PMMF_WAVE;
    if (li < nq) {
      const int x = qci[q0 + li];
      qv[h] = qcv[q0 + li];
      ri[h] = run_ptr[x];
      r1[h] = run_ptr[x + 1];
      wend[h] = wcnt ? wrp[x] + wcnt[x] : wrp[x + 1];
      if (ri[h] < r1[h]) {
        cl[h] = run_cl[ri[h]];
        rs[h] = wrs[ri[h]];
        re[h] = ri[h] + 1 < r1[h] ? wrs[ri[h] + 1] : wend[h];
      }
    }
  }
  const int na = next[a];
  const bool surv = na >= 0;
  int64_t ocur = (fill && surv) ? orp[na] : 0;
  double loss = 0.0;
  while (true) {
    const int vmin = pmmf_wave_min_int(NS == 2 ? min(cl[0], cl[1]) : cl[0]);
    if (vmin == INT_MAX) break;
    const int ov = off[vmin];
    const bool part0 = cl[0] == vmin, part1 = NS == 2 && cl[1] == vmin;
    const int len0 = part0 ? (int)(re[0] - rs[0]) : 0;
    const int len1 = part1 ? (int)(re[1] - rs[1]) : 0;
    int bmin = INT_MAX, bmax = -1;
    {
      // participating runs in list order: lists 0..63 (h = 0), then 64..127 (h = 1)
      uint64_t left0 = __ballot(len0 > 0), left1 = NS == 2 ? __ballot(len1 > 0) : 0;
      bool live = false;
      int qn = 0, qoff = 0;
      int64_t qb = 0;
      float qw = 0.f;
      auto next_run = [&]() {
        const bool h1 = left0 == 0;
        const uint64_t m = h1 ? left1 : left0;
        live = m != 0;
        const int l = live ? (int)__builtin_ctzll(m) : 0;
        if (h1) left1 &= left1 - 1;
        else left0 &= left0 - 1;
        const int n0 = __builtin_amdgcn_readlane(len0, l), n1 = __builtin_amdgcn_readlane(len1, l);
        const int64_t b0 = ((int64_t)__builtin_amdgcn_readlane((int)(rs[0] >> 32), l) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)rs[0], l);
        const int64_t b1 = ((int64_t)__builtin_amdgcn_readlane((int)(rs[1] >> 32), l) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)rs[1], l);
        const float w0 = pmmf_readlane_f(qv[0], l), w1 = pmmf_readlane_f(qv[1], l);
        qn = h1 ? n1 : n0;
        qb = h1 ? b1 : b0;
        qw = h1 ? w1 : w0;
        qoff = 0;
      };
      next_run();
      // an exhausted cursor yields empty items at the last run's start (a valid address)
      auto take = [&](GramItem& g) {
        g.base = qb;
        g.off = live ? qoff : 0;
        g.rem = live ? qn - qoff : 0;
        g.w = qw;
        qoff += GRAM_ITEM * PMMF_WAVE;
        if (live && qoff >= qn) next_run();
      };
      auto load = [&](const GramItem& g, int* col, float* val) {
        const char* cp = reinterpret_cast<const char*>(wci + g.base);
        const char* vp = reinterpret_cast<const char*>(wcv + g.base);
        const int last = max(g.rem - 1, 0);
#pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          const uint32_t eb = 4u * (uint32_t)(g.off + min(lane + t * PMMF_WAVE, last));
          col[t] = *reinterpret_cast<const int32_t*>(cp + eb);
          val[t] = *reinterpret_cast<const float*>(vp + eb);
        }
      };
      auto add = [&](const GramItem& g, const int* col, const float* val) {
#pragma unroll
        for (int t = 0; t < GRAM_ITEM; ++t) {
          const bool ok = lane + t * PMMF_WAVE < g.rem;
          const int b = col[t] - ov;
          acc[ok ? b : spare] += ok ? g.w * val[t] : 0.f;
          bmin = ok ? min(bmin, b) : bmin;
          bmax = ok ? max(bmax, b) : bmax;
        }
      };
      GramItem g0, g1;
      int c0[GRAM_ITEM], c1[GRAM_ITEM];
      float v0[GRAM_ITEM], v1[GRAM_ITEM];
      // a fixed, even number of items: no exit test sits between a load and its add
      constexpr int IE = GRAM_ITEM * PMMF_WAVE;
      const int nit = __builtin_amdgcn_readlane(
          pmmf_wave_incl_scan_dpp((len0 + IE - 1) / IE + (len1 + IE - 1) / IE), PMMF_WAVE - 1);
      const int pairs = (nit + 1) / 2;
      take(g0);
      load(g0, c0, v0);
      for (int it = 0; it < pairs; ++it) {
        take(g1);
        load(g1, c1, v1);
        add(g0, c0, v0);
        take(g0);
        load(g0, c0, v0);
        add(g1, c1, v1);
      }
    }
    // the participating lists move to their next run
#pragma unroll
    for (int h = 0; h < NS; ++h) {
      if (cl[h] == vmin) {
        ++ri[h];
        cl[h] = ri[h] < r1[h] ? run_cl[ri[h]] : INT_MAX;
        rs[h] = re[h];
        re[h] = ri[h] + 1 < r1[h] ? wrs[ri[h] + 1] : wend[h];
      }
    }
    bmin = pmmf_wave_min_int(bmin);
    bmax = pmmf_wave_max_int(bmax);
    // the cluster's accumulated run, eight 64-column chunks per round (their next positions are
    // requested together, only where the value is nonzero)
    for (int bb0 = bmin; bb0 <= bmax; bb0 += 8 * PMMF_WAVE) {
      float vv[8];
      int nxv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int j = bb0 + t * PMMF_WAVE + lane;
        vv[t] = 0.f;
        nxv[t] = -1;
        if (j <= bmax) {
          vv[t] = acc[j];
          acc[j] = 0.f;
          if (vv[t] != 0.f) nxv[t] = next[ov + j];
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (bb0 + t * PMMF_WAVE > bmax) break;
        const int colpos = ov + bb0 + t * PMMF_WAVE + lane;
        const float val = vv[t];
        if (surv) {
          const bool keep = val != 0.f && nxv[t] >= 0;
          const uint64_t b = __ballot(keep);
          if (fill && keep) {
            const int64_t pos = ocur + pmmf_lanes_below(b);
            oci[pos] = nxv[t];
            ocv[pos] = val;
          }
          ocur += __popcll(b);
        } else if (fill && val != 0.f && colpos != a) {
          const double v2 = (double)val * (double)val;
          loss += nxv[t] >= 0 ? 2.0 * v2 : v2;
        }
      }
    }
  }
  if (fill && !surv) {
    loss = pmmf_wave_sum_double(loss);
    if (lane == 0) loss_row[a] = loss;
  } else if (fill && lane == 0) {
    loss_row[a] = 0.0;
  }
  if (lane == 0 && surv) cnt[na] = (int32_t)(fill ? ocur - orp[na] : ocur);
}

// Row capacities for writing a product straight into staging storage (no counting pass): a row
// of W = M Qbar^T has at most sum_y nnz(Qbar^T_y) entries over its entries y, and a row of
// A_p = Qbar W at most sum_x nnz(W_x) over the entries x of its Qbar row; both at most `cap`.
__global__ void k_bound_right(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const int64_t* __restrict__ qrp, int64_t cap,
                              int32_t* __restrict__ ub) {
  const int x = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (x >= S) return;
  int64_t acc = 0;
  for (int64_t t = rp[x] + pmmf_lane(); t < rp[x + 1]; t += PMMF_WAVE) {
    const int y = ci[t];
    acc += qrp[y + 1] - qrp[y];
  }
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (pmmf_lane() == 0) ub[x] = (int32_t)min<int64_t>(acc, cap);
}

__global__ void k_bound_left(int S, const int64_t* __restrict__ qrp, const int32_t* __restrict__ qci,
                             const int32_t* __restrict__ wcnt, const int32_t* __restrict__ next,
                             int64_t cap, int32_t* __restrict__ ub) {
  const int a = blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (a >= S) return;
  const int na = next[a];
  if (na < 0) return;
  int64_t acc = 0;
  for (int64_t t = qrp[a] + pmmf_lane(); t < qrp[a + 1]; t += PMMF_WAVE) acc += wcnt[qci[t]];
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (pmmf_lane() == 0) ub[na] = (int32_t)min<int64_t>(acc, cap);
}

// staging rows (start sb[r], cnt[r] entries) -> compact CSR rows at rp[r]
__global__ void k_compact_rows(int64_t n, const int64_t* __restrict__ sb,
                               const int32_t* __restrict__ cnt, const int32_t* __restrict__ sci,
                               const float* __restrict__ scv, const int64_t* __restrict__ rp,
                               int32_t* __restrict__ ci, float* __restrict__ cv) {
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (r >= n) return;
  const int64_t src = sb[r], dst = rp[r];
  for (int t = pmmf_lane(); t < cnt[r]; t += PMMF_WAVE) {
    ci[dst + t] = sci[src + t];
    cv[dst + t] = scv[src + t];
  }
}

hipError_t launch_bound_right(int S, const int64_t* rp, const int32_t* ci, const int64_t* qrp,
                              int64_t cap, int32_t* ub, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_bound_right<<<(S + 3) / 4, 256, 0, s>>>(S, rp, ci, qrp, cap, ub);
  return hipGetLastError();
}

hipError_t launch_bound_left(int S, const int64_t* qrp, const int32_t* qci, const int32_t* wcnt,
                             const int32_t* next, int64_t cap, int32_t* ub, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_bound_left<<<(S + 3) / 4, 256, 0, s>>>(S, qrp, qci, wcnt, next, cap, ub);
  return hipGetLastError();
}

hipError_t launch_compact_rows(int64_t n, const int64_t* sb, const int32_t* cnt,
                               const int32_t* sci, const float* scv, const int64_t* rp,
                               int32_t* ci, float* cv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_compact_rows<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, sb, cnt, sci, scv, rp, ci, cv);
  return hipGetLastError();
}

hipError_t launch_left(int S, int fill, const int64_t* qrp, const int32_t* qci, const float* qcv,
                       const int64_t* wrp, const int32_t* wcnt, const int32_t* wci,
                       const float* wcv, const int64_t* run_ptr, const int32_t* run_cl,
                       const int64_t* wrs,
                       const int32_t* off, const int32_t* cl_of, const int32_t* next,
                       int32_t* cnt, const int64_t* orp, int32_t* oci, float* ocv,
                       double* loss_row, int32_t* overflow, int cmax, hipStream_t s) {
  if (S == 0) return hipSuccess;
  // One wave (one row) per workgroup: a workgroup's LDS is released only when its last wave
  // ends, and rows differ widely in work, so several rows per workgroup hold LDS idle (four per
  // workgroup: rotate phase 26.7 ms, one: 22.6 ms on the 262k factor).
  auto go = [&](auto kern, int qcap) -> hipError_t {
    const size_t per_wave = (size_t)cmax * 4 + (size_t)qcap * LEFT_PER_LIST;
    int wpb = 1;
    while (wpb > 1 && wpb * per_wave > 64 * 1024) wpb >>= 1;
    const size_t lds = wpb * per_wave;
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    kern<<<(S + wpb - 1) / wpb, wpb * PMMF_WAVE, lds, s>>>(S, fill, qrp, qci, qcv, wrp, wcnt, wci,
                                                           wcv, off, cl_of, next, cnt, orp, oci,
                                                           ocv, loss_row, overflow, cmax);
    return hipGetLastError();
  };
  {
    const size_t per_wave = ((size_t)cmax + PMMF_WAVE) * 4;
    int wpb = 1;
    while (wpb > 1 && wpb * per_wave > 64 * 1024) wpb >>= 1;
    const unsigned grid = (unsigned)((S + wpb - 1) / wpb);
    k_left_seg<<<grid, wpb * PMMF_WAVE, wpb * per_wave, s>>>(
        S, fill, qrp, qci, qcv, wrp, wcnt, wci, wcv, run_ptr, run_cl, wrs, off, next, cnt, orp,
        oci, ocv, loss_row, cmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return go(k_left<LEFT_QMAX>, LEFT_QMAX);
}

// ------------------------------------------------------------------------------------------
// positions of the survivors in the next stage, and the global ids there
__global__ void k_keep_flags(int S, const uint8_t* __restrict__ retflag, int32_t* __restrict__ keep) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < S) keep[q] = retflag[q] ? 0 : 1;
}
hipError_t launch_keep_flags(int S, const uint8_t* retflag, int32_t* keep, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_keep_flags<<<(S + 255) / 256, 256, 0, s>>>(S, retflag, keep);
  return hipGetLastError();
}

__global__ void k_next_positions(int S, const uint8_t* __restrict__ retflag,
                                 const int64_t* __restrict__ scan, const int32_t* __restrict__ gid,
                                 int32_t* __restrict__ next, int32_t* __restrict__ gid_new) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S) return;
  if (retflag[q]) {
    next[q] = -gid[q] - 1;
  } else {
    const int np = (int)scan[q];
    next[q] = np;
    gid_new[np] = gid[q];
  }
}
hipError_t launch_next_positions(int S, const uint8_t* retflag, const int64_t* scan,
                                 const int32_t* gid, int32_t* next, int32_t* gid_new,
                                 hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_next_positions<<<(S + 255) / 256, 256, 0, s>>>(S, retflag, scan, gid, next, gid_new);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// exclusive scan of int32 counts into int64 offsets out[0..n] (out[n] = total)
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_B = SCAN_T * SCAN_I;

__global__ void k_scan_block(const int32_t* __restrict__ in32, const int64_t* __restrict__ in64,
                             int64_t n, int64_t* __restrict__ out, int64_t* __restrict__ bsum) {
  __shared__ int64_t wsum[SCAN_T / PMMF_WAVE];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_B;
  int64_t v[SCAN_I];
  int64_t tot = 0;
  for (int q = 0; q < SCAN_I; ++q) {
    const int64_t idx = b0 + (int64_t)threadIdx.x * SCAN_I + q;
    int64_t x = 0;
    if (idx < n) x = in32 ? (int64_t)in32[idx] : in64[idx];
    v[q] = tot;
    tot += x;
  }
  // exclusive scan of thread totals across the block
  int64_t incl = tot;
  const int lane = pmmf_lane();
  for (int o = 1; o < PMMF_WAVE; o <<= 1) {
    int64_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == PMMF_WAVE - 1) wsum[pmmf_wave()] = incl;
  __syncthreads();
  int64_t wpre = 0;
  for (int q = 0; q < pmmf_wave(); ++q) wpre += wsum[q];
  const int64_t texcl = wpre + incl - tot;
  for (int q = 0; q < SCAN_I; ++q) {
    const int64_t idx = b0 + (int64_t)threadIdx.x * SCAN_I + q;
    if (idx < n) out[idx] = texcl + v[q];
  }
  if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = texcl + tot;
}

__global__ void k_scan_add(int64_t n, int64_t* __restrict__ out, const int64_t* __restrict__ boff) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] += boff[idx / SCAN_B];
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t tot = 0;
  int64_t m = n;
  while (true) {
    const int64_t nb = (m + SCAN_B - 1) / SCAN_B;
    tot += 2 * (nb + 1);
    if (nb <= 1) break;
    m = nb;
  }
  return tot + 8;
}

static hipError_t scan_rec(const int32_t* in32, const int64_t* in64, int64_t n, int64_t* out,
                           int64_t* tmp, hipStream_t s) {
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  int64_t* bsum = tmp;
  int64_t* boff = tmp + nb + 1;
  k_scan_block<<<(unsigned)nb, SCAN_T, 0, s>>>(in32, in64, n, out, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb > 1) {
    e = scan_rec(nullptr, bsum, nb, boff, tmp + 2 * (nb + 1), s);
    if (e != hipSuccess) return e;
    k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, out, boff);
    e = hipGetLastError();
  }
  return e;
}

// total is written to out[n]
__global__ void k_scan_total(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  out[n] = (n > 0 ? out[n - 1] + in[n - 1] : 0);
}

hipError_t launch_scan(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  if (n > 0) {
    hipError_t e = scan_rec(in, nullptr, n, out, tmp, s);
    if (e != hipSuccess) return e;
  }
  k_scan_total<<<1, 1, 0, s>>>(in, n, out);
  return hipGetLastError();
}

// deterministic FP64 sum (one block, fixed order)
// one workgroup, a fixed summation order (four interleaved partial sums per thread, so four
// loads are in flight per thread, then the waves' sums in wave order)
__global__ void k_sum_double(const double* __restrict__ in, int64_t n, double* __restrict__ out) {
  __shared__ double part[1024 / PMMF_WAVE];
  const int64_t bd = blockDim.x;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 3 * bd < n; i += 4 * bd) {
    v0 += in[i];
    v1 += in[i + bd];
    v2 += in[i + 2 * bd];
    v3 += in[i + 3 * bd];
  }
  for (; i < n; i += bd) v0 += in[i];
  double v = (v0 + v1) + (v2 + v3);
  v = pmmf_wave_sum_double(v);
  if (pmmf_lane() == 0) part[pmmf_wave()] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x / PMMF_WAVE); ++q) t += part[q];
    *out = t;
  }
}
hipError_t launch_sum_double(const double* in, int64_t n, double* out, hipStream_t s) {
  k_sum_double<<<1, 1024, 0, s>>>(in, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// input checks and statistics: per row FP64 partial sums of squares (fro2_trace[2*row]) and the
// diagonal (fro2_trace[2*row+1]); flags bit 0 = non-finite, bit 1 = not symmetric
__global__ void k_csr_stats(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const float* __restrict__ cv, int check_sym,
                            double* __restrict__ part, int32_t* __restrict__ flags) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double f2 = 0.0, tr = 0.0;
  int fl = 0;
  for (int64_t t = rp[a]; t < rp[a + 1]; ++t) {
    const float v = cv[t];
    const int b = ci[t];
    if (!isfinite(v)) fl |= 1;
    if (b < 0 || b >= n) fl |= 4;
    if (t > rp[a] && b <= ci[t - 1]) fl |= 8;
    f2 += (double)v * v;
    if (b == a) tr += v;
    if (check_sym && b >= 0 && b < n) {
      const int64_t q = lower_bound_i32(ci, rp[b], rp[b + 1], (int32_t)a);
      if (q >= rp[b + 1] || ci[q] != a || __float_as_uint(cv[q]) != __float_as_uint(v)) fl |= 2;
    }
  }
  part[a] = f2;
  part[n + a] = tr;
  if (fl) atomicOr(flags, fl);
}
hipError_t launch_csr_stats(int64_t n, const int64_t* rp, const int32_t* ci, const float* cv,
                            int check_sym, double* part, int32_t* flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_csr_stats<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, rp, ci, cv, check_sym, part, flags);
  return hipGetLastError();
}

__global__ void k_core_dense(int S, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const float* __restrict__ cv, float* __restrict__ hcore) {
  const int a = blockIdx.x;
  for (int64_t t = rp[a] + threadIdx.x; t < rp[a + 1]; t += blockDim.x)
    hcore[(size_t)a * S + ci[t]] = cv[t];
}
hipError_t launch_core_dense(int S, const int64_t* rp, const int32_t* ci, const float* cv,
                             float* hcore, hipStream_t s) {
  if (S == 0) return hipSuccess;
  k_core_dense<<<S, 64, 0, s>>>(S, rp, ci, cv, hcore);
  return hipGetLastError();
}

// out[0] = ||H||_F^2, out[1] = trace(H), FP64 accumulation in a fixed order
__global__ void k_h_stats(int64_t n, const float* __restrict__ hdiag, int64_t core,
                          const float* __restrict__ hcore, double* __restrict__ out) {
  __shared__ double p1[1024 / PMMF_WAVE], p2[1024 / PMMF_WAVE];
  const int64_t bd = blockDim.x;
  // sums of squares over hdiag and hcore, two interleaved partial sums per thread; trace of
  // hdiag plus the core's diagonal
  double f0 = 0.0, f1 = 0.0, t = 0.0;
  int64_t i = threadIdx.x;
  for (; i + bd < n; i += 2 * bd) {
    const double a = hdiag[i], b = hdiag[i + bd];
    f0 += a * a;
    f1 += b * b;
    t += a + b;
  }
  for (; i < n; i += bd) {
    const double a = hdiag[i];
    f0 += a * a;
    t += a;
  }
  // the core (up to a few million entries): eight loads in flight per thread
  const int64_t cc = core * core;
  double g[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (i = threadIdx.x; i + 7 * bd < cc; i += 8 * bd) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double a = hcore[i + q * bd];
      g[q] += a * a;
    }
  }
  for (; i < cc; i += bd) {
    const double a = hcore[i];
    f0 += a * a;
  }
  f0 += ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]));
  for (i = threadIdx.x; i < core; i += bd) t += hcore[i * core + i];
  double f = f0 + f1;
  f = pmmf_wave_sum_double(f);
  t = pmmf_wave_sum_double(t);
  if (pmmf_lane() == 0) { p1[pmmf_wave()] = f; p2[pmmf_wave()] = t; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < (int)(blockDim.x / PMMF_WAVE); ++q) { a += p1[q]; b += p2[q]; }
    out[0] = a;
    out[1] = b;
  }
}
hipError_t launch_h_stats(int64_t n, const float* hdiag, int64_t core, const float* hcore,
                          double* out, hipStream_t s) {
  k_h_stats<<<1, 1024, 0, s>>>(n, hdiag, core, hcore, out);
  return hipGetLastError();
}

__global__ void k_copy_csr(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const float* __restrict__ cv, int64_t* __restrict__ orp,
                           int32_t* __restrict__ oci, float* __restrict__ ocv) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a > n) return;
  orp[a] = rp[a];
  if (a == n) return;
  for (int64_t t = rp[a]; t < rp[a + 1]; ++t) {
    oci[t] = ci[t];
    ocv[t] = cv[t];
  }
}
hipError_t launch_copy_csr(int64_t n, const int64_t* rp, const int32_t* ci, const float* cv,
                           int64_t* orp, int32_t* oci, float* ocv, hipStream_t s) {
  k_copy_csr<<<(unsigned)((n + 256) / 256), 256, 0, s>>>(n, rp, ci, cv, orp, oci, ocv);
  return hipGetLastError();
}

__global__ void k_iota(int32_t* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}
hipError_t launch_iota(int32_t* a, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, n);
  return hipGetLastError();
}

}  // namespace pmmf
