// Preconditioned conjugate gradients with the pMMF inverse as preconditioner (Sec. 4), for a block
// of right-hand sides solved in lockstep.  Inner iterations run in FP32 with the matrix-free
// inverse (mmf_apply_inverse); an outer loop recomputes the residual b - A x in FP64 and corrects
// the FP64 solution (iterative refinement), until ||b_j - A x_j|| / ||b_j|| <= tol for every column.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "dev_alloc.h"
#include "pmmf.h"

namespace pmmf {

// Y[n][ld] = A X for CSR A (float32); one wave per row, lanes over the columns
__global__ void k_spmm_f32(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const float* __restrict__ cv, const float* __restrict__ X,
                           float* __restrict__ Y, int64_t nrhs, int64_t ld) {
  // one wave per row, lane = right-hand side; eight nonzeros per round so their rows of X are
  // requested together (summed in ascending nonzero order)
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (row >= n) return;
  const int lane = pmmf_lane();
  const int64_t b0 = rp[row], b1 = rp[row + 1];
  for (int64_t c0 = 0; c0 < nrhs; c0 += PMMF_WAVE) {
    const int64_t col = c0 + lane;
    const int64_t colc = col < nrhs ? col : nrhs - 1;
    float acc = 0.f;
    for (int64_t t0 = b0; t0 < b1; t0 += 8) {
      float w[8], xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t t = t0 + q < b1 ? t0 + q : b1 - 1;
        w[q] = t0 + q < b1 ? cv[t] : 0.f;
        xv[q] = X[(int64_t)ci[t] * ld + colc];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += w[q] * xv[q];
    }
    if (col < nrhs) Y[row * ld + col] = acc;
  }
}

// R = B - A X in FP64 (A and B float32, X float64)
__global__ void k_residual_f64(int64_t n, const int64_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, const float* __restrict__ cv,
                               const double* __restrict__ X, const float* __restrict__ B,
                               double* __restrict__ R, int64_t nrhs, int64_t ld) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / PMMF_WAVE) + pmmf_wave();
  if (row >= n) return;
  const int lane = pmmf_lane();
  const int64_t b0 = rp[row], b1 = rp[row + 1];
  for (int64_t c0 = 0; c0 < nrhs; c0 += PMMF_WAVE) {
    const int64_t col = c0 + lane;
    if (col >= nrhs) continue;
    double acc = 0.0;
    for (int64_t t = b0; t < b1; ++t) acc += (double)cv[t] * X[(int64_t)ci[t] * ld + col];
    R[row * ld + col] = (double)B[row * ld + col] - acc;
  }
}

// partial column dot products sum_rows U[r][j] V[r][j] over a row chunk per block (FP64),
// written to part[block][j]; fixed summation order
template <class TU, class TV>
__global__ void k_coldot_part(int64_t n, const TU* __restrict__ U, const TV* __restrict__ V,
                              int64_t nrhs, int64_t ld, int64_t rows_per_block,
                              double* __restrict__ part) {
  __shared__ double red[4][64];
  const int cl = threadIdx.x % 64, rg = threadIdx.x / 64;
  const int64_t col = (int64_t)blockIdx.y * 64 + cl;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  double acc = 0.0;
  if (col < nrhs)
    for (int64_t r = r0 + rg; r < r1; r += 4) acc += (double)U[r * ld + col] * (double)V[r * ld + col];
  red[rg][cl] = acc;
  __syncthreads();
  if (rg == 0 && col < nrhs)
    part[(int64_t)blockIdx.x * nrhs + col] = red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl];
}

__global__ void k_coldot_final(int64_t nblocks, int64_t nrhs, const double* __restrict__ part,
                               double* __restrict__ out) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= nrhs) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) s += part[b * nrhs + col];
  out[col] = s;
}

// per-column scalars of one CG step: alpha = rz / pAp (0 when pAp is 0 or the column is done)
__global__ void k_cg_alpha(int64_t nrhs, const double* __restrict__ rz,
                           const double* __restrict__ pap, const int32_t* __restrict__ active,
                           float* __restrict__ alpha) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  alpha[j] = (active[j] && pap[j] != 0.0) ? (float)(rz[j] / pap[j]) : 0.f;
}
__global__ void k_cg_beta(int64_t nrhs, const double* __restrict__ rz_new,
                          const double* __restrict__ rz_old, float* __restrict__ beta) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  beta[j] = rz_old[j] != 0.0 ? (float)(rz_new[j] / rz_old[j]) : 0.f;
}

// D += alpha P ; R -= alpha AP
__global__ void k_cg_update(int64_t n, int64_t nrhs, int64_t ld, const float* __restrict__ alpha,
                            const float* __restrict__ P, const float* __restrict__ AP,
                            float* __restrict__ Dx, float* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t r = i / nrhs, j = i % nrhs;
  const float a = alpha[j];
  Dx[r * ld + j] += a * P[r * ld + j];
  R[r * ld + j] -= a * AP[r * ld + j];
}
// P = Z + beta P
__global__ void k_cg_direction(int64_t n, int64_t nrhs, int64_t ld, const float* __restrict__ beta,
                               const float* __restrict__ Z, float* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t r = i / nrhs, j = i % nrhs;
  P[r * ld + j] = Z[r * ld + j] + beta[j] * P[r * ld + j];
}
// R32 = R64 / scale_j (scale = ||r_j||, 1 when zero); X64 += scale_j D32
__global__ void k_to_f32_scaled(int64_t n, int64_t nrhs, int64_t ld, const double* __restrict__ R,
                                const double* __restrict__ nrm2, float* __restrict__ R32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t r = i / nrhs, j = i % nrhs;
  const double s = nrm2[j] > 0.0 ? sqrt(nrm2[j]) : 1.0;
  R32[r * ld + j] = (float)(R[r * ld + j] / s);
}
__global__ void k_accumulate_scaled(int64_t n, int64_t nrhs, int64_t ld,
                                    const double* __restrict__ nrm2, const float* __restrict__ D,
                                    double* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t r = i / nrhs, j = i % nrhs;
  const double s = nrm2[j] > 0.0 ? sqrt(nrm2[j]) : 1.0;
  X[r * ld + j] += s * (double)D[r * ld + j];
}

}  // namespace pmmf

namespace {

struct Buf {
  void* p = nullptr;
  pmmf_alloc::How how;
  explicit Buf(size_t bytes) { p = pmmf_alloc::alloc(std::max<size_t>(bytes, 16), &how); }
  ~Buf() { pmmf_alloc::release(p, how); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct PcgErr {
  int code;
  std::string msg;
};

void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw PcgErr{MMF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

}  // namespace

namespace pmmf_host_detail {
void set_error(const std::string& msg);
}

// split = false: CG on M^{-1} A (left preconditioning, z = M^{-1} r);
// split = true:  CG on the symmetric M^{-1/2} A M^{-1/2} y = M^{-1/2} r with d = M^{-1/2} y.
static int pcg_impl(mmf_handle h, int64_t n, const int64_t* d_rowptr, const int32_t* d_colind,
                    const float* d_val, const float* d_b, double* d_x, int64_t nrhs, double tol,
                    int32_t max_iter, double inner_reduction, void* stream, mmf_pcg_info* out,
                    bool split) {
  using namespace pmmf;
  try {
    if (!h || !d_rowptr || !d_colind || !d_val || !d_b || !d_x || nrhs < 1 || n < 1 ||
        !(tol > 0.0) || max_iter < 1 || !(inner_reduction > 0.0 && inner_reduction < 1.0))
      throw PcgErr{MMF_EINVAL, "bad PCG arguments"};
    mmf_info inf;
    int rc = mmf_get_info(h, &inf);
    if (rc != MMF_OK) return rc;
    if (inf.n != n) throw PcgErr{MMF_EINVAL, "the factorization has another dimension"};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    pmmf_alloc::StreamScope alloc_scope(stream);
    const int64_t ld = nrhs, N = n * nrhs;
    hipEvent_t e0, e1;
    chk(hipEventCreate(&e0), "event");
    chk(hipEventCreate(&e1), "event");
    chk(hipEventRecord(e0, s), "event");
    Buf R64(N * 8), R(N * 4), Z(N * 4), P(N * 4), AP(N * 4), Dx(N * 4);
    const int64_t rpb = 4096;
    const int64_t nblk = (n + rpb - 1) / rpb;
    Buf part(nblk * nrhs * 8), bb(nrhs * 8), rr(nrhs * 8), rz(nrhs * 8), rz2(nrhs * 8),
        pap(nrhs * 8), alpha(nrhs * 4), beta(nrhs * 4), active(nrhs * 4), scale(nrhs * 8);
    for (Buf* b : {&R64, &R, &Z, &P, &AP, &Dx, &part, &bb, &rr, &rz, &rz2, &pap, &alpha, &beta,
                   &active, &scale})
      if (!b->p) throw PcgErr{MMF_ENOMEM, "PCG workspace allocation failed"};
    const dim3 dgrid((unsigned)nblk, (unsigned)((nrhs + 63) / 64));
    const unsigned ewb = (unsigned)((N + 255) / 256);
    const unsigned rowb = (unsigned)((n + 3) / 4);
    auto coldot32 = [&](const float* U, const float* V, double* dst) {
      k_coldot_part<float, float><<<dgrid, 256, 0, s>>>(n, U, V, nrhs, ld, rpb, part.as<double>());
      k_coldot_final<<<(unsigned)((nrhs + 255) / 256), 256, 0, s>>>(nblk, nrhs, part.as<double>(), dst);
    };
    auto coldot64 = [&](const double* U, const double* V, double* dst) {
      k_coldot_part<double, double><<<dgrid, 256, 0, s>>>(n, U, V, nrhs, ld, rpb, part.as<double>());
      k_coldot_final<<<(unsigned)((nrhs + 255) / 256), 256, 0, s>>>(nblk, nrhs, part.as<double>(), dst);
    };
    // ||b||^2 and the initial residual
    {
      Buf b64(N * 8);
      if (!b64.p) throw PcgErr{MMF_ENOMEM, "PCG workspace allocation failed"};
      chk(hipMemsetAsync(d_x, 0, N * 8, s), "memset");
      k_residual_f64<<<rowb, 256, 0, s>>>(n, d_rowptr, d_colind, d_val, d_x, d_b, b64.as<double>(),
                                         nrhs, ld);
      coldot64(b64.as<double>(), b64.as<double>(), bb.as<double>());
      chk(hipGetLastError(), "kernels");
      chk(hipStreamSynchronize(s), "sync");
    }
    // the preconditioner products are captured once as graphs and replayed after that: R -> Z
    // (M^{-1}); split form: P -> T1 and T2 -> AP (M^{-1/2})
    struct GraphGuard {
      mmf_graph g = nullptr;
      ~GraphGuard() { if (g) (void)mmf_graph_destroy(g); }
    } pre, half1, half2;
    auto precondition = [&]() -> int {
      if (!pre.g) return mmf_graph_capture(h, 1, R.as<float>(), Z.as<float>(), nrhs, ld, stream, &pre.g);
      return mmf_graph_launch(pre.g, stream);
    };
    Buf T1(split ? N * 4 : 16), T2(split ? N * 4 : 16);
    if (!T1.p || !T2.p) throw PcgErr{MMF_ENOMEM, "PCG workspace allocation failed"};
    auto half = [&](GraphGuard& gg, const float* src, float* dst) -> int {
      if (!gg.g) return mmf_graph_capture(h, 2, src, dst, nrhs, ld, stream, &gg.g);
      return mmf_graph_launch(gg.g, stream);
    };
    // split form: AP = M^{-1/2} A M^{-1/2} P
    auto split_product = [&]() -> int {
      int r2 = half(half1, P.as<float>(), T1.as<float>());
      if (r2 != MMF_OK) return r2;
      k_spmm_f32<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, d_rowptr, d_colind, d_val,
                                                         T1.as<float>(), T2.as<float>(), nrhs, ld);
      return half(half2, T2.as<float>(), AP.as<float>());
    };
    std::vector<double> bn(nrhs), rn(nrhs), rzh(nrhs);
    chk(hipMemcpy(bn.data(), bb.p, nrhs * 8, hipMemcpyDeviceToHost), "copy");
    int total_it = 0, outer = 0;
    double worst = 0.0;
    std::vector<int32_t> act(nrhs, 1);
    while (true) {
      k_residual_f64<<<rowb, 256, 0, s>>>(n, d_rowptr, d_colind, d_val, d_x, d_b, R64.as<double>(),
                                         nrhs, ld);
      coldot64(R64.as<double>(), R64.as<double>(), rr.as<double>());
      chk(hipGetLastError(), "kernels");
      chk(hipMemcpyAsync(rn.data(), rr.p, nrhs * 8, hipMemcpyDeviceToHost, s), "copy");
      chk(hipStreamSynchronize(s), "sync");
      worst = 0.0;
      int done = 0;
      for (int64_t j = 0; j < nrhs; ++j) {
        const double rel = bn[j] > 0.0 ? std::sqrt(rn[j] / bn[j]) : std::sqrt(rn[j]);
        worst = std::max(worst, rel);
        act[j] = rel > tol ? 1 : 0;
        done += act[j] ? 0 : 1;
      }
      if (done == nrhs || total_it >= max_iter) break;
      ++outer;
      // inner FP32 PCG on A d = r / ||r|| (per column), from d = 0
      chk(hipMemcpyAsync(active.p, act.data(), nrhs * 4, hipMemcpyHostToDevice, s), "copy");
      chk(hipMemcpyAsync(scale.p, rr.p, nrhs * 8, hipMemcpyDeviceToDevice, s), "copy");
      k_to_f32_scaled<<<ewb, 256, 0, s>>>(n, nrhs, ld, R64.as<double>(), scale.as<double>(),
                                          R.as<float>());
      chk(hipMemsetAsync(Dx.p, 0, N * 4, s), "memset");
      std::vector<double> r0n(nrhs, 1.0);  // split form: ||M^{-1/2} r|| at the start
      if (split) {
        // R <- M^{-1/2} R: the residual of the symmetric system in y (Dx holds y)
        rc = mmf_apply_inverse_sqrt(h, R.as<float>(), Z.as<float>(), nrhs, ld, stream);
        if (rc != MMF_OK) return rc;
        chk(hipMemcpyAsync(R.p, Z.p, N * 4, hipMemcpyDeviceToDevice, s), "copy");
        coldot32(R.as<float>(), R.as<float>(), rr.as<double>());
        chk(hipMemcpyAsync(r0n.data(), rr.p, nrhs * 8, hipMemcpyDeviceToHost, s), "copy");
        chk(hipStreamSynchronize(s), "sync");
        for (auto& v : r0n) v = std::sqrt(v);
      } else {
        rc = precondition();
        if (rc != MMF_OK) return rc;
      }
      chk(hipMemcpyAsync(P.p, Z.p, N * 4, hipMemcpyDeviceToDevice, s), "copy");
      coldot32(R.as<float>(), Z.as<float>(), rz.as<double>());
      while (total_it < max_iter) {
        if (split) {
          rc = split_product();
          if (rc != MMF_OK) return rc;
        } else {
          k_spmm_f32<<<rowb, 256, 0, s>>>(n, d_rowptr, d_colind, d_val, P.as<float>(),
                                          AP.as<float>(), nrhs, ld);
        }
        coldot32(P.as<float>(), AP.as<float>(), pap.as<double>());
        k_cg_alpha<<<(unsigned)((nrhs + 255) / 256), 256, 0, s>>>(
            nrhs, rz.as<double>(), pap.as<double>(), active.as<int32_t>(), alpha.as<float>());
        k_cg_update<<<ewb, 256, 0, s>>>(n, nrhs, ld, alpha.as<float>(), P.as<float>(),
                                        AP.as<float>(), Dx.as<float>(), R.as<float>());
        ++total_it;
        // convergence of the inner solve: every active column reduced by inner_reduction
        coldot32(R.as<float>(), R.as<float>(), rr.as<double>());
        chk(hipGetLastError(), "kernels");
        chk(hipMemcpyAsync(rn.data(), rr.p, nrhs * 8, hipMemcpyDeviceToHost, s), "copy");
        chk(hipStreamSynchronize(s), "sync");
        bool inner_done = true;
        for (int64_t j = 0; j < nrhs; ++j)
          if (act[j] && !(std::sqrt(rn[j]) <= inner_reduction * r0n[j])) inner_done = false;
        if (inner_done) break;
        if (split) {
          // unpreconditioned CG on the symmetric operator: the direction follows the residual
          chk(hipMemcpyAsync(Z.p, R.p, N * 4, hipMemcpyDeviceToDevice, s), "copy");
        } else {
          rc = precondition();
          if (rc != MMF_OK) return rc;
        }
        coldot32(R.as<float>(), Z.as<float>(), rz2.as<double>());
        k_cg_beta<<<(unsigned)((nrhs + 255) / 256), 256, 0, s>>>(nrhs, rz2.as<double>(),
                                                                 rz.as<double>(), beta.as<float>());
        k_cg_direction<<<ewb, 256, 0, s>>>(n, nrhs, ld, beta.as<float>(), Z.as<float>(),
                                           P.as<float>());
        chk(hipMemcpyAsync(rz.p, rz2.p, nrhs * 8, hipMemcpyDeviceToDevice, s), "copy");
      }
      if (split) {
        // d = M^{-1/2} y
        rc = mmf_apply_inverse_sqrt(h, Dx.as<float>(), T1.as<float>(), nrhs, ld, stream);
        if (rc != MMF_OK) return rc;
        chk(hipMemcpyAsync(Dx.p, T1.p, N * 4, hipMemcpyDeviceToDevice, s), "copy");
      }
      k_accumulate_scaled<<<ewb, 256, 0, s>>>(n, nrhs, ld, scale.as<double>(), Dx.as<float>(),
                                              d_x);
      chk(hipGetLastError(), "kernels");
    }
    chk(hipEventRecord(e1, s), "event");
    chk(hipEventSynchronize(e1), "sync");
    float ms = 0.f;
    chk(hipEventElapsedTime(&ms, e0, e1), "event");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (out) {
      out->iterations = total_it;
      out->refinements = outer;
      int conv = 0;
      for (int64_t j = 0; j < nrhs; ++j) conv += act[j] ? 0 : 1;
      out->converged = conv;
      out->pad = 0;
      out->max_rel_residual = worst;
      out->solve_ms = ms;
    }
    return MMF_OK;
  } catch (const PcgErr& e) {
    pmmf_host_detail::set_error(e.msg);
    return e.code;
  }
}

extern "C" int mmf_pcg(mmf_handle h, int64_t n, const int64_t* d_rowptr, const int32_t* d_colind,
                       const float* d_val, const float* d_b, double* d_x, int64_t nrhs,
                       double tol, int32_t max_iter, double inner_reduction, void* stream,
                       mmf_pcg_info* out) {
  return pcg_impl(h, n, d_rowptr, d_colind, d_val, d_b, d_x, nrhs, tol, max_iter,
                  inner_reduction, stream, out, false);
}

extern "C" int mmf_pcg_split(mmf_handle h, int64_t n, const int64_t* d_rowptr,
                             const int32_t* d_colind, const float* d_val, const float* d_b,
                             double* d_x, int64_t nrhs, double tol, int32_t max_iter,
                             double inner_reduction, void* stream, mmf_pcg_info* out) {
  return pcg_impl(h, n, d_rowptr, d_colind, d_val, d_b, d_x, nrhs, tol, max_iter,
                  inner_reduction, stream, out, true);
}

extern "C" int mmf_spmm(int64_t n, const int64_t* d_rowptr, const int32_t* d_colind,
                        const float* d_val, const float* d_x, float* d_y, int64_t nrhs,
                        int64_t ld, void* stream) {
  if (n < 0 || nrhs < 0 || ld < nrhs || (n > 0 && (!d_rowptr || !d_colind || !d_val)) ||
      (n > 0 && nrhs > 0 && (!d_x || !d_y)) || (d_x && d_x == d_y)) {
    pmmf_host_detail::set_error("mmf_spmm: bad arguments");
    return MMF_EINVAL;
  }
  if (n == 0 || nrhs == 0) return MMF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned blocks = (unsigned)((n + 3) / 4);
  pmmf::k_spmm_f32<<<blocks, 256, 0, s>>>(n, d_rowptr, d_colind, d_val, d_x, d_y, nrhs, ld);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    pmmf_host_detail::set_error(std::string("mmf_spmm: ") + hipGetErrorString(e));
    return MMF_EDEVICE;
  }
  return MMF_OK;
}
