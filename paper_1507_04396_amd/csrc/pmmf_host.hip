// Host side of the pMMF library: the C ABI declared in include/pmmf.h.
#include "pmmf.h"

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "dev_alloc.h"
#include "factor_kernels.h"
#include "sweep_kernels.h"

namespace pmmf_alloc {
namespace {
std::mutex g_mu;
void* (*g_alloc)(size_t, void*, void*) = nullptr;
void (*g_release)(void*, void*, void*) = nullptr;
void* g_ctx = nullptr;
thread_local void* g_stream = nullptr;

// Blocks of the default allocator.  A released block is kept for reuse: at once by later
// allocations on the stream it was released on (stream order keeps them behind the work that
// used it), by other streams only after the device has been synchronized since its release.
struct Block {
  void* p;
  size_t bytes;
  int dev;
  void* stream;    // stream of the releasing call
  bool idle;       // the device has been synchronized since the release
  uint64_t epoch;  // release count when it was released
};
struct Live {
  size_t bytes;
  int dev;
};
std::vector<Block> g_kept;               // released blocks, oldest first
std::map<void*, Live> g_out;            // blocks handed out by the default allocator
size_t g_kept_bytes = 0;
uint64_t g_releases = 0;  // releases so far (a synchronization covers those made before it)
constexpr size_t kKeepMax = 64ull << 30;  // at most this much is kept for reuse

// best-fitting kept block for `bytes` on `dev` (sizes up to twice the request), or -1
int fit(size_t bytes, int dev, void* stream, bool usable_only) {
  int best = -1;
  for (int i = 0; i < (int)g_kept.size(); ++i) {
    const Block& b = g_kept[i];
    if (b.dev != dev || b.bytes < bytes || b.bytes > 2 * bytes) continue;
    if (usable_only && !b.idle && b.stream != stream) continue;
    if (best < 0 || b.bytes < g_kept[best].bytes) best = i;
  }
  return best;
}

// frees every kept block (after waiting for the device); g_mu must not be held
void drop_kept() {
  std::vector<Block> all;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    all.swap(g_kept);
    g_kept_bytes = 0;
  }
  for (const Block& b : all) (void)hipFree(b.p);
}

void* default_alloc(size_t bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  void* const stream = g_stream;
  for (int pass = 0; pass < 2; ++pass) {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      int i = fit(bytes, dev, stream, true);
      if (i >= 0) {
        const Block b = g_kept[i];
        g_kept.erase(g_kept.begin() + i);
        g_kept_bytes -= b.bytes;
        g_out[b.p] = Live{b.bytes, dev};
        return b.p;
      }
      if (pass == 1 || fit(bytes, dev, stream, false) < 0) break;
    }
    // a kept block would fit once the work that used it has finished: a device
    // synchronization covers the blocks released before it starts, not those released by
    // other threads meanwhile
    uint64_t before;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      before = g_releases;
    }
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(g_mu);
    for (Block& b : g_kept)
      if (b.epoch <= before) b.idle = true;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    drop_kept();
    p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_out[p] = Live{bytes, dev};
  return p;
}

void default_release(void* p) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_out.find(p);
    if (it == g_out.end()) return;
    g_kept.push_back(Block{p, it->second.bytes, it->second.dev, g_stream, false, ++g_releases});
    g_kept_bytes += it->second.bytes;
    g_out.erase(it);
    while (g_kept_bytes > kKeepMax && !g_kept.empty()) {
      drop.push_back(g_kept.front().p);
      g_kept_bytes -= g_kept.front().bytes;
      g_kept.erase(g_kept.begin());
    }
  }
  for (void* q : drop) (void)hipFree(q);  // hipFree waits for the device
}
}  // namespace

void* alloc(size_t bytes, How* how) {
  void* (*a)(size_t, void*, void*);
  void (*r)(void*, void*, void*);
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    a = g_alloc;
    r = g_release;
    ctx = g_ctx;
  }
  if (a) {
    how->release = r;
    how->ctx = ctx;
    how->stream = g_stream;
    return a(bytes, g_stream, ctx);
  }
  *how = How{};
  return default_alloc(bytes);
}

void release(void* p, const How& how) {
  if (!p) return;
  if (how.release) {
    (void)hipDeviceSynchronize();
    how.release(p, how.stream, how.ctx);
  } else {
    default_release(p);
  }
}

void trim() { drop_kept(); }

StreamScope::StreamScope(void* stream) : prev(g_stream) { g_stream = stream; }
StreamScope::~StreamScope() { g_stream = prev; }

void set(void* (*a)(size_t, void*, void*), void (*r)(void*, void*, void*), void* ctx) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_alloc = a;
  g_release = r;
  g_ctx = ctx;
}
}  // namespace pmmf_alloc

namespace {

thread_local std::string g_err;

struct Err {
  int code;
  std::string msg;
};

[[noreturn]] void raise(int code, const std::string& msg) { throw Err{code, msg}; }

void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) raise(MMF_ENOMEM, std::string(what) + ": out of device memory");
    raise(MMF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HIPCHK(x) hipchk((x), #x)

// Owned device buffer.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  pmmf_alloc::How how;  // the allocator that produced p
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) pmmf_alloc::release(p, how);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) b = 16;
    p = pmmf_alloc::alloc(b, &how);
    if (!p) raise(MMF_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    bytes = b;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
  void swap_with(DBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(how, o.how);
  }
};

// Host -> device copy on the stream; waits for it, since the host vector may be a temporary.
template <class T>
void upload(DBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.ensure(h.size() * sizeof(T));
  if (h.empty()) return;
  HIPCHK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

// Host -> device copies that do not wait: the data is copied into a pinned staging area of the
// calling thread, which is reused once the stream its copies were queued on has been waited for
// (staging_synced, called after each such wait) or by waiting for it when the area is full.
struct Staging {
  char* buf = nullptr;
  size_t cap = 0, used = 0;
  hipStream_t stream = nullptr;  // stream of the copies not known to be complete (used > 0)
  ~Staging() {
    if (buf) (void)hipHostFree(buf);
  }
};
thread_local Staging g_staging;

void staging_synced(hipStream_t s) {
  if (g_staging.stream == s) g_staging.used = 0;
}

template <class T>
void upload_async(DBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.ensure(h.size() * sizeof(T));
  if (h.empty()) return;
  Staging& g = g_staging;
  const size_t b = h.size() * sizeof(T);
  if (g.used > 0 && (g.stream != s || g.used + b > g.cap)) {
    HIPCHK(hipStreamSynchronize(g.stream));
    g.used = 0;
  }
  if (b > g.cap) {
    if (g.buf) HIPCHK(hipHostFree(g.buf));
    g.buf = nullptr;
    g.cap = 0;
    const size_t cap = std::max<size_t>(b, 64 * 1024);
    HIPCHK(hipHostMalloc((void**)&g.buf, cap, hipHostMallocDefault));
    g.cap = cap;
  }
  std::memcpy(g.buf + g.used, h.data(), b);
  HIPCHK(hipMemcpyAsync(d.p, g.buf + g.used, b, hipMemcpyHostToDevice, s));
  g.used = (g.used + b + 255) & ~(size_t)255;
  g.stream = s;
}

// Device -> host reads of a few values between the stages of a factorization: copied into a
// pinned area of the calling thread (a copy into pageable memory goes through the runtime's own
// staging buffer).  Each use waits for its copies before it takes the area again, so one area
// per thread serves every call; it grows to the largest request.
struct Readback {
  char* buf = nullptr;
  size_t cap = 0;
  ~Readback() {
    if (buf) (void)hipHostFree(buf);
  }
};
thread_local Readback g_readback;

char* readback_area(size_t bytes = 64) {
  Readback& r = g_readback;
  if (bytes > r.cap) {
    if (r.buf) HIPCHK(hipHostFree(r.buf));
    r.buf = nullptr;
    r.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 4096);
    HIPCHK(hipHostMalloc((void**)&r.buf, cap, hipHostMallocDefault));
    r.cap = cap;
  }
  return r.buf;
}

int64_t read_i64(const int64_t* dptr, hipStream_t s) {
  int64_t* v = reinterpret_cast<int64_t*>(readback_area());
  HIPCHK(hipMemcpyAsync(v, dptr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  staging_synced(s);
  return *v;
}

// active matrices with at most this many rows and at least this fill get the dense Gram
constexpr int64_t DENSE_GRAM_MAX_ROWS = 16384;
constexpr double DENSE_GRAM_MIN_FILL = 0.1;
constexpr int CMAX_LIMIT = 3072;   // largest cluster (dense c x c Gram, diagonal block, Q;
                                    // the search keeps four of its rows in LDS)

}  // namespace

struct StageDev {
  int64_t size = 0, t = 0, rot_base = 0, nnz = 0;
  int m = 0, cmax = 0, rmax = 0, lvl_stride = 0, depth_max = 0;
  std::vector<int32_t> off_h, rcnt_h, roff_h;
  std::vector<int64_t> gbase_h;
  DBuf off, rcnt, roff, order, gbase, next, gid, cl_of, lvl_ptr, depth, sw_loc, sw_o, sw_idx;
  double loss = 0.0;
  double gram_ms = 0.0, find_ms = 0.0, rotate_ms = 0.0;
  bool dense_gram = false;
  int64_t bf16_long = 0, bf16_rescored = 0;  // BF16 form: long shortlists, candidates rescored
  double gram_flops = 0.0, gram_useful_flops = 0.0;  // performed / algorithmic Gram flops
  // sweep plan (built on first use): units of whole rotation components, and the clusters
  // holding a component larger than a unit, which the level kernel handles
  int nu = 0, nbig = 0, big_cmax = 0, big_rmax = 0;
  DBuf u_cnt, u_slot, u_rot, big_list;
};

// HIP events bracketing the phases of one stage
struct PhaseEvents {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  PhaseEvents() {
    for (auto& x : e) HIPCHK(hipEventCreate(&x));
  }
  ~PhaseEvents() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  double ms(int a, int b) const {
    float v = 0.f;
    HIPCHK(hipEventElapsedTime(&v, e[a], e[b]));
    return v;
  }
};

// launch configuration of the sweeps (chosen by the autotuner)
struct SweepCfg {
  int wpb = 2;  // units (waves) per workgroup of the unit sweep
  int W = 0;    // column tile of the level sweep
  // largest first active set of the fused trailing stages of the products (capped by the
  // handle's mmf_set_tail_rows); untuned: 4096, the best of 0 / 2048 / 4096 / 8192 measured on
  // the 256 x 256 grid factorization with 256 vectors
  int tail = 4096;
};

struct mmf_plan {
  int64_t n = 0, core = 0, R = 0;
  int elims = 1;  // indices retired per rotation (MMF_TWO_ELIMINATIONS: 2)
  int k = 2;
  mmf_params prm{};
  std::vector<std::unique_ptr<StageDev>> st;
  DBuf rot_loc, rot_gid, rot_o, rot_ret, rot_margin, theta, rot_lit;
  DBuf rot_lvl;  // level of each rotation, recorded by the search (one retirement per rotation)
  DBuf rot_o0;  // k = 3: the rotations as found (angles w = 0), O_t = expm(W(w_t)) O0_t
  DBuf hdiag, hcore, core_ids, is_core;
  DBuf hinv, chol_L, chol_X, status;
  DBuf hisqrt, eig_A, eig_D, eig_E, eig_info;  // H_core^{-1/2} and its eigendecomposition
  bool inv_ready = false;
  bool isqrt_ready = false;
  bool units_ready = false;
  // trailing stages as one launch per direction (tables built with the units, for the stages
  // from tail_first on that qualify; tail_plan picks the first trailing stage per call)
  int tail_first = -1;
  int64_t tail_rows = (int64_t)pmmf::TAIL_THREADS * pmmf::TAIL_J;  // mmf_set_tail_rows
  int lds_cap = 0;
  std::vector<pmmf::TailStage> tail_st;
  DBuf tail_blob, tail_trans, tail_pos, tail_gid, tail_pidx, tail_odst;
  int64_t tail_entries = 0;
  uint64_t version = 0;  // bumped whenever theta, H or the rotations change
  std::map<std::pair<std::string, int64_t>, SweepCfg> tune;  // (product, width) -> config
  DBuf ws[18];
  mmf_info info{};
  hipStream_t stream = nullptr;
};

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------------------------------------
// schedule (Alg. 1 stages, Alg. 2 rotation counts, seeded cluster sizes)
struct SchedStage {
  int64_t size, t;
  std::vector<int32_t> sizes, rcnt;
};

// rotations per cluster: floor share plus leftovers by largest remainder (lower u on ties)
void allocate_stage_rotations(SchedStage& st, const mmf_params& p) {
  const int64_t s = st.size, t = st.t;
  const size_t m = st.sizes.size();
  std::vector<int64_t> base(m), rem(m);
  int64_t sum = 0;
  for (size_t u = 0; u < m; ++u) {
    base[u] = (t * st.sizes[u]) / s;
    rem[u] = (t * st.sizes[u]) % s;
    sum += base[u];
  }
  std::vector<size_t> ord(m);
  for (size_t u = 0; u < m; ++u) ord[u] = u;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return rem[a] > rem[b]; });
  for (int64_t q = 0; q < t - sum; ++q) base[ord[q]] += 1;
  st.rcnt.clear();
  for (size_t u = 0; u < m; ++u) {
    if (st.sizes[u] > CMAX_LIMIT)
      raise(MMF_EINVAL, "cluster of " + std::to_string(st.sizes[u]) + " exceeds the limit " +
                            std::to_string(CMAX_LIMIT) + " (set cluster bounds)");
    if (base[u] > st.sizes[u] - (p.k - 1))
      raise(MMF_EINVAL, "a cluster has fewer than k live indices at its last step");
    st.rcnt.push_back((int32_t)base[u]);
  }
}

// Data-driven cluster sizes (MMF_CUT_CLUSTERS): contiguous clusters with sizes in [lo, hi] whose
// boundaries separate the fewest entries of the active matrix; w[b] is the count at boundary b
// (b = 0..S).  f(b) = least total count of a partition of [0, b) into clusters (counting b itself
// when b < S) = w(b) + min f(b') over b' in [b - hi, b - lo]; the window minimum comes from a
// monotone deque, which keeps the smallest b' among equal minima, so the sizes read backwards are
// the lexicographically largest optimal ones.  O(S).
std::vector<int32_t> cut_cluster_sizes(const std::vector<int64_t>& w, int64_t S, int64_t lo,
                                       int64_t hi) {
  if (S <= hi) return {(int32_t)S};
  const int64_t INF = INT64_MAX;
  std::vector<int64_t> f(S + 1, INF), back(S + 1, -1);
  f[0] = 0;
  std::vector<int64_t> dq(S + 1);
  size_t head = 0, tail = 0;  // candidates b' in ascending order, f non-decreasing
  for (int64_t b = lo; b <= S; ++b) {
    const int64_t add = b - lo;  // enters the window
    if (f[add] != INF) {
      while (tail > head && f[dq[tail - 1]] > f[add]) --tail;
      dq[tail++] = add;
    }
    while (tail > head && dq[head] < b - hi) ++head;  // leaves the window
    if (tail > head) {
      f[b] = f[dq[head]] + (b < S ? w[b] : 0);
      back[b] = dq[head];
    }
  }
  if (f[S] == INF) raise(MMF_EINVAL, "the active set cannot be split into clusters of [lo, hi]");
  std::vector<int32_t> sizes;
  for (int64_t b = S; b > 0; b = back[b]) sizes.push_back((int32_t)(b - back[b]));
  std::reverse(sizes.begin(), sizes.end());
  return sizes;
}

std::vector<SchedStage> make_schedule(const mmf_params& p, int64_t n) {
  std::vector<SchedStage> out;
  int64_t s = n;
  int stage = 0;
  const bool cut = (p.flags & MMF_CUT_CLUSTERS) != 0;
  if (cut && (p.flags & MMF_EVEN_CLUSTERS))
    raise(MMF_EINVAL, "MMF_CUT_CLUSTERS and MMF_EVEN_CLUSTERS exclude each other");
  if (cut && p.cluster_max > CMAX_LIMIT)
    raise(MMF_EINVAL, "cluster_max exceeds the limit " + std::to_string(CMAX_LIMIT));
  while (s > p.core_size) {
    ++stage;
    const int64_t t = std::min<int64_t>(s - p.core_size, (int64_t)std::floor(p.eta * (double)s));
    if (t < 1) raise(MMF_EINVAL, "eta * |S| < 1: the schedule cannot reach the core");
    SchedStage st;
    st.size = s;
    st.t = t;
    if (p.cluster_min == 0 && p.cluster_max == 0) {
      st.sizes.push_back((int32_t)s);
    } else if (cut && s > p.cluster_max) {
      // sizes chosen at the start of the stage from the active matrix
    } else if (cut) {
      st.sizes.push_back((int32_t)s);
    } else {
      int64_t r = s;
      uint64_t q = 0;
      const int64_t lo = p.cluster_min, hi = p.cluster_max;
      while (r > hi) {
        int64_t c = lo + (int64_t)pmmf_mulhi(pmmf_hash4(p.seed, PMMF_TAG_CLUSTER_SIZE,
                                                        (uint64_t)stage, q, 0),
                                             (uint64_t)(hi - lo + 1));
        c = std::min(c, r - lo);
        if (p.flags & MMF_EVEN_CLUSTERS) c -= c % 2;
        st.sizes.push_back((int32_t)c);
        r -= c;
        ++q;
      }
      st.sizes.push_back((int32_t)r);
    }
    if (!st.sizes.empty()) allocate_stage_rotations(st, p);
    out.push_back(std::move(st));
    s -= t;
  }
  return out;
}

void validate(int64_t n, const mmf_params* p) {
  if (!p) raise(MMF_EINVAL, "params is NULL");
  if (n < 1 || n > (int64_t)INT32_MAX - 1) raise(MMF_EINVAL, "n out of range");
  if (p->k != 2 && p->k != 3) raise(MMF_EINVAL, "k must be 2 or 3");
  if (!(p->eta > 0.0 && p->eta <= 0.5)) raise(MMF_EINVAL, "eta must be in (0, 0.5]");
  if (p->core_size < 1 || p->core_size > n) raise(MMF_EINVAL, "core_size must be in [1, n]");
  const bool single = p->cluster_min == 0 && p->cluster_max == 0;
  if (!single && (p->cluster_min < 2 || p->cluster_max < 2 * p->cluster_min))
    raise(MMF_EINVAL, "cluster bounds need cluster_min >= 2 and cluster_max >= 2 cluster_min");
  if (p->gram_mode != 0 && p->gram_mode != 1)
    raise(MMF_EINVAL, "gram_mode must be 0 (FP32 Gram) or 1 (BF16 Gram, FP32 rescoring)");
  if ((p->flags & MMF_TWO_ELIMINATIONS) && (p->k != 3 || p->gram_mode != 0))
    raise(MMF_EINVAL, "MMF_TWO_ELIMINATIONS needs k = 3 and the FP32 Gram form");
}

// sparse matrix in CSR
struct Csr {
  int64_t n = 0, nnz = 0;
  DBuf rp, ci, cv;
};

void build_stage_geometry(StageDev& sd, const SchedStage& sc, int64_t rot_base, hipStream_t s) {
  sd.size = sc.size;
  sd.t = sc.t;
  sd.m = (int)sc.sizes.size();
  sd.rot_base = rot_base;
  sd.off_h.assign(sd.m + 1, 0);
  sd.roff_h.assign(sd.m + 1, 0);
  sd.rcnt_h = sc.rcnt;
  sd.gbase_h.assign(sd.m, 0);
  int64_t gb = 0;
  sd.cmax = 0;
  sd.rmax = 0;
  for (int u = 0; u < sd.m; ++u) {
    sd.off_h[u + 1] = sd.off_h[u] + sc.sizes[u];
    sd.roff_h[u + 1] = sd.roff_h[u] + sc.rcnt[u];
    sd.gbase_h[u] = gb;
    gb += (int64_t)sc.sizes[u] * pmmf::gd_stride(sc.sizes[u]);
    sd.cmax = std::max(sd.cmax, sc.sizes[u]);
    sd.rmax = std::max(sd.rmax, sc.rcnt[u]);
  }
  sd.lvl_stride = sd.rmax + 1;
  std::vector<int32_t> order(sd.m);
  for (int u = 0; u < sd.m; ++u) order[u] = u;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return sc.sizes[a] > sc.sizes[b]; });
  upload_async(sd.off, sd.off_h, s);
  upload_async(sd.rcnt, sd.rcnt_h, s);
  upload_async(sd.roff, sd.roff_h, s);
  upload_async(sd.order, order, s);
  upload_async(sd.gbase, sd.gbase_h, s);
  sd.next.ensure(sd.size * sizeof(int32_t));
  sd.gid.ensure(sd.size * sizeof(int32_t));
  sd.cl_of.ensure(sd.size * sizeof(int32_t));
  sd.lvl_ptr.ensure((size_t)sd.m * sd.lvl_stride * sizeof(int32_t));
  sd.depth.ensure(sd.m * sizeof(int32_t));
  sd.sw_idx.ensure(sd.t * sizeof(int32_t));
  HIPCHK(pmmf::launch_fill_cluster_of(sd.off.as<int32_t>(), sd.m, (int)sd.size,
                                      sd.cl_of.as<int32_t>(), s));
}

int round_cmax(int c) { return (c + 63) / 64 * 64; }

// workgroup size of the greedy search (PMMF_FIND_THREADS = 256 or 512; 256 by default)
// threads per cluster in the search (512 measured faster than 256 on the 262k kNN workload;
// PMMF_FIND_THREADS=256 selects the other form)
int find_threads() {
  static int nt = [] {
    const char* e = std::getenv("PMMF_FIND_THREADS");
    return (e && std::atoi(e) == 256) ? 256 : 512;
  }();
  return nt;
}

// level-kernel view of a stage restricted to its big clusters (those not split into units)
pmmf::SweepStage sweep_view(const mmf_plan& h, const StageDev& sd) {
  pmmf::SweepStage v;
  v.m = sd.nbig;
  v.k = h.k;
  v.cmax = round_cmax(std::max(sd.big_cmax, 1));
  v.rmax = std::max(sd.big_rmax, 1);
  v.lvl_stride = sd.lvl_stride;
  v.off = sd.off.as<int32_t>();
  v.lvl_ptr = sd.lvl_ptr.as<int32_t>();
  v.depth = sd.depth.as<int32_t>();
  v.sw_loc = sd.sw_loc.as<int32_t>();
  v.sw_o = sd.sw_o.as<float>();
  v.next = sd.next.as<int32_t>();
  v.gid = sd.gid.as<int32_t>();
  v.sw_idx = sd.sw_idx.as<int32_t>();
  v.rot_base = sd.rot_base;
  v.clist = sd.big_list.as<int32_t>();
  return v;
}

pmmf::UnitStage unit_view(const mmf_plan& h, const StageDev& sd) {
  pmmf::UnitStage v;
  v.nu = sd.nu;
  v.k = h.k;
  v.cnt = sd.u_cnt.as<int2>();
  v.slot = sd.u_slot.as<int4>();
  v.rot = sd.u_rot.as<int2>();
  v.rot_o = h.rot_o.as<float>();
  v.rot_base = sd.rot_base;
  return v;
}

void build_tail(mmf_plan& h, const std::vector<std::vector<int32_t>>& all_cnt,
                const std::vector<std::vector<int32_t>>& all_slot,
                const std::vector<std::vector<int32_t>>& all_rot, hipStream_t s);

void ensure_units(mmf_plan& h, hipStream_t s) {
  if (h.units_ready) return;
  const int k = h.k;
  constexpr int UM = pmmf::UNIT_MAX;
  std::vector<std::vector<int32_t>> all_cnt, all_slot, all_rot;
  for (auto& sp : h.st) {
    StageDev& sd = *sp;
    std::vector<int32_t> loc3(std::max<int64_t>(sd.t, 1) * 3);
    std::vector<int32_t> nxt(std::max<int64_t>(sd.size, 1)), gidv(std::max<int64_t>(sd.size, 1));
    if (sd.t)
      HIPCHK(hipMemcpy(loc3.data(), h.rot_loc.as<int32_t>() + sd.rot_base * 3,
                       sd.t * 3 * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(nxt.data(), sd.next.p, sd.size * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(gidv.data(), sd.gid.p, sd.size * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> ucnt, uslot, urot, big;
    sd.big_cmax = 0;
    sd.big_rmax = 0;
    std::vector<int> parent, cid, comp_rows_ptr, comp_rot_ptr, slot;
    for (int u = 0; u < sd.m; ++u) {
      const int o = sd.off_h[u], c = sd.off_h[u + 1] - o, r = sd.rcnt_h[u], rb = sd.roff_h[u];
      parent.assign(c, 0);
      for (int j = 0; j < c; ++j) parent[j] = j;
      auto find = [&](int x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
      };
      for (int q = 0; q < r; ++q)
        for (int a = 1; a < k; ++a) {
          const int x = find(loc3[(rb + q) * 3]), y = find(loc3[(rb + q) * 3 + a]);
          if (x != y) parent[std::max(x, y)] = std::min(x, y);
        }
      // components numbered by their smallest row
      cid.assign(c, -1);
      int nc = 0;
      std::vector<int> csize;
      for (int j = 0; j < c; ++j) {
        const int rt = find(j);
        if (cid[rt] < 0) {
          cid[rt] = nc++;
          csize.push_back(0);
        }
        csize[cid[rt]] += 1;
      }
      int maxc = 0;
      for (int z : csize) maxc = std::max(maxc, z);
      if (maxc > UM) {
        big.push_back(u);
        sd.big_cmax = std::max(sd.big_cmax, c);
        sd.big_rmax = std::max(sd.big_rmax, r);
        continue;
      }
      // rows and rotations grouped by component (ascending rows, rotations in order)
      comp_rows_ptr.assign(nc + 1, 0);
      comp_rot_ptr.assign(nc + 1, 0);
      for (int j = 0; j < c; ++j) comp_rows_ptr[cid[find(j)] + 1] += 1;
      for (int q = 0; q < r; ++q) comp_rot_ptr[cid[find(loc3[(rb + q) * 3])] + 1] += 1;
      for (int z = 0; z < nc; ++z) {
        comp_rows_ptr[z + 1] += comp_rows_ptr[z];
        comp_rot_ptr[z + 1] += comp_rot_ptr[z];
      }
      std::vector<int> crow(c), crot(r);
      {
        std::vector<int> fill(comp_rows_ptr.begin(), comp_rows_ptr.end() - 1);
        for (int j = 0; j < c; ++j) crow[fill[cid[find(j)]]++] = j;
        std::vector<int> fr(comp_rot_ptr.begin(), comp_rot_ptr.end() - 1);
        for (int q = 0; q < r; ++q) crot[fr[cid[find(loc3[(rb + q) * 3])]]++] = q;
      }
      slot.assign(c, -1);
      int z = 0;
      while (z < nc) {
        // pack components z..z2-1 into one unit
        int z2 = z, nrow = 0;
        while (z2 < nc && nrow + (comp_rows_ptr[z2 + 1] - comp_rows_ptr[z2]) <= UM) {
          nrow += comp_rows_ptr[z2 + 1] - comp_rows_ptr[z2];
          ++z2;
        }
        const size_t sbase = uslot.size(), rbase = urot.size();
        uslot.resize(sbase + 4 * UM, 0);
        urot.resize(rbase + 2 * UM, 0);
        int li = 0;
        for (int i = comp_rows_ptr[z]; i < comp_rows_ptr[z2]; ++i) {
          const int pos = o + crow[i];
          slot[crow[i]] = li;
          uslot[sbase + 4 * li + 0] = pos;
          uslot[sbase + 4 * li + 1] = nxt[pos];
          uslot[sbase + 4 * li + 2] = gidv[pos];
          ++li;
        }
        int nq = 0;
        for (int i = comp_rot_ptr[z]; i < comp_rot_ptr[z2]; ++i) {
          const int q = crot[i];
          if (nq >= UM) raise(MMF_EDEVICE, "unit with more rotations than slots");
          int packed = 0;
          for (int a = 0; a < k; ++a) packed |= slot[loc3[(rb + q) * 3 + a]] << (5 * a);
          urot[rbase + 2 * nq + 0] = packed;
          urot[rbase + 2 * nq + 1] = (int32_t)(sd.rot_base + rb + q);
          ++nq;
        }
        ucnt.push_back(li);
        ucnt.push_back(nq);
        z = z2;
      }
    }
    sd.nu = (int)(ucnt.size() / 2);
    sd.nbig = (int)big.size();
    upload(sd.u_cnt, ucnt, s);
    upload(sd.u_slot, uslot, s);
    upload(sd.u_rot, urot, s);
    upload(sd.big_list, big, s);
    all_cnt.push_back(std::move(ucnt));
    all_slot.push_back(std::move(uslot));
    all_rot.push_back(std::move(urot));
  }
  build_tail(h, all_cnt, all_slot, all_rot, s);
  HIPCHK(hipStreamSynchronize(s));
  h.units_ready = true;
}

// Tables of the trailing stages: every stage from the first one on after which all stages are
// made of units and have at most TAIL_THREADS * TAIL_J rows (and at most TAIL_MAX_STAGES of them).
// Per stage: the program block (units, unit-local slots, rotation blocks filled from the
// canonical blocks by k_tail_params), and per LDS slot (units' rows in unit order) the slot of the
// next stage (or the core position, or -(gid + 1)), the position in S_{p-1} and the global id.
void build_tail(mmf_plan& h, const std::vector<std::vector<int32_t>>& all_cnt,
                const std::vector<std::vector<int32_t>>& all_slot,
                const std::vector<std::vector<int32_t>>& all_rot, hipStream_t s) {
  constexpr int UM = pmmf::UNIT_MAX;
  h.tail_first = -1;
  h.tail_st.clear();
  h.tail_entries = 0;
  const int P = (int)h.st.size();
  int first = P;
  while (first > 0 && P - (first - 1) <= pmmf::TAIL_MAX_STAGES) {
    const StageDev& sd = *h.st[first - 1];
    if (sd.nbig != 0 || sd.size > (int64_t)pmmf::TAIL_THREADS * pmmf::TAIL_J) break;
    --first;
  }
  if (P - first < 2) return;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&h.lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const int k = h.k, KK = k * k;
  // LDS slot of each position, per stage
  std::vector<std::vector<int32_t>> slot_of(P);
  for (int i = first; i < P; ++i) {
    const StageDev& sd = *h.st[i];
    slot_of[i].assign(sd.size, -1);
    const int nu = (int)(all_cnt[i].size() / 2);
    int sb = 0;
    for (int u = 0; u < nu; ++u) {
      const int ns = all_cnt[i][2 * u];
      for (int li = 0; li < ns; ++li) slot_of[i][all_slot[i][((size_t)u * UM + li) * 4]] = sb + li;
      sb += ns;
    }
    if (sb != sd.size) raise(MMF_EDEVICE, "trailing stage: units do not cover the active set");
  }
  std::vector<uint8_t> blob;
  std::vector<int32_t> trans, pos, gid, pidx;
  std::vector<int64_t> odst;
  for (int i = first; i < P; ++i) {
    const StageDev& sd = *h.st[i];
    const int nu = (int)(all_cnt[i].size() / 2);
    const int t = (int)sd.t;
    pmmf::TailStage ts{};
    ts.rows = (int)sd.size;
    ts.t = t;
    ts.nu = nu;
    ts.blob_bytes = pmmf::tail_blob_bytes(nu, t, k);
    ts.blob_off = (int64_t)blob.size();
    ts.slot_off = (int64_t)trans.size();
    blob.resize(blob.size() + ts.blob_bytes, 0);
    int32_t* units = reinterpret_cast<int32_t*>(blob.data() + ts.blob_off);
    int32_t* prog = reinterpret_cast<int32_t*>(blob.data() + ts.blob_off + pmmf::tail_prog_off(nu));
    const int64_t o_base = (ts.blob_off + pmmf::tail_o_off(nu, t)) / 4;
    int sb = 0, rb = 0;
    for (int u = 0; u < nu; ++u) {
      const int ns = all_cnt[i][2 * u], nq = all_cnt[i][2 * u + 1];
      units[2 * u] = sb;
      units[2 * u + 1] = rb;
      for (int li = 0; li < ns; ++li) {
        const int32_t* e = &all_slot[i][((size_t)u * UM + li) * 4];
        const int nx = e[1];
        trans.push_back(nx >= 0 && i + 1 < P ? slot_of[i + 1][nx] : nx);
        pos.push_back(e[0]);
        gid.push_back(e[2]);
      }
      for (int q = 0; q < nq; ++q) {
        prog[rb + q] = all_rot[i][((size_t)u * UM + q) * 2];
        pidx.push_back(all_rot[i][((size_t)u * UM + q) * 2 + 1]);
        odst.push_back(o_base + (int64_t)(rb + q) * KK);
      }
      sb += ns;
      rb += nq;
    }
    if (rb != t) raise(MMF_EDEVICE, "trailing stage: units do not hold every rotation");
    units[2 * nu] = sb;
    units[2 * nu + 1] = rb;
    h.tail_st.push_back(ts);
  }
  upload(h.tail_blob, blob, s);
  upload(h.tail_trans, trans, s);
  upload(h.tail_pos, pos, s);
  upload(h.tail_gid, gid, s);
  upload(h.tail_pidx, pidx, s);
  upload(h.tail_odst, odst, s);
  h.tail_entries = (int64_t)pidx.size();
  h.tail_first = first;
  HIPCHK(pmmf::launch_tail_params(h.tail_entries, k, h.tail_pidx.as<int32_t>(),
                                  h.tail_odst.as<int64_t>(), h.rot_o.as<float>(),
                                  h.tail_blob.as<uint8_t>(), s));
}

// The trailing stages this call runs as one launch per direction: from the first stage with
// tail tables whose rows are within max_rows and h.tail_rows and whose rows and consecutive program blocks fit
// one workgroup's LDS (nst = 0: none)
pmmf::TailPlan tail_plan(const mmf_plan& h, int64_t max_rows) {
  pmmf::TailPlan tp;
  if (h.tail_first < 0) return tp;
  const int P = (int)h.st.size();
  for (int i = h.tail_first; i + 2 <= P; ++i) {
    const pmmf::TailStage& f = h.tail_st[i - h.tail_first];
    if (f.rows > std::min(max_rows, h.tail_rows)) continue;
    int maxpair = 0;
    for (int q = i; q + 1 < P; ++q)
      maxpair = std::max(maxpair, h.tail_st[q - h.tail_first].blob_bytes +
                                      h.tail_st[q + 1 - h.tail_first].blob_bytes);
    const int data_bytes = (4 * f.rows + 15) & ~15;
    if (data_bytes + maxpair > h.lds_cap) continue;
    tp.nst = P - i;
    tp.data_bytes = data_bytes;
    tp.lds_bytes = data_bytes + maxpair;
    tp.blob = h.tail_blob.as<uint8_t>();
    tp.trans = h.tail_trans.as<int32_t>();
    tp.pos = h.tail_pos.as<int32_t>();
    tp.gid = h.tail_gid.as<int32_t>();
    for (int q = i; q < P; ++q) tp.st[q - i] = h.tail_st[q - h.tail_first];
    return tp;
  }
  return tp;
}

// widest column tile whose LDS footprint allows two workgroups per CU (fallback: one)
int pick_tile(const mmf_plan& h, int nv, int64_t nrhs) {
  int cmax = 64, rmax = 1;
  for (auto& sp : h.st) {
    if (!sp->nbig) continue;
    cmax = std::max(cmax, round_cmax(sp->big_cmax));
    rmax = std::max(rmax, sp->big_rmax);
  }
  int wmax = 1;
  while (wmax < nrhs && wmax < 32) wmax <<= 1;
  for (size_t budget : {80u * 1024u, 160u * 1024u}) {
    for (int W = wmax; W >= 1; W >>= 1)
      if (pmmf::sweep_lds_bytes(h.k, W, nv, cmax, rmax) <= budget) return W;
  }
  raise(MMF_ECAPACITY, "clusters too large for the sweep's LDS tile");
}

}  // namespace

// ------------------------------------------------------------------------------------------
extern "C" const char* mmf_last_error(void) { return g_err.c_str(); }

extern "C" int mmf_set_allocator(void* (*alloc)(size_t, void*, void*),
                                 void (*release)(void*, void*, void*), void* ctx) {
  g_err.clear();
  if ((alloc == nullptr) != (release == nullptr)) {
    g_err = "mmf_set_allocator: alloc and release must both be set or both be NULL";
    return MMF_EINVAL;
  }
  pmmf_alloc::set(alloc, release, ctx);
  return MMF_OK;
}

extern "C" int mmf_trim(void) {
  g_err.clear();
  pmmf_alloc::trim();
  return MMF_OK;
}

namespace pmmf_host_detail {
void set_error(const std::string& msg) { g_err = msg; }
}

#define ABI_BEGIN try {
#define ABI_END                                      \
  }                                                  \
  catch (const Err& e) {                             \
    g_err = e.msg;                                   \
    return e.code;                                   \
  }                                                  \
  catch (const std::exception& e) {                  \
    g_err = e.what();                                \
    return MMF_EDEVICE;                              \
  }

static std::mutex g_live_mu;
static std::set<mmf_plan*> g_live;

static void register_handle(mmf_plan* h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.insert(h);
}

static mmf_plan* checked(mmf_handle h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  if (!h || !g_live.count(h)) raise(MMF_ESTATE, "invalid or destroyed handle");
  return h;
}

// k = 3: three angles per rotation, all zero, about the rotations as found
static void init_params3(mmf_plan& h, hipStream_t s) {
  if (h.k != 3) return;
  const int64_t R = std::max<int64_t>(h.R, 1);
  h.theta.ensure(R * 3 * sizeof(float));
  HIPCHK(hipMemsetAsync(h.theta.p, 0, R * 3 * sizeof(float), s));
  h.rot_o0.ensure(R * 9 * sizeof(float));
  HIPCHK(hipMemcpyAsync(h.rot_o0.p, h.rot_o.p, R * 9 * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

// rotations (canonical and sweep-log copies) from the current angles
static void sync_rotations(mmf_plan& h, hipStream_t s) {
  if (h.k == 2) {
    HIPCHK(pmmf::launch_sync_angles(h.R, h.theta.as<float>(), h.rot_o.as<float>(), s));
    for (auto& sp : h.st)
      HIPCHK(pmmf::launch_sync_sweep((int)sp->t, sp->sw_idx.as<int32_t>(), h.theta.as<float>(),
                                     sp->sw_o.as<float>(), s));
  } else {
    HIPCHK(pmmf::launch_sync_rot3(h.R, h.theta.as<float>(), h.rot_o0.as<float>(),
                                  h.rot_o.as<float>(), s));
    for (auto& sp : h.st)
      HIPCHK(pmmf::launch_sync_sweep3((int)sp->t, sp->sw_idx.as<int32_t>(), h.rot_o.as<float>(),
                                      sp->sw_o.as<float>(), s));
  }
  if (h.tail_entries)
    HIPCHK(pmmf::launch_tail_params(h.tail_entries, h.k, h.tail_pidx.as<int32_t>(),
                                    h.tail_odst.as<int64_t>(), h.rot_o.as<float>(),
                                    h.tail_blob.as<uint8_t>(), s));
}

namespace {
// launch configuration of the sparse cluster Gram (waves per block, item form), chosen by the
// autotuner below; defined with it
struct GramCfg {
  int wpb = 0;   // waves (rows) per workgroup; 0: the default
  int form = -1; // 1: items of one row segment, 0: items of consecutive short segments; -1: default
};
GramCfg gram_config(const mmf_plan& h, int S, int64_t nnz, int cmax, hipStream_t s,
                    const std::function<void(const GramCfg&)>& run);
}  // namespace

extern "C" int mmf_factor(int64_t n, int64_t nnz, const int64_t* d_rowptr, const int32_t* d_colind,
                          const float* d_val, const mmf_params* p, void* stream, mmf_handle* out) {
  ABI_BEGIN
  g_err.clear();
  if (!out) raise(MMF_EINVAL, "out is NULL");
  *out = nullptr;
  validate(n, p);
  if (nnz < 0 || (nnz > 0 && (!d_rowptr || !d_colind || !d_val)) || !d_rowptr)
    raise(MMF_EINVAL, "bad CSR arguments");
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  auto h = std::make_unique<mmf_plan>();
  h->n = n;
  h->core = p->core_size;
  h->k = p->k;
  h->prm = *p;
  h->elims = (p->flags & MMF_TWO_ELIMINATIONS) ? 2 : 1;
  h->stream = s;
  h->R = n - p->core_size;
  std::vector<SchedStage> sched = make_schedule(*p, n);

  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, s));

  // input checks and ||A||_F^2, trace(A)
  DBuf part, flags, dsum, scan_tmp;
  part.ensure(2 * n * sizeof(double));
  flags.ensure(sizeof(int32_t));
  dsum.ensure(8 * sizeof(double));
  HIPCHK(hipMemsetAsync(flags.p, 0, sizeof(int32_t), s));
  HIPCHK(pmmf::launch_csr_stats(n, d_rowptr, d_colind, d_val,
                                (p->flags & MMF_CHECK_SYMMETRY) ? 1 : 0, part.as<double>(),
                                flags.as<int32_t>(), s));
  HIPCHK(pmmf::launch_sum_double(part.as<double>(), n, dsum.as<double>() + 0, s));
  HIPCHK(pmmf::launch_sum_double(part.as<double>() + n, n, dsum.as<double>() + 1, s));
  int32_t fl = 0;
  double stats_a[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&fl, flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(stats_a, dsum.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl & 4) raise(MMF_EINVAL, "column index out of range");
  if (fl & 8) raise(MMF_EINVAL, "column indices must be strictly ascending within each row");
  if (fl & 1) raise(MMF_ENONFINITE, "matrix has NaN or Inf entries");
  if (fl & 2) raise(MMF_ENOTSYM, "matrix is not exactly symmetric");

  const int64_t R = h->R;
  h->rot_loc.ensure(std::max<int64_t>(R, 1) * 3 * sizeof(int32_t));
  h->rot_gid.ensure(std::max<int64_t>(R, 1) * 3 * sizeof(int32_t));
  h->rot_o.ensure(std::max<int64_t>(R, 1) * 9 * sizeof(float));
  h->rot_ret.ensure(std::max<int64_t>(R, 1) * sizeof(int32_t));
  h->rot_margin.ensure(std::max<int64_t>(R, 1) * sizeof(float));
  h->theta.ensure(std::max<int64_t>(R, 1) * sizeof(float));
  h->rot_lit.ensure(std::max<int64_t>(R, 1) * sizeof(double));
  h->rot_lvl.ensure(std::max<int64_t>(R, 1) * sizeof(int32_t));
  h->hdiag.ensure(n * sizeof(float));
  HIPCHK(hipMemsetAsync(h->hdiag.p, 0, n * sizeof(float), s));
  HIPCHK(hipMemsetAsync(h->theta.p, 0, std::max<int64_t>(R, 1) * sizeof(float), s));

  // working copy of the active matrix
  Csr M, W, M2, Qr, Qt;
  M.n = n;
  M.nnz = nnz;
  M.rp.ensure((n + 1) * sizeof(int64_t));
  M.ci.ensure(std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  M.cv.ensure(std::max<int64_t>(nnz, 1) * sizeof(float));
  HIPCHK(pmmf::launch_copy_csr(n, d_rowptr, d_colind, d_val, M.rp.as<int64_t>(),
                               M.ci.as<int32_t>(), M.cv.as<float>(), s));

  int64_t pool = 1;
  for (auto& sc : sched) {
    int64_t g = 0;
    for (int32_t c : sc.sizes) g += (int64_t)c * pmmf::gd_stride(c);
    // sizes chosen during the factorization: every cluster has at most cluster_max positions
    if (sc.sizes.empty()) g = sc.size * (std::min<int64_t>(sc.size, p->cluster_max) + 1);
    pool = std::max(pool, g);
  }
  DBuf GD, retflag, keep, scan, cnt, loss_row, overflow, gid_cur, dense_buf;
  DBuf qs_ci, qs_cv;  // per-column scratch slots of the accumulated rotations (nonzeros only)
  DBuf bf_bm, bf_pre, bf_R, bf_off, bf_slab, bf_slab16, bf_stats;  // BF16 form only
  DBuf wstart, wcnt, abase, stage_ci, stage_cv;  // staging rows of the two products
  DBuf tcur;                                     // column cursors of the Qbar transpose
  DBuf qtmp_ci, qtmp_cv;                         // Qbar's rows before they are put in order
  DBuf run_ptr, run_cl, run_start, wrs;            // run table of the active matrix, run starts in W
  if (p->gram_mode == 1) bf_stats.ensure(2 * sizeof(unsigned long long));
  GD.ensure(pool * sizeof(float2));
  qs_ci.ensure(pool * sizeof(int32_t));
  qs_cv.ensure(pool * sizeof(float));
  retflag.ensure(n);
  keep.ensure((n + 1) * sizeof(int32_t));
  scan.ensure((n + 2) * sizeof(int64_t));
  cnt.ensure((n + 1) * sizeof(int32_t));
  loss_row.ensure(n * sizeof(double));
  overflow.ensure(2 * sizeof(int32_t));
  scan_tmp.ensure(pmmf::scan_tmp_elems(n + 1) * sizeof(int64_t));
  HIPCHK(hipMemsetAsync(overflow.p, 0, 2 * sizeof(int32_t), s));

  int64_t rot_base = 0;
  h->info.fro2_a = stats_a[0];
  h->info.trace_a = stats_a[1];
  std::vector<double> stage_loss_dev;
  DBuf stage_loss, gram_work;
  stage_loss.ensure(std::max<size_t>(sched.size(), 1) * sizeof(double));
  gram_work.ensure(std::max<size_t>(sched.size(), 1) * sizeof(unsigned long long));
  HIPCHK(hipMemsetAsync(gram_work.p, 0, std::max<size_t>(sched.size(), 1) * 8, s));

  std::vector<std::unique_ptr<PhaseEvents>> stage_events;
  DBuf cut_d, cut_w;  // boundary cut counts (data-driven clustering)
  for (size_t pi = 0; pi < sched.size(); ++pi) {
    SchedStage& sc = sched[pi];
    if (sc.sizes.empty()) {
      // data-driven clustering of this stage's active matrix (MMF_CUT_CLUSTERS)
      const int64_t S0 = sc.size;
      cut_d.ensure((S0 + 2) * sizeof(int32_t));
      cut_w.ensure((S0 + 2) * sizeof(int64_t));
      HIPCHK(pmmf::launch_cut_counts((int)S0, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                                     cut_d.as<int32_t>(), cut_w.as<int64_t>(),
                                     scan_tmp.as<int64_t>(), s));
      std::vector<int64_t> wb(S0 + 2);
      HIPCHK(hipMemcpyAsync(wb.data(), cut_w.p, (S0 + 2) * sizeof(int64_t), hipMemcpyDeviceToHost,
                            s));
      HIPCHK(hipStreamSynchronize(s));
      staging_synced(s);
      std::vector<int64_t> w(wb.begin() + 1, wb.end());  // w[b] = count at boundary b
      sc.sizes = cut_cluster_sizes(w, S0, p->cluster_min, p->cluster_max);
      allocate_stage_rotations(sc, *p);
    }
    auto sdp = std::make_unique<StageDev>();
    StageDev& sd = *sdp;
    build_stage_geometry(sd, sc, rot_base, s);
    sd.nnz = M.nnz;
    const int S = (int)sd.size;
    const int cm = round_cmax(sd.cmax);
    if (pi == 0) HIPCHK(pmmf::launch_iota(sd.gid.as<int32_t>(), S, s));
    else HIPCHK(hipMemcpyAsync(sd.gid.p, gid_cur.p, S * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(retflag.p, 0, S, s));

    // phase timings, read once the factorization has finished
    stage_events.push_back(std::make_unique<PhaseEvents>());
    PhaseEvents& pev = *stage_events.back();
    HIPCHK(hipEventRecord(pev.e[0], s));
    // cluster Grams, diagonal blocks, identity accumulators: sparse row merges, or dense column
    // slices on the matrix cores once the active matrix is dense enough
    const bool dense_gram = (int64_t)S <= DENSE_GRAM_MAX_ROWS &&
                            (double)M.nnz >= DENSE_GRAM_MIN_FILL * (double)S * (double)S;
    sd.dense_gram = dense_gram;
    const bool bf16 = h->prm.gram_mode == 1;
    // run table of the active matrix (each row's column runs per cluster): read by the sparse
    // Gram, the right rotation and, through the runs' starts in W, the left rotation
    {
      HIPCHK(pmmf::launch_runs(S, 0, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                               sd.cl_of.as<int32_t>(), cnt.as<int32_t>(), nullptr, nullptr,
                               nullptr, s));
      run_ptr.ensure((S + 1) * sizeof(int64_t));
      HIPCHK(pmmf::launch_scan(cnt.as<int32_t>(), run_ptr.as<int64_t>(), S,
                               scan_tmp.as<int64_t>(), s));
      // a run holds at least one entry, and a row meets each cluster in at most one run
      const int64_t nrun = std::min<int64_t>(M.nnz, (int64_t)S * sd.m);
      run_cl.ensure(std::max<int64_t>(nrun, 1) * sizeof(int32_t));
      run_start.ensure(std::max<int64_t>(nrun, 1) * sizeof(int64_t));
      wrs.ensure(std::max<int64_t>(nrun, 1) * sizeof(int64_t));
      HIPCHK(pmmf::launch_runs(S, 1, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                               sd.cl_of.as<int32_t>(), nullptr, run_ptr.as<int64_t>(),
                               run_cl.as<int32_t>(), run_start.as<int64_t>(), s));
      HIPCHK(pmmf::launch_gram_work(S, M.rp.as<int64_t>(), run_ptr.as<int64_t>(),
                                    run_start.as<int64_t>(),
                                    gram_work.as<unsigned long long>() + pi, s));
    }
    if (bf16) {
      // slab rows R_u, slab sizes (host), then FP32 + BF16 slabs, G~ on the matrix cores, D
      // and the exact column norms
      sd.dense_gram = true;
      const int64_t W = (S + 31) / 32;
      bf_bm.ensure((size_t)sd.m * W * sizeof(uint32_t));
      bf_pre.ensure((size_t)sd.m * W * sizeof(int32_t));
      bf_R.ensure((size_t)sd.m * sizeof(int32_t));
      HIPCHK(pmmf::launch_slab_rows(S, sd.m, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                                    sd.cl_of.as<int32_t>(), W, bf_bm.as<uint32_t>(),
                                    bf_pre.as<int32_t>(), bf_R.as<int32_t>(), s));
      std::vector<int32_t> Rh(sd.m);
      HIPCHK(hipMemcpyAsync(Rh.data(), bf_R.p, sd.m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::vector<int64_t> soff(sd.m + 1, 0);
      for (int u = 0; u < sd.m; ++u)
        soff[u + 1] = soff[u] + (int64_t)Rh[u] * (sd.off_h[u + 1] - sd.off_h[u]);
      upload(bf_off, soff, s);
      bf_slab.ensure(std::max<int64_t>(soff[sd.m], 1) * sizeof(float));
      bf_slab16.ensure(std::max<int64_t>(soff[sd.m], 1) * sizeof(uint16_t));
      // matrix-core work: upper-triangle 32 x 32 tiles, slab rows in 64-row slices
      for (int u = 0; u < sd.m; ++u) {
        const double nt = (double)((sd.off_h[u + 1] - sd.off_h[u] + 31) / 32);
        sd.gram_flops += nt * (nt + 1) / 2 * 2.0 * 32 * 32 * (double)((Rh[u] + 63) / 64 * 64);
      }
      HIPCHK(pmmf::launch_gram_bf16(S, sd.m, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                                    M.cv.as<float>(), sd.off.as<int32_t>(),
                                    sd.cl_of.as<int32_t>(), W, bf_bm.as<uint32_t>(),
                                    bf_pre.as<int32_t>(), bf_off.as<int64_t>(),
                                    bf_R.as<int32_t>(), soff[sd.m], bf_slab.as<float>(),
                                    bf_slab16.as<unsigned short>(), sd.gbase.as<int64_t>(),
                                    GD.as<float2>(), sd.cmax, s));
    } else if (dense_gram) {
      // matrix-core work: upper-triangle 32 x 32 tiles over all S rows in 128-row slices
      for (int u = 0; u < sd.m; ++u) {
        const double nt = (double)((sd.off_h[u + 1] - sd.off_h[u] + 31) / 32);
        sd.gram_flops += nt * (nt + 1) / 2 * 2.0 * 32 * 32 * (double)((S + 127) / 128 * 128);
      }
      dense_buf.ensure((size_t)S * S * sizeof(float));
      HIPCHK(pmmf::launch_gram_dense(S, M.rp.as<int64_t>(), M.ci.as<int32_t>(), M.cv.as<float>(),
                                     dense_buf.as<float>(), sd.off.as<int32_t>(), sd.m,
                                     sd.gbase.as<int64_t>(), GD.as<float2>(), sd.cmax, s));
    } else {
      auto gram = [&](const GramCfg& gc) {
        HIPCHK(pmmf::launch_gram(S, M.nnz, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                                 M.cv.as<float>(), sd.off.as<int32_t>(), sd.cl_of.as<int32_t>(),
                                 sd.gbase.as<int64_t>(), run_ptr.as<int64_t>(),
                                 run_cl.as<int32_t>(), run_start.as<int64_t>(), GD.as<float2>(),
                                 cm, s, gc.wpb, gc.form));
      };
      // every configuration forms the same Gram (each row summed in one fixed order), so the
      // tuner's trial runs leave the right values behind
      gram(gram_config(*h, S, M.nnz, cm, s, gram));
    }
    // greedy rotation search in every cluster
    pmmf::FindArgs fa;
    fa.p = (int)pi + 1;
    fa.k = h->k;
    fa.elims = (p->flags & MMF_TWO_ELIMINATIONS) ? 2 : 1;
    fa.seed = p->seed;
    fa.order = sd.order.as<int32_t>();
    fa.off = sd.off.as<int32_t>();
    fa.rcnt = sd.rcnt.as<int32_t>();
    fa.roff = sd.roff.as<int32_t>();
    fa.gbase = sd.gbase.as<int64_t>();
    fa.GD = GD.as<float2>();
    fa.gid = sd.gid.as<int32_t>();
    fa.rot0 = rot_base;
    fa.rot_loc = h->rot_loc.as<int32_t>();
    fa.rot_gid = h->rot_gid.as<int32_t>();
    fa.rot_o = h->rot_o.as<float>();
    fa.rot_ret = h->rot_ret.as<int32_t>();
    fa.rot_margin = h->rot_margin.as<float>();
    fa.rot_lit = h->rot_lit.as<double>();
    fa.rot_lvl = h->rot_lvl.as<int32_t>();
    fa.hdiag = h->hdiag.as<float>();
    fa.retflag = retflag.as<uint8_t>();
    fa.err = overflow.as<int32_t>() + 1;
    HIPCHK(hipEventRecord(pev.e[1], s));
    if (bf16) {
      HIPCHK(hipMemsetAsync(bf_stats.p, 0, 2 * sizeof(unsigned long long), s));
      fa.slab = bf_slab.as<float>();
      fa.slab_off = bf_off.as<int64_t>();
      fa.slab_rows = bf_R.as<int32_t>();
      fa.sl_stats = bf_stats.as<unsigned long long>();
      HIPCHK(pmmf::launch_find_bf16(fa, sd.m, cm, s));
      unsigned long long st2[2];
      HIPCHK(hipMemcpyAsync(st2, bf_stats.p, sizeof(st2), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      sd.bf16_long = (int64_t)st2[0];
      sd.bf16_rescored = (int64_t)st2[1];
    } else {
      HIPCHK(pmmf::launch_find(fa, sd.m, cm, find_threads(), s));
    }
    HIPCHK(hipEventRecord(pev.e[2], s));
    // rotation levels (recorded by the search for one retirement per rotation) and the sweep log
    const int32_t* lvl_in = (!bf16 && h->elims != 2) ? h->rot_lvl.as<int32_t>() : nullptr;
    sd.sw_loc.ensure(sd.t * h->k * sizeof(int32_t));
    sd.sw_o.ensure(sd.t * h->k * h->k * sizeof(float));
    HIPCHK(pmmf::launch_levelize(sd.m, h->k, sd.off.as<int32_t>(), sd.rcnt.as<int32_t>(),
                                 sd.roff.as<int32_t>(), rot_base, h->rot_loc.as<int32_t>(),
                                 h->rot_o.as<float>(), lvl_in, sd.lvl_stride,
                                 sd.lvl_ptr.as<int32_t>(),
                                 sd.depth.as<int32_t>(), sd.sw_loc.as<int32_t>(),
                                 sd.sw_o.as<float>(), sd.sw_idx.as<int32_t>(),
                                 h->theta.as<float>(), cm, s));
    // survivors' positions in the next stage
    HIPCHK(pmmf::launch_keep_flags(S, retflag.as<uint8_t>(), keep.as<int32_t>(), s));
    HIPCHK(pmmf::launch_scan(keep.as<int32_t>(), scan.as<int64_t>(), S, scan_tmp.as<int64_t>(), s));
    gid_cur.ensure(S * sizeof(int32_t));
    DBuf gid_new;
    gid_new.ensure(S * sizeof(int32_t));
    HIPCHK(pmmf::launch_next_positions(S, retflag.as<uint8_t>(), scan.as<int64_t>(),
                                       sd.gid.as<int32_t>(), sd.next.as<int32_t>(),
                                       gid_new.as<int32_t>(), s));
    const int64_t Snext = sd.size - sd.t;

    // the clusters' accumulated rotations Qbar, rebuilt from the sweep log: each column's nonzeros
    // into its scratch slots, then packed into the CSR of Qbar^T; Qbar's rows from its transpose,
    // put in column order
    Qt.n = S;
    Qt.rp.ensure((S + 1) * sizeof(int64_t));
    HIPCHK(pmmf::launch_qsparse(sd.m, h->k, sd.off.as<int32_t>(), sd.gbase.as<int64_t>(),
                                sd.lvl_ptr.as<int32_t>(), sd.lvl_stride, sd.depth.as<int32_t>(),
                                sd.sw_loc.as<int32_t>(), sd.sw_o.as<float>(), cnt.as<int32_t>(),
                                qs_ci.as<int32_t>(), qs_cv.as<float>(), sd.cmax, s));
    HIPCHK(pmmf::launch_scan(cnt.as<int32_t>(), Qt.rp.as<int64_t>(), S, scan_tmp.as<int64_t>(), s));
    Qt.nnz = read_i64(Qt.rp.as<int64_t>() + S, s);
    Qt.ci.ensure(std::max<int64_t>(Qt.nnz, 1) * sizeof(int32_t));
    Qt.cv.ensure(std::max<int64_t>(Qt.nnz, 1) * sizeof(float));
    HIPCHK(pmmf::launch_qt_compact(S, sd.off.as<int32_t>(), sd.cl_of.as<int32_t>(),
                                   sd.gbase.as<int64_t>(), qs_ci.as<int32_t>(), qs_cv.as<float>(),
                                   Qt.rp.as<int64_t>(), Qt.ci.as<int32_t>(), Qt.cv.as<float>(), s));
    Qr.n = S;
    Qr.nnz = Qt.nnz;
    Qr.rp.ensure((S + 1) * sizeof(int64_t));
    Qr.ci.ensure(std::max<int64_t>(Qr.nnz, 1) * sizeof(int32_t));
    Qr.cv.ensure(std::max<int64_t>(Qr.nnz, 1) * sizeof(float));
    qtmp_ci.ensure(std::max<int64_t>(Qr.nnz, 1) * sizeof(int32_t));
    qtmp_cv.ensure(std::max<int64_t>(Qr.nnz, 1) * sizeof(float));
    tcur.ensure(std::max<int64_t>(S, 1) * sizeof(int64_t));
    HIPCHK(pmmf::launch_csr_transpose(S, Qt.nnz, Qt.rp.as<int64_t>(), Qt.ci.as<int32_t>(),
                                      Qt.cv.as<float>(), cnt.as<int32_t>(), Qr.rp.as<int64_t>(),
                                      scan_tmp.as<int64_t>(), tcur.as<int64_t>(),
                                      qtmp_ci.as<int32_t>(), qtmp_cv.as<float>(), s));
    HIPCHK(pmmf::launch_sort_rows(S, Qr.rp.as<int64_t>(), qtmp_ci.as<int32_t>(),
                                  qtmp_cv.as<float>(), Qr.ci.as<int32_t>(), Qr.cv.as<float>(), s));
    // W = M Qbar^T, written once into staging rows sized by a capacity bound (row x of W keeps
    // its entries at [wstart[x], wstart[x] + wcnt[x]); k_left reads it in that form)
    HIPCHK(pmmf::launch_bound_right(S, M.rp.as<int64_t>(), M.ci.as<int32_t>(), Qt.rp.as<int64_t>(),
                                    S, cnt.as<int32_t>(), s));
    wstart.ensure((S + 1) * sizeof(int64_t));
    HIPCHK(pmmf::launch_scan(cnt.as<int32_t>(), wstart.as<int64_t>(), S, scan_tmp.as<int64_t>(), s));
    const int64_t wcap = read_i64(wstart.as<int64_t>() + S, s);
    W.n = S;
    W.ci.ensure(std::max<int64_t>(wcap, 1) * sizeof(int32_t));
    W.cv.ensure(std::max<int64_t>(wcap, 1) * sizeof(float));
    wcnt.ensure(S * sizeof(int32_t));
    HIPCHK(pmmf::launch_right(S, 1, M.rp.as<int64_t>(), M.ci.as<int32_t>(), M.cv.as<float>(),
                              sd.off.as<int32_t>(), run_ptr.as<int64_t>(), run_cl.as<int32_t>(),
                              run_start.as<int64_t>(), Qt.rp.as<int64_t>(), Qt.ci.as<int32_t>(),
                              Qt.cv.as<float>(), wcnt.as<int32_t>(), wstart.as<int64_t>(),
                              W.ci.as<int32_t>(), W.cv.as<float>(), wrs.as<int64_t>(), cm, s));
    // A_p = Qbar W, peeled to the survivors, plus the exact residual of the retired rows: written
    // into staging rows, then compacted into the next stage's CSR
    HIPCHK(pmmf::launch_bound_left(S, Qr.rp.as<int64_t>(), Qr.ci.as<int32_t>(), wcnt.as<int32_t>(),
                                   sd.next.as<int32_t>(), Snext, cnt.as<int32_t>(), s));
    abase.ensure((Snext + 1) * sizeof(int64_t));
    HIPCHK(pmmf::launch_scan(cnt.as<int32_t>(), abase.as<int64_t>(), Snext, scan_tmp.as<int64_t>(), s));
    const int64_t acap = read_i64(abase.as<int64_t>() + Snext, s);
    stage_ci.ensure(std::max<int64_t>(acap, 1) * sizeof(int32_t));
    stage_cv.ensure(std::max<int64_t>(acap, 1) * sizeof(float));
    HIPCHK(pmmf::launch_left(S, 1, Qr.rp.as<int64_t>(), Qr.ci.as<int32_t>(), Qr.cv.as<float>(),
                             wstart.as<int64_t>(), wcnt.as<int32_t>(), W.ci.as<int32_t>(),
                             W.cv.as<float>(), run_ptr.as<int64_t>(), run_cl.as<int32_t>(),
                             wrs.as<int64_t>(), sd.off.as<int32_t>(), sd.cl_of.as<int32_t>(),
                             sd.next.as<int32_t>(), cnt.as<int32_t>(), abase.as<int64_t>(),
                             stage_ci.as<int32_t>(), stage_cv.as<float>(), loss_row.as<double>(),
                             overflow.as<int32_t>(), cm, s));
    M2.n = Snext;
    M2.rp.ensure((Snext + 1) * sizeof(int64_t));
    HIPCHK(pmmf::launch_scan(cnt.as<int32_t>(), M2.rp.as<int64_t>(), Snext, scan_tmp.as<int64_t>(), s));
    {
      // the error flags and the next active matrix's entry count, in one wait
      char* rb = readback_area();
      int32_t* fl2 = reinterpret_cast<int32_t*>(rb);
      int64_t* nnz2p = reinterpret_cast<int64_t*>(rb + 8);
      HIPCHK(hipMemcpyAsync(fl2, overflow.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(nnz2p, M2.rp.as<int64_t>() + Snext, sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      staging_synced(s);
      const int64_t nnz2 = *nnz2p;
      if (fl2[1]) raise(MMF_EDEVICE, "greedy search found no partner in a cluster");
      if (fl2[0]) raise(MMF_ECAPACITY, "a row of Qbar has more than 512 entries");
      M2.nnz = nnz2;
    }
    M2.ci.ensure(std::max<int64_t>(M2.nnz, 1) * sizeof(int32_t));
    M2.cv.ensure(std::max<int64_t>(M2.nnz, 1) * sizeof(float));
    HIPCHK(pmmf::launch_compact_rows(Snext, abase.as<int64_t>(), cnt.as<int32_t>(),
                                     stage_ci.as<int32_t>(), stage_cv.as<float>(),
                                     M2.rp.as<int64_t>(), M2.ci.as<int32_t>(), M2.cv.as<float>(),
                                     s));
    HIPCHK(hipEventRecord(pev.e[3], s));
    HIPCHK(pmmf::launch_sum_double(loss_row.as<double>(), S, stage_loss.as<double>() + pi, s));
    M.rp.swap_with(M2.rp);
    M.ci.swap_with(M2.ci);
    M.cv.swap_with(M2.cv);
    std::swap(M.nnz, M2.nnz);
    M.n = Snext;
    gid_cur.swap_with(gid_new);
    rot_base += sd.t;
    h->st.push_back(std::move(sdp));
  }

  // core: the final active block, dense
  const int64_t core = h->core;
  h->hcore.ensure(std::max<int64_t>(core * core, 1) * sizeof(float));
  HIPCHK(hipMemsetAsync(h->hcore.p, 0, core * core * sizeof(float), s));
  HIPCHK(pmmf::launch_core_dense((int)core, M.rp.as<int64_t>(), M.ci.as<int32_t>(),
                                 M.cv.as<float>(), h->hcore.as<float>(), s));
  h->core_ids.ensure(std::max<int64_t>(core, 1) * sizeof(int32_t));
  if (sched.empty()) HIPCHK(pmmf::launch_iota(h->core_ids.as<int32_t>(), core, s));
  else HIPCHK(hipMemcpyAsync(h->core_ids.p, gid_cur.p, core * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, s));
  // H statistics and the literal loss
  HIPCHK(pmmf::launch_h_stats(n, h->hdiag.as<float>(), core, h->hcore.as<float>(),
                              dsum.as<double>() + 2, s));
  HIPCHK(pmmf::launch_sum_double(h->rot_lit.as<double>(), R, dsum.as<double>() + 4, s));
  HIPCHK(hipEventRecord(ev1, s));
  double hst[4] = {0, 0, 0, 0};
  std::vector<double> sl(sched.size(), 0.0);
  int32_t ovf = 0;
  std::vector<unsigned long long> gw(sched.size(), 0);
  {
    // one wait for the H statistics, the overflow flag and the per-stage losses and Gram work
    const size_t ns = sched.size();
    char* rb = readback_area(32 + 16 * ns);
    double* hst_p = reinterpret_cast<double*>(rb);
    int32_t* ovf_p = reinterpret_cast<int32_t*>(rb + 24);
    double* sl_p = reinterpret_cast<double*>(rb + 32);
    unsigned long long* gw_p = reinterpret_cast<unsigned long long*>(rb + 32 + 8 * ns);
    HIPCHK(hipMemcpyAsync(hst_p, dsum.as<double>() + 2, 3 * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    if (ns > 0) {
      HIPCHK(hipMemcpyAsync(sl_p, stage_loss.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(gw_p, gram_work.p, ns * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipMemcpyAsync(ovf_p, overflow.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    staging_synced(s);
    std::copy(hst_p, hst_p + 3, hst);
    std::copy(sl_p, sl_p + ns, sl.begin());
    std::copy(gw_p, gw_p + ns, gw.begin());
    ovf = *ovf_p;
  }
  if (ovf) raise(MMF_ECAPACITY, "a row of a stage rotation had more than 512 terms");
  for (size_t pi = 0; pi < stage_events.size(); ++pi) {
    StageDev& sd = *h->st[pi];
    const PhaseEvents& pev = *stage_events[pi];
    sd.gram_ms = pev.ms(0, 1);
    sd.find_ms = pev.ms(1, 2);
    sd.rotate_ms = pev.ms(2, 3);
  }
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);

  // is_core flags for the sweeps
  {
    std::vector<int32_t> cid(core);
    HIPCHK(hipMemcpy(cid.data(), h->core_ids.p, core * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<uint8_t> flag(n, 0);
    for (int32_t g : cid) flag[g] = 1;
    upload(h->is_core, flag, s);
    HIPCHK(hipStreamSynchronize(s));
  }
  mmf_info& inf = h->info;
  inf.n = n;
  inf.core_size = core;
  inf.k = h->k;
  inf.num_stages = (int32_t)h->st.size();
  inf.num_rotations = R;
  inf.max_clusters = 0;
  inf.loss = 0.0;
  for (size_t q = 0; q < sl.size(); ++q) {
    h->st[q]->gram_useful_flops = 2.0 * (double)gw[q];
    if (!h->st[q]->dense_gram) h->st[q]->gram_flops = h->st[q]->gram_useful_flops;
    h->st[q]->loss = sl[q];
    inf.loss += sl[q];
    inf.max_clusters = std::max<int64_t>(inf.max_clusters, h->st[q]->m);
  }
  inf.fro2_h = hst[0];
  inf.trace_h = hst[1];
  inf.loss_literal = hst[2];
  inf.factor_ms = ms;
  // stage depths for the stage info
  for (auto& sp : h->st) {
    std::vector<int32_t> dep(sp->m);
    HIPCHK(hipMemcpy(dep.data(), sp->depth.p, sp->m * sizeof(int32_t), hipMemcpyDeviceToHost));
    sp->depth_max = 0;
    for (int32_t d : dep) sp->depth_max = std::max(sp->depth_max, d);
  }
  init_params3(*h, s);
  *out = h.release();
  register_handle(*out);
  return MMF_OK;
  ABI_END
}

// ------------------------------------------------------------------------------------------
namespace {

float* wsbuf(mmf_plan& h, int slot, size_t floats) {
  h.ws[slot].ensure(std::max<size_t>(floats, 1) * sizeof(float));
  return h.ws[slot].as<float>();
}

void ensure_inverse(mmf_plan& h, hipStream_t s) {
  if (h.inv_ready) return;
  const int64_t c = h.core;
  h.hinv.ensure(std::max<int64_t>(c * c, 1) * sizeof(float));
  h.chol_L.ensure(std::max<int64_t>(c * c, 1) * sizeof(float));
  h.chol_X.ensure(std::max<int64_t>(c * c, 1) * sizeof(float));
  h.status.ensure(sizeof(int32_t));
  HIPCHK(hipMemsetAsync(h.status.p, 0, sizeof(int32_t), s));
  if (c > 0)
    HIPCHK(hipMemcpyAsync(h.chol_L.p, h.hcore.p, c * c * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(pmmf::launch_core_inverse((int)c, h.chol_L.as<float>(), h.chol_X.as<float>(),
                                   h.hinv.as<float>(), h.n, h.hdiag.as<float>(),
                                   h.is_core.as<uint8_t>(), h.status.as<int32_t>(), s));
  int32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, h.status.p, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st & 2) raise(MMF_ESINGULAR, "H has a zero retired diagonal entry");
  if (st & 1) raise(MMF_ESINGULAR, "the core of H is not positive definite");
  h.inv_ready = true;
}

// H^{-1/2} for Y = U^T H^{-1/2} U X: positive retired diagonal (checked), and the core's inverse
// square root from an FP64 symmetric eigendecomposition (LAPACK syevd through rocSOLVER, once per
// handle and parameter set)
std::mutex g_rb_mu;
rocblas_handle g_rb = nullptr;

void ensure_inverse_sqrt(mmf_plan& h, hipStream_t s) {
  if (h.isqrt_ready) return;
  const int64_t c = h.core;
  h.hisqrt.ensure(std::max<int64_t>(c * c, 1) * sizeof(float));
  h.status.ensure(sizeof(int32_t));
  HIPCHK(hipMemsetAsync(h.status.p, 0, sizeof(int32_t), s));
  HIPCHK(pmmf::launch_check_hdiag_pos(h.n, h.hdiag.as<float>(), h.is_core.as<uint8_t>(),
                                      h.status.as<int32_t>(), s));
  if (c > 0) {
    h.eig_A.ensure(c * c * sizeof(double));
    h.eig_D.ensure(c * sizeof(double));
    h.eig_E.ensure(c * sizeof(double));
    h.eig_info.ensure(sizeof(rocblas_int));
    HIPCHK(pmmf::launch_f32_to_f64(c * c, h.hcore.as<float>(), h.eig_A.as<double>(), s));
    std::lock_guard<std::mutex> lk(g_rb_mu);
    if (!g_rb && rocblas_create_handle(&g_rb) != rocblas_status_success)
      raise(MMF_EDEVICE, "rocblas_create_handle failed");
    if (rocblas_set_stream(g_rb, s) != rocblas_status_success)
      raise(MMF_EDEVICE, "rocblas_set_stream failed");
    // the core is symmetric, so its row-major array is also its column-major array
    const rocblas_status st = rocsolver_dsyevd(g_rb, rocblas_evect_original, rocblas_fill_upper,
                                               (rocblas_int)c, h.eig_A.as<double>(),
                                               (rocblas_int)c, h.eig_D.as<double>(),
                                               h.eig_E.as<double>(),
                                               h.eig_info.as<rocblas_int>());
    if (st != rocblas_status_success) raise(MMF_EDEVICE, "rocsolver_dsyevd failed");
    HIPCHK(pmmf::launch_isqrt_assemble((int)c, h.eig_A.as<double>(), h.eig_D.as<double>(),
                                       h.hisqrt.as<float>(), h.status.as<int32_t>(), s));
  }
  int32_t st = 0;
  rocblas_int info = 0;
  HIPCHK(hipMemcpyAsync(&st, h.status.p, sizeof(st), hipMemcpyDeviceToHost, s));
  if (c > 0) HIPCHK(hipMemcpyAsync(&info, h.eig_info.p, sizeof(info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info != 0) raise(MMF_EDEVICE, "the core eigendecomposition did not converge");
  if (st & 4) raise(MMF_ESINGULAR, "H has a retired diagonal entry that is not positive");
  if (st & 8) raise(MMF_ESINGULAR, "the core of H is not positive definite");
  h.isqrt_ready = true;
}

// Y = U^T op(H) U X with op = H (which = 0), H^{-1} (1) or H^{-1/2} (2)
// ------------------------------------------------------------------------------------------
// Sweep autotuner.  The first product (or adjoint) of a handle with a given column count times each
// candidate configuration of the sweep kernels on the caller's own buffers (the products are
// idempotent) and keeps the fastest: waves per workgroup of the unit sweep (1, 2, 4) and, when
// some cluster needs the level kernel, its column tile (widest that fits, half, quarter).  Results
// persist in a small JSON file (PMMF_TUNE_CACHE, default $HOME/.cache/pmmf_tune.json), keyed by
// device, rotation order, size, core, vectors per sweep, column count and the sweep plan's shape,
// so later processes reuse them.  PMMF_AUTOTUNE=0 keeps the default configuration.
struct TuneCache {
  std::mutex mu;
  bool loaded = false;
  std::string path;
  std::map<std::string, std::pair<SweepCfg, double>> entries;
};
TuneCache g_tune;

bool autotune_enabled() {
  const char* e = std::getenv("PMMF_AUTOTUNE");
  return !(e && std::strcmp(e, "0") == 0);
}

std::string tune_path() {
  const char* e = std::getenv("PMMF_TUNE_CACHE");
  if (e && *e) return e;
  const char* home = std::getenv("HOME");
  return std::string(home && *home ? home : "/tmp") + "/.cache/pmmf_tune.json";
}

// one entry per line:  "key": {"wpb": 2, "W": 16, "tail": 4096, "ms": 0.123},
void tune_load_locked() {
  g_tune.path = tune_path();
  g_tune.loaded = true;
  FILE* f = std::fopen(g_tune.path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* q0 = std::strchr(line, '"');
    const char* q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
    const char* br = q1 ? std::strchr(q1, '{') : nullptr;
    if (!br) continue;
    SweepCfg c;
    double ms = 0.0;
    if (std::sscanf(br, "{\"wpb\": %d, \"W\": %d, \"tail\": %d, \"ms\": %lf}", &c.wpb, &c.W,
                    &c.tail, &ms) == 4 ||
        std::sscanf(br, "{\"wpb\": %d, \"W\": %d, \"ms\": %lf}", &c.wpb, &c.W, &ms) == 3)
      g_tune.entries[std::string(q0 + 1, q1)] = {c, ms};
  }
  std::fclose(f);
}

void tune_save_locked() {
  const std::string& path = g_tune.path;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);
    for (size_t k = 1; k <= dir.size(); ++k)  // mkdir -p, one level at a time
      if (k == dir.size() || dir[k] == '/') (void)mkdir(dir.substr(0, k).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : g_tune.entries) {
    std::fprintf(f, "  \"%s\": {\"wpb\": %d, \"W\": %d, \"tail\": %d, \"ms\": %.6f}%s\n",
                 kv.first.c_str(), kv.second.first.wpb, kv.second.first.W, kv.second.first.tail,
                 kv.second.second, ++k < g_tune.entries.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
  (void)std::rename(tmp.c_str(), path.c_str());
}

std::string tune_key(const mmf_plan& h, const char* what, int nv, int64_t nrhs) {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    std::strcpy(prop.gcnArchName, "unknown");
  int64_t nu = 0, nbig = 0;
  for (const auto& sp : h.st) {
    nu += sp->nu;
    nbig += sp->nbig;
  }
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == '"' || ch == '\\') ch = '_';
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s|%s|k%d|n%lld|core%lld|nv%d|cols%lld|units%lld|big%lld",
                arch.c_str(), what, h.k, (long long)h.n, (long long)h.core, nv, (long long)nrhs,
                (long long)nu, (long long)nbig);
  return buf;
}

// the configuration for (what, nv, nrhs): from the handle, the cache file, or by timing `run`
template <class Run>
SweepCfg sweep_config(mmf_plan& h, const char* what, int nv, int64_t nrhs, hipStream_t s,
                      Run run) {
  const auto hk = std::make_pair(std::string(what) + std::to_string(nv), nrhs);
  auto it = h.tune.find(hk);
  if (it != h.tune.end()) return it->second;
  SweepCfg def;
  def.W = pick_tile(h, nv, nrhs);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (!autotune_enabled() || hipStreamIsCapturing(s, &cap) != hipSuccess ||
      cap != hipStreamCaptureStatusNone) {
    return def;
  }
  const std::string key = tune_key(h, what, nv, nrhs);
  {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    if (!g_tune.loaded || g_tune.path != tune_path()) {
      g_tune.entries.clear();
      tune_load_locked();
    }
    auto f = g_tune.entries.find(key);
    if (f != g_tune.entries.end()) {
      h.tune[hk] = f->second.first;
      return f->second.first;
    }
  }
  bool big = false;
  for (const auto& sp : h.st) big = big || sp->nbig > 0;
  std::vector<int> Ws{def.W};
  if (big)
    for (int w = def.W / 2; w >= std::max(1, def.W / 4); w /= 2) Ws.push_back(w);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  SweepCfg best = def;
  double best_ms = 1e300;
  // fused trailing stages: only the one-vector products use them; otherwise one candidate
  std::vector<int> tails{def.tail};
  if (nv == 1 && h.tail_first >= 0) tails = {0, 2048, 4096, 8192};
  for (int tl : tails)
  for (int wpb : {1, 2, 4})
    for (int W : Ws) {
      SweepCfg c{wpb, W, tl};
      run(c);  // warm
      HIPCHK(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) run(c);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms / 3.0 < best_ms) {
        best_ms = ms / 3.0;
        best = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h.tune[hk] = best;
  {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.entries[key] = {best, best_ms};
    tune_save_locked();
  }
  return best;
}

// The sparse cluster Gram: waves per workgroup (1, 2, 4 within the LDS budget) and item form,
// tuned per stage shape (rows, nonzeros, largest cluster) with the same cache as the sweeps.
GramCfg gram_config(const mmf_plan& h, int S, int64_t nnz, int cmax, hipStream_t s,
                    const std::function<void(const GramCfg&)>& run) {
  GramCfg def;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (!autotune_enabled() || hipStreamIsCapturing(s, &cap) != hipSuccess ||
      cap != hipStreamCaptureStatusNone)
    return def;
  char what[128];
  std::snprintf(what, sizeof what, "gram_S%d_nnz%lld_c%d", S, (long long)nnz, cmax);
  const std::string key = tune_key(h, what, 0, 0);
  {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    if (!g_tune.loaded || g_tune.path != tune_path()) {
      g_tune.entries.clear();
      tune_load_locked();
    }
    auto f = g_tune.entries.find(key);
    if (f != g_tune.entries.end()) return GramCfg{f->second.first.wpb, f->second.first.W};
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  GramCfg best = def;
  double best_ms = 1e300;
  for (int form : {0, 1})
    for (int wpb : {1, 2, 4}) {
      if ((size_t)wpb * (cmax + 64) * 4 > 64 * 1024) continue;
      const GramCfg c{wpb, form};
      run(c);  // warm
      HIPCHK(hipEventRecord(e0, s));
      run(c);
      run(c);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms / 2.0 < best_ms) {
        best_ms = ms / 2.0;
        best = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    g_tune.entries[key] = {SweepCfg{best.wpb, best.form, 0}, best_ms};
    tune_save_locked();
  }
  return best;
}

void apply_body(mmf_plan& h, const float* x, float* y, int64_t nrhs, int64_t ld, hipStream_t s,
                int which, float* ws0, float* ws1, const SweepCfg& cfg) {
  const float* Hc = which == 2 ? h.hisqrt.as<float>()
                               : (which == 1 ? h.hinv.as<float>() : h.hcore.as<float>());
  const int P = (int)h.st.size();
  const int64_t core = h.core;
  if (P == 0) {
    HIPCHK(pmmf::launch_gemm((int)core, (int)nrhs, (int)core, Hc, (int)core, 0, x, (int)ld, 0, y,
                             (int)ld, 0.f, s));
    return;
  }
  const int64_t s1 = h.st[0]->size - h.st[0]->t;
  float* buf[2] = {ws0 ? ws0 : wsbuf(h, 0, s1 * nrhs), ws1 ? ws1 : wsbuf(h, 1, s1 * nrhs)};
  const int W = cfg.W;
  const pmmf::TailPlan tp = tail_plan(h, cfg.tail);
  const int p0 = tp.nst ? P - tp.nst + 1 : P + 1;  // first trailing stage
  for (int p = 1; p <= P; ++p) {
    const StageDev& sd = *h.st[p - 1];
    pmmf::FwdIO io{};
    io.src[0] = p == 1 ? x : buf[(p - 1) % 2];
    io.ld_src = p == 1 ? ld : nrhs;
    io.dst_c[0] = buf[p % 2];
    io.ld_c = nrhs;
    io.dst_nat[0] = y;
    io.ld_nat = ld;
    io.mode[0] = which == 2 ? 3 : (which == 1 ? 2 : 1);
    io.hdiag = h.hdiag.as<float>();
    io.nrhs = nrhs;
    if (p == p0) {
      io.dst_c[0] = buf[P % 2];
      HIPCHK(pmmf::launch_tail_fwd(h.k, tp, io, s));
      break;
    }
    HIPCHK(pmmf::launch_unit_fwd(unit_view(h, sd), io, 1, cfg.wpb, s));
    HIPCHK(pmmf::launch_sweep_fwd(sweep_view(h, sd), io, W, 1, s));
  }
  HIPCHK(pmmf::launch_gemm((int)core, (int)nrhs, (int)core, Hc, (int)core, 0, buf[P % 2],
                           (int)nrhs, 0, buf[(P + 1) % 2], (int)nrhs, 0.f, s));
  for (int p = P; p >= 1; --p) {
    if (p >= p0 && p != p0) continue;
    const StageDev& sd = *h.st[p - 1];
    pmmf::RevIO io{};
    io.src_c[0] = buf[(p + 1) % 2];
    io.ld_c = nrhs;
    io.src_nat[0] = y;
    io.ld_nat = ld;
    io.mode[0] = 0;
    io.hdiag = h.hdiag.as<float>();
    if (p == 1) {
      io.dst_nat[0] = y;
      io.ld_dnat = ld;
    } else {
      io.dst_c[0] = buf[p % 2];
      io.ld_out = nrhs;
    }
    io.nrhs = nrhs;
    if (p == p0) {
      io.src_c[0] = buf[(P + 1) % 2];
      HIPCHK(pmmf::launch_tail_rev(h.k, tp, io, s));
      continue;
    }
    HIPCHK(pmmf::launch_unit_rev(unit_view(h, sd), io, 1, false, cfg.wpb, s));
    HIPCHK(pmmf::launch_sweep_rev(sweep_view(h, sd), io, W, 1, false, s));
  }
}

void apply_impl(mmf_plan& h, const float* x, float* y, int64_t nrhs, int64_t ld, hipStream_t s,
                int which, float* ws0 = nullptr, float* ws1 = nullptr) {
  if (nrhs < 0 || ld < nrhs || (!x && nrhs > 0) || (!y && nrhs > 0))
    raise(MMF_EINVAL, "bad vector arguments");
  if (nrhs == 0) return;
  if (which == 1) ensure_inverse(h, s);
  if (which == 2) ensure_inverse_sqrt(h, s);
  ensure_units(h, s);
  const SweepCfg cfg = sweep_config(h, "apply", 1, nrhs, s, [&](const SweepCfg& c) {
    apply_body(h, x, y, nrhs, ld, s, which, ws0, ws1, c);
  });
  apply_body(h, x, y, nrhs, ld, s, which, ws0, ws1, cfg);
}

}  // namespace

extern "C" int mmf_apply(mmf_handle hh, const float* d_x, float* d_y, int64_t nrhs, int64_t ld,
                         void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  apply_impl(h, d_x, d_y, nrhs, ld, as_stream(stream), 0);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_apply_inverse(mmf_handle hh, const float* d_x, float* d_y, int64_t nrhs,
                                 int64_t ld, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  apply_impl(h, d_x, d_y, nrhs, ld, as_stream(stream), 1);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_apply_inverse_sqrt(mmf_handle hh, const float* d_x, float* d_y, int64_t nrhs,
                                      int64_t ld, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  apply_impl(h, d_x, d_y, nrhs, ld, as_stream(stream), 2);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_set_tail_rows(mmf_handle hh, int64_t rows) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (rows < 0) raise(MMF_EINVAL, "mmf_set_tail_rows: rows < 0");
  h.tail_rows = rows;
  return MMF_OK;
  ABI_END
}

// ------------------------------------------------------------------------------------------
// y = A~ x without allocating (mmf_apply_noalloc): the two ping-pong blocks of compacted vectors
// live in a fixed array of this library's device code instead of handle-owned memory.  Each
// device holds its own copy; in host code `scratch` only names it, so its address on the current
// device is looked up once per device and kept.
constexpr int64_t NOALLOC_FLOATS = int64_t(1) << 24;  // 64 MiB
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];
static std::mutex g_scratch_mu;
static std::map<int, float*> g_scratch_ptr;  // device ordinal -> that device's copy of scratch

static float* scratch_on_current_device() {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    raise(MMF_EDEVICE, std::string("address of the library's scratch array: ") +
                           hipGetErrorString(e));
  g_scratch_ptr[dev] = static_cast<float*>(ptr);
  return static_cast<float*>(ptr);
}

extern "C" int mmf_apply_noalloc(mmf_handle hh, const float* d_x, float* d_y, int64_t nrhs,
                                 int64_t ld, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (nrhs < 0 || ld < nrhs || (!d_x && nrhs > 0) || (!d_y && nrhs > 0))
    raise(MMF_EINVAL, "bad vector arguments");
  if (nrhs == 0) return MMF_OK;
  if (!h.units_ready)
    raise(MMF_ESTATE, "mmf_apply_noalloc: the handle's sweep plan is built by its first "
                      "mmf_apply, mmf_apply_inverse or mmf_graph_capture; call one of them once");
  const int64_t s1 = h.st.empty() ? 0 : h.st[0]->size - h.st[0]->t;
  if (2 * s1 * nrhs > NOALLOC_FLOATS)
    raise(MMF_ECAPACITY, "mmf_apply_noalloc: 2 x " + std::to_string(s1) + " survivors x " +
                             std::to_string(nrhs) + " right-hand sides exceed the " +
                             std::to_string(NOALLOC_FLOATS) + "-float scratch array");
  float* ws = scratch_on_current_device();
  // the tile the tuner chose for this width, else the default (no tuning runs here)
  SweepCfg cfg;
  const auto it = h.tune.find(std::make_pair(std::string("apply1"), nrhs));
  if (it != h.tune.end()) cfg = it->second;
  else cfg.W = pick_tile(h, 1, nrhs);
  apply_body(h, d_x, d_y, nrhs, ld, as_stream(stream), 0, ws, ws + s1 * nrhs, cfg);
  return MMF_OK;
  ABI_END
}

// ------------------------------------------------------------------------------------------
// Captured products: one mmf_apply / mmf_apply_inverse on fixed buffers recorded as a HIP graph
// (kernel nodes only: every size-dependent preparation runs in an eager call before capture).
// The graph owns its ping-pong workspace, so later eager calls cannot move it.
struct mmf_graph_s {
  mmf_plan* h = nullptr;
  int which = 0;  // 0 A~, 1 A~^{-1}, 2 A~^{-1/2}
  uint64_t version = 0;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  DBuf ws0, ws1;
};
static std::set<mmf_graph_s*> g_graphs;  // guarded by g_live_mu

static void graph_free(mmf_graph_s* G) {
  if (G->ge) (void)hipGraphExecDestroy(G->ge);
  if (G->g) (void)hipGraphDestroy(G->g);
  delete G;
}

extern "C" int mmf_graph_capture(mmf_handle hh, int32_t inverse, const float* d_x, float* d_y,
                                 int64_t nrhs, int64_t ld, void* stream, mmf_graph* out) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (!out || nrhs < 1 || ld < nrhs || !d_x || !d_y || d_x == d_y || inverse < 0 || inverse > 2)
    raise(MMF_EINVAL, "bad graph capture arguments");
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  std::unique_ptr<mmf_graph_s, void (*)(mmf_graph_s*)> G(new mmf_graph_s, graph_free);
  G->h = &h;
  G->which = inverse;
  const int64_t s1 = h.st.empty() ? 0 : h.st[0]->size - h.st[0]->t;
  G->ws0.ensure(std::max<int64_t>(s1 * nrhs, 1) * sizeof(float));
  G->ws1.ensure(std::max<int64_t>(s1 * nrhs, 1) * sizeof(float));
  // eager call: sweep units, core inverse and tile choice are prepared here, and y is produced
  apply_impl(h, d_x, d_y, nrhs, ld, s, G->which, G->ws0.as<float>(), G->ws1.as<float>());
  HIPCHK(hipStreamSynchronize(s));
  G->version = h.version;
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (ce != hipSuccess) {
    (void)hipStreamDestroy(cs);
    raise(MMF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
  }
  try {
    apply_impl(h, d_x, d_y, nrhs, ld, cs, G->which, G->ws0.as<float>(), G->ws1.as<float>());
  } catch (...) {
    hipGraph_t dead = nullptr;
    (void)hipStreamEndCapture(cs, &dead);
    if (dead) (void)hipGraphDestroy(dead);
    (void)hipStreamDestroy(cs);
    throw;
  }
  ce = hipStreamEndCapture(cs, &G->g);
  (void)hipStreamDestroy(cs);
  if (ce != hipSuccess) raise(MMF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
  HIPCHK(hipGraphInstantiate(&G->ge, G->g, nullptr, nullptr, 0));
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_graphs.insert(G.get());
  }
  *out = G.release();
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_graph_launch(mmf_graph gg, void* stream) {
  ABI_BEGIN
  mmf_graph_s* G = gg;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!G || !g_graphs.count(G)) raise(MMF_ESTATE, "invalid or destroyed graph");
    if (!g_live.count(G->h)) raise(MMF_ESTATE, "the graph's factorization was destroyed");
    if (G->which != 0 && G->version != G->h->version)
      raise(MMF_ESTATE, "parameters changed since the inverse graph was captured");
  }
  HIPCHK(hipGraphLaunch(G->ge, as_stream(stream)));
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_graph_destroy(mmf_graph gg) {
  ABI_BEGIN
  mmf_graph_s* G = gg;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!G || !g_graphs.count(G)) raise(MMF_ESTATE, "invalid or destroyed graph");
    g_graphs.erase(G);
  }
  (void)hipDeviceSynchronize();  // no replay may still use the workspace
  graph_free(G);
  return MMF_OK;
  ABI_END
}

void backward_body(mmf_plan& h, const float* d_x, const float* d_ybar, float* d_xbar,
                   float* d_hdiag_bar, float* d_hcore_bar, float* d_theta_bar, int64_t nrhs,
                   int64_t ld, hipStream_t s, const SweepCfg& cfg) {
  const int P = (int)h.st.size();
  const int64_t n = h.n, core = h.core;
  const float* Hc = h.hcore.as<float>();
  // forward sweeps of x and ybar together: a = U x, b = U ybar
  float* a_nat = wsbuf(h, 2, n * nrhs);
  float* b_nat = wsbuf(h, 3, n * nrhs);
  const int64_t s1 = P > 0 ? h.st[0]->size - h.st[0]->t : core;
  float* F[2][2] = {{wsbuf(h, 4, s1 * nrhs), wsbuf(h, 5, s1 * nrhs)},
                    {wsbuf(h, 6, s1 * nrhs), wsbuf(h, 7, s1 * nrhs)}};  // F[vector][pingpong]
  float* ga_core = wsbuf(h, 8, core * nrhs);
  float* gb_core = wsbuf(h, 9, core * nrhs);
  const float* a_core;
  const float* b_core;
  if (P == 0) {
    a_core = d_x;
    b_core = d_ybar;
  }
  const int W2 = cfg.W;
  // the trailing stages of both forward sweeps in one launch (as in the products)
  const pmmf::TailPlan tp = tail_plan(h, cfg.tail);
  const int p0 = tp.nst ? P - tp.nst + 1 : P + 1;
  for (int p = 1; p <= P; ++p) {
    const StageDev& sd = *h.st[p - 1];
    pmmf::FwdIO io{};
    io.src[0] = p == 1 ? d_x : F[0][(p - 1) % 2];
    io.src[1] = p == 1 ? d_ybar : F[1][(p - 1) % 2];
    io.ld_src = p == 1 ? ld : nrhs;
    io.dst_c[0] = F[0][p % 2];
    io.dst_c[1] = F[1][p % 2];
    io.ld_c = nrhs;
    io.dst_nat[0] = a_nat;
    io.dst_nat[1] = b_nat;
    io.ld_nat = nrhs;
    io.mode[0] = io.mode[1] = 0;
    io.hdiag = h.hdiag.as<float>();
    io.nrhs = nrhs;
    if (p == p0) {
      io.dst_c[0] = F[0][P % 2];
      io.dst_c[1] = F[1][P % 2];
      HIPCHK(pmmf::launch_tail_fwd(h.k, tp, io, s));
      break;
    }
    HIPCHK(pmmf::launch_unit_fwd(unit_view(h, sd), io, 2, cfg.wpb, s));
    HIPCHK(pmmf::launch_sweep_fwd(sweep_view(h, sd), io, W2, 2, s));
  }
  int64_t lda_core = nrhs;
  if (P > 0) {
    a_core = F[0][P % 2];
    b_core = F[1][P % 2];
  } else {
    lda_core = ld;
  }
  // H gradients: hdiag_bar on retired rows, hcore_bar = b_core a_core^T
  if (d_hdiag_bar) {
    if (P > 0)
      HIPCHK(pmmf::launch_rowdot(n, a_nat, b_nat, nrhs, nrhs, h.is_core.as<uint8_t>(),
                                 d_hdiag_bar, s));
    else
      HIPCHK(hipMemsetAsync(d_hdiag_bar, 0, n * sizeof(float), s));
  }
  // adjoint seeds on the core, g_a = H a and g_b = H^T b, and hcore_bar = b_core a_core^T: three
  // independent products in one launch
  {
    pmmf::GemmArgs ga[3] = {
        {(int)core, (int)nrhs, (int)core, Hc, (int)core, 0, a_core, (int)lda_core, 0, ga_core,
         (int)nrhs, 0.f},
        {(int)core, (int)nrhs, (int)core, Hc, (int)core, 1, b_core, (int)lda_core, 0, gb_core,
         (int)nrhs, 0.f},
        {(int)core, (int)core, (int)nrhs, b_core, (int)lda_core, 0, a_core, (int)lda_core, 1,
         d_hcore_bar, (int)core, 0.f}};
    HIPCHK(pmmf::launch_gemm_batch(d_hcore_bar ? 3 : 2, ga, s));
  }
  if (P == 0) {
    if (d_xbar)
      HIPCHK(hipMemcpy2DAsync(d_xbar, ld * sizeof(float), gb_core, nrhs * sizeof(float),
                              nrhs * sizeof(float), core, hipMemcpyDeviceToDevice, s));
    return;
  }
  // reverse passes: A carries (z = U-states of ybar, g_a), B carries (z = states of x, g_b)
  float* RA[2][2] = {{wsbuf(h, 10, s1 * nrhs), wsbuf(h, 11, s1 * nrhs)},
                     {wsbuf(h, 12, s1 * nrhs), wsbuf(h, 13, s1 * nrhs)}};
  float* RB[2][2] = {{wsbuf(h, 16, s1 * nrhs), wsbuf(h, 17, s1 * nrhs)},
                     {wsbuf(h, 14, s1 * nrhs), wsbuf(h, 15, s1 * nrhs)}};
  // the reverse passes read the forward states of the core (F[.][P % 2]) in place: no buffer is
  // read and written by the same sweep
  // column tiles of the angle partials: the unit sweep's (64 columns) and, where a stage has
  // clusters with a larger component, the level sweep's (W2 columns); a launch with fewer tiles
  // zero-fills the rest
  int ntiles = 1;
  for (auto& sp : h.st)
    ntiles = (int)std::max<int64_t>(ntiles, std::max(sp->nu > 0 ? (nrhs + 63) / 64 : 0,
                                                     sp->nbig > 0 ? (nrhs + W2 - 1) / W2 : 0));
  // per-tile angle partials of every rotation, [tile][rotation * NP], reduced once at the end
  const int64_t RT = std::max<int64_t>(h.R, 1);
  // angle partials per rotation: one (k = 2) or one per plane of its slots (k = 3)
  const int NP = h.k == 3 ? 3 : 1;
  const bool want_theta = h.k == 2 || d_theta_bar;
  DBuf pa_buf, pb_buf;
  pa_buf.ensure((size_t)ntiles * RT * NP * sizeof(float));
  pb_buf.ensure((size_t)ntiles * RT * NP * sizeof(float));
  for (int p = P; p >= 1; --p) {
    const StageDev& sd = *h.st[p - 1];
    const pmmf::SweepStage v = sweep_view(h, sd);
    // the two passes touch disjoint buffers: their unit sweeps share one launch
    pmmf::RevIO iop[2];
    for (int pass = 0; pass < 2; ++pass) {
      float* (*Rb)[2] = pass == 0 ? RA : RB;
      pmmf::RevIO& io = iop[pass];
      io = pmmf::RevIO{};
      if (p == P) {
        io.src_c[0] = pass == 0 ? b_core : a_core;
        io.src_c[1] = pass == 0 ? ga_core : gb_core;
      } else {
        io.src_c[0] = Rb[0][(p + 1) % 2];
        io.src_c[1] = Rb[1][(p + 1) % 2];
      }
      io.ld_c = nrhs;
      io.src_nat[0] = pass == 0 ? b_nat : a_nat;
      io.src_nat[1] = pass == 0 ? a_nat : b_nat;
      io.ld_nat = nrhs;
      io.mode[0] = 0;
      io.mode[1] = 1;
      io.hdiag = h.hdiag.as<float>();
      if (p == 1) {
        io.dst_nat[0] = nullptr;
        io.dst_nat[1] = pass == 1 ? d_xbar : nullptr;
        io.ld_dnat = ld;
      } else {
        io.dst_c[0] = Rb[0][p % 2];
        io.dst_c[1] = Rb[1][p % 2];
        io.ld_out = nrhs;
      }
      io.nrhs = nrhs;
      io.theta_part = (pass == 0 ? pa_buf.as<float>() : pb_buf.as<float>()) + sd.rot_base * NP;
      io.theta_stride = RT * NP;
      io.theta_tiles = ntiles;
      HIPCHK(pmmf::launch_sweep_rev(v, io, W2, 2, want_theta, s));
    }
    HIPCHK(pmmf::launch_unit_rev(unit_view(h, sd), iop[0], 2, want_theta, cfg.wpb, s, &iop[1]));
  }
  if (d_theta_bar)
    HIPCHK(pmmf::launch_theta_reduce((int)(h.R * NP), ntiles, RT * NP, pa_buf.as<float>(),
                                     pb_buf.as<float>(), 0, d_theta_bar, s));
  // k = 3: plane derivatives -> derivatives in the angles (derivative of the exponential map)
  if (d_theta_bar && h.k == 3)
    HIPCHK(pmmf::launch_theta3_chain(h.R, h.theta.as<float>(), d_theta_bar, s));
  // keep the temporaries alive until the stream has consumed them
  HIPCHK(hipStreamSynchronize(s));
}

extern "C" int mmf_backward(mmf_handle hh, const float* d_x, const float* d_ybar, float* d_xbar,
                            float* d_hdiag_bar, float* d_hcore_bar, float* d_theta_bar,
                            int64_t nrhs, int64_t ld, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  if (nrhs < 1 || ld < nrhs || !d_x || !d_ybar) raise(MMF_EINVAL, "bad vector arguments");
  ensure_units(h, s);
  const SweepCfg cfg = sweep_config(h, "adjoint", 2, nrhs, s, [&](const SweepCfg& c) {
    backward_body(h, d_x, d_ybar, d_xbar, d_hdiag_bar, d_hcore_bar, d_theta_bar, nrhs, ld, s, c);
  });
  backward_body(h, d_x, d_ybar, d_xbar, d_hdiag_bar, d_hcore_bar, d_theta_bar, nrhs, ld, s, cfg);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_get_info(mmf_handle hh, mmf_info* out) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (!out) raise(MMF_EINVAL, "out is NULL");
  *out = h.info;
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_get_stage_info(mmf_handle hh, int32_t stage, mmf_stage_info* out) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (!out || stage < 0 || stage >= (int32_t)h.st.size()) raise(MMF_EINVAL, "bad stage");
  const StageDev& sd = *h.st[stage];
  out->size = sd.size;
  out->rotations = sd.t;
  out->clusters = sd.m;
  out->nnz = sd.nnz;
  out->max_cluster = sd.cmax;
  out->max_depth = sd.depth_max;
  out->dense_gram = sd.dense_gram ? 1 : 0;
  out->loss = sd.loss;
  out->gram_ms = sd.gram_ms;
  out->find_ms = sd.find_ms;
  out->rotate_ms = sd.rotate_ms;
  out->find_bytes = 0;
  for (int u = 0; u < sd.m; ++u) {
    const int64_t c = sd.off_h[u + 1] - sd.off_h[u];
    const int64_t steps = (sd.rcnt_h[u] + h.elims - 1) / h.elims;
    out->find_bytes += steps * 4 * c * (1 + 8 * h.k);
  }
  out->gram_flops = sd.gram_flops;
  out->gram_useful_flops = sd.gram_useful_flops;
  out->bf16_long = sd.bf16_long;
  out->bf16_rescored = sd.bf16_rescored;
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_export(mmf_handle hh, int32_t* rot_ids, float* rot_o, int32_t* rot_retired,
                          float* rot_margin, float* hdiag, int32_t* core_ids, float* hcore) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  HIPCHK(hipStreamSynchronize(h.stream));
  const int64_t R = h.R;
  const int k = h.k;
  if (rot_ids || rot_o) {
    std::vector<int32_t> ids(R * 3);
    std::vector<float> o(R * 9);
    if (R) {
      HIPCHK(hipMemcpy(ids.data(), h.rot_gid.p, R * 3 * sizeof(int32_t), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(o.data(), h.rot_o.p, R * 9 * sizeof(float), hipMemcpyDeviceToHost));
    }
    for (int64_t r = 0; r < R; ++r) {
      for (int a = 0; a < k; ++a) {
        if (rot_ids) rot_ids[r * k + a] = ids[r * 3 + a];
        for (int b = 0; b < k; ++b)
          if (rot_o) rot_o[(r * k + a) * k + b] = o[r * 9 + a * 3 + b];
      }
    }
  }
  if (rot_retired && R)
    HIPCHK(hipMemcpy(rot_retired, h.rot_ret.p, R * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (rot_margin && R)
    HIPCHK(hipMemcpy(rot_margin, h.rot_margin.p, R * sizeof(float), hipMemcpyDeviceToHost));
  if (hdiag) HIPCHK(hipMemcpy(hdiag, h.hdiag.p, h.n * sizeof(float), hipMemcpyDeviceToHost));
  if (core_ids && h.core)
    HIPCHK(hipMemcpy(core_ids, h.core_ids.p, h.core * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (hcore && h.core)
    HIPCHK(hipMemcpy(hcore, h.hcore.p, h.core * h.core * sizeof(float), hipMemcpyDeviceToHost));
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_import(int64_t n, int32_t k, int64_t core_size, int32_t num_stages,
                          const int64_t* stage_sizes, const int64_t* stage_clusters,
                          const int64_t* cluster_sizes, const int32_t* rot_ids,
                          const float* rot_o, const int32_t* rot_retired, const float* hdiag,
                          const int32_t* core_ids, const float* hcore, void* stream,
                          mmf_handle* out) {
  ABI_BEGIN
  g_err.clear();
  if (!out) raise(MMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || (k != 2 && k != 3) || core_size < 1 || core_size > n || num_stages < 0)
    raise(MMF_EINVAL, "bad sizes");
  if (num_stages > 0 && (!stage_sizes || !stage_clusters || !cluster_sizes || !rot_ids ||
                         !rot_o || !rot_retired))
    raise(MMF_EINVAL, "missing stage or rotation arrays");
  if (!hdiag || !core_ids || !hcore) raise(MMF_EINVAL, "missing H arrays");
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  auto h = std::make_unique<mmf_plan>();
  h->n = n;
  h->core = core_size;
  h->k = k;
  h->stream = s;
  h->R = n - core_size;
  h->prm.k = k;
  h->prm.core_size = core_size;
  const int64_t R = h->R;
  std::vector<int32_t> loc(std::max<int64_t>(R, 1) * 3, -1), gidv(std::max<int64_t>(R, 1) * 3, -1),
      ret(std::max<int64_t>(R, 1), 0);
  std::vector<float> ob(std::max<int64_t>(R, 1) * 9, 0.f), th(std::max<int64_t>(R, 1), 0.f);
  std::vector<int32_t> active(n);
  for (int64_t i = 0; i < n; ++i) active[i] = (int32_t)i;
  std::vector<int32_t> pos_of(n, -1);
  int64_t rbase = 0, cbase = 0;
  std::vector<uint8_t> retired(n, 0);
  for (int32_t p = 0; p < num_stages; ++p) {
    const int64_t S = stage_sizes[p];
    const int64_t Snext = p + 1 < num_stages ? stage_sizes[p + 1] : core_size;
    if (S != (int64_t)active.size() || Snext >= S) raise(MMF_EINVAL, "inconsistent stage sizes");
    SchedStage sc;
    sc.size = S;
    sc.t = S - Snext;
    const int64_t m = stage_clusters[p];
    std::vector<int32_t> off(m + 1, 0);
    for (int64_t u = 0; u < m; ++u) {
      sc.sizes.push_back((int32_t)cluster_sizes[cbase + u]);
      off[u + 1] = off[u] + (int32_t)cluster_sizes[cbase + u];
    }
    if (off[m] != S) raise(MMF_EINVAL, "cluster sizes do not add up to the stage size");
    cbase += m;
    for (int64_t q = 0; q < S; ++q) pos_of[active[q]] = (int32_t)q;
    sc.rcnt.assign(m, 0);
    int64_t last_u = 0;
    for (int64_t r = rbase; r < rbase + sc.t; ++r) {
      const int32_t q0 = pos_of[rot_ids[r * k]];
      if (q0 < 0) raise(MMF_EINVAL, "rotation touches an inactive index");
      const int64_t u = std::upper_bound(off.begin(), off.end(), q0) - off.begin() - 1;
      if (u < last_u) raise(MMF_EINVAL, "rotations are not grouped by cluster");
      last_u = u;
      sc.rcnt[u] += 1;
      for (int a = 0; a < k; ++a) {
        const int32_t g = rot_ids[r * k + a];
        const int32_t q = pos_of[g];
        if (q < off[u] || q >= off[u + 1]) raise(MMF_EINVAL, "rotation crosses clusters");
        loc[r * 3 + a] = q - off[u];
        gidv[r * 3 + a] = g;
        for (int b = 0; b < k; ++b) ob[r * 9 + a * 3 + b] = rot_o[(r * k + a) * k + b];
      }
      ret[r] = rot_retired[r];
      if (pos_of[ret[r]] < 0 || retired[ret[r]]) raise(MMF_EINVAL, "bad retired index");
      retired[ret[r]] = 1;
      if (k == 2) th[r] = std::atan2(rot_o[(r * 2 + 1) * 2 + 0], rot_o[(r * 2 + 0) * 2 + 0]);
    }
    auto sdp = std::make_unique<StageDev>();
    StageDev& sd = *sdp;
    build_stage_geometry(sd, sc, rbase, s);
    std::vector<int32_t> next(S), gid(S);
    std::vector<int32_t> nact;
    for (int64_t q = 0; q < S; ++q) {
      const int32_t g = active[q];
      gid[q] = g;
      if (retired[g]) {
        next[q] = -g - 1;
      } else {
        next[q] = (int32_t)nact.size();
        nact.push_back(g);
      }
    }
    if ((int64_t)nact.size() != Snext) raise(MMF_EINVAL, "retirements do not match stage sizes");
    upload(sd.next, next, s);
    upload(sd.gid, gid, s);
    for (int64_t q = 0; q < S; ++q) pos_of[active[q]] = -1;
    active.swap(nact);
    rbase += sc.t;
    h->st.push_back(std::move(sdp));
  }
  if (rbase != R) raise(MMF_EINVAL, "rotation count does not equal n - core_size");
  upload(h->rot_loc, loc, s);
  upload(h->rot_gid, gidv, s);
  upload(h->rot_o, ob, s);
  upload(h->rot_ret, ret, s);
  upload(h->theta, th, s);
  h->rot_margin.ensure(std::max<int64_t>(R, 1) * sizeof(float));
  HIPCHK(hipMemsetAsync(h->rot_margin.p, 0, std::max<int64_t>(R, 1) * sizeof(float), s));
  for (auto& sp : h->st) {
    StageDev& sd = *sp;
    sd.sw_loc.ensure(sd.t * k * sizeof(int32_t));
    sd.sw_o.ensure(sd.t * k * k * sizeof(float));
    HIPCHK(pmmf::launch_levelize(sd.m, k, sd.off.as<int32_t>(), sd.rcnt.as<int32_t>(),
                                 sd.roff.as<int32_t>(), sd.rot_base, h->rot_loc.as<int32_t>(),
                                 h->rot_o.as<float>(), nullptr, sd.lvl_stride,
                                 sd.lvl_ptr.as<int32_t>(),
                                 sd.depth.as<int32_t>(), sd.sw_loc.as<int32_t>(),
                                 sd.sw_o.as<float>(), sd.sw_idx.as<int32_t>(),
                                 h->theta.as<float>(), round_cmax(sd.cmax), s));
  }
  std::vector<float> hd(hdiag, hdiag + n), hc(hcore, hcore + core_size * core_size);
  std::vector<int32_t> cid(core_ids, core_ids + core_size);
  std::vector<uint8_t> flag(n, 0);
  for (int32_t g : cid) {
    if (g < 0 || g >= n || flag[g]) raise(MMF_EINVAL, "bad core ids");
    flag[g] = 1;
  }
  upload(h->hdiag, hd, s);
  upload(h->hcore, hc, s);
  upload(h->core_ids, cid, s);
  upload(h->is_core, flag, s);
  HIPCHK(hipStreamSynchronize(s));
  for (auto& sp : h->st) {
    std::vector<int32_t> dep(sp->m);
    HIPCHK(hipMemcpy(dep.data(), sp->depth.p, sp->m * sizeof(int32_t), hipMemcpyDeviceToHost));
    sp->depth_max = 0;
    for (int32_t d : dep) sp->depth_max = std::max(sp->depth_max, d);
  }
  h->info.n = n;
  h->info.core_size = core_size;
  h->info.k = k;
  h->info.num_stages = num_stages;
  h->info.num_rotations = R;
  init_params3(*h, s);
  *out = h.release();
  register_handle(*out);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_param_ptrs(mmf_handle hh, float** theta, float** hdiag, float** hcore) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  if (theta) *theta = h.theta.as<float>();
  if (hdiag) *hdiag = h.hdiag.as<float>();
  if (hcore) *hcore = h.hcore.as<float>();
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_sync_angles(mmf_handle hh, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  h.inv_ready = false;
  h.isqrt_ready = false;
  ++h.version;
  sync_rotations(h, s);
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_set_params(mmf_handle hh, const float* d_theta, const float* d_hdiag,
                              const float* d_hcore, void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  pmmf_alloc::StreamScope alloc_scope(stream);
  hipStream_t s = as_stream(stream);
  h.inv_ready = false;
  h.isqrt_ready = false;
  ++h.version;
  if (d_hdiag)
    HIPCHK(hipMemcpyAsync(h.hdiag.p, d_hdiag, h.n * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (d_hcore && h.core)
    HIPCHK(hipMemcpyAsync(h.hcore.p, d_hcore, h.core * h.core * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
  if (d_theta && h.R) {
    const int64_t na = h.R * (h.k == 3 ? 3 : 1);
    HIPCHK(hipMemcpyAsync(h.theta.p, d_theta, na * sizeof(float), hipMemcpyDeviceToDevice, s));
    sync_rotations(h, s);
  }
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_get_params(mmf_handle hh, float* d_theta, float* d_hdiag, float* d_hcore,
                              void* stream) {
  ABI_BEGIN
  mmf_plan& h = *checked(hh);
  hipStream_t s = as_stream(stream);
  if (d_hdiag)
    HIPCHK(hipMemcpyAsync(d_hdiag, h.hdiag.p, h.n * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (d_hcore && h.core)
    HIPCHK(hipMemcpyAsync(d_hcore, h.hcore.p, h.core * h.core * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
  if (d_theta && h.R)
    HIPCHK(hipMemcpyAsync(d_theta, h.theta.p, h.R * (h.k == 3 ? 3 : 1) * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
  return MMF_OK;
  ABI_END
}

extern "C" int mmf_destroy(mmf_handle hh) {
  ABI_BEGIN
  checked(hh);
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(hh);
  }
  // the handle's buffers may still be read by work on any stream (products run on the caller's
  // streams), and a released block is reused at once by later work on the stream it is released
  // with: wait for the whole device before releasing them
  (void)hipDeviceSynchronize();
  delete hh;
  return MMF_OK;
  ABI_END
}
