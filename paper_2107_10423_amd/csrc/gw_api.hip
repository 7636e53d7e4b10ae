// Host side of libgw: the C-ABI of include/gw.h, the per-molecule context,
// the stage-A pipeline (Pi build -> blocked Cholesky -> W^c table), the
// batched residue solver driver and the quasiparticle step tree.
//
// Method: Mejia-Rodriguez et al., "Scalable Molecular GW Calculations:
// Valence and Core Spectra", Implementation - Contour Deformation, Algorithm 1
// and Implementation - Solution of the Quasiparticle Equations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gw.h"
#include "../../include/gw_audit.h"
#include "gw_internal.h"

using namespace gw;

namespace {

thread_local std::string g_err;
std::atomic<bool> g_contexts_created{false};

// Host-side trace of every stage, to stderr, when GW_TRACE is set.
bool trace_on() {
  static const bool on = getenv("GW_TRACE") != nullptr;
  return on;
}
void trace(const char* fmt, ...) {
  if (!trace_on()) return;
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "[gw] ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  fflush(stderr);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  // GW_TRACE_ERRORS=1: every error is also printed where it arises (worker
  // threads of the request server included)
  static const bool show = [] {
    const char* e = getenv("GW_TRACE_ERRORS");
    return e && *e && *e != '0';
  }();
  if (show || trace_on()) fprintf(stderr, "gw: error %d: %s\n", code, buf);
  return code;
}

// GW_DEBUG_SYNC=1: every runtime call and launch is followed by a device
// synchronisation, so an asynchronous fault is reported at the call that
// caused it (graphs are then off: a capture cannot synchronise)
bool debug_sync() {
  static const bool on = [] {
    const char* e = getenv("GW_DEBUG_SYNC");
    return e && atoi(e) != 0;
  }();
  return on;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ == hipSuccess && debug_sync() && !gw::audit_mode()) e_ = hipDeviceSynchronize();  \
    if (e_ != hipSuccess)                                                                    \
      return fail(GW_EDEVICE, "%s failed: %s [%s] (%s:%d)", #expr, hipGetErrorString(e_),    \
                  gw::launch_error(), __FILE__, __LINE__);                                   \
  } while (0)

#define RCHK(expr)            \
  do {                        \
    int r_ = (expr);          \
    if (r_ != 0) return r_;   \
  } while (0)

// Runtime calls go through these wrappers.  In launch-audit mode (see
// include/gw_audit.h) device buffers are host memory, copies are memcpy and
// nothing is launched; the kernel wrappers only run their bounds guards.
hipError_t rt_malloc(void** p, size_t bytes) {
  if (audit_mode()) {
    size_t b = (bytes + 255) / 256 * 256;
    *p = aligned_alloc(256, b);
    if (!*p) return hipErrorOutOfMemory;
    memset(*p, 0, b);
    return hipSuccess;
  }
  return hipMalloc(p, bytes);
}
void rt_free(void* p) {
  if (audit_mode()) free(p);
  else hipFree(p);
}
hipError_t rt_memcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st) {
  if (audit_mode()) {
    if (bytes) memcpy(dst, src, bytes);
    return hipSuccess;
  }
  return hipMemcpyAsync(dst, src, bytes, kind, st);
}
hipError_t rt_memcpy2d(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                       size_t height, hipMemcpyKind kind, hipStream_t st) {
  if (audit_mode()) {
    for (size_t r = 0; r < height; ++r)
      memcpy((char*)dst + r * dpitch, (const char*)src + r * spitch, width);
    return hipSuccess;
  }
  return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, kind, st);
}
hipError_t rt_memset(void* p, int v, size_t bytes, hipStream_t st) {
  if (audit_mode()) {
    memset(p, v, bytes);
    return hipSuccess;
  }
  return hipMemsetAsync(p, v, bytes, st);
}
hipError_t rt_sync(hipStream_t st) { return audit_mode() ? hipSuccess : hipStreamSynchronize(st); }

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Default residue systems per MINRES batch.  At (H2O)30 (rounds of about 400
// systems) the stage took 262 ms with 384, 273 with 256, 290 with 320, 283
// with 448 and 512: a batch of 384 runs on three 128-row pass tiles, and the
// few systems left over form a second, short batch.
constexpr int MINRES_BATCH = 384;
inline long round_up_l(long x, long m) { return (x + m - 1) / m * m; }

constexpr int PANEL = 128;  // Cholesky panel width (matches chol.hip)

// Split counts of the two MINRES operator passes for kp systems: about 1024
// workgroups each.  Pass 1 (64 x 64 tiles over n_ov, split over N_aux, at
// least 4 K-steps per split); pass 2 (64 x 128 tiles over N_aux, split over
// n_ov, at least 16 K-steps per split).
void minres_splits(int kp, int Np, int Kp, int* splitk, int* splitk1) {
  // K chunks of about `chunk2` (pass 2) and `chunk1` (pass 1) elements bound the
  // latency chain of each workgroup; GW_TUNE_MINRES="chunk1,chunk2" replaces
  // the rule below by those chunks
  int chunk1 = 384, chunk2 = 4096;
  const int t1 = (kp / 64) * (Kp / 64);
  const int t2 = (kp / 64) * (Np / 128);
  if (const char* e = getenv("GW_TUNE_MINRES")) {
    if (sscanf(e, "%d,%d", &chunk1, &chunk2) == 2) {
      chunk1 = std::max(16, chunk1);
      chunk2 = std::max(16, chunk2);
      *splitk = std::max(1, std::min(Kp / chunk2, Kp / 16));
      *splitk1 = std::max(1, std::min(Np / chunk1, Np / 16));
      return;
    }
  }
  // pass 2 (kp x N_aux outputs): about 1024 workgroups, or K chunks of about
  // chunk2 where that makes more; pass 1 is split only when its kp x N_ov
  // outputs make fewer than 2048 tiles
  *splitk = std::max(1, std::min(std::max(1024 / std::max(t2, 1), Kp / chunk2), Kp / 64));
  *splitk1 = t1 >= 2048 ? 1 : std::max(1, std::min(Np / chunk1, Np / 16));
}

// Split-K slabs of the preconditioner product r M^-1 (K = Np, a multiple of
// 128, so each slab's K range is a multiple of 16)
constexpr int PRE_SPLIT = 8;

// Residue systems the dense fallback builds and solves at once (one
// workgroup each): the fallback's workspace is FB_MAX dielectric matrices
constexpr int FB_MAX = 32;

// Elements of the MINRES partial-product buffer for a capacity of kp systems.
// The splits follow the capacity, and a smaller capacity can need more (the
// first pass is split over N_aux only while it has few tiles), so the buffer
// and the footprint take the largest need of every capacity up to kp.
size_t minres_part_elems(int kp, int Np, int Kp) {
  size_t part = 0;
  for (int q = 64; q <= std::max(kp, 64); q += 64) {
    int splitk = 1, splitk1 = 1;
    minres_splits(q, Np, Kp, &splitk, &splitk1);
    part = std::max({part, (size_t)splitk * q * Np, (size_t)(Kp / 64) * q,
                     (size_t)splitk1 * q * Kp, (size_t)PRE_SPLIT * q * Np});
  }
  return part;
}

long lower_tile_count(int tiles_m, int tiles_n, int BM, int BN) {
  long n = 0;
  for (int I = 0; I < tiles_m; ++I) {
    int c = ((I + 1) * BM - 1) / BN + 1;
    n += std::min(c, tiles_n);
  }
  return n;
}

// Residue system of one Sigma evaluation
struct System {
  int q;        // row of the right-hand side in the padded R buffer (r * n_mo + m)
  double w;     // real frequency eps_m - omega
  double tol;   // MINRES residual target relative to |b| (0: the context default)
};

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st = nullptr;
  void start(hipStream_t s) {
    st = s;
    if (!audit_mode()) hipEventRecord(a, st);
  }
  double stop() {
    if (audit_mode()) return 0.0;
    hipEventRecord(b, st);
    hipEventSynchronize(b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    return ms;
  }
};

}  // namespace

// Block cache for the contexts a server creates: device blocks and pinned host
// blocks freed by a context go to per-size free lists and are handed out again
// to later contexts, so that requests of recurring shapes run without
// hipMalloc / hipFree (hipFree waits for the whole device) once the cache is
// warm.  Blocks are returned to the runtime only when a new allocation would
// exceed the cap, and when the cache is destroyed.
struct gw_devcache {
  std::mutex mu;
  std::multimap<size_t, void*> free_dev, free_host;
  std::map<void*, size_t> size_of;     // every block handed out or cached -> its size
  size_t cap = 0;                      // device bytes (live + cached) the cache may hold
  size_t live = 0, cached = 0;
  long n_malloc = 0, n_free = 0, n_hits = 0;

  // Size classes: multiples of 256 B below 1 MiB; above, eight classes per
  // octave (m 2^(e-3), m = 8..15: at most 12.5% over the request), so that
  // requests of neighbouring shapes share classes and the blocks of every
  // shape a server sees fit in the cache together.  GW_CACHE_CLASSES=fine
  // keeps 64 KiB steps above 1 MiB instead.
  static size_t round(size_t b) {
    b = std::max<size_t>(b, 8);
    if (b < (1u << 20)) return (b + 255) / 256 * 256;
    static const bool fine = [] {
      const char* e = getenv("GW_CACHE_CLASSES");
      return e && strcmp(e, "fine") == 0;
    }();
    if (fine) return (b + (64u << 10) - 1) / (64u << 10) * (64u << 10);
    int e = 63 - __builtin_clzll((unsigned long long)b);   // 2^e <= b < 2^(e+1)
    const size_t step = (size_t)1 << (e - 3);
    return (b + step - 1) / step * step;
  }
  // a block of exactly this size class: a recurring sequence of allocations
  // (the same request shapes again) then finds every block it needs, which a
  // best fit that lets one class take another's block does not guarantee
  static void* take(std::multimap<size_t, void*>& fl, size_t want, size_t* got) {
    auto it = fl.find(want);
    if (it == fl.end()) return nullptr;
    void* p = it->second;
    *got = it->first;
    fl.erase(it);
    return p;
  }
  hipError_t get_dev(void** p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    const size_t want = round(bytes);
    size_t got = 0;
    if ((*p = take(free_dev, want, &got))) {
      cached -= got;
      live += got;
      ++n_hits;
      if (audit_mode()) memset(*p, 0, got);   // as fresh audit-mode memory (no kernel runs)
      return hipSuccess;
    }
    while (live + cached + want > cap && !free_dev.empty()) {   // make room: largest first
      auto last = std::prev(free_dev.end());
      rt_free(last->second);
      size_of.erase(last->second);
      cached -= last->first;
      ++n_free;
      free_dev.erase(last);
    }
    trace("block cache: new device block of %zu bytes", want);
    hipError_t e = rt_malloc(p, want);
    if (e != hipSuccess && !free_dev.empty()) {   // the runtime is short: drop the rest
      (void)hipGetLastError();
      for (auto& kv : free_dev) {
        rt_free(kv.second);
        size_of.erase(kv.second);
        ++n_free;
      }
      free_dev.clear();
      cached = 0;
      e = rt_malloc(p, want);
    }
    if (e != hipSuccess) return e;
    ++n_malloc;
    size_of[*p] = want;
    live += want;
    return hipSuccess;
  }
  void put_dev(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = size_of.find(p);
    if (it == size_of.end()) return;
    live -= it->second;
    cached += it->second;
    free_dev.emplace(it->second, p);
  }
  hipError_t get_host(void** p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    const size_t want = round(bytes);
    size_t got = 0;
    if ((*p = take(free_host, want, &got))) {
      ++n_hits;
      return hipSuccess;
    }
    trace("block cache: new pinned block of %zu bytes", want);
    if (audit_mode()) {
      *p = calloc(want, 1);
      if (!*p) return hipErrorOutOfMemory;
    } else {
      hipError_t e = hipHostMalloc(p, want, hipHostMallocDefault);
      if (e != hipSuccess) return e;
    }
    ++n_malloc;
    size_of[*p] = want;
    return hipSuccess;
  }
  void put_host(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = size_of.find(p);
    if (it != size_of.end()) free_host.emplace(it->second, p);
  }
  ~gw_devcache() {
    for (auto& kv : free_dev) rt_free(kv.second);
    for (auto& kv : free_host) {
      if (audit_mode()) free(kv.second);
      else hipHostFree(kv.second);
    }
  }
};

namespace {
// pinned host memory of a context: from its cache, else the runtime
hipError_t host_alloc(gw_devcache* cache, void** p, size_t bytes) {
  if (cache) return cache->get_host(p, bytes);
  if (audit_mode()) {
    *p = calloc(bytes, 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}
void host_free(gw_devcache* cache, void* p) {
  if (!p) return;
  if (cache) cache->put_host(p);
  else if (audit_mode()) free(p);
  else hipHostFree(p);
}
}  // namespace

struct gw_ctx {
  // device and pinned host blocks come from this cache when set (server contexts)
  gw_devcache* cache = nullptr;
  // sizes
  int n_mo = 0, n_occ = 0, n_virt = 0, n_aux = 0, n_rows = 0;
  // spins: 1 (closed shell) or 2 (open shell, up then down); per-spin
  // occupations; levels, dsig_x and state names run over n_spin * n_mo
  // spin-orbitals (sigma * n_mo + n)
  int n_spin = 1;
  int n_occ_s[2] = {0, 0};
  int Np = 0;      // n_aux padded to 128
  int Kov = 0;     // n_occ * n_virt
  int Kp = 0;      // Kov padded to 128
  int nR = 0;      // n_rows * n_mo
  int Rp = 0;      // nR padded to 128
  // options
  int pi_prec = GW_PI_FP64;
  int wc_prec = GW_PI_FP64;    // W^c contraction: FP64 GEMM, or the BF16x3 form
  int minres_max_iter = 200;
  double minres_rtol = 1e-12;
  double qp_tol = 1e-10;
  int qp_max_iter = 100;
  double cluster_width = 0.0;  // > 0: cluster initial-guess layer
  int minres_batch = MINRES_BATCH;  // systems per MINRES batch (bounds the workspace)
  size_t mem_budget = 0, work_budget = 16ull << 30;
  size_t mem_used = 0;
  // host copies: eps_ks are the mean-field eigenvalues (the QP equation's
  // constant term); eps the energies in G (the poles of G in the residue set,
  // the residue frequencies and the quadrature), equal to eps_ks except while
  // gw_evgw runs; d_eps mirrors eps, d_D holds the transition energies of W
  std::vector<double> eps_ks, eps, dsig_x;
  std::vector<int> row_ids;
  std::vector<int> row_spin;   // spin of each row
  std::map<int, int> row_of;
  // stream
  hipStream_t st = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;    // stage timers
  hipEvent_t ev0b = nullptr, ev1b = nullptr;  // whole-call timer
  hipEvent_t evk[4] = {nullptr, nullptr, nullptr, nullptr};  // Pi / W^c kernel launches
  // MINRES convergence polling: per-iteration active counts land in pinned
  // host memory and are read one iteration late, so the host never idles the GPU
  hipEvent_t ev_poll[2] = {nullptr, nullptr};
  int* h_poll = nullptr;
  hipEvent_t ev_quad[2] = {nullptr, nullptr};   // brackets the imaginary-axis quadrature
  // pinned host staging for the small per-round transfers (QP frequencies in,
  // Sigma parts out; MINRES parameters in, results out), so that they are
  // plain DMA commands on the stream and a QP round synchronises once;
  // stage_off is where the MINRES region starts (after the Sigma region)
  char* h_stage = nullptr;
  size_t h_stage_cap = 0, stage_off = 0;
  // MINRES iterations 2, 3, ... replay a captured graph per (padded batch,
  // iteration parity); valid while the MINRES workspace is not reallocated
  std::map<int, std::array<hipGraphExec_t, 2>> mr_graphs;
  bool graphs_off = false;     // opts.no_graphs, or the stream cannot be captured
  void drop_graphs() {
    for (auto& kv : mr_graphs)
      for (hipGraphExec_t g : kv.second)
        if (g) hipGraphExecDestroy(g);
    mr_graphs.clear();
  }
  // device data
  double* d_eps = nullptr;
  double* d_D = nullptr;       // [Kp]
  double* d_Bov = nullptr;     // [Np][Kp]
  double* d_R = nullptr;       // [Rp][Np]
  double* d_bn = nullptr;      // [Rp]
  // mixed-precision copies of B_ov (lazily built)
  float* d_B32 = nullptr;
  uint16_t* d_Bhi = nullptr;
  uint16_t* d_Blo = nullptr;
  // stage-A workspace
  double* d_work = nullptr;
  size_t work_bytes = 0;
  int chunk = 0;
  double* d_Linv = nullptr;
  int* d_info = nullptr;
  double* d_scale = nullptr;   // [chunk][Kp]
  float* d_scale32 = nullptr;  // [chunk][Kp], the same scales rounded for the mixed builds
  double* d_parts = nullptr;   // [chunk][Np/128][Rp] squared-norm partials
  // mixed W^c contraction: R split once, F = L^-1 - I split per grid point
  uint16_t* d_Rh = nullptr;    // [Rp][Np] (hi; lo follows at Rp Np)
  uint16_t* d_F = nullptr;     // [2][f_cap][Np][Np] (hi block, then lo block)
  int f_cap = 0;
  double* d_grid = nullptr;    // [2][Gmax]
  int grid_cap = 0;
  // W^c table cache
  double* d_wtab = nullptr;    // [nR][wtab_G]
  int wtab_G = 0;              // table columns
  int quad_G = 0;              // quadrature points (wtab_G, or wtab_G - 1 with wtab_w0)
  int wtab_w0 = 0;             // the table was built with xi = 0 as its last point
  bool wtab_w0col = false;     // ... and its last column holds W^c(0)
  int quad_split = 0;          // the quadrature integrates the W^c(0) part exactly (evGW)
  // MINRES preconditioner M^-1 = (1 - Pi(0))^-1, formed from the xi = 0 point
  // of a table build; systems with |omega| < pre_w use it
  bool no_precond = false;
  bool pre_valid = false;
  double* d_pre = nullptr;     // [Np][Np]
  double pre_w = 0.0;
  bool test_indefinite = false;
  bool wtab_valid = false;
  std::vector<double> wtab_xi, wtab_w;
  int wtab_prec = -1;
  int wtab_wcprec = -1;
  // Sigma quadrature buffers
  int* d_rowsel = nullptr;
  int* d_rowspin = nullptr;      // [n_rows] (open shell only)
  double* d_omega = nullptr;
  double* d_sig = nullptr;
  double* d_dsig = nullptr;
  double* d_sigpart = nullptr;   // [n][16][2] quadrature partial sums
  char* d_mrin = nullptr;        // MINRES parameters [omega | rtol | rhs index | warm |
                                 // preconditioned], cap each
  char* d_mrout = nullptr;       // MINRES results [W^c | dW^c | convergence], cap each
  int sig_cap = 0;
  // MINRES workspace
  MinresBufs mr{};
  int mr_cap = 0;       // kp capacity
  int mr_splitk = 1;    // split-K of the B_ov V^T pass
  int mr_splitk1 = 1;   // split over N_aux of the B_ov^T v pass
  size_t part_cap = 0;  // doubles
  int* d_rhs_idx = nullptr;
  int* d_warm = nullptr;       // [kp] 1 when the system starts from the cached solution
  double* d_xcache = nullptr;  // [Rp][Np] last solution of each right-hand side row
  std::vector<char> xvalid;    // host flags: d_xcache row holds a solution of this call
  double* d_wc = nullptr;
  double* d_dwc = nullptr;
  int* d_conv = nullptr;
  // spectral-decomposition route (built on first use; dropped when the
  // transition energies change)
  bool sd_valid = false;
  double* d_sdM = nullptr;     // [Kp][Kp] Casida matrix, diagonalised in place
  double* d_sdT = nullptr;     // [Kp][Kp] its eigenvectors (columns)
  double* d_sdV = nullptr;     // [Kp/64][64][64] rotations of one Jacobi round
  double* d_sdY = nullptr;     // [Rp][Kp] R B_ov, then the pole strengths rho
  double* d_sdRho = nullptr;   // [Rp][Kp]
  double* d_sdO = nullptr;     // [Kp] Omega
  double* d_sdPart = nullptr;  // [2][SD_NORM_BLOCKS]
  int sd_sweeps = 0;
  // dense fallback workspace
  double* d_dense = nullptr;
  double* d_dscale = nullptr;
  double* d_db = nullptr;
  int* d_dinfo = nullptr;
  int* d_dpiv = nullptr;
  gw_timing timing{};

  std::vector<void*> allocs;

  int alloc(void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (mem_budget && mem_used + bytes > mem_budget)
      return fail(GW_ENOMEM, "device memory budget exceeded: need %zu more bytes, %zu of %zu used",
                  bytes, mem_used, mem_budget);
    hipError_t e = cache ? cache->get_dev(p, bytes) : rt_malloc(p, bytes);
    if (e != hipSuccess) return fail(GW_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    allocs.push_back(*p);
    mem_used += bytes;
    alloc_sizes[*p] = bytes;
    return 0;
  }
  void release(void* p) {
    if (!p) return;
    auto it = alloc_sizes.find(p);
    if (it != alloc_sizes.end()) {
      mem_used -= it->second;
      alloc_sizes.erase(it);
    }
    allocs.erase(std::remove(allocs.begin(), allocs.end(), p), allocs.end());
    if (cache) cache->put_dev(p);
    else rt_free(p);
  }
  // elements of size `elem` reachable from p inside its allocation (0 if none)
  long ext(const void* p, size_t elem) const {
    if (!p) return 0;
    auto it = alloc_sizes.upper_bound(const_cast<void*>(p));
    if (it == alloc_sizes.begin()) return 0;
    --it;
    const char* base = (const char*)it->first;
    const char* q = (const char*)p;
    if (q < base || q >= base + it->second) return 0;
    return (long)((size_t)(base + it->second - q) / elem);
  }
  std::map<void*, size_t> alloc_sizes;

  ~gw_ctx() {
    if (st) hipStreamSynchronize(st);
    drop_graphs();
    for (void* p : allocs) {
      if (cache) cache->put_dev(p);
      else rt_free(p);
    }
    for (hipEvent_t e : {ev0, ev1, ev0b, ev1b, ev_poll[0], ev_poll[1], ev_quad[0], ev_quad[1],
                         evk[0], evk[1], evk[2], evk[3]})
      if (e) hipEventDestroy(e);
    host_free(cache, h_stage);
    host_free(cache, h_poll);
    if (own_stream && st) hipStreamDestroy(st);
  }
};

namespace {

template <class T>
int ensure(gw_ctx* c, T** p, size_t count, size_t* cap_bytes = nullptr) {
  size_t bytes = count * sizeof(T);
  if (*p && cap_bytes && *cap_bytes >= bytes) return 0;
  if (*p) c->release(*p);
  *p = nullptr;
  RCHK(c->alloc(reinterpret_cast<void**>(p), bytes));
  if (cap_bytes) *cap_bytes = bytes;
  return 0;
}

// GEMM launch with operand extents taken from the context's allocation map
int run_gemm(gw_ctx* c, GemmArgs a, int kind, int la, int lb, int epi) {
  trace("gemm kind=%d la=%d lb=%d epi=%d tiles=%dx%d n=%d batch=%d split=%d K=%d", kind, la, lb,
        epi, a.tiles_m, a.tiles_n, a.n_tiles, a.batch, a.splitk, a.K);
  a.nA = c->ext(a.A, sizeof(double));
  a.nB = c->ext(a.B, sizeof(double));
  a.nS = c->ext(a.scale, sizeof(double));
  a.nC = c->ext(a.C, sizeof(double));
  a.nD = c->ext(a.Dvec, sizeof(double));
  a.nW = c->ext(a.wrow, sizeof(double));
  HIPCHK(gemm_f64(a, kind, la, lb, epi, c->st));
  return 0;
}

// ---------------------------------------------------------------------------
// Stage A: W^c table for a grid

int ensure_mixed_operands(gw_ctx* c);
int pi_build_chunk(gw_ctx* c, int G, long per_g, long ldA);

// Stage-A layout of one grid point: rows [0, Np) the dielectric matrix (then
// L), rows [Np, 2 Np) the identity (then L^-T), 128 rows and 128 columns of
// padding that tiles overrunning a 64-aligned edge may touch.
inline long work_ld(const gw_ctx* c) { return c->Np + 128; }
inline long work_per_g(const gw_ctx* c) { return (2L * c->Np + 128) * work_ld(c); }
inline int parts_ld(const gw_ctx* c) { return c->Rp; }
inline long parts_per_g(const gw_ctx* c) { return (long)(c->Np / 128) * c->Rp; }

int setup_work(gw_ctx* c, int G) {
  const long per_g = work_per_g(c);
  size_t per_bytes = (size_t)per_g * sizeof(double) + (size_t)c->Kp * (sizeof(double) + sizeof(float)) +
                     PANEL * PANEL * sizeof(double) + (size_t)parts_per_g(c) * sizeof(double);
  if (c->wc_prec == GW_PI_BF16X3) per_bytes += (size_t)c->Np * c->Np * 2 * sizeof(uint16_t);
  const int chunk = (int)std::min<size_t>(std::max<size_t>(1, c->work_budget / per_bytes),
                                          (size_t)std::max(G, 1));
  if (c->d_work && c->chunk >= chunk) return 0;
  if (c->d_work) c->release(c->d_work);
  if (c->d_Linv) c->release(c->d_Linv);
  if (c->d_info) c->release(c->d_info);
  if (c->d_scale) c->release(c->d_scale);
  if (c->d_scale32) c->release(c->d_scale32);
  if (c->d_parts) c->release(c->d_parts);
  c->d_work = nullptr;
  c->d_Linv = nullptr;
  c->d_info = nullptr;
  c->d_scale = nullptr;
  c->d_scale32 = nullptr;
  c->d_parts = nullptr;
  RCHK(c->alloc((void**)&c->d_work, (size_t)per_g * chunk * sizeof(double)));
  RCHK(c->alloc((void**)&c->d_parts, (size_t)parts_per_g(c) * chunk * sizeof(double)));
  HIPCHK(rt_memset(c->d_work, 0, (size_t)per_g * chunk * sizeof(double), c->st));
  RCHK(c->alloc((void**)&c->d_Linv, (size_t)chunk * PANEL * PANEL * sizeof(double)));
  RCHK(c->alloc((void**)&c->d_info, (size_t)chunk * sizeof(int)));
  RCHK(c->alloc((void**)&c->d_scale, (size_t)chunk * c->Kp * sizeof(double)));
  RCHK(c->alloc((void**)&c->d_scale32, (size_t)chunk * c->Kp * sizeof(float)));
  c->chunk = chunk;
  return 0;
}

int upload_grid(gw_ctx* c, int n, const double* xi, const double* w) {
  if (n > c->grid_cap) {
    if (c->d_grid) c->release(c->d_grid);
    c->d_grid = nullptr;
    RCHK(c->alloc((void**)&c->d_grid, 2 * (size_t)n * sizeof(double)));
    c->grid_cap = n;
  }
  HIPCHK(rt_memcpy(c->d_grid, xi, n * sizeof(double), hipMemcpyHostToDevice, c->st));
  HIPCHK(rt_memcpy(c->d_grid + c->grid_cap, w, n * sizeof(double), hipMemcpyHostToDevice,
                        c->st));
  return 0;
}

int check_grid(const gw_grid* grid) {
  if (!grid || grid->n < 1 || !grid->xi || !grid->w)
    return fail(GW_EINVAL, "grid must have n >= 1 and non-NULL xi, w");
  for (int g = 0; g < grid->n; ++g)
    if (!(std::isfinite(grid->xi[g]) && std::isfinite(grid->w[g]) && grid->xi[g] >= 0.0))
      return fail(GW_EINVAL, "grid point %d is not finite and non-negative", g);
  return 0;
}

// Pi build of `G` grid points (scales already in d_scale) into the work buffer
int pi_build_chunk(gw_ctx* c, int G, long per_g, long ldA) {
  if (c->pi_prec == GW_PI_FP64) {
    GemmArgs a{};
    a.A = c->d_Bov; a.lda = c->Kp; a.sA = 0;
    a.B = c->d_Bov; a.ldb = c->Kp; a.sB = 0;
    a.scale = c->d_scale; a.sS = c->Kp;
    a.C = c->d_work; a.ldc = ldA; a.sC = per_g;
    a.M = c->Np; a.N = c->Np; a.K = c->Kp;
    a.row0 = 0; a.col0 = 0; a.k0 = 0;
    a.map = MAP_LOWER;
    a.tiles_m = c->Np / 128; a.tiles_n = c->Np / 128;
    a.n_tiles = (int)lower_tile_count(a.tiles_m, a.tiles_n, 128, 128);
    a.batch = G; a.splitk = 1; a.sSplit = 0;
    RCHK(run_gemm(c, a, 0, KC, KC, EPI_ONE_PLUS_4));
    return 0;
  }
  RCHK(ensure_mixed_operands(c));
  if (c->pi_prec == GW_PI_FP32) {
    HIPCHK(pi_build_f32(c->d_B32, c->Kp, c->d_scale32, c->Kp, c->d_work, ldA, per_g, c->Np,
                        c->Kp, G, c->ext(c->d_B32, 4), c->ext(c->d_scale32, 4),
                        c->ext(c->d_work, 8), c->st));
    return 0;
  }
  const long nB = std::min({c->ext(c->d_Bhi, 2), c->ext(c->d_Blo, 2), c->ext(c->d_B32, 4)});
  HIPCHK(pi_build_bf16x3(c->d_Bhi, c->d_Blo, c->Kp, c->d_B32, c->d_scale32, c->Kp, c->d_work,
                         ldA, per_g, c->Np, c->Kp, G, nB, c->ext(c->d_scale32, 4),
                         c->ext(c->d_work, 8), c->st));
  return 0;
}

// Operands of the mixed W^c contraction: R split once per context, the F
// buffer sized for the current chunk.
int ensure_r_split(gw_ctx* c) {
  if (!c->d_Rh) {
    const size_t n = (size_t)c->Rp * c->Np;
    RCHK(c->alloc((void**)&c->d_Rh, 2 * n * sizeof(uint16_t)));
    HIPCHK(split_bf16(c->d_R, c->d_Rh, c->d_Rh + n, nullptr, (long)n, c->st));
  }
  return 0;
}

int ensure_wc_mixed(gw_ctx* c) {
  RCHK(ensure_r_split(c));
  if (c->f_cap < c->chunk) {
    if (c->d_F) c->release(c->d_F);
    c->d_F = nullptr;
    c->f_cap = 0;
    RCHK(c->alloc((void**)&c->d_F, 2 * (size_t)c->chunk * c->Np * c->Np * sizeof(uint16_t)));
    c->f_cap = c->chunk;
  }
  return 0;
}

int ensure_mixed_operands(gw_ctx* c) {
  const size_t n = (size_t)c->Np * c->Kp;
  if (!c->d_B32) {
    RCHK(c->alloc((void**)&c->d_B32, n * sizeof(float)));
    RCHK(c->alloc((void**)&c->d_Bhi, n * sizeof(uint16_t)));
    RCHK(c->alloc((void**)&c->d_Blo, n * sizeof(uint16_t)));
    HIPCHK(split_bf16(c->d_Bov, c->d_Bhi, c->d_Blo, c->d_B32, (long)n, c->st));
  }
  return 0;
}

// Blocked left-looking Cholesky of every item of the chunk over the rows
// [0, Np) of 1 - Pi and the appended identity rows; panel k carries the
// appended rows up to Np + k + PANEL only (the later ones are still unit rows
// that the panel does not touch).
// deferred: the pivot flags are left in d_info for the caller to read (no host
// synchronisation, no memset: the sequence can be captured into a graph)
int cholesky_chunk(gw_ctx* c, int G, long per_g, long ldA, bool deferred = false) {
  const int Np = c->Np;
  if (deferred) HIPCHK(fill_int(c->d_info, G, 0, c->ext(c->d_info, 4), c->st));
  else HIPCHK(rt_memset(c->d_info, 0, G * sizeof(int), c->st));
  if (c->test_indefinite)
    HIPCHK(reflect_unit(c->d_work, ldA, per_g, Np, G, c->ext(c->d_work, 8), c->st));
  HIPCHK(set_identity_rows(c->d_work, ldA, per_g, Np, Np, Np, G, c->ext(c->d_work, 8), c->st));
  // Left-looking (Crout) panels over the augmented rows: panel k is first
  // brought up to date with every factored column to its left (one GEMM with
  // K = k over rows [k, Np + k); identity row Np + s is zero left of column s,
  // so its tile starts its k loop at s), then its diagonal block is factored
  // and inverted, then the rows below are solved against that block.  Only
  // the panel is read-modified-written per step, never the trailing matrix.
  for (int k = 0; k < Np; k += PANEL) {
    trace("cholesky panel k=%d", k);
    if (k > 0) {  // P[r][k:k+128] -= L[r][0:k] L[k:k+128][0:k]^T, r in [k, Np + k)
      GemmArgs a{};
      a.A = c->d_work; a.lda = ldA; a.sA = per_g;
      a.B = c->d_work; a.ldb = ldA; a.sB = per_g;
      a.C = c->d_work; a.ldc = ldA; a.sC = per_g;
      a.K = k; a.row0 = k; a.col0 = k; a.k0 = 0; a.kb0 = 0;
      a.klo_from = Np;
      a.map = MAP_FULL;
      a.tiles_m = Np / 64; a.tiles_n = 1;
      a.M = Np; a.N = PANEL;
      a.n_tiles = a.tiles_m; a.batch = G; a.splitk = 1;
      a.alpha = -1.0; a.beta = 1.0;
      RCHK(run_gemm(c, a, 2, KC, KC, EPI_AXPBY));
    }
    HIPCHK(chol_diag(c->d_work, ldA, per_g, c->d_Linv, k, G, c->d_info, c->ext(c->d_work, 8),
                     c->ext(c->d_Linv, 8), c->ext(c->d_info, 4), c->st));
    const int rows_below = Np;  // rows [k + PANEL, Np + k + PANEL)
    {  // panel solve: L[i][k:k+128] = P[i][k:k+128] Linv_kk^T
      GemmArgs a{};
      a.A = c->d_work; a.lda = ldA; a.sA = per_g;
      a.B = c->d_Linv; a.ldb = PANEL; a.sB = PANEL * PANEL;
      a.C = c->d_work + k; a.ldc = ldA; a.sC = per_g;
      a.K = PANEL; a.row0 = k + PANEL; a.col0 = 0; a.k0 = k; a.kb0 = 0;
      a.map = MAP_FULL;
      a.tiles_m = (rows_below + 63) / 64; a.tiles_n = 1;
      a.M = a.tiles_m * 64; a.N = PANEL;
      a.n_tiles = a.tiles_m; a.batch = G; a.splitk = 1;
      a.alpha = 1.0; a.beta = 0.0;
      RCHK(run_gemm(c, a, 2, KC, KC, EPI_AXPBY));
    }
  }
  if (deferred) return 0;
  std::vector<int> info(G);
  HIPCHK(rt_memcpy(info.data(), c->d_info, G * sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(rt_sync(c->st));
  for (int g = 0; g < G; ++g)
    if (info[g] != 0)
      return fail(GW_ENOTSPD, "1 - Pi(i xi) is not positive definite (item %d, pivot %d)", g,
                  info[g]);
  return 0;
}

// Copy the leading n_aux x n_aux block of each chunk item to host memory and
// zero its strict upper triangle (only the lower triangle is maintained).
int copy_out_blocks(gw_ctx* c, double* dst, int Gc, long per_g, long ldA) {
  const int n = c->n_aux;
  for (int g = 0; g < Gc; ++g)
    HIPCHK(rt_memcpy2d(dst + (size_t)g * n * n, n * sizeof(double), c->d_work + g * per_g,
                            ldA * sizeof(double), n * sizeof(double), n, hipMemcpyDeviceToHost,
                            c->st));
  HIPCHK(rt_sync(c->st));
  for (int g = 0; g < Gc; ++g)
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) dst[(size_t)g * n * n + (size_t)i * n + j] = 0.0;
  return 0;
}

// Build the W^c table for `grid` unless cached.  mode: 0 normal; 1/2 write
// the dielectric matrix / Cholesky factor of each point to `dbg_out`.
// with_w0 (mode 0): one more column, W^c at xi = 0, for the split quadrature.
// need_w0_col: the W^c(0) column itself is read (evGW); otherwise the xi = 0
// point serves the preconditioner only and its W^c GEMM is skipped.
int build_wtable(gw_ctx* c, const gw_grid* grid_in, int mode = 0, double* dbg_out = nullptr,
                 bool with_w0 = false, bool need_w0_col = false) {
  RCHK(check_grid(grid_in));
  std::vector<double> ext_xi, ext_w;
  gw_grid ext = *grid_in;
  if (with_w0) {
    ext_xi.assign(grid_in->xi, grid_in->xi + grid_in->n);
    ext_w.assign(grid_in->w, grid_in->w + grid_in->n);
    ext_xi.push_back(0.0);
    ext_w.push_back(0.0);
    ext.n = grid_in->n + 1;
    ext.xi = ext_xi.data();
    ext.w = ext_w.data();
  }
  const gw_grid* grid = &ext;
  const int G = grid->n;
  if (mode == 0 && c->wtab_valid && c->wtab_G == G && c->wtab_w0 == (int)with_w0 &&
      (!need_w0_col || c->wtab_w0col) && c->wtab_prec == c->pi_prec &&
      c->wtab_wcprec == c->wc_prec &&
      std::equal(grid->xi, grid->xi + G, c->wtab_xi.begin()) &&
      std::equal(grid->w, grid->w + G, c->wtab_w.begin())) {
    c->timing.wtab_cached = 1;
    return 0;
  }
  c->timing.wtab_cached = 0;
  RCHK(setup_work(c, G));
  RCHK(upload_grid(c, G, grid->xi, grid->w));
  if (mode == 0) {
    if (c->d_wtab && c->wtab_G < G) {
      c->release(c->d_wtab);
      c->d_wtab = nullptr;
    }
    if (!c->d_wtab) {
      RCHK(c->alloc((void**)&c->d_wtab, (size_t)std::max(c->nR, 1) * G * sizeof(double)));
    }
    c->wtab_valid = false;
  }
  const long ldA = work_ld(c);
  const long per_g = work_per_g(c);
  Timer tm;
  tm.a = c->ev0; tm.b = c->ev1;
  double pi_ms = 0, chol_ms = 0, wt_ms = 0;
  for (int g0 = 0; g0 < G; g0 += c->chunk) {
    const int Gc = std::min(c->chunk, G - g0);
    trace("stage A mode=%d g0=%d Gc=%d prec=%d Np=%d Kp=%d Rp=%d", mode, g0, Gc, c->pi_prec, c->Np,
          c->Kp, c->Rp);
    tm.start(c->st);
    HIPCHK(make_scale_imag(c->d_D, c->Kov, c->Kp, c->d_grid + g0, Gc, c->d_scale,
                           c->pi_prec == GW_PI_FP64 ? nullptr : c->d_scale32, c->ext(c->d_D, 8),
                           G - g0, c->ext(c->d_scale, 8), c->ext(c->d_scale32, 4), c->st));
    if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[0], c->st));
    RCHK(pi_build_chunk(c, Gc, per_g, ldA));
    if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[1], c->st));
    pi_ms += tm.stop();
    if (!audit_mode()) {
      float kms = 0.f;
      HIPCHK(hipEventElapsedTime(&kms, c->evk[0], c->evk[1]));
      c->timing.pi_kernel_ms += kms;
    }
    c->timing.pi_launches++;
    if (mode == 1) {
      RCHK(copy_out_blocks(c, dbg_out + (size_t)g0 * c->n_aux * c->n_aux, Gc, per_g, ldA));
      continue;
    }
    tm.start(c->st);
    RCHK(cholesky_chunk(c, Gc, per_g, ldA));
    chol_ms += tm.stop();
    if (mode == 2) {
      RCHK(copy_out_blocks(c, dbg_out + (size_t)g0 * c->n_aux * c->n_aux, Gc, per_g, ldA));
      continue;
    }
    tm.start(c->st);
    // items of this chunk whose W^c column is formed (the xi = 0 point, last,
    // only when its column is read)
    const int Gw = (with_w0 && !need_w0_col && g0 + Gc == G) ? Gc - 1 : Gc;
    if (c->nR > 0 && Gw > 0 && c->wc_prec == GW_PI_BF16X3) {
      // 2 b^T y + |y|^2, y = (L^-1 - I) b, in BF16x3 products: F split from
      // the k-major L^-T rows, then one contraction with the split R
      RCHK(ensure_wc_mixed(c));
      const long nRR = (long)c->Rp * c->Np;
      const long sF = (long)c->Np * c->Np;
      const long nF = (long)c->f_cap * sF;
      uint16_t* Fh = c->d_F;
      uint16_t* Fl = c->d_F + nF;
      HIPCHK(split_linv(c->d_work + (long)c->Np * ldA, ldA, per_g, c->Np, Gw, Fh, Fl, sF,
                        c->ext(c->d_work + (long)c->Np * ldA, 8), nF, c->st));
      if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[2], c->st));
      HIPCHK(wc_bf16x3(c->d_Rh, c->d_Rh + nRR, c->Np, c->Rp, Fh, Fl, sF, c->Np, Gw, c->d_parts,
                       parts_ld(c), parts_per_g(c), nRR, nF, c->ext(c->d_parts, 8), c->st));
      if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[3], c->st));
      HIPCHK(wc_from_parts(c->d_parts, parts_per_g(c), wc_bf16x3_panels(c->Np), parts_ld(c),
                           nullptr, c->nR,
                           Gw, G, g0, c->d_wtab, c->ext(c->d_parts, 8), 0, c->ext(c->d_wtab, 8),
                           c->st));
    } else if (c->nR > 0 && Gw > 0) {
      // |L^-1 b|^2 for every b = (P|nm): rows of R times L^-T (k-major rows
      // Np.. of the work buffer), k limited to the lower triangle
      GemmArgs a{};
      a.A = c->d_R; a.lda = c->Np; a.sA = 0;
      a.B = c->d_work + (long)c->Np * ldA; a.ldb = ldA; a.sB = per_g;
      a.C = c->d_parts; a.ldc = parts_ld(c); a.sC = parts_per_g(c);
      a.M = c->Rp; a.N = c->Np; a.K = c->Np;
      a.map = MAP_FULL_J; a.tiles_m = c->Rp / 128; a.tiles_n = c->Np / 128;
      a.n_tiles = a.tiles_m * a.tiles_n; a.batch = Gw; a.splitk = 1; a.ktri = 1;
      if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[2], c->st));
      RCHK(run_gemm(c, a, 0, KC, KM, EPI_SQNORM));
      if (!audit_mode()) HIPCHK(hipEventRecord(c->evk[3], c->st));
      HIPCHK(wc_from_parts(c->d_parts, parts_per_g(c), c->Np / 128, parts_ld(c), c->d_bn, c->nR,
                           Gw, G, g0, c->d_wtab, c->ext(c->d_parts, 8), c->ext(c->d_bn, 8),
                           c->ext(c->d_wtab, 8), c->st));
    }
    wt_ms += tm.stop();
    if (c->nR > 0 && Gw > 0) {
      if (!audit_mode()) {
        float kms = 0.f;
        HIPCHK(hipEventElapsedTime(&kms, c->evk[2], c->evk[3]));
        c->timing.wc_kernel_ms += kms;
      }
      c->timing.wc_launches++;
    }
  }
  if (mode == 0 && with_w0 && !c->no_precond) {
    // the xi = 0 point is the last one, still in the work buffer after the
    // last chunk: its rows [Np, 2 Np) hold X = L0^-T, and M^-1 = X X^T
    const int g_last = G - 1 - ((G - 1) / c->chunk) * c->chunk;
    if (!c->d_pre) RCHK(c->alloc((void**)&c->d_pre, (size_t)c->Np * c->Np * sizeof(double)));
    const double* X = c->d_work + (long)g_last * per_g + (long)c->Np * ldA;
    GemmArgs a{};
    a.A = X; a.lda = ldA; a.sA = 0;
    a.B = X; a.ldb = ldA; a.sB = 0;
    a.C = c->d_pre; a.ldc = c->Np; a.sC = 0;
    a.M = c->Np; a.N = c->Np; a.K = c->Np;
    a.map = MAP_FULL; a.tiles_m = c->Np / 64; a.tiles_n = c->Np / 128;
    a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1; a.splitk = 1;
    a.alpha = 1.0; a.beta = 0.0;
    RCHK(run_gemm(c, a, 2, KC, KC, EPI_AXPBY));
    // preconditioned window: |omega| below 0.9 of the lowest transition
    // energy, where 1 - Pi(omega) stays positive definite and close to M
    double dmin = INFINITY;
    for (int sp = 0; sp < c->n_spin; ++sp) {
      const double* e = c->eps.data() + (size_t)sp * c->n_mo;
      const int no = c->n_occ_s[sp];
      dmin = std::min(dmin, *std::min_element(e + no, e + c->n_mo) -
                                *std::max_element(e, e + no));
    }
    c->pre_w = 0.9 * dmin;
    c->pre_valid = true;
  }
  c->timing.pi_ms += pi_ms;
  c->timing.chol_ms += chol_ms;
  c->timing.wtab_ms += wt_ms;
  if (mode == 0) {
    c->wtab_valid = true;
    c->wtab_G = G;
    c->wtab_w0 = with_w0 ? 1 : 0;
    c->wtab_w0col = with_w0 && need_w0_col;
    c->quad_G = with_w0 ? G - 1 : G;
    c->wtab_prec = c->pi_prec;
    c->wtab_wcprec = c->wc_prec;
    c->wtab_xi.assign(grid->xi, grid->xi + G);
    c->wtab_w.assign(grid->w, grid->w + G);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Residues: batched MINRES with dense fallback

// Pinned staging of at least `bytes`.  Growing it first drains the stream
// (copies into the old buffer complete) and carries the old contents over, so
// callers re-derive their pointers from h_stage after this call.
int ensure_stage(gw_ctx* c, size_t bytes) {
  if (bytes <= c->h_stage_cap) return 0;
  HIPCHK(rt_sync(c->st));
  const size_t cap = std::max<size_t>(64 << 10, 2 * bytes);
  char* p = nullptr;
  if (host_alloc(c->cache, (void**)&p, cap) != hipSuccess)
    return fail(GW_ENOMEM, "pinned host allocation of %zu bytes failed", cap);
  if (c->h_stage) {
    memcpy(p, c->h_stage, c->h_stage_cap);
    host_free(c->cache, c->h_stage);
  }
  c->h_stage = p;
  c->h_stage_cap = cap;
  return 0;
}


// Padded size of a batch of k residue systems: whole 64-row tiles, and whole
// 128-row tiles above 256 so that large batches run the 128 x 128 pass tiles
// (padding rows are 16-row blocks past the batch, whose MFMAs are skipped).
inline int mr_kp(int k) {
  const int kp = round_up(k, 64);
  return kp > 256 ? round_up(k, 128) : kp;
}

// Staging bytes of one MINRES batch of kp systems: rhs index, warm flag,
// frequency, tolerance in; W^c, dW^c, convergence out.
inline size_t mr_stage_bytes(int cap) { return (size_t)cap * (4 + 4 + 4 + 8 + 8 + 8 + 8 + 4); }

int ensure_minres(gw_ctx* c, int kp) {
  if (kp <= c->mr_cap) return 0;
  c->drop_graphs();
  MinresBufs& m = c->mr;
  void* olds[] = {m.x, m.w, m.w2, m.r1, m.r2, m.y, m.v, m.x0, m.scal, m.V, m.part, m.active,
                  m.blk, c->d_mrin, c->d_mrout};
  for (void* p : olds) c->release(p);
  const size_t vec = (size_t)kp * c->Np;
  double** vecs[] = {&m.x, &m.w, &m.w2, &m.r1, &m.r2, &m.y, &m.v, &m.x0};
  for (double** p : vecs) RCHK(c->alloc((void**)p, vec * sizeof(double)));
  RCHK(c->alloc((void**)&m.scal, (size_t)kp * 16 * sizeof(double)));
  RCHK(c->alloc((void**)&m.V, (size_t)kp * c->Kp * sizeof(double)));
  // split-K partials: aim for about 1024 workgroups in both operator passes
  int splitk = 1, splitk1 = 1;
  minres_splits(kp, c->Np, c->Kp, &splitk, &splitk1);
  c->mr_splitk = splitk;
  c->mr_splitk1 = splitk1;
  const size_t part = minres_part_elems(kp, c->Np, c->Kp);
  RCHK(c->alloc((void**)&m.part, part * sizeof(double)));
  c->part_cap = part;
  RCHK(c->alloc((void**)&m.active, 2 * sizeof(int)));
  RCHK(c->alloc((void**)&m.blk, 2 * (size_t)(kp / 16) * sizeof(int)));
  // parameters and results each in one block, moved by one copy per batch
  RCHK(c->alloc((void**)&c->d_mrin, (size_t)kp * (2 * sizeof(double) + 3 * sizeof(int))));
  m.omega = (double*)c->d_mrin;
  m.rtol = m.omega + kp;
  c->d_rhs_idx = (int*)(m.rtol + kp);
  c->d_warm = c->d_rhs_idx + kp;
  m.preflag = c->d_warm + kp;
  RCHK(c->alloc((void**)&c->d_mrout, (size_t)kp * (2 * sizeof(double) + sizeof(int))));
  c->d_wc = (double*)c->d_mrout;
  c->d_dwc = c->d_wc + kp;
  c->d_conv = (int*)(c->d_dwc + kp);
  c->mr_cap = kp;
  return 0;
}

// mask (nullable): per 16-system block, 0 where every system's vector is zero
// Tiles of the MINRES operator passes for a batch of kp systems: 128 x 128
// (kind 0) for kp a multiple of 128 from 256 systems up, else the 64 x 64
// first pass (kind 3) and 64 x 128 back-projection (kind 2).  Measured: at
// (H2O)30 the stage takes 281 against 289 ms with the larger tiles; at
// (H2O)10 (kp 128) 6.51 against 6.41 ms, so small batches keep the 64-row
// tiles.  GW_TUNE_MINRES_TILE=0 / 1: never / whenever kp is a multiple of 128.
bool mr_wide_tiles(int kp) {
  static const int mode = [] {
    const char* e = getenv("GW_TUNE_MINRES_TILE");
    return e ? atoi(e) : -1;
  }();
  if (kp % 128 != 0) return false;
  return mode < 0 ? kp >= 256 : mode == 1;
}

// Partials of the derivative pass: one per column tile of the first pass
inline int deriv_parts(const gw_ctx* c, int kp) {
  return mr_wide_tiles(kp) ? c->Kp / 128 : c->Kp / 64;
}

int matvec_pass(gw_ctx* c, const double* X, int kp, int epi, double* out, long ldc,
                const int* mask = nullptr) {
  const bool wide = mr_wide_tiles(kp);
  const int T = wide ? 128 : 64, kind = wide ? 0 : 3;
  // out = scale(X B_ov): rows = systems, cols = ia.  The system tiles that
  // read one B_ov column panel are adjacent in the launch order (and so run
  // together on one XCD), so the panel comes from HBM once, not kp / 64 times
  GemmArgs a{};
  a.A = X; a.lda = c->Np; a.sA = 0;
  a.B = c->d_Bov; a.ldb = c->Kp; a.sB = 0;
  a.C = out; a.ldc = ldc; a.sC = 0;
  a.M = kp; a.N = c->Kp; a.K = c->Np;
  a.map = MAP_FULL_J; a.tiles_m = kp / T; a.tiles_n = c->Kp / T;
  a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1; a.splitk = 1;
  a.mrows = mask ? 0 : c->mr.k;   // a mask also marks the padding systems
  a.rowmask = mask; a.nMask = c->ext(mask, sizeof(int));
  a.Dvec = c->d_D; a.wrow = c->mr.omega;
  if (epi == EPI_RES_SCALE && c->mr_splitk1 > 1) {
    // split over N_aux for parallelism: partials, then a deterministic sum + scale
    a.C = c->mr.part; a.ldc = c->Kp; a.splitk = c->mr_splitk1; a.sSplit = (long)kp * c->Kp;
    RCHK(run_gemm(c, a, kind, KC, KM, EPI_STORE));
    HIPCHK(minres_scale_sum(c->mr, c->mr_splitk1, c->d_D, c->ext(c->d_D, 8), mask,
                            c->ext(mask, sizeof(int)), c->st));
    return 0;
  }
  RCHK(run_gemm(c, a, kind, KC, KM, epi));
  return 0;
}

int backproject_pass(gw_ctx* c, int kp, const int* mask = nullptr) {
  // part[s][sys][P] = sum_{ia in split s} V[sys][ia] B_ov[P][ia]
  GemmArgs a{};
  a.A = c->mr.V; a.lda = c->Kp; a.sA = 0;
  a.B = c->d_Bov; a.ldb = c->Kp; a.sB = 0;
  a.C = c->mr.part; a.ldc = c->Np; a.sC = 0;
  a.M = kp; a.N = c->Np; a.K = c->Kp;
  const bool wide = mr_wide_tiles(kp);
  a.map = MAP_FULL; a.tiles_m = kp / (wide ? 128 : 64); a.tiles_n = c->Np / 128;
  a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1;
  a.splitk = c->mr_splitk; a.sSplit = (long)kp * c->Np;
  a.mrows = mask ? 0 : c->mr.k;
  a.rowmask = mask; a.nMask = c->ext(mask, sizeof(int));
  RCHK(run_gemm(c, a, wide ? 0 : 2, KC, KC, EPI_STORE));
  return 0;
}

// part[s] = X M^-1 over the K slab s (X [kp][Np], M^-1 symmetric, so its rows
// serve as the B operand); mask as for the operator passes
int precond_pass(gw_ctx* c, const double* X, int kp, const int* mask = nullptr) {
  GemmArgs a{};
  a.A = X; a.lda = c->Np; a.sA = 0;
  a.B = c->d_pre; a.ldb = c->Np; a.sB = 0;
  a.C = c->mr.part; a.ldc = c->Np; a.sC = 0;
  a.M = kp; a.N = c->Np; a.K = c->Np;
  a.map = MAP_FULL; a.tiles_m = kp / 64; a.tiles_n = c->Np / 128;
  a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1;
  a.splitk = PRE_SPLIT; a.sSplit = (long)kp * c->Np;
  a.mrows = mask ? 0 : c->mr.k;
  a.rowmask = mask; a.nMask = c->ext(mask, sizeof(int));
  RCHK(run_gemm(c, a, 2, KC, KC, EPI_STORE));
  return 0;
}

// One MINRES iteration: both operator passes (from the second iteration on
// skipping the 16-system blocks the previous step found converged), the apply
// and step kernels (with a preconditioner, the product r2 M^-1 between two
// step kernels), and the copy of this iteration's count of active systems to
// pinned host memory.  Its launches depend on the iteration only through its
// parity.
int minres_iteration(gw_ctx* c, int kp, int itn) {
  MinresBufs& m = c->mr;
  const int par = itn & 1;
  const int* mask = itn > 1 ? m.blk + (par ^ 1) * (kp / 16) : nullptr;
  RCHK(matvec_pass(c, m.v, kp, EPI_RES_SCALE, m.V, c->Kp, mask));
  RCHK(backproject_pass(c, kp, mask));
  HIPCHK(minres_apply(m, c->mr_splitk, mask, c->ext(mask, sizeof(int)), c->st));
  if (m.pre) {
    HIPCHK(minres_pre_step_a(m, par, c->st));
    RCHK(precond_pass(c, m.r2, kp, mask));
    HIPCHK(minres_pre_step_b(m, par, c->st));
  } else {
    HIPCHK(minres_finish_step(m, par, c->st));
  }
  HIPCHK(rt_memcpy(c->h_poll + par, m.active + par, sizeof(int), hipMemcpyDeviceToHost, c->st));
  return 0;
}

// The same iteration (itn >= 2) replayed from a graph captured on first use.
// A stream that refuses capture switches the context to eager launches.
int minres_iteration_graph(gw_ctx* c, int kp, int itn) {
  const int par = itn & 1;
  // value-initialised: no graphs yet; the launch sequence depends on whether
  // a preconditioner is in use
  auto& slot = c->mr_graphs[2 * kp + (c->mr.pre ? 1 : 0)];
  if (!slot[par]) {
    if (hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      c->graphs_off = true;
      return minres_iteration(c, kp, itn);
    }
    const int rc = minres_iteration(c, kp, itn);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->st, &g);
    if (rc != 0 || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      if (rc != 0) return rc;
      HIPCHK(e);
    }
    const hipError_t ei = hipGraphInstantiate(&slot[par], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHK(ei);
    trace("minres graph captured kp=%d parity=%d", kp, par);
  }
  HIPCHK(hipGraphLaunch(slot[par], c->st));
  return 0;
}

// Solve all systems; fills wc, dwc (host) and iteration counts (negative if
// not converged by MINRES; fallback marks them solved when enabled).
int solve_residues_batch(gw_ctx* c, const std::vector<System>& sys, bool use_fallback,
                         std::vector<double>& wc, std::vector<double>& dwc, std::vector<int>& iters,
                         std::vector<double>* x_out);

// Systems are solved in batches of at most minres_batch, which bounds the
// MINRES workspace of a context.
int solve_residues(gw_ctx* c, const std::vector<System>& sys, bool use_fallback,
                   std::vector<double>& wc, std::vector<double>& dwc, std::vector<int>& iters,
                   std::vector<double>* x_out = nullptr) {
  const int k = (int)sys.size();
  const int cap = c->minres_batch;
  if (k <= cap) return solve_residues_batch(c, sys, use_fallback, wc, dwc, iters, x_out);
  wc.assign(k, 0.0);
  dwc.assign(k, 0.0);
  iters.assign(k, 0);
  if (x_out) x_out->assign((size_t)k * c->n_aux, 0.0);
  for (int j0 = 0; j0 < k; j0 += cap) {
    const int j1 = std::min(k, j0 + cap);
    std::vector<System> part(sys.begin() + j0, sys.begin() + j1);
    std::vector<double> a, b, xs;
    std::vector<int> it;
    RCHK(solve_residues_batch(c, part, use_fallback, a, b, it, x_out ? &xs : nullptr));
    std::copy(a.begin(), a.end(), wc.begin() + j0);
    std::copy(b.begin(), b.end(), dwc.begin() + j0);
    std::copy(it.begin(), it.end(), iters.begin() + j0);
    if (x_out) std::copy(xs.begin(), xs.end(), x_out->begin() + (size_t)j0 * c->n_aux);
  }
  return 0;
}

int solve_residues_batch(gw_ctx* c, const std::vector<System>& sys, bool use_fallback,
                         std::vector<double>& wc, std::vector<double>& dwc, std::vector<int>& iters,
                         std::vector<double>* x_out) {
  const int k = (int)sys.size();
  wc.assign(k, 0.0);
  dwc.assign(k, 0.0);
  iters.assign(k, 0);
  if (k == 0) return 0;
  const int kp = mr_kp(k);
  RCHK(ensure_minres(c, kp));
  MinresBufs& m = c->mr;
  m.k = k; m.kp = kp; m.Np = c->Np; m.Kp = c->Kp;
  m.n_vec = std::min({c->ext(m.x, 8), c->ext(m.w, 8), c->ext(m.w2, 8), c->ext(m.r1, 8),
                      c->ext(m.r2, 8), c->ext(m.y, 8), c->ext(m.v, 8), c->ext(m.x0, 8)});
  m.n_scal = c->ext(m.scal, 8);
  m.n_part = c->ext(m.part, 8);
  m.n_V = c->ext(m.V, 8);
  m.n_blk = c->ext(m.blk, sizeof(int));
  m.pre = (c->pre_valid && !c->no_precond) ? c->d_pre : nullptr;
  m.splitp = PRE_SPLIT;
  // host mirror of the device parameter and result blocks (same layout)
  const int cap = c->mr_cap;
  RCHK(ensure_stage(c, c->stage_off + mr_stage_bytes(cap)));
  char* h_in = c->h_stage + c->stage_off;
  double* om = (double*)h_in;
  double* tol = om + cap;
  int* idx = (int*)(tol + cap);
  int* warm = idx + cap;
  int* pref = warm + cap;
  char* h_out = (char*)(pref + cap);
  double* h_wc = (double*)h_out;
  double* h_dwc = h_wc + cap;
  int* h_conv = (int*)(h_dwc + cap);
  const size_t in_bytes = (size_t)cap * (2 * sizeof(double) + 3 * sizeof(int));
  const size_t out_bytes = (size_t)cap * (2 * sizeof(double) + sizeof(int));
  for (int j = 0; j < kp; ++j) {
    idx[j] = j < k ? sys[j].q : 0;
    om[j] = j < k ? sys[j].w : 0.0;
    tol[j] = (j < k && sys[j].tol > 0) ? std::max(sys[j].tol, c->minres_rtol) : c->minres_rtol;
    // preconditioned window (a device flag, so replayed graphs read the current one)
    pref[j] = (m.pre && j < k && std::fabs(sys[j].w) < c->pre_w) ? 1 : 0;
  }
  Timer tm;
  tm.a = c->ev0; tm.b = c->ev1;
  tm.start(c->st);

  trace("minres k=%d kp=%d splitk=%d", k, kp, c->mr_splitk);
  // warm start: a right-hand side solved earlier in this call starts from that
  // solution; one operator pass gives A x0 for the start vector b - A x0
  if (!c->d_xcache) {
    RCHK(c->alloc((void**)&c->d_xcache, (size_t)c->Rp * c->Np * sizeof(double)));
    c->xvalid.assign(c->Rp, 0);
  }
  int n_warm = 0;
  for (int j = 0; j < kp; ++j) {
    warm[j] = (j < k && c->xvalid[idx[j]]) ? 1 : 0;
    n_warm += warm[j];
  }
  const long n_cache = c->ext(c->d_xcache, 8);
  HIPCHK(rt_memcpy(c->d_mrin, h_in, in_bytes, hipMemcpyHostToDevice, c->st));
  HIPCHK(minres_gather(m, c->d_xcache, c->d_rhs_idx, idx, c->Rp, c->d_warm, n_cache, c->st));
  if (n_warm > 0) {
    RCHK(matvec_pass(c, m.v, kp, EPI_RES_SCALE, m.V, c->Kp));
    RCHK(backproject_pass(c, kp));
    HIPCHK(minres_apply(m, c->mr_splitk, nullptr, 0, c->st));
  }
  if (m.pre) {
    // preconditioned start: r = b - A x0, |b| and beta1 in the M^-1 norm
    HIPCHK(minres_pre_init_a(m, c->d_R, c->d_rhs_idx, idx, c->Rp, n_warm > 0, c->st));
    RCHK(precond_pass(c, m.w, kp));
    HIPCHK(minres_pre_init_b(m, c->st));
    RCHK(precond_pass(c, m.r1, kp));
    HIPCHK(minres_pre_init_c(m, c->st));
  } else {
    HIPCHK(minres_init(m, c->d_R, c->d_rhs_idx, idx, c->Rp, n_warm > 0, c->st));
  }
  int itn = 0;
  // Each iteration's count of still-active systems is copied to pinned host
  // memory behind its step kernel; the host reads iteration i's count after
  // queueing iteration i + 1, so polling never drains the stream and at most
  // one extra iteration (with every system frozen by the step kernel) runs.
  for (itn = 1; itn <= c->minres_max_iter; ++itn) {
    if (itn >= 2 && !c->graphs_off && !audit_mode())
      RCHK(minres_iteration_graph(c, kp, itn));
    else
      RCHK(minres_iteration(c, kp, itn));
    if (!audit_mode()) HIPCHK(hipEventRecord(c->ev_poll[itn & 1], c->st));
    if (itn > 1) {
      const int prev = (itn - 1) & 1;
      if (!audit_mode()) HIPCHK(hipEventSynchronize(c->ev_poll[prev]));
      if (c->h_poll[prev] == 0) break;
    }
  }
  c->timing.minres_iters += std::min(itn, c->minres_max_iter);
  c->timing.minres_systems += k;
  trace("minres done k=%d iterations=%d warm=%d", k, std::min(itn, c->minres_max_iter), n_warm);
  // x = x0 + correction; remember it for later solves of the same right-hand side
  HIPCHK(minres_finalize(m, c->d_xcache, c->d_rhs_idx, idx, c->Rp, n_cache, c->st));
  for (int j = 0; j < k; ++j) c->xvalid[idx[j]] = 1;
  // derivative partials: sum over ia of (B^T x)^2 * 2 D w/(D^2 - w^2)^2
  const int nparts = deriv_parts(c, kp);
  RCHK(matvec_pass(c, m.x, kp, EPI_RES_DERIV, m.part, kp));
  HIPCHK(minres_results(m, c->d_R, c->d_rhs_idx, c->Rp, nparts, c->d_wc, c->d_dwc, c->d_conv,
                        c->ext(c->d_wc, 8), c->st));
  HIPCHK(rt_memcpy(h_out, c->d_mrout, out_bytes, hipMemcpyDeviceToHost, c->st));
  HIPCHK(rt_sync(c->st));
  c->timing.minres_ms += tm.stop();
  std::copy(h_wc, h_wc + k, wc.begin());
  std::copy(h_dwc, h_dwc + k, dwc.begin());
  std::copy(h_conv, h_conv + k, iters.begin());

  if (audit_mode())  // no results exist; walk the fallback launches for every system
    for (int j = 0; j < k; ++j) iters[j] = -1;
  std::vector<int> bad;
  for (int j = 0; j < k; ++j)
    if (iters[j] < 0) bad.push_back(j);
  if (!bad.empty() && use_fallback) {
    tm.start(c->st);
    const long ld = c->Np, sq = (long)c->Np * c->Np;
    if (!c->d_dense) {   // room for FB_MAX systems at once (counted in the footprint)
      RCHK(c->alloc((void**)&c->d_dense, (size_t)FB_MAX * sq * sizeof(double)));
      RCHK(c->alloc((void**)&c->d_dscale, (size_t)FB_MAX * c->Kp * sizeof(double)));
      RCHK(c->alloc((void**)&c->d_db, (size_t)FB_MAX * c->Np * sizeof(double)));
      RCHK(c->alloc((void**)&c->d_dinfo, FB_MAX * sizeof(int)));
      RCHK(c->alloc((void**)&c->d_dpiv, (size_t)FB_MAX * c->Np * sizeof(int)));
    }
    for (size_t j0 = 0; j0 < bad.size(); j0 += FB_MAX) {
      const int nb = (int)std::min<size_t>(FB_MAX, bad.size() - j0);
      for (int i = 0; i < nb; ++i) {
        const System& y = sys[bad[j0 + i]];
        double* sc = c->d_dscale + (long)i * c->Kp;
        HIPCHK(make_scale_real(c->d_D, c->Kov, c->Kp, y.w, sc, c->ext(c->d_D, 8),
                               c->ext(sc, 8), c->st));
        HIPCHK(copy_vec(c->d_R + (long)y.q * c->Np, c->d_db + (long)i * c->Np, c->Np,
                        c->ext(c->d_R + (long)y.q * c->Np, 8),
                        c->ext(c->d_db + (long)i * c->Np, 8), c->st));
      }
      GemmArgs a{};   // 1 - Pi(w) of every system of the batch, full matrices
      a.A = c->d_Bov; a.lda = c->Kp;
      a.B = c->d_Bov; a.ldb = c->Kp;
      a.scale = c->d_dscale; a.sS = c->Kp;
      a.C = c->d_dense; a.ldc = ld; a.sC = sq;
      a.M = c->Np; a.N = c->Np; a.K = c->Kp;
      a.map = MAP_FULL; a.tiles_m = c->Np / 128; a.tiles_n = c->Np / 128;
      a.n_tiles = a.tiles_m * a.tiles_n; a.batch = nb; a.splitk = 1;
      RCHK(run_gemm(c, a, 0, KC, KC, EPI_ONE_PLUS_4));
      HIPCHK(rt_memset(c->d_dinfo, 0, nb * sizeof(int), c->st));
      HIPCHK(dense_solve(c->d_dense, ld, sq, c->Np, c->d_db, c->Np, c->d_dpiv, c->Np,
                         c->d_dinfo, nb, c->ext(c->d_dense, 8), c->ext(c->d_db, 8),
                         c->ext(c->d_dpiv, 4), c->ext(c->d_dinfo, 4), c->st));
      for (int i = 0; i < nb; ++i) {
        const int j = bad[j0 + i];
        const double* xb = c->d_db + (long)i * c->Np;
        HIPCHK(copy_vec(xb, m.x + (long)j * c->Np, c->Np, c->ext(xb, 8),
                        c->ext(m.x + (long)j * c->Np, 8), c->st));
        HIPCHK(copy_vec(xb, c->d_xcache + (long)sys[j].q * c->Np, c->Np, c->ext(xb, 8),
                        c->ext(c->d_xcache + (long)sys[j].q * c->Np, 8), c->st));
      }
      int dinfo[FB_MAX] = {0};
      HIPCHK(rt_memcpy(dinfo, c->d_dinfo, nb * sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCHK(rt_sync(c->st));
      for (int i = 0; i < nb; ++i)
        if (dinfo[i] != 0)
          return fail(GW_EDEVICE, "dense fallback: singular dielectric matrix at w = %.17g",
                      sys[bad[j0 + i]].w);
    }
    RCHK(matvec_pass(c, m.x, kp, EPI_RES_DERIV, m.part, kp));
    HIPCHK(minres_results(m, c->d_R, c->d_rhs_idx, c->Rp, nparts, c->d_wc, c->d_dwc, c->d_conv,
                        c->ext(c->d_wc, 8), c->st));
    HIPCHK(rt_memcpy(wc.data(), c->d_wc, k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(rt_memcpy(dwc.data(), c->d_dwc, k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(rt_sync(c->st));
    c->timing.fallback_ms += tm.stop();
    c->timing.fallback_systems += (int)bad.size();
  }
  if (x_out) {
    x_out->assign((size_t)k * c->n_aux, 0.0);
    for (int j = 0; j < k; ++j)
      HIPCHK(rt_memcpy(x_out->data() + (size_t)j * c->n_aux, m.x + (long)j * c->Np,
                            c->n_aux * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(rt_sync(c->st));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Sigma^c at a batch of (state, omega)

// Residue weight of the residue term R_nn: occupied m carry -theta(eps_m - w),
// virtual m carry +theta(w - eps_m), with theta(0) = 1/2.
double residue_weight(const gw_ctx* c, int spin, int m, double w) {
  const double e = c->eps[(size_t)spin * c->n_mo + m];
  if (m < c->n_occ_s[spin]) {
    double x = e - w;
    return x > 0 ? -1.0 : (x == 0 ? -0.5 : 0.0);
  }
  double x = w - e;
  return x > 0 ? 1.0 : (x == 0 ? 0.5 : 0.0);
}

int ensure_sig(gw_ctx* c, int n) {
  if (n <= c->sig_cap) return 0;
  // a multiple of 8, so that the pinned mirror [omega | rows | sig | dsig]
  // keeps its doubles 8-byte aligned after the int block
  n = round_up(n, 8);
  c->release(c->d_omega);
  c->release(c->d_sig);
  c->release(c->d_sigpart);
  // inputs [omega | rows] and outputs [sig | dsig] each in one block
  RCHK(c->alloc((void**)&c->d_omega, (size_t)n * (sizeof(double) + sizeof(int))));
  c->d_rowsel = (int*)(c->d_omega + n);
  RCHK(c->alloc((void**)&c->d_sig, 2 * (size_t)n * sizeof(double)));
  c->d_dsig = c->d_sig + n;
  RCHK(c->alloc((void**)&c->d_sigpart, (size_t)n * 32 * sizeof(double)));
  c->sig_cap = n;
  return 0;
}

// Requires a valid W^c table for the grid in the context.
int eval_sigma(gw_ctx* c, const std::vector<int>& states, const std::vector<double>& omega,
               std::vector<double>& sig, std::vector<double>& dsig, std::vector<int>& nres,
               std::vector<int>& flags, const std::vector<double>* tols = nullptr) {
  const int n = (int)states.size();
  sig.assign(n, 0.0);
  dsig.assign(n, 0.0);
  nres.assign(n, 0);
  flags.assign(n, 0);
  if (n == 0) return 0;
  RCHK(ensure_sig(c, n));
  std::vector<int> rows(n);
  for (int j = 0; j < n; ++j) rows[j] = c->row_of[states[j]];
  // residue systems of every entry (host only)
  std::vector<System> sys;
  std::vector<int> owner;
  std::vector<double> weight;
  for (int j = 0; j < n; ++j) {
    const int sp = c->row_spin[rows[j]];
    const double* e = c->eps.data() + (size_t)sp * c->n_mo;
    for (int m = 0; m < c->n_mo; ++m) {
      double f = residue_weight(c, sp, m, omega[j]);
      if (f == 0.0) continue;
      sys.push_back(System{rows[j] * c->n_mo + m, e[m] - omega[j],
                           tols ? (*tols)[j] : 0.0});
      owner.push_back(j);
      weight.push_back(f);
      nres[j]++;
    }
  }
  // pinned staging mirrors the device blocks: [omega cap | rows cap] in,
  // [sig cap | dsig cap] out, then the MINRES region; the quadrature's results
  // are read after the round's single synchronisation
  const int sc = c->sig_cap;
  const size_t sig_bytes = ((size_t)sc * (3 * sizeof(double) + sizeof(int)) + 63) / 64 * 64;
  const int kmax = std::min((int)sys.size(), c->minres_batch);
  RCHK(ensure_stage(c, sig_bytes + mr_stage_bytes(std::max(c->mr_cap, mr_kp(std::max(kmax, 1))))));
  {
    double* h_om = (double*)c->h_stage;
    int* h_row = (int*)(h_om + sc);
    double* h_sig = (double*)(h_row + sc);
    std::copy(omega.begin(), omega.end(), h_om);
    std::copy(rows.begin(), rows.end(), h_row);
    if (!audit_mode()) HIPCHK(hipEventRecord(c->ev_quad[0], c->st));
    HIPCHK(rt_memcpy(c->d_omega, h_om, (size_t)sc * (sizeof(double) + sizeof(int)),
                     hipMemcpyHostToDevice, c->st));
    HIPCHK(sigma_quad(c->d_wtab, c->n_mo, c->quad_G, c->wtab_G, c->quad_split, c->d_rowsel,
                      c->n_spin > 1 ? c->d_rowspin : nullptr, c->d_omega, c->d_eps, c->d_grid,
                      c->d_grid + c->grid_cap, n, c->d_sig, c->d_dsig, c->d_sigpart, c->n_rows,
                      c->ext(c->d_wtab, 8), c->ext(c->d_sigpart, 8), c->ext(c->d_eps, 8),
                      c->ext(c->d_grid, 8), c->ext(c->d_grid + c->grid_cap, 8), c->st));
    HIPCHK(rt_memcpy(h_sig, c->d_sig, 2 * (size_t)sc * sizeof(double), hipMemcpyDeviceToHost,
                     c->st));
    if (!audit_mode()) HIPCHK(hipEventRecord(c->ev_quad[1], c->st));
  }
  std::vector<double> wc, dwc;
  std::vector<int> it;
  c->stage_off = sig_bytes;
  const int rc = solve_residues(c, sys, true, wc, dwc, it);
  c->stage_off = 0;
  RCHK(rc);
  HIPCHK(rt_sync(c->st));   // (already drained when there were residue systems)
  if (!audit_mode()) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_quad[0], c->ev_quad[1]));
    c->timing.quad_ms += ms;
  }
  {
    // (h_stage may have moved; the layout is unchanged)
    const double* h_sig = (const double*)((const int*)((const double*)c->h_stage + sc) + sc);
    for (int j = 0; j < n; ++j) {
      sig[j] = h_sig[j];
      dsig[j] = h_sig[sc + j];
    }
  }
  for (size_t s = 0; s < sys.size(); ++s) {
    const int j = owner[s];
    sig[j] += weight[s] * wc[s];
    // the residue frequency eps_m - omega moves opposite to omega
    dsig[j] -= weight[s] * dwc[s];
    if (it[s] < 0) flags[j] |= GW_ST_FALLBACK;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Spectral-decomposition route (Implementation - Spectral Decomposition)

constexpr int SD_NORM_BLOCKS = 256;
constexpr int SD_MAX_KP = 16384;    // the dense Kp x Kp eigenproblem is for small systems

// Casida matrix M = D^2 + 4 D^1/2 B_ov^T B_ov D^1/2, its eigendecomposition
// M = T Omega^2 T^T by block Jacobi, and the pole strengths
// rho = 2 (R B_ov) D^1/2 T of every supplied row.
int build_sd(gw_ctx* c) {
  if (c->sd_valid) return 0;
  const int Kp = c->Kp;
  if (Kp > SD_MAX_KP)
    return fail(GW_EINVAL, "the spectral-decomposition route holds N_ov x N_ov matrices; "
                "N_ov = %d exceeds its limit %d", c->Kov, SD_MAX_KP);
  Timer tm;
  tm.a = c->ev0; tm.b = c->ev1;
  tm.start(c->st);
  if (!c->d_sdM) {
    RCHK(c->alloc((void**)&c->d_sdM, (size_t)Kp * Kp * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdT, (size_t)Kp * Kp * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdV, (size_t)(Kp / 64) * 64 * 64 * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdY, (size_t)c->Rp * Kp * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdRho, (size_t)c->Rp * Kp * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdO, (size_t)Kp * sizeof(double)));
    RCHK(c->alloc((void**)&c->d_sdPart, 2 * (size_t)SD_NORM_BLOCKS * sizeof(double)));
  }
  {  // B_ov^T B_ov (both operands k-major), then the Casida scaling
    GemmArgs a{};
    a.A = c->d_Bov; a.lda = Kp;
    a.B = c->d_Bov; a.ldb = Kp;
    a.C = c->d_sdM; a.ldc = Kp;
    a.M = Kp; a.N = Kp; a.K = c->Np;
    a.map = MAP_FULL; a.tiles_m = Kp / 128; a.tiles_n = Kp / 128;
    a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1; a.splitk = 1;
    RCHK(run_gemm(c, a, 0, KM, KM, EPI_STORE));
  }
  HIPCHK(casida_matrix(c->d_sdM, Kp, c->d_D, c->Kov, Kp, c->ext(c->d_sdM, 8), c->ext(c->d_D, 8),
                       c->st));
  HIPCHK(set_identity(c->d_sdT, Kp, Kp, c->ext(c->d_sdT, 8), c->st));
  const int nb = Kp / 32;
  // inner Jacobi sweeps per 64 x 64 subproblem (GW_TUNE_SD="sweeps" replaces the default)
  int inner = 1;
  if (const char* e = getenv("GW_TUNE_SD")) inner = std::max(1, std::min(16, atoi(e)));
  std::vector<double> part(2 * SD_NORM_BLOCKS);
  int sweeps = 0;
  double off_prev = -1.0;
  for (; sweeps < 40; ++sweeps) {
    HIPCHK(offnorm(c->d_sdM, Kp, c->Kov, c->d_sdPart, SD_NORM_BLOCKS, c->ext(c->d_sdM, 8),
                   c->ext(c->d_sdPart, 8), c->st));
    HIPCHK(rt_memcpy(part.data(), c->d_sdPart, part.size() * sizeof(double),
                     hipMemcpyDeviceToHost, c->st));
    HIPCHK(rt_sync(c->st));
    double off = 0.0, dia = 0.0;
    for (int b = 0; b < SD_NORM_BLOCKS; ++b) {
      off += part[2 * b];
      dia += part[2 * b + 1];
    }
    trace("sd sweep %d: off/diag = %.3e", sweeps, dia > 0 ? std::sqrt(off / dia) : 0.0);
    // converged: off-diagonal norm below 1e-15 of the diagonal's, or stalled
    // at the rounding floor once below 1e-10 of it
    const bool stalled = off_prev >= 0.0 && off < 1e-20 * dia && off > 0.25 * off_prev;
    if (audit_mode() ? sweeps >= 1 : (!(off > 1e-30 * dia) || stalled)) break;
    off_prev = off;
    for (int r = 0; r < nb - 1; ++r)
      HIPCHK(jacobi_round(c->d_sdM, c->d_sdT, Kp, Kp, r, c->d_sdV, inner, c->ext(c->d_sdM, 8),
                          c->ext(c->d_sdT, 8), c->ext(c->d_sdV, 8), c->st));
  }
  if (sweeps >= 40) return fail(GW_EDEVICE, "block Jacobi did not converge in 40 sweeps");
  c->sd_sweeps = sweeps;
  HIPCHK(diag_sqrt(c->d_sdM, Kp, c->Kov, c->d_sdO, c->ext(c->d_sdM, 8), c->ext(c->d_sdO, 8),
                   c->st));
  if (c->nR > 0) {
    GemmArgs a{};  // Y = R B_ov: rows of (P|nm) times B_ov [P][ia] (k-major)
    a.A = c->d_R; a.lda = c->Np;
    a.B = c->d_Bov; a.ldb = Kp;
    a.C = c->d_sdY; a.ldc = Kp;
    a.M = c->Rp; a.N = Kp; a.K = c->Np;
    a.map = MAP_FULL; a.tiles_m = c->Rp / 64; a.tiles_n = Kp / 64;
    a.n_tiles = a.tiles_m * a.tiles_n; a.batch = 1; a.splitk = 1;
    RCHK(run_gemm(c, a, 3, KC, KM, EPI_STORE));
    HIPCHK(pole_scale(c->d_sdY, Kp, c->Rp, c->d_D, c->Kov, Kp, c->ext(c->d_sdY, 8),
                      c->ext(c->d_D, 8), c->st));
    GemmArgs b{};  // rho = Y T, T [k][s] (k-major for the product over k)
    b.A = c->d_sdY; b.lda = Kp;
    b.B = c->d_sdT; b.ldb = Kp;
    b.C = c->d_sdRho; b.ldc = Kp;
    b.M = c->Rp; b.N = Kp; b.K = Kp;
    b.map = MAP_FULL; b.tiles_m = c->Rp / 64; b.tiles_n = Kp / 64;
    b.n_tiles = b.tiles_m * b.tiles_n; b.batch = 1; b.splitk = 1;
    RCHK(run_gemm(c, b, 3, KC, KM, EPI_STORE));
  }
  c->timing.sd_ms += tm.stop();
  c->timing.sd_sweeps = sweeps;
  c->sd_valid = true;
  return 0;
}

// Re Sigma^c and its derivative from the pole form (requires build_sd).
int eval_sigma_sd(gw_ctx* c, const std::vector<int>& states, const std::vector<double>& omega,
                  std::vector<double>& sig, std::vector<double>& dsig) {
  const int n = (int)states.size();
  sig.assign(n, 0.0);
  dsig.assign(n, 0.0);
  if (n == 0) return 0;
  RCHK(ensure_sig(c, n));
  const int sc = c->sig_cap;
  RCHK(ensure_stage(c, (size_t)sc * (3 * sizeof(double) + sizeof(int)) + 64));
  double* h_om = (double*)c->h_stage;
  int* h_row = (int*)(h_om + sc);
  double* h_sig = (double*)(h_row + sc);
  for (int j = 0; j < n; ++j) {
    h_om[j] = omega[j];
    h_row[j] = c->row_of[states[j]];
  }
  HIPCHK(rt_memcpy(c->d_omega, h_om, (size_t)sc * (sizeof(double) + sizeof(int)),
                   hipMemcpyHostToDevice, c->st));
  HIPCHK(sigma_sd(c->d_sdRho, c->Kp, c->n_mo, c->Kov, c->n_rows, c->d_rowsel,
                  c->n_spin > 1 ? c->d_rowspin : nullptr, c->n_occ_s[0], c->n_occ_s[1],
                  c->d_omega, c->d_eps, c->d_sdO, n, c->d_sig, c->d_dsig, c->d_sigpart,
                  c->ext(c->d_sdRho, 8), c->ext(c->d_eps, 8), c->ext(c->d_sdO, 8),
                  c->ext(c->d_sigpart, 8), c->st));
  HIPCHK(rt_memcpy(h_sig, c->d_sig, 2 * (size_t)sc * sizeof(double), hipMemcpyDeviceToHost,
                   c->st));
  HIPCHK(rt_sync(c->st));
  for (int j = 0; j < n; ++j) {
    sig[j] = h_sig[j];
    dsig[j] = h_sig[sc + j];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Quasiparticle step tree (Implementation - Solution of the Quasiparticle
// Equations, step-selection tree figure).  f(w) = eps_n + dsig_x_n +
// Re Sigma^c(w) - w, Z = -1/f'(w).
//   iteration 0: scaled residual, dw = a f with a = min(0.1, 0.1/|f|)
//   Z >= 0.3: Newton, dw = Z f
//   else bracketed: golden section, next = s + 0.381966 (e - s) with s the
//       bracket end of smaller |f|
//   else Z >= 0.1: scaled Newton, dw = 0.7 Z f
//   else: scaled residual
// Brackets come from consecutive points: a sign change with f > 0 on the
// left end, or the same sign with growing |f| after a step taken along the
// residual (a pole was crossed and a root skipped).  A point inside an
// existing bracket replaces one of its ends.  Converged when |f| < qp_tol.

struct QPState {
  int n;
  double w;
  bool done = false;
  int iter = 0;
  bool has_prev = false;
  double wp = 0, fp = 0;
  bool has_br = false;
  double s = 0, fs = 0, e = 0, fe = 0;
  double E = 0, sig = 0, Z = 0;
  double last_f = -1;   // |f| at the previous evaluation (-1: none yet)
  int status = 0;
};

inline int sgn(double x) { return (x > 0) - (x < 0); }

void order_bracket(QPState& q) {
  if (std::fabs(q.fe) < std::fabs(q.fs)) {
    std::swap(q.s, q.e);
    std::swap(q.fs, q.fe);
  }
}

void update_bracket(QPState& q, double w, double f) {
  if (!q.has_prev) return;
  if (q.has_br && std::min(q.s, q.e) < w && w < std::max(q.s, q.e)) {
    if (sgn(q.fs) != sgn(q.fe)) {
      if (sgn(f) == sgn(q.fs)) { q.s = w; q.fs = f; }
      else { q.e = w; q.fe = f; }
    } else {
      if (sgn(f) == sgn(q.fs) && std::fabs(f) < std::fabs(q.fs)) { q.s = w; q.fs = f; }
      else { q.e = w; q.fe = f; }
    }
    order_bracket(q);
    return;
  }
  const double wp = q.wp, fp = q.fp;
  if (fp * f < 0) {
    double lo = wp, flo = fp, hi = w, fhi = f;
    if (w < wp) { lo = w; flo = f; hi = wp; fhi = fp; }
    if (flo > 0 && fhi < 0) {
      q.has_br = true;
      q.s = lo; q.fs = flo; q.e = hi; q.fe = fhi;
      order_bracket(q);
    }
  } else if (fp * f > 0 && std::fabs(f) > std::fabs(fp) && sgn(w - wp) == sgn(fp)) {
    q.has_br = true;
    q.s = wp; q.fs = fp; q.e = w; q.fe = f;
    order_bracket(q);
  }
}

double alpha_of(double f) { return f != 0.0 ? std::min(0.1, 0.1 / std::fabs(f)) : 0.1; }

// One step-tree decision for a state that has just been evaluated.
void qp_step(gw_ctx* c, QPState& q, double sigma, double dsigma) {
  const double f = c->eps_ks[q.n] + c->dsig_x[q.n] + sigma - q.w;
  q.last_f = std::fabs(f);
  const double fprime = dsigma - 1.0;
  const double Z = (fprime != 0.0) ? -1.0 / fprime : INFINITY;
  update_bracket(q, q.w, f);
  if (std::fabs(f) < c->qp_tol) {
    q.done = true;
    q.E = q.w;
    q.sig = sigma;
    q.Z = Z;
    if (Z < 0.1) q.status |= GW_ST_SMALL_Z;
    return;
  }
  double wn;
  if (q.iter == 0) wn = q.w + alpha_of(f) * f;
  else if (Z >= 0.3) wn = q.w + Z * f;
  else if (q.has_br) wn = q.s + 0.3819660112501051 * (q.e - q.s);
  else if (Z >= 0.1) wn = q.w + 0.7 * Z * f;
  else wn = q.w + alpha_of(f) * f;
  q.has_prev = true;
  q.wp = q.w;
  q.fp = f;
  q.w = wn;
  q.iter++;
  if (q.iter >= c->qp_max_iter) {
    q.status |= GW_ST_MAXITER;
  }
}

// Result-returning entry points end here: in launch-audit mode nothing was
// computed, so they report GW_EAUDIT instead of success.
// A public call starts without remembered residue solutions, so its results
// do not depend on earlier calls.
void forget_solutions(gw_ctx* c) { std::fill(c->xvalid.begin(), c->xvalid.end(), 0); }

int finish() {
  if (audit_mode()) return fail(GW_EAUDIT, "launch audit: every launch was checked, none was run");
  return 0;
}

int validate_states(gw_ctx* c, int n, const int* states) {
  if (n < 0 || (n > 0 && !states)) return fail(GW_EINVAL, "bad state list");
  for (int j = 0; j < n; ++j)
    if (!c->row_of.count(states[j]))
      return fail(GW_EINVAL, "state %d was not among the rows given to gw_setup", states[j]);
  return 0;
}

// The QP equations of `states` on the context's current W^c table, the
// states advancing together one step-tree decision per round (one batched
// Sigma evaluation per round); start: first frequency per state (NULL: the
// energy of the state in G).
//
// Cluster initial-guess layer ([QP], the layer after the step tree): with
// cluster_width > 0 the states, sorted by start energy (ties in request
// order), split into clusters wherever neighbours are more than the width
// apart.  A cluster's median member (the lower one for an even count) starts
// at once; the other members wait, and join the rounds after it is done,
// starting at their own energy plus its QP shift (their own energy if it hit
// the iteration cap).  A state's trajectory depends only on its start, so the
// schedule does not change results.
int solve_qp(gw_ctx* c, int n_states, const int* states, std::vector<QPState>& qs, int* rounds,
             const double* start = nullptr, bool sd = false) {
  qs.assign(n_states, QPState{});
  std::vector<double> e0(n_states);
  for (int j = 0; j < n_states; ++j) {
    qs[j].n = states[j];
    e0[j] = start ? start[j] : c->eps[states[j]];
    qs[j].w = e0[j];
  }
  std::vector<int> waits_for(n_states, -1);   // representative a member waits for
  if (c->cluster_width > 0.0 && n_states > 1) {
    std::vector<int> order(n_states);
    for (int j = 0; j < n_states; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return e0[a] < e0[b]; });
    for (int i = 0; i < n_states;) {
      int j = i + 1;
      while (j < n_states && e0[order[j]] - e0[order[j - 1]] <= c->cluster_width) ++j;
      const int rep = order[i + (j - i - 1) / 2];
      for (int k = i; k < j; ++k)
        if (order[k] != rep) waits_for[order[k]] = rep;
      i = j;
    }
  }
  *rounds = 0;
  while (true) {
    std::vector<int> act, st;
    std::vector<double> om, tol;
    for (int j = 0; j < n_states; ++j)
      if (!qs[j].done && waits_for[j] < 0) {
        act.push_back(j);
        st.push_back(qs[j].n);
        om.push_back(qs[j].w);
        // inexact Newton: residue solves need an error well below the current
        // |f| only; the last evaluations run at the full tolerance
        const double lf = qs[j].last_f < 0 ? 1.0 : qs[j].last_f;
        tol.push_back(std::min(1e-6, std::max(c->minres_rtol, 1e-4 * lf)));
      }
    if (act.empty()) break;   // (members are released as soon as their representative is done)
    std::vector<double> sg, dsg;
    std::vector<int> nres, flags;
    if (sd) {
      RCHK(eval_sigma_sd(c, st, om, sg, dsg));
      flags.assign(st.size(), 0);
    } else {
      RCHK(eval_sigma(c, st, om, sg, dsg, nres, flags, &tol));
    }
    (*rounds)++;
    for (size_t a = 0; a < act.size(); ++a) {
      QPState& q = qs[act[a]];
      q.status |= flags[a];
      qp_step(c, q, sg[a], dsg[a]);
      if (!q.done && q.iter >= c->qp_max_iter) {
        // report the last evaluated point
        q.done = true;
        q.E = q.wp;
        q.sig = sg[a];
        const double fprime = dsg[a] - 1.0;
        q.Z = fprime != 0.0 ? -1.0 / fprime : INFINITY;
        if (q.Z < 0.1) q.status |= GW_ST_SMALL_Z;
      }
    }
    for (int r : act) {
      if (!qs[r].done) continue;
      const bool guess = !(qs[r].status & GW_ST_MAXITER);
      for (int j = 0; j < n_states; ++j)
        if (waits_for[j] == r) {
          waits_for[j] = -1;
          if (guess) qs[j].w = e0[j] + (qs[r].E - e0[r]);
        }
    }
  }
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device-memory footprint of one context over gw_setup + gw_qp, mirroring
// every allocation above (requested bytes).  n_states bounds the number of
// residue systems per Sigma evaluation (n_states * n_mo, in batches of at
// most minres_batch; 0: a context's default batch).
size_t footprint_bytes(int n_mo, int n_occ, int n_aux, int n_rows, int n_states, int G_in,
                       int pi_prec, int wc_prec, size_t work_budget, int minres_batch) {
  if (minres_batch <= 0) minres_batch = MINRES_BATCH;
  const size_t d = sizeof(double);
  const int G = G_in + 1;   // the xi = 0 point of the preconditioner (on by default)
  const int Np = round_up(n_aux, 128);
  const int Kov = n_occ * (n_mo - n_occ);
  const int Kp = round_up(Kov, 128);
  const int nR = n_rows * n_mo;
  const int Rp = round_up(std::max(nR, 1), 128);
  size_t b = 0;
  b += (size_t)n_mo * d + (size_t)Kp * d + (size_t)Np * Kp * d + (size_t)Rp * Np * d +
       (size_t)Rp * d;
  if (pi_prec != GW_PI_FP64) b += (size_t)Np * Kp * (4 + 2 + 2);
  // stage A
  const size_t per_g = (size_t)(2L * Np + 128) * (Np + 128);
  const size_t parts = (size_t)(Np / 128) * Rp;
  const size_t f_bytes = wc_prec == GW_PI_BF16X3 ? (size_t)Np * Np * 4 : 0;
  const size_t per_bytes = per_g * d + (size_t)Kp * (d + 4) + PANEL * PANEL * d + parts * d + f_bytes;
  int chunk = (int)std::max<size_t>(1, work_budget / per_bytes);
  if (chunk > G) chunk = G;
  b += (size_t)chunk * (per_g * d + parts * d + PANEL * PANEL * d + sizeof(int) + (size_t)Kp * (d + 4));
  if (wc_prec == GW_PI_BF16X3) b += (size_t)chunk * f_bytes + (size_t)Rp * Np * 4;
  b += 2 * (size_t)G * d + (size_t)std::max(nR, 1) * G * d;
  // Sigma evaluation buffers
  b += (size_t)round_up(std::max(n_states, 1), 8) * (sizeof(int) + 3 * d + 32 * d);
  // MINRES workspace for the largest batch
  const int kmax = std::min(std::max(n_states, 1) * n_mo, minres_batch);
  const int kp = mr_kp(kmax);
  const size_t part = minres_part_elems(kp, Np, Kp);
  b += 8 * (size_t)kp * Np * d + (size_t)kp * 16 * d + (size_t)kp * Kp * d + part * d +
       (size_t)kp * (2 * d + 2 * sizeof(int) + 2 * d + sizeof(int)) + 2 * sizeof(int) +
       2 * (size_t)(kp / 16) * sizeof(int);
  b += (size_t)Rp * Np * d;  // remembered residue solutions
  b += (size_t)Np * Np * d;  // preconditioner
  // dense fallback (FB_MAX systems at once)
  b += FB_MAX * ((size_t)Np * Np * d + (size_t)Kp * d + (size_t)Np * d + (size_t)Np * sizeof(int) +
                 sizeof(int));
  return b;
}

// First flat index of a non-finite value in src[0, n), or -1; with dst, src is
// also copied to dst chunk by chunk (the check then reads the copy while it is
// still in cache).  Exponent-bit test over chunks (vectorisable); arrays above
// 4 Mi values are split over up to 8 host threads.
long copy_check_finite(double* dst, const double* src, long n) {
  auto scan = [dst, src](long lo, long hi) -> long {
    const long CH = 4096;
    for (long c = lo; c < hi; c += CH) {
      const long e = std::min(hi, c + CH);
      const double* x = src + c;
      if (dst) {
        memcpy(dst + c, src + c, (size_t)(e - c) * sizeof(double));
        x = dst + c;
      }
      unsigned long long bad = 0;
      for (long i = 0; i < e - c; ++i) {
        unsigned long long b;
        memcpy(&b, x + i, sizeof b);
        bad |= ((b >> 52) & 0x7ffULL) == 0x7ffULL;
      }
      if (bad)
        for (long i = c; i < e; ++i)
          if (!std::isfinite(src[i])) return i;
    }
    return -1;
  };
  const long big = 1L << 22;
  if (n < big) return scan(0, n);
  const int nt = 8;
  std::vector<long> found(nt, -1);
  std::vector<std::thread> th;
  const long per = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] { found[t] = scan(std::min(n, t * per), std::min(n, (t + 1) * per)); });
  for (auto& t : th) t.join();
  for (long f : found)
    if (f >= 0) return f;
  return -1;
}

// Host-side checks of gw_setup's inputs (sizes, ordering, finiteness; the
// finiteness of B_ov and B_rows only when check_arrays).
int validate_inputs(int n_mo, int n_occ, int n_aux, const double* eps, const double* B_ov,
                    int n_rows, const int* row_ids, const double* B_rows, bool check_arrays) {
  if (n_mo < 2 || n_occ < 1 || n_occ >= n_mo || n_aux < 1 || n_rows < 0)
    return fail(GW_EINVAL, "bad sizes: n_mo=%d n_occ=%d n_aux=%d n_rows=%d", n_mo, n_occ, n_aux,
                n_rows);
  if (!eps || !B_ov || (n_rows > 0 && (!row_ids || !B_rows)))
    return fail(GW_EINVAL, "NULL input array");
  for (int i = 0; i < n_mo; ++i) {
    if (!std::isfinite(eps[i])) return fail(GW_EINVAL, "eps[%d] is not finite", i);
    if (i > 0 && !(eps[i] > eps[i - 1])) return fail(GW_EINVAL, "eps is not strictly ascending at %d", i);
  }
  const long Kov = (long)n_occ * (n_mo - n_occ);
  if (Kov > 0x3fffffffL || (long)n_aux * n_mo > 0x3fffffffL)
    return fail(GW_EINVAL, "sizes too large");
  if (!check_arrays) return 0;
  long f = copy_check_finite(nullptr, B_ov, (long)n_aux * Kov);
  if (f >= 0) return fail(GW_EINVAL, "B_ov has a non-finite entry at %ld", f);
  f = copy_check_finite(nullptr, B_rows, (long)n_rows * n_mo * n_aux);
  if (f >= 0) return fail(GW_EINVAL, "B_rows has a non-finite entry at %ld", f);
  return 0;
}

int setup_validated(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                    const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
                    const gw_opts* opts);

// Validated inputs of one context: n_spin = 1 (closed shell) or 2 (open
// shell); eps [n_spin][n_mo]; B_ov[s] [n_aux][n_occ[s] * (n_mo - n_occ[s])];
// row ids name spin-orbitals s * n_mo + n.
struct SetupIn {
  int n_spin, n_mo, n_occ[2], n_aux;
  const double* eps;
  const double* B_ov[2];
  int n_rows;
  const int* row_ids;
  const double* B_rows;
};

int setup_core(gw_ctx** out, const SetupIn& in, const gw_opts* opts,
               gw_devcache* cache = nullptr);

// ===========================================================================
// C-ABI

extern "C" {

const char* gw_last_error(void) { return g_err.c_str(); }

int gw_grid_gauss_legendre(int n, double x0, double* xi, double* w) {
  if (n < 1 || !(x0 > 0.0) || !xi || !w) return fail(GW_EINVAL, "need n >= 1, x0 > 0");
  // Gauss-Legendre nodes by Newton's method on P_n (three-term recurrence)
  std::vector<double> t(n), u(n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0; }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    // final derivative at the converged node
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = x; p0 = 1.0; }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    t[i] = x;
    u[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // ascending t
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return t[a] < t[b]; });
  for (int i = 0; i < n; ++i) {
    double tt = t[ord[i]], uu = u[ord[i]];
    xi[i] = x0 * (1.0 + tt) / (1.0 - tt);
    w[i] = uu * 2.0 * x0 / ((1.0 - tt) * (1.0 - tt));
  }
  return 0;
}

int gw_setup(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps, const double* B_ov,
             int n_rows, const int* row_ids, const double* B_rows, const gw_opts* opts) {
  if (!out) return fail(GW_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (int rc = validate_inputs(n_mo, n_occ, n_aux, eps, B_ov, n_rows, row_ids, B_rows, true))
    return rc;
  return setup_validated(out, n_mo, n_occ, n_aux, eps, B_ov, n_rows, row_ids, B_rows, opts);
}

int gw_setup_full(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                  const double* B, const gw_opts* opts) {
  if (!out) return fail(GW_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (!B) return fail(GW_EINVAL, "NULL input array");
  if (n_mo < 2 || n_occ < 1 || n_occ >= n_mo || n_aux < 1 ||
      (double)n_aux * n_mo * n_mo > 4.0e9)
    return fail(GW_EINVAL, "bad sizes: n_mo=%d n_occ=%d n_aux=%d", n_mo, n_occ, n_aux);
  // B_ov[P][i*n_virt + a] = B[P][i][n_occ + a]; rows of every state,
  // B_rows[n][m][P] = B[P][n][m]
  const int n_virt = n_mo - n_occ;
  std::vector<double> B_ov((size_t)n_aux * n_occ * n_virt);
  std::vector<double> rows((size_t)n_mo * n_mo * n_aux);
  std::vector<int> ids(n_mo);
  for (int n = 0; n < n_mo; ++n) ids[n] = n;
  for (int P = 0; P < n_aux; ++P) {
    const double* BP = B + (size_t)P * n_mo * n_mo;
    for (int i = 0; i < n_occ; ++i)
      memcpy(&B_ov[((size_t)P * n_occ + i) * n_virt], BP + (size_t)i * n_mo + n_occ,
             (size_t)n_virt * sizeof(double));
    for (int n = 0; n < n_mo; ++n)
      for (int m = 0; m < n_mo; ++m) rows[((size_t)n * n_mo + m) * n_aux + P] = BP[(size_t)n * n_mo + m];
  }
  if (int rc = validate_inputs(n_mo, n_occ, n_aux, eps, B_ov.data(), n_mo, ids.data(),
                               rows.data(), true))
    return rc;
  return setup_validated(out, n_mo, n_occ, n_aux, eps, B_ov.data(), n_mo, ids.data(),
                         rows.data(), opts);
}

int gw_setup_uhf(gw_ctx** out, int n_mo, const int* n_occ, int n_aux, const double* eps,
                 const double* B_ov_up, const double* B_ov_down, int n_rows, const int* row_ids,
                 const double* B_rows, const gw_opts* opts) {
  if (!out) return fail(GW_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (!n_occ) return fail(GW_EINVAL, "n_occ is NULL");
  const double* Bs[2] = {B_ov_up, B_ov_down};
  for (int sp = 0; sp < 2; ++sp) {
    // each spin's levels and integrals pass the closed-shell checks (the rows
    // are checked once, with spin up)
    if (int rc = validate_inputs(n_mo, n_occ[sp], n_aux, eps ? eps + (size_t)sp * n_mo : nullptr,
                                 Bs[sp], sp == 0 ? n_rows : 0, row_ids, B_rows, true))
      return fail(rc, "spin %d: %s", sp, gw_last_error());
  }
  SetupIn in{2, n_mo, {n_occ[0], n_occ[1]}, n_aux, eps, {B_ov_up, B_ov_down}, n_rows, row_ids,
             B_rows};
  return setup_core(out, in, opts);
}

}  // extern "C"

int setup_core(gw_ctx** out, const SetupIn& in, const gw_opts* opts, gw_devcache* cache) {
  *out = nullptr;
  const int n_mo = in.n_mo, n_aux = in.n_aux, n_rows = in.n_rows, n_spin = in.n_spin;
  long Ks[2] = {0, 0};
  for (int sp = 0; sp < n_spin; ++sp) Ks[sp] = (long)in.n_occ[sp] * (n_mo - in.n_occ[sp]);
  const long Kov = Ks[0] + Ks[1];
  if (Kov > 0x3fffffffL) return fail(GW_EINVAL, "sizes too large");
  gw_opts o{};
  if (opts) o = *opts;
  if (o.pi_prec < 0 || o.pi_prec > 2) return fail(GW_EINVAL, "unknown pi_prec %d", o.pi_prec);
  if (o.wc_prec != GW_PI_FP64 && o.wc_prec != GW_PI_BF16X3)
    return fail(GW_EINVAL, "wc_prec must be GW_PI_FP64 or GW_PI_BF16X3, not %d", o.wc_prec);
  if (o.minres_max_iter < 0 || o.qp_max_iter < 0 || o.minres_rtol < 0 || o.qp_tol < 0 ||
      !(o.cluster_width >= 0.0) || !std::isfinite(o.cluster_width))
    return fail(GW_EINVAL, "negative or non-finite option");

  gw_ctx* c = new gw_ctx();
  c->cache = cache;
  g_contexts_created = true;
  c->n_spin = n_spin;
  c->n_occ_s[0] = in.n_occ[0];
  c->n_occ_s[1] = n_spin > 1 ? in.n_occ[1] : in.n_occ[0];
  c->n_mo = n_mo; c->n_occ = in.n_occ[0]; c->n_virt = n_mo - in.n_occ[0]; c->n_aux = n_aux;
  c->n_rows = n_rows;
  c->Np = round_up(n_aux, 128);
  c->Kov = (int)Kov;
  c->Kp = round_up((int)Kov, 128);
  c->nR = n_rows * n_mo;
  c->Rp = round_up(std::max(c->nR, 1), 128);
  c->pi_prec = o.pi_prec;
  c->wc_prec = o.wc_prec;
  if (o.minres_max_iter > 0) c->minres_max_iter = o.minres_max_iter;
  if (o.minres_rtol > 0) c->minres_rtol = o.minres_rtol;
  if (o.qp_tol > 0) c->qp_tol = o.qp_tol;
  if (o.qp_max_iter > 0) c->qp_max_iter = o.qp_max_iter;
  c->mem_budget = o.mem_budget_bytes;
  if (o.work_budget_bytes > 0) c->work_budget = o.work_budget_bytes;
  if (o.minres_batch > 0) c->minres_batch = std::max(64, o.minres_batch);
  c->graphs_off = o.no_graphs != 0 || debug_sync();
  c->no_precond = o.no_precond != 0;
  // test hook: GW_TEST_INDEFINITE=1 replaces 1 - Pi(i xi) by 1 + Pi(i xi) before
  // the Cholesky, so that the factorisation meets a non-positive pivot
  if (const char* e = getenv("GW_TEST_INDEFINITE")) c->test_indefinite = atoi(e) != 0;
  c->cluster_width = o.cluster_width;
  const int n_so = n_spin * n_mo;   // spin-orbitals
  c->eps.assign(in.eps, in.eps + n_so);
  c->eps_ks = c->eps;
  c->dsig_x.assign(n_so, 0.0);
  if (o.dsig_x) {
    for (int i = 0; i < n_so; ++i) {
      if (!std::isfinite(o.dsig_x[i])) {
        delete c;
        return fail(GW_EINVAL, "dsig_x[%d] is not finite", i);
      }
      c->dsig_x[i] = o.dsig_x[i];
    }
  }
  for (int r = 0; r < n_rows; ++r) {
    const int id = in.row_ids[r];
    if (id < 0 || id >= n_so || c->row_of.count(id)) {
      delete c;
      return fail(GW_EINVAL, "row_ids[%d] = %d is out of range or repeated", r, id);
    }
    c->row_of[id] = r;
    c->row_ids.push_back(id);
    c->row_spin.push_back(id / n_mo);
  }
  int rc = 0;
  auto cleanup = [&](int code) {
    std::string keep = g_err;
    delete c;
    g_err = keep;
    return code;
  };
  if (audit_mode()) {
    c->st = nullptr;
  } else if (o.stream) {
    c->st = (hipStream_t)o.stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(GW_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
    c->own_stream = true;
  }
  if (!audit_mode() &&
      (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
       hipEventCreate(&c->ev0b) != hipSuccess || hipEventCreate(&c->ev1b) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_poll[0], hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&c->ev_poll[1], hipEventDisableTiming) != hipSuccess ||
       hipEventCreate(&c->ev_quad[0]) != hipSuccess || hipEventCreate(&c->ev_quad[1]) != hipSuccess ||
       hipEventCreate(&c->evk[0]) != hipSuccess || hipEventCreate(&c->evk[1]) != hipSuccess ||
       hipEventCreate(&c->evk[2]) != hipSuccess || hipEventCreate(&c->evk[3]) != hipSuccess))
    return cleanup(fail(GW_EDEVICE, "hipEventCreate failed"));
  if (host_alloc(c->cache, (void**)&c->h_poll, 2 * sizeof(int)) != hipSuccess)
    return cleanup(fail(GW_ENOMEM, "pinned host allocation failed"));
  if ((rc = c->alloc((void**)&c->d_eps, (size_t)n_so * sizeof(double)))) return cleanup(rc);
  if ((rc = c->alloc((void**)&c->d_D, (size_t)c->Kp * sizeof(double)))) return cleanup(rc);
  if ((rc = c->alloc((void**)&c->d_Bov, (size_t)c->Np * c->Kp * sizeof(double)))) return cleanup(rc);
  if ((rc = c->alloc((void**)&c->d_R, (size_t)c->Rp * c->Np * sizeof(double)))) return cleanup(rc);
  if ((rc = c->alloc((void**)&c->d_bn, (size_t)c->Rp * sizeof(double)))) return cleanup(rc);
  if (n_spin > 1 &&
      (rc = c->alloc((void**)&c->d_rowspin, (size_t)std::max(n_rows, 1) * sizeof(int))))
    return cleanup(rc);
  hipStream_t st = c->st;
#define SETUP_CHK(expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ == hipSuccess && debug_sync() && !audit_mode()) e_ = hipDeviceSynchronize();     \
    if (e_ != hipSuccess)                                                                   \
      return cleanup(fail(GW_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)));      \
  } while (0)
  SETUP_CHK(rt_memcpy(c->d_eps, in.eps, (size_t)n_so * sizeof(double), hipMemcpyHostToDevice, st));
  SETUP_CHK(transition_energies(c->d_eps, n_spin, n_mo, c->n_occ_s, c->Kp, c->d_D,
                                c->ext(c->d_eps, 8), c->ext(c->d_D, 8), st));
  SETUP_CHK(rt_memset(c->d_Bov, 0, (size_t)c->Np * c->Kp * sizeof(double), st));
  // the spins' transitions side by side: columns [0, K_up) then [K_up, K_up + K_down)
  for (int sp = 0; sp < n_spin; ++sp)
    SETUP_CHK(rt_memcpy2d(c->d_Bov + (sp ? Ks[0] : 0), (size_t)c->Kp * sizeof(double),
                          in.B_ov[sp], (size_t)Ks[sp] * sizeof(double),
                          (size_t)Ks[sp] * sizeof(double), n_aux, hipMemcpyHostToDevice, st));
  // Pi = -2 sum_s B_s diag(.) B_s^T for two spins is the closed-shell form
  // -4 B diag(.) B^T of the stacked B / sqrt(2): every kernel keeps its factor 4
  if (n_spin > 1)
    SETUP_CHK(scale_inplace(c->d_Bov, (long)c->Np * c->Kp, std::sqrt(0.5), c->ext(c->d_Bov, 8),
                            st));
  SETUP_CHK(rt_memset(c->d_R, 0, (size_t)c->Rp * c->Np * sizeof(double), st));
  if (c->nR > 0) {
    SETUP_CHK(rt_memcpy2d(c->d_R, (size_t)c->Np * sizeof(double), in.B_rows,
                               (size_t)n_aux * sizeof(double), (size_t)n_aux * sizeof(double),
                               c->nR, hipMemcpyHostToDevice, st));
  }
  if (n_spin > 1 && n_rows > 0)
    SETUP_CHK(rt_memcpy(c->d_rowspin, c->row_spin.data(), (size_t)n_rows * sizeof(int),
                        hipMemcpyHostToDevice, st));
  SETUP_CHK(row_norm2(c->d_R, c->Rp, c->Np, c->d_bn, c->ext(c->d_R, 8), c->ext(c->d_bn, 8), st));
  SETUP_CHK(rt_sync(st));
#undef SETUP_CHK
  *out = c;
  return 0;
}

int setup_validated(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                    const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
                    const gw_opts* opts) {
  SetupIn in{1, n_mo, {n_occ, n_occ}, n_aux, eps, {B_ov, nullptr}, n_rows, row_ids, B_rows};
  return setup_core(out, in, opts);
}

// A server context: its device and pinned host blocks come from `cache`.
int setup_cached(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                 const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
                 const gw_opts* opts, gw_devcache* cache) {
  SetupIn in{1, n_mo, {n_occ, n_occ}, n_aux, eps, {B_ov, nullptr}, n_rows, row_ids, B_rows};
  return setup_core(out, in, opts, cache);
}

extern "C" {

void gw_free(gw_ctx* ctx) { delete ctx; }

int gw_set_pi_prec(gw_ctx* c, int prec) {
  if (!c) return fail(GW_EINVAL, "NULL ctx");
  if (prec < 0 || prec > 2) return fail(GW_EINVAL, "unknown pi_prec %d", prec);
  if (prec != c->pi_prec) c->wtab_valid = false;
  c->pi_prec = prec;
  return 0;
}

size_t gw_footprint(int n_mo, int n_occ, int n_aux, int n_rows, int n_states, int grid_n,
                    const gw_opts* opts) {
  gw_opts o{};
  if (opts) o = *opts;
  const size_t wb = o.work_budget_bytes ? o.work_budget_bytes : (16ull << 30);
  const int mb = o.minres_batch > 0 ? std::max(64, o.minres_batch) : MINRES_BATCH;
  if (n_mo < 2 || n_occ < 1 || n_occ >= n_mo || n_aux < 1 || n_rows < 0 || grid_n < 1) return 0;
  return footprint_bytes(n_mo, n_occ, n_aux, n_rows, n_states, grid_n, o.pi_prec, o.wc_prec, wb, mb);
}

int gw_reset_cache(gw_ctx* c) {
  if (!c) return fail(GW_EINVAL, "NULL ctx");
  c->wtab_valid = false;
  c->sd_valid = false;
  return 0;
}

int gw_get_timing(gw_ctx* c, gw_timing* out) {
  if (!c || !out) return fail(GW_EINVAL, "NULL argument");
  *out = c->timing;
  return 0;
}

int gw_dielectric(gw_ctx* c, int n_xi, const double* xi, double* out) {
  if (!c || n_xi < 1 || !xi || !out) return fail(GW_EINVAL, "bad arguments");
  std::vector<double> w(n_xi, 1.0);
  gw_grid g{n_xi, xi, w.data()};
  c->timing = gw_timing{};
  RCHK(build_wtable(c, &g, 1, out));
  return finish();
}

int gw_cholesky(gw_ctx* c, int n_xi, const double* xi, double* out) {
  if (!c || n_xi < 1 || !xi || !out) return fail(GW_EINVAL, "bad arguments");
  std::vector<double> w(n_xi, 1.0);
  gw_grid g{n_xi, xi, w.data()};
  c->timing = gw_timing{};
  RCHK(build_wtable(c, &g, 2, out));
  return finish();
}

int gw_wtable(gw_ctx* c, const gw_grid* grid, double* out) {
  if (!c) return fail(GW_EINVAL, "NULL ctx");
  c->timing = gw_timing{};
  RCHK(build_wtable(c, grid, 0));
  if (out && c->nR > 0) {
    HIPCHK(rt_memcpy(out, c->d_wtab, (size_t)c->nR * grid->n * sizeof(double),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(rt_sync(c->st));
  }
  return finish();
}

int gw_sigma(gw_ctx* c, int n, const int* states, const double* omega, const gw_grid* grid,
             double* sigma, double* dsigma, int* n_res) {
  if (!c || n < 0 || (n > 0 && (!omega || !sigma || !dsigma)))
    return fail(GW_EINVAL, "bad arguments");
  RCHK(validate_states(c, n, states));
  for (int j = 0; j < n; ++j)
    if (!std::isfinite(omega[j])) return fail(GW_EINVAL, "omega[%d] is not finite", j);
  forget_solutions(c);
  c->timing = gw_timing{};
  RCHK(build_wtable(c, grid, 0, nullptr, !c->no_precond));
  c->quad_split = 0;
  std::vector<int> st(states, states + n), nres, flags;
  std::vector<double> om(omega, omega + n), sg, dsg;
  RCHK(eval_sigma(c, st, om, sg, dsg, nres, flags));
  for (int j = 0; j < n; ++j) {
    sigma[j] = sg[j];
    dsigma[j] = dsg[j];
    if (n_res) n_res[j] = nres[j];
  }
  return finish();
}

int gw_residues(gw_ctx* c, int k, const int* states, const int* m, const double* w,
                int use_fallback, double* x, double* wc, double* dwc, int* iters) {
  if (!c || k < 0 || (k > 0 && (!states || !m || !w))) return fail(GW_EINVAL, "bad arguments");
  RCHK(validate_states(c, k, states));
  std::vector<System> sys(k);
  for (int j = 0; j < k; ++j) {
    if (m[j] < 0 || m[j] >= c->n_mo || !std::isfinite(w[j]))
      return fail(GW_EINVAL, "bad system %d", j);
    sys[j] = System{c->row_of[states[j]] * c->n_mo + m[j], w[j], 0.0};
  }
  forget_solutions(c);
  c->timing = gw_timing{};
  std::vector<double> a, b, xs;
  std::vector<int> it;
  RCHK(solve_residues(c, sys, use_fallback != 0, a, b, it, x ? &xs : nullptr));
  for (int j = 0; j < k; ++j) {
    if (wc) wc[j] = a[j];
    if (dwc) dwc[j] = b[j];
    if (iters) iters[j] = it[j];
  }
  if (x) std::copy(xs.begin(), xs.end(), x);
  return finish();
}

int gw_qp(gw_ctx* c, int n_states, const int* states, const gw_grid* grid, double* E_qp,
          double* sigma_c, double* Z, int* status) {
  if (!c || n_states < 0 || (n_states > 0 && (!E_qp || !sigma_c || !Z)))
    return fail(GW_EINVAL, "bad arguments");
  RCHK(validate_states(c, n_states, states));
  forget_solutions(c);
  c->timing = gw_timing{};
  Timer total;
  total.a = c->ev0b;
  total.b = c->ev1b;
  total.start(c->st);
  // (the xi = 0 point also gives the MINRES preconditioner)
  int rc = build_wtable(c, grid, 0, nullptr, !c->no_precond);
  if (rc) return rc;
  c->quad_split = 0;
  std::vector<QPState> qs;
  int rounds = 0;
  rc = solve_qp(c, n_states, states, qs, &rounds);
  const double ms = total.stop();
  if (rc) return rc;
  c->timing.total_ms = ms;
  c->timing.qp_rounds = rounds;
  for (int j = 0; j < n_states; ++j) {
    E_qp[j] = qs[j].E;
    sigma_c[j] = qs[j].sig;
    Z[j] = qs[j].Z;
    if (status) status[j] = qs[j].status;
  }
  return finish();
}

int gw_qp_sd(gw_ctx* c, int n_states, const int* states, double* E_qp, double* sigma_c,
             double* Z, int* status) {
  if (!c || n_states < 0 || (n_states > 0 && (!E_qp || !sigma_c || !Z)))
    return fail(GW_EINVAL, "bad arguments");
  RCHK(validate_states(c, n_states, states));
  c->timing = gw_timing{};
  Timer total;
  total.a = c->ev0b;
  total.b = c->ev1b;
  total.start(c->st);
  int rc = build_sd(c);
  if (rc) return rc;
  std::vector<QPState> qs;
  int rounds = 0;
  rc = solve_qp(c, n_states, states, qs, &rounds, nullptr, true);
  const double ms = total.stop();
  if (rc) return rc;
  c->timing.total_ms = ms;
  c->timing.qp_rounds = rounds;
  for (int j = 0; j < n_states; ++j) {
    E_qp[j] = qs[j].E;
    sigma_c[j] = qs[j].sig;
    Z[j] = qs[j].Z;
    if (status) status[j] = qs[j].status;
  }
  return finish();
}

int gw_rpa_excitations(gw_ctx* c, double* Omega) {
  if (!c || !Omega) return fail(GW_EINVAL, "bad arguments");
  c->timing = gw_timing{};
  RCHK(build_sd(c));
  std::vector<double> om(c->Kov);
  HIPCHK(rt_memcpy(om.data(), c->d_sdO, (size_t)c->Kov * sizeof(double), hipMemcpyDeviceToHost,
                   c->st));
  HIPCHK(rt_sync(c->st));
  std::sort(om.begin(), om.end());
  std::copy(om.begin(), om.end(), Omega);
  return finish();
}

int gw_evgw(gw_ctx* c, int mode, int n_cycles, double ev_tol, int n_states, const int* states,
            const gw_grid* grid, double* E_qp, double* sigma_c, double* Z, int* status,
            double* E_cycles, int* cycles_done) {
  if (!c || n_states < 0 || (n_states > 0 && (!E_qp || !sigma_c || !Z)))
    return fail(GW_EINVAL, "bad arguments");
  if (mode != GW_EVGW0 && mode != GW_EVGW) return fail(GW_EINVAL, "unknown mode %d", mode);
  if (n_cycles < 1 || !(ev_tol >= 0.0) || !std::isfinite(ev_tol))
    return fail(GW_EINVAL, "need n_cycles >= 1 and a finite ev_tol >= 0");
  if (c->n_spin != 1) return fail(GW_EINVAL, "gw_evgw needs a closed-shell context");
  RCHK(validate_states(c, n_states, states));
  forget_solutions(c);
  c->timing = gw_timing{};
  Timer total;
  total.a = c->ev0b;
  total.b = c->ev1b;
  total.start(c->st);
  // Whatever happens below, the context leaves with its mean-field energies in
  // G and W again; a W^c table built from moved energies is dropped.
  bool w_moved = false;
  auto restore = [&]() -> int {
    c->quad_split = 0;
    c->eps = c->eps_ks;
    HIPCHK(rt_memcpy(c->d_eps, c->eps.data(), c->eps.size() * sizeof(double),
                     hipMemcpyHostToDevice, c->st));
    if (w_moved) {
      c->wtab_valid = false;
      c->sd_valid = false;
      HIPCHK(transition_energies(c->d_eps, c->n_spin, c->n_mo, c->n_occ_s, c->Kp, c->d_D,
                                 c->ext(c->d_eps, 8), c->ext(c->d_D, 8), c->st));
    }
    HIPCHK(rt_sync(c->st));
    return 0;
  };
  std::vector<double> prev(n_states, 0.0), cur(n_states, 0.0);
  std::vector<QPState> qs;
  int rc = 0, rounds = 0, cycles = 0;
  for (int cyc = 0; cyc < n_cycles; ++cyc) {
    if (mode == GW_EVGW && cyc > 0) {
      // W from the current energies: transition energies, then a fresh table
      for (int sp = 0; sp < c->n_spin && rc == 0; ++sp) {
        const auto e = c->eps.begin() + (size_t)sp * c->n_mo;
        const double homo = *std::max_element(e, e + c->n_occ_s[sp]);
        const double lumo = *std::min_element(e + c->n_occ_s[sp], e + c->n_mo);
        if (!(lumo > homo))
          rc = fail(GW_ENOTSPD, "evGW: the updated energies close the gap of spin %d "
                    "(%.17g >= %.17g)", sp, homo, lumo);
      }
      if (rc) break;
      w_moved = true;
      c->wtab_valid = false;
      c->sd_valid = false;
      if (transition_energies(c->d_eps, c->n_spin, c->n_mo, c->n_occ_s, c->Kp, c->d_D,
                              c->ext(c->d_eps, 8), c->ext(c->d_D, 8), c->st) != hipSuccess) {
        rc = fail(GW_EDEVICE, "transition energies failed");
        break;
      }
    }
    if ((rc = build_wtable(c, grid, 0, nullptr, true, true))) break;
    c->quad_split = 1;
    // each cycle starts its solves from the current energies in G
    std::vector<double> start(n_states);
    for (int j = 0; j < n_states; ++j) start[j] = c->eps[states[j]];
    int r = 0;
    if ((rc = solve_qp(c, n_states, states, qs, &r, start.data()))) break;
    rounds += r;
    for (int j = 0; j < n_states; ++j) cur[j] = qs[j].E;
    if (E_cycles) std::copy(cur.begin(), cur.end(), E_cycles + (size_t)cyc * n_states);
    cycles = cyc + 1;
    double change = 0.0;
    for (int j = 0; j < n_states; ++j) change = std::max(change, std::fabs(cur[j] - prev[j]));
    const bool converged = cyc > 0 && change < ev_tol;
    trace("evgw mode=%d cycle=%d max change=%.3e", mode, cyc, cyc > 0 ? change : 0.0);
    prev = cur;
    // the requested states' QP energies become their energies in G (and W)
    for (int j = 0; j < n_states; ++j) c->eps[states[j]] = cur[j];
    if (rt_memcpy(c->d_eps, c->eps.data(), c->eps.size() * sizeof(double),
                  hipMemcpyHostToDevice, c->st) != hipSuccess) {
      rc = fail(GW_EDEVICE, "energy upload failed");
      break;
    }
    if (converged) break;
  }
  const std::string err = g_err;
  const int rrc = restore();
  const double ms = total.stop();
  if (rc) {
    g_err = err;
    return rc;
  }
  if (rrc) return rrc;
  c->timing.total_ms = ms;
  c->timing.qp_rounds = rounds;
  for (int j = 0; j < n_states; ++j) {
    E_qp[j] = qs[j].E;
    sigma_c[j] = qs[j].sig;
    Z[j] = qs[j].Z;
    if (status) status[j] = qs[j].status;
  }
  if (cycles_done) *cycles_done = cycles;
  return finish();
}

// ---- launch audit (include/gw_audit.h)

int gw_audit_enable(void) {
  if (g_contexts_created) return fail(GW_EINVAL, "launch audit must be enabled before any context exists");
  set_audit_mode(true);
  return 0;
}

long gw_audit_launch_count(void) { return audit_count(); }

}  // extern "C"

// ===========================================================================
// Grouped stage A (serving).  Requests of one padded shape (Np, Kp, Rp) share
// one set of stage-A launches: batch item b = j * Gx + g is grid point g of
// request j (the serving grid extended by xi = 0 for the preconditioner), the
// per-request operands (B_ov and its mixed copies, D, R and its split, |b|^2,
// the W^c table and M^-1) are read through device tables of pointers, and the
// per-item work (scales, 1 - Pi, Cholesky, L^-1, W^c partials) lives in the
// group's own workspace.  The launch sequence for n requests is captured once
// into a graph and replayed for every later batch of n: only the pointer
// tables change between replays.

namespace {
enum { T_BOV, T_D, T_R, T_BN, T_WTAB, T_PRE, T_B32, T_BHI, T_BLO, T_RH, T_COUNT };
}

struct gw_group {
  gw_ctx* lead = nullptr;   // owns the workspace for n_max * Gx items and the stream
  int Np = 0, Kp = 0, Rp = 0, Gx = 0, n_max = 0;
  int pi_prec = 0, wc_prec = 0;
  std::vector<double> xi, w;          // serving grid, then xi = 0 (weight 0)
  void** d_tab = nullptr;             // [T_COUNT][n_max] pointers, then n_max ints (Kov)
  void** h_tab = nullptr;             // pinned host copy
  int* h_info = nullptr;              // pinned: Cholesky pivot flags of a batch
  std::vector<hipGraphExec_t> graphs; // [n]: the launch sequence for n requests
  long batches = 0, items = 0, replays = 0;
  size_t tab_bytes() const { return (size_t)n_max * (T_COUNT * sizeof(void*) + sizeof(int)); }
  ~gw_group() {
    for (hipGraphExec_t g : graphs)
      if (g) hipGraphExecDestroy(g);
    if (lead) {
      host_free(lead->cache, h_tab);
      host_free(lead->cache, h_info);
      delete lead;
    }
  }
};

namespace {

// device elements each member operand must hold (checked per member per batch;
// the launch guards are evaluated against these)
struct GroupExt {
  long bov, d, r, bn, wtab, pre, b32, bhalf, rh;
};
GroupExt group_ext(const gw_group* g) {
  const long NK = (long)g->Np * g->Kp, RN = (long)g->Rp * g->Np;
  return GroupExt{NK, g->Kp, RN, g->Rp, (long)g->Rp * g->Gx, (long)g->Np * g->Np, NK, NK, 2 * RN};
}

// the stage-A launches of a batch of n requests (tables already on the device)
int group_sequence(gw_group* g, int n) {
  gw_ctx* L = g->lead;
  const int G = n * g->Gx, Np = g->Np, Kp = g->Kp, Rp = g->Rp;
  const long ldA = work_ld(L), per_g = work_per_g(L);
  const GroupExt ex = group_ext(g);
  void** tab = g->d_tab;
  auto T = [&](int k) { return tab + (size_t)k * g->n_max; };
  const int* kov = reinterpret_cast<const int*>(T(T_COUNT));
  HIPCHK(make_scale_imag_tab((const double* const*)T(T_D), kov, Kp, L->d_grid, g->Gx, G,
                             L->d_scale, g->pi_prec == GW_PI_FP64 ? nullptr : L->d_scale32, ex.d,
                             L->ext(L->d_grid, 8), L->ext(L->d_scale, 8),
                             L->ext(L->d_scale32, 4), L->st));
  if (g->pi_prec == GW_PI_FP64) {
    GemmArgs a{};
    a.Atab = (const double* const*)T(T_BOV); a.lda = Kp;
    a.Btab = (const double* const*)T(T_BOV); a.ldb = Kp;
    a.grp = g->Gx;
    a.scale = L->d_scale; a.sS = Kp;
    a.C = L->d_work; a.ldc = ldA; a.sC = per_g;
    a.M = Np; a.N = Np; a.K = Kp;
    a.map = MAP_LOWER;
    a.tiles_m = Np / 128; a.tiles_n = Np / 128;
    a.n_tiles = (int)lower_tile_count(a.tiles_m, a.tiles_n, 128, 128);
    a.batch = G; a.splitk = 1;
    a.nA = ex.bov; a.nB = ex.bov;
    a.nS = L->ext(L->d_scale, 8); a.nC = L->ext(L->d_work, 8);
    HIPCHK(gemm_f64(a, 0, KC, KC, EPI_ONE_PLUS_4, L->st));
  } else {
    OperandTabs tb{};
    tb.B32 = (const float* const*)T(T_B32);
    tb.Bhi = (const uint16_t* const*)T(T_BHI);
    tb.Blo = (const uint16_t* const*)T(T_BLO);
    tb.grp = g->Gx;
    if (g->pi_prec == GW_PI_FP32)
      HIPCHK(pi_build_f32_tab(tb, Kp, L->d_scale32, Kp, L->d_work, ldA, per_g, Np, Kp, G, ex.b32,
                              L->ext(L->d_scale32, 4), L->ext(L->d_work, 8), L->st));
    else
      HIPCHK(pi_build_bf16x3_tab(tb, Kp, L->d_scale32, Kp, L->d_work, ldA, per_g, Np, Kp, G,
                                 std::min(ex.b32, ex.bhalf), L->ext(L->d_scale32, 4),
                                 L->ext(L->d_work, 8), L->st));
  }
  RCHK(cholesky_chunk(L, G, per_g, ldA, true));
  const double* X = L->d_work + (long)Np * ldA;   // L^-T rows of every item
  if (g->wc_prec == GW_PI_BF16X3) {
    const long sF = (long)Np * Np;
    const long nF = (long)L->f_cap * sF;
    uint16_t* Fh = L->d_F;
    uint16_t* Fl = L->d_F + nF;
    HIPCHK(split_linv(X, ldA, per_g, Np, G, Fh, Fl, sF, L->ext(X, 8), nF, L->st));
    OperandTabs tb{};
    tb.Rh = (const uint16_t* const*)T(T_RH);
    tb.grp = g->Gx;
    HIPCHK(wc_bf16x3_tab(tb, (long)Rp * Np, Np, Rp, Fh, Fl, sF, Np, G, L->d_parts, parts_ld(L),
                         parts_per_g(L), ex.rh / 2, nF, L->ext(L->d_parts, 8), L->st));
    HIPCHK(wc_from_parts_tab(L->d_parts, parts_per_g(L), wc_bf16x3_panels(Np), parts_ld(L),
                             nullptr, Rp, G,
                             g->Gx, (double* const*)T(T_WTAB), L->ext(L->d_parts, 8), 0, ex.wtab,
                             L->st));
  } else {
    GemmArgs a{};
    a.Atab = (const double* const*)T(T_R); a.lda = Np; a.grp = g->Gx;
    a.B = X; a.ldb = ldA; a.sB = per_g;
    a.C = L->d_parts; a.ldc = parts_ld(L); a.sC = parts_per_g(L);
    a.M = Rp; a.N = Np; a.K = Np;
    a.map = MAP_FULL_J; a.tiles_m = Rp / 128; a.tiles_n = Np / 128;
    a.n_tiles = a.tiles_m * a.tiles_n; a.batch = G; a.splitk = 1; a.ktri = 1;
    a.nA = ex.r; a.nB = L->ext(X, 8); a.nC = L->ext(L->d_parts, 8);
    HIPCHK(gemm_f64(a, 0, KC, KM, EPI_SQNORM, L->st));
    HIPCHK(wc_from_parts_tab(L->d_parts, parts_per_g(L), Np / 128, parts_ld(L),
                             (const double* const*)T(T_BN), Rp, G, g->Gx,
                             (double* const*)T(T_WTAB), L->ext(L->d_parts, 8), ex.bn, ex.wtab,
                             L->st));
  }
  {  // M^-1 = X0 X0^T of each request, X0 from its xi = 0 item (the last)
    GemmArgs a{};
    const double* X0 = X + (long)(g->Gx - 1) * per_g;
    a.A = X0; a.lda = ldA; a.sA = (long)g->Gx * per_g;
    a.B = X0; a.ldb = ldA; a.sB = (long)g->Gx * per_g;
    a.Ctab = (double* const*)T(T_PRE); a.ldc = Np; a.grp = 1;
    a.M = Np; a.N = Np; a.K = Np;
    a.map = MAP_FULL; a.tiles_m = Np / 64; a.tiles_n = Np / 128;
    a.n_tiles = a.tiles_m * a.tiles_n; a.batch = n; a.splitk = 1;
    a.alpha = 1.0; a.beta = 0.0;
    a.nA = L->ext(X0, 8); a.nB = a.nA; a.nC = ex.pre;
    HIPCHK(gemm_f64(a, 2, KC, KC, EPI_AXPBY, L->st));
  }
  return 0;
}

// a member context of the group's shape, made ready for one batch: its W^c
// table and M^-1 buffers allocated, its mixed copies split
int group_member_prepare(gw_group* g, gw_ctx* m) {
  if (m->Np != g->Np || m->Kp != g->Kp || m->Rp != g->Rp || m->n_spin != 1 ||
      m->pi_prec != g->pi_prec || m->wc_prec != g->wc_prec || m->no_precond)
    return fail(GW_EINVAL, "request does not match the group's shape or options");
  const size_t wt = (size_t)g->Rp * g->Gx;
  if (m->d_wtab && m->ext(m->d_wtab, 8) < (long)wt) {
    m->release(m->d_wtab);
    m->d_wtab = nullptr;
  }
  if (!m->d_wtab) RCHK(m->alloc((void**)&m->d_wtab, wt * sizeof(double)));
  if (!m->d_pre) RCHK(m->alloc((void**)&m->d_pre, (size_t)g->Np * g->Np * sizeof(double)));
  // the grid (nodes and weights) the member's quadrature reads, as its own
  // stage A would have left it
  RCHK(upload_grid(m, g->Gx, g->xi.data(), g->w.data()));
  if (g->pi_prec != GW_PI_FP64) RCHK(ensure_mixed_operands(m));
  if (g->wc_prec == GW_PI_BF16X3) RCHK(ensure_r_split(m));
  const GroupExt ex = group_ext(g);
  const bool ok = m->ext(m->d_Bov, 8) >= ex.bov && m->ext(m->d_D, 8) >= ex.d &&
                  m->ext(m->d_R, 8) >= ex.r && m->ext(m->d_bn, 8) >= ex.bn &&
                  m->ext(m->d_wtab, 8) >= ex.wtab && m->ext(m->d_pre, 8) >= ex.pre &&
                  (g->pi_prec == GW_PI_FP64 ||
                   (m->ext(m->d_B32, 4) >= ex.b32 && m->ext(m->d_Bhi, 2) >= ex.bhalf &&
                    m->ext(m->d_Blo, 2) >= ex.bhalf)) &&
                  (g->wc_prec != GW_PI_BF16X3 || m->ext(m->d_Rh, 2) >= ex.rh);
  if (!ok) return fail(GW_EINVAL, "member buffers smaller than the group's shape");
  return 0;
}

// the member's W^c table (and preconditioner) now hold the group's results
void group_member_finish(gw_group* g, gw_ctx* m) {
  m->wtab_valid = true;
  m->wtab_G = g->Gx;
  m->wtab_w0 = 1;
  m->wtab_w0col = true;
  m->quad_G = g->Gx - 1;
  m->wtab_prec = g->pi_prec;
  m->wtab_wcprec = g->wc_prec;
  m->wtab_xi = g->xi;
  m->wtab_w = g->w;
  double dmin = INFINITY;
  const double* e = m->eps.data();
  dmin = *std::min_element(e + m->n_occ, e + m->n_mo) - *std::max_element(e, e + m->n_occ);
  m->pre_w = 0.9 * dmin;
  m->pre_valid = true;
}

}  // namespace

// Creates a group for requests of padded shape (Np, Kp, Rp) on `grid` (the
// xi = 0 point is appended), batches of at most n_max, with its own stream and
// workspace; device and pinned blocks from `cache` (nullable).
int group_create(gw_group** out, int Np, int Kp, int Rp, const gw_grid* grid, int n_max,
                 int pi_prec, int wc_prec, gw_devcache* cache, bool graphs) {
  *out = nullptr;
  RCHK(check_grid(grid));
  if (Np < 128 || Np % 128 || Kp < 128 || Kp % 128 || Rp < 128 || Rp % 128 || n_max < 1 ||
      n_max > 64)
    return fail(GW_EINVAL, "bad group shape");
  gw_group* g = new gw_group();
  g->Np = Np; g->Kp = Kp; g->Rp = Rp; g->Gx = grid->n + 1; g->n_max = n_max;
  g->pi_prec = pi_prec; g->wc_prec = wc_prec;
  g->xi.assign(grid->xi, grid->xi + grid->n);
  g->w.assign(grid->w, grid->w + grid->n);
  g->xi.push_back(0.0);
  g->w.push_back(0.0);
  g->graphs.assign(n_max + 1, nullptr);
  gw_ctx* L = new gw_ctx();
  g->lead = L;
  L->cache = cache;
  L->n_mo = 2; L->n_occ = 1; L->n_virt = 1; L->n_aux = Np;
  L->Np = Np; L->Kp = Kp; L->Kov = Kp; L->Rp = Rp; L->nR = Rp;
  L->pi_prec = pi_prec; L->wc_prec = wc_prec;
  L->work_budget = (size_t)1 << 62;     // one chunk holds every item of a full batch
  L->graphs_off = !graphs || debug_sync();
  if (const char* e = getenv("GW_TEST_INDEFINITE")) L->test_indefinite = atoi(e) != 0;
  auto bad = [&](int rc) {
    std::string keep = g_err;
    delete g;
    g_err = keep;
    return rc;
  };
  if (!audit_mode()) {
    if (hipStreamCreateWithFlags(&L->st, hipStreamNonBlocking) != hipSuccess)
      return bad(fail(GW_EDEVICE, "hipStreamCreate failed"));
    L->own_stream = true;
  }
  int rc;
  if ((rc = setup_work(L, n_max * g->Gx))) return bad(rc);
  if ((rc = upload_grid(L, g->Gx, g->xi.data(), g->w.data()))) return bad(rc);
  if (wc_prec == GW_PI_BF16X3) {
    if ((rc = L->alloc((void**)&L->d_F, 2 * (size_t)L->chunk * Np * Np * sizeof(uint16_t))))
      return bad(rc);
    L->f_cap = L->chunk;
  }
  if ((rc = L->alloc((void**)&g->d_tab, g->tab_bytes()))) return bad(rc);
  if (host_alloc(cache, (void**)&g->h_tab, g->tab_bytes()) != hipSuccess ||
      host_alloc(cache, (void**)&g->h_info, (size_t)n_max * g->Gx * sizeof(int)) != hipSuccess)
    return bad(fail(GW_ENOMEM, "pinned host allocation failed"));
  if (rt_sync(L->st) != hipSuccess) return bad(fail(GW_EDEVICE, "group setup failed"));
  *out = g;
  return 0;
}

void group_free(gw_group* g) { delete g; }

// Moves a context to another stream (its pending work on the old one is
// finished first); the server uses it to run a request's quasiparticle stage
// on the pipeline that picks it up.
int ctx_set_stream(gw_ctx* c, hipStream_t st) {
  if (c->st == st) return 0;
  HIPCHK(rt_sync(c->st));
  if (c->own_stream && c->st) hipStreamDestroy(c->st);
  c->own_stream = false;
  c->st = st;
  return 0;
}

// padded shape of a closed-shell request (the context's Np, Kp, Rp)
void padded_shape(int n_mo, int n_occ, int n_aux, int n_rows, int* Np, int* Kp, int* Rp) {
  *Np = round_up(n_aux, 128);
  *Kp = round_up(n_occ * (n_mo - n_occ), 128);
  *Rp = round_up(std::max(n_rows * n_mo, 1), 128);
}

// device bytes of a group's workspace for batches of n (the pointer tables aside)
size_t group_bytes(int Np, int Kp, int Rp, int grid_n, int n, int pi_prec, int wc_prec) {
  const size_t d = sizeof(double);
  const size_t items = (size_t)n * (grid_n + 1);
  const size_t per_g = (size_t)(2L * Np + 128) * (Np + 128);
  size_t b = items * (per_g * d + (size_t)(Np / 128) * Rp * d + PANEL * PANEL * d + sizeof(int) +
                      (size_t)Kp * (d + 4));
  if (wc_prec == GW_PI_BF16X3) b += items * (size_t)Np * Np * 4;
  (void)pi_prec;
  return b;
}

// Stage A of n member contexts (created with the group's padded shape and
// options) in one replay of the group's graph.  rc[j] receives each member's
// outcome: 0 (its W^c table and preconditioner are then cached, so gw_qp on it
// goes straight to the quasiparticle stage) or GW_ENOTSPD.  Returns a hard
// error for the whole batch (bad arguments, device failure) or 0.
int group_run(gw_group* g, gw_ctx* const* m, int n, int* rc) {
  if (!g || !m || n < 1 || n > g->n_max) return fail(GW_EINVAL, "bad group batch");
  gw_ctx* L = g->lead;
  for (int j = 0; j < n; ++j) RCHK(group_member_prepare(g, m[j]));
  for (int j = 0; j < n; ++j) HIPCHK(rt_sync(m[j]->st));   // uploads and splits are done
  void** T = g->h_tab;
  std::fill(T, T + (size_t)T_COUNT * g->n_max, nullptr);
  int* kov = reinterpret_cast<int*>(T + (size_t)T_COUNT * g->n_max);
  for (int j = 0; j < g->n_max; ++j) {
    gw_ctx* c = m[std::min(j, n - 1)];   // unused entries repeat the last member
    T[T_BOV * g->n_max + j] = c->d_Bov;
    T[T_D * g->n_max + j] = c->d_D;
    T[T_R * g->n_max + j] = c->d_R;
    T[T_BN * g->n_max + j] = c->d_bn;
    T[T_WTAB * g->n_max + j] = c->d_wtab;
    T[T_PRE * g->n_max + j] = c->d_pre;
    T[T_B32 * g->n_max + j] = c->d_B32;
    T[T_BHI * g->n_max + j] = c->d_Bhi;
    T[T_BLO * g->n_max + j] = c->d_Blo;
    T[T_RH * g->n_max + j] = c->d_Rh;
    kov[j] = c->Kov;
  }
  HIPCHK(rt_memcpy(g->d_tab, g->h_tab, g->tab_bytes(), hipMemcpyHostToDevice, L->st));
  if (!L->graphs_off && !audit_mode()) {
    if (!g->graphs[n]) {
      if (hipStreamBeginCapture(L->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        L->graphs_off = true;
      } else {
        const int r = group_sequence(g, n);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(L->st, &gr);
        if (r != 0 || e != hipSuccess) {
          if (gr) hipGraphDestroy(gr);
          if (r != 0) return r;
          HIPCHK(e);
        }
        const hipError_t ei = hipGraphInstantiate(&g->graphs[n], gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        HIPCHK(ei);
        trace("group graph captured Np=%d Kp=%d Rp=%d n=%d", g->Np, g->Kp, g->Rp, n);
      }
    }
  }
  if (g->graphs[n]) {
    HIPCHK(hipGraphLaunch(g->graphs[n], L->st));
    g->replays++;
  } else {
    RCHK(group_sequence(g, n));
  }
  const int items = n * g->Gx;
  HIPCHK(rt_memcpy(g->h_info, L->d_info, (size_t)items * sizeof(int), hipMemcpyDeviceToHost, L->st));
  HIPCHK(rt_sync(L->st));
  g->batches++;
  g->items += items;
  for (int j = 0; j < n; ++j) {
    rc[j] = 0;
    for (int q = 0; q < g->Gx; ++q)
      if (g->h_info[j * g->Gx + q] != 0) rc[j] = GW_ENOTSPD;
    if (rc[j] == 0) group_member_finish(g, m[j]);
    else m[j]->wtab_valid = false;
  }
  return 0;
}

void group_stats(const gw_group* g, long* batches, long* items, long* replays) {
  *batches = g->batches;
  *items = g->items;
  *replays = g->replays;
}

gw_devcache* devcache_create(size_t cap) {
  gw_devcache* c = new gw_devcache();
  c->cap = cap;
  return c;
}
void devcache_destroy(gw_devcache* c) { delete c; }
void devcache_stats(gw_devcache* c, long* mallocs, long* hits, long* frees, size_t* live,
                    size_t* cached) {
  std::lock_guard<std::mutex> lk(c->mu);
  *mallocs = c->n_malloc;
  *hits = c->n_hits;
  *frees = c->n_free;
  *live = c->live;
  *cached = c->cached;
}

extern "C" int gw_group_stage_a(int n, gw_ctx* const* ctxs, const gw_grid* grid, int use_graph,
                                int* rc) {
  if (n < 1 || !ctxs || !rc) return fail(GW_EINVAL, "bad arguments");
  for (int j = 0; j < n; ++j)
    if (!ctxs[j]) return fail(GW_EINVAL, "NULL context");
  const gw_ctx* c0 = ctxs[0];
  gw_group* g = nullptr;
  RCHK(group_create(&g, c0->Np, c0->Kp, c0->Rp, grid, n, c0->pi_prec, c0->wc_prec, nullptr,
                    use_graph != 0));
  const int r = group_run(g, ctxs, n, rc);
  group_free(g);
  return r == 0 ? finish() : r;
}

// ===========================================================================
// Allocation-free form of gw_dielectric (include/gw.h): the scale vectors live
// in a file-scope device array instead of the context's stage-A workspace, and
// the matrices go straight into the caller's device buffer.

namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = 32ull << 20;
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// per-device address of `scratch` (the array's name is no device address in
// host code), looked up once per device with that device current
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_ptr(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(GW_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GW_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}
}  // namespace

extern "C" int gw_dielectric_noalloc(gw_ctx* c, int n_xi, const double* d_xi, double* d_out,
                                     long ld_out, long out_stride) {
  if (!c || n_xi < 1 || !d_xi || !d_out) return fail(GW_EINVAL, "bad arguments");
  if (audit_mode()) return fail(GW_EINVAL, "gw_dielectric_noalloc has no launch-audit form");
  if (ld_out < c->Np || out_stride < (long)c->Np * ld_out || (ld_out & 1))
    return fail(GW_EINVAL, "output layout: need ld_out >= %d (even) and out_stride >= %d * ld_out",
                c->Np, c->Np);
  const bool mixed = c->pi_prec != GW_PI_FP64;
  const size_t need = (size_t)n_xi * c->Kp * (sizeof(double) + (mixed ? sizeof(float) : 0));
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(GW_EINVAL, "n_xi = %d needs %zu bytes of scratch, more than its %zu (at most %zu "
                "grid points for this context)", n_xi, need, NOALLOC_SCRATCH_BYTES,
                NOALLOC_SCRATCH_BYTES / ((size_t)c->Kp * (sizeof(double) + (mixed ? 4 : 0))));
  if (mixed && !c->d_B32)
    return fail(GW_EINVAL, "the context's split copies of B_ov are not built yet (a first "
                "gw_dielectric, gw_wtable or gw_qp call builds them)");
  char* base = nullptr;
  RCHK(scratch_ptr(&base));
  double* s64 = reinterpret_cast<double*>(base);
  float* s32 = mixed ? reinterpret_cast<float*>(base + (size_t)n_xi * c->Kp * sizeof(double))
                     : nullptr;
  const long nS = (long)n_xi * c->Kp;
  const long nOut = (long)(n_xi - 1) * out_stride + (long)(c->Np - 1) * ld_out + c->Np;
  // every scale entry the builds read is written here first (no clearing needed)
  HIPCHK(make_scale_imag(c->d_D, c->Kov, c->Kp, d_xi, n_xi, s64, s32, c->ext(c->d_D, 8), n_xi, nS,
                         nS, c->st));
  if (!mixed) {
    GemmArgs a{};
    a.A = c->d_Bov; a.lda = c->Kp; a.sA = 0;
    a.B = c->d_Bov; a.ldb = c->Kp; a.sB = 0;
    a.scale = s64; a.sS = c->Kp;
    a.C = d_out; a.ldc = ld_out; a.sC = out_stride;
    a.M = c->Np; a.N = c->Np; a.K = c->Kp;
    a.map = MAP_LOWER;
    a.tiles_m = c->Np / 128; a.tiles_n = c->Np / 128;
    a.n_tiles = (int)lower_tile_count(a.tiles_m, a.tiles_n, 128, 128);
    a.batch = n_xi; a.splitk = 1;
    a.nA = c->ext(c->d_Bov, 8); a.nB = a.nA; a.nS = nS; a.nC = nOut;
    HIPCHK(gemm_f64(a, 0, KC, KC, EPI_ONE_PLUS_4, c->st));
  } else if (c->pi_prec == GW_PI_FP32) {
    HIPCHK(pi_build_f32(c->d_B32, c->Kp, s32, c->Kp, d_out, ld_out, out_stride, c->Np, c->Kp, n_xi,
                        c->ext(c->d_B32, 4), nS, nOut, c->st));
  } else {
    const long nB = std::min({c->ext(c->d_Bhi, 2), c->ext(c->d_Blo, 2), c->ext(c->d_B32, 4)});
    HIPCHK(pi_build_bf16x3(c->d_Bhi, c->d_Blo, c->Kp, c->d_B32, s32, c->Kp, d_out, ld_out,
                           out_stride, c->Np, c->Kp, n_xi, nB, nS, nOut, c->st));
  }
  return 0;
}
