// Batched MINRES (Paige and Saunders) for the residue systems
// (1 - Pi(w_j)) x_j = b_j, one system per real frequency w_j.  The matrix is
// never formed: A v = v + 4 B_ov diag(D/(D^2 - w^2)) B_ov^T v is applied as
// two MFMA GEMM passes over B_ov (see gemm_f64.hip) for all systems at once.
// This file holds the per-system Lanczos / Givens recurrences, one
// workgroup per system.
#include <algorithm>

#include "gw_internal.h"

namespace gw {

enum {
  S_BETA1 = 0, S_BETA, S_OLDB, S_DBAR, S_EPS, S_PHIBAR, S_CS, S_SN, S_DONE, S_ITERS, S_RATIO,
  S_BNORM, S_ALPHA
};

static hipError_t check_bufs(const MinresBufs& m, const char* kn) {
  if (m.k < 0 || m.k > m.kp || m.kp % 64 != 0) return refuse(kn, "system count");
  GW_GUARD(kn, "vectors", (long)m.kp * m.Np - 1, m.n_vec);
  GW_GUARD(kn, "scalars", (long)m.kp * 16 - 1, m.n_scal);
  return hipSuccess;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  return s;
}

__global__ void k_minres_gather(MinresBufs m, const double* xcache, const int* rhs_idx,
                                const int* warm) {
  const int j = blockIdx.y;
  const long o = (long)j * m.Np;
  const bool w = j < m.k && warm[j] != 0;
  const double* src = w ? xcache + (long)rhs_idx[j] * m.Np : nullptr;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m.Np; p += gridDim.x * blockDim.x) {
    const double v = w ? src[p] : 0.0;
    m.x0[o + p] = v;
    m.v[o + p] = v;
  }
}

static hipError_t check_rows(const MinresBufs& m, const char* kn, const int* host_idx, int n_rows,
                             long n_cache) {
  for (int j = 0; j < m.k; ++j)
    if (host_idx[j] < 0 || host_idx[j] >= n_rows) return refuse(kn, "rhs index");
  GW_GUARD(kn, "xcache", (long)n_rows * m.Np - 1, n_cache);
  return hipSuccess;
}

hipError_t minres_gather(MinresBufs& m, const double* xcache, const int* rhs_idx,
                         const int* host_idx, int n_rows, const int* warm, long n_cache,
                         hipStream_t st) {
  if (hipError_t e = check_bufs(m, "minres_gather")) return e;
  if (hipError_t e = check_rows(m, "minres_gather", host_idx, n_rows, n_cache)) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_gather, dim3((m.Np + 255) / 256, m.kp), dim3(256), 0, st, m, xcache,
                     rhs_idx, warm);
  return hipGetLastError();
}

// Start vectors: r = b - A x0 when use_y (y = A x0), else r = b.  Block 0
// also clears the convergence counters and block flags of both parities.
__global__ __launch_bounds__(256) void k_minres_init(MinresBufs m, const double* rhs_base,
                                                     const int* rhs_idx, int use_y) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  if (j == 0) {
    if (t < 2) m.active[t] = 0;
    for (int i = t; i < 2 * (m.kp / 16); i += 256) m.blk[i] = 0;
  }
  const long o = (long)j * m.Np;
  const double* b = (j < m.k) ? rhs_base + (long)rhs_idx[j] * m.Np : nullptr;
  double s = 0.0, sb = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    const double bv = b ? b[p] : 0.0;
    const double rv = use_y ? bv - m.y[o + p] : bv;
    m.r1[o + p] = rv;
    m.r2[o + p] = rv;
    m.y[o + p] = rv;
    m.x[o + p] = 0.0;
    m.w[o + p] = 0.0;
    m.w2[o + p] = 0.0;
    s += rv * rv;
    sb += bv * bv;
  }
  const double beta1 = sqrt(block_sum(s, red));
  const double bnorm = sqrt(block_sum(sb, red));
  const double inv = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  for (int p = t; p < m.Np; p += 256) m.v[o + p] = m.y[o + p] * inv;
  if (t == 0) {
    double* sc = m.scal + j * 16;
    sc[S_BETA1] = beta1;
    sc[S_BETA] = beta1;
    sc[S_OLDB] = 0.0;
    sc[S_DBAR] = 0.0;
    sc[S_EPS] = 0.0;
    sc[S_PHIBAR] = beta1;
    sc[S_CS] = -1.0;
    sc[S_SN] = 0.0;
    sc[S_DONE] = (j < m.k && beta1 > 0.0) ? 0.0 : 1.0;
    sc[S_ITERS] = 0.0;
    sc[S_RATIO] = 0.0;
    sc[S_BNORM] = bnorm;
  }
}

hipError_t minres_init(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                       const int* host_idx, int n_rhs_rows, int use_y, hipStream_t st) {
  if (hipError_t e = check_bufs(m, "minres_init")) return e;
  GW_GUARD("minres_init", "blk", 2L * (m.kp / 16) - 1, m.n_blk);
  for (int j = 0; j < m.k; ++j)
    if (host_idx[j] < 0 || host_idx[j] >= n_rhs_rows) return refuse("minres_init", "rhs index");
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_init, dim3(m.kp), dim3(256), 0, st, m, rhs_base, rhs_idx, use_y);
  return hipGetLastError();
}

__global__ void k_minres_finalize(MinresBufs m, double* xcache, const int* rhs_idx) {
  const int j = blockIdx.y;
  if (j >= m.k) return;
  const long o = (long)j * m.Np;
  double* dst = xcache + (long)rhs_idx[j] * m.Np;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m.Np; p += gridDim.x * blockDim.x) {
    const double v = m.x[o + p] + m.x0[o + p];
    m.x[o + p] = v;
    dst[p] = v;
  }
}

hipError_t minres_finalize(MinresBufs& m, double* xcache, const int* rhs_idx,
                           const int* host_idx, int n_rows, long n_cache, hipStream_t st) {
  if (m.k <= 0) return hipSuccess;
  if (hipError_t e = check_bufs(m, "minres_finalize")) return e;
  if (hipError_t e = check_rows(m, "minres_finalize", host_idx, n_rows, n_cache)) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_finalize, dim3((m.Np + 255) / 256, m.k), dim3(256), 0, st, m, xcache,
                     rhs_idx);
  return hipGetLastError();
}

// V[j][ia] = D_ia/(D_ia^2 - w_j^2) sum_s part[s][j][ia]: finishes the first
// operator pass from its partials over N_aux, in a fixed order.  One block row
// per system; with a mask, systems of 16-system blocks flagged converged are
// skipped (the second pass does not multiply their rows of V).
__global__ void k_minres_scale_sum(MinresBufs m, int splits, const double* D, const int* mask) {
  const int j = blockIdx.y;
  if (mask && mask[j >> 4] == 0) return;
  const long n = (long)m.kp * m.Kp;
  const double w = m.omega[j];
  for (int ia = blockIdx.x * blockDim.x + threadIdx.x; ia < m.Kp; ia += gridDim.x * blockDim.x) {
    const long i = (long)j * m.Kp + ia;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += m.part[s * n + i];
    const double d = D[ia];
    m.V[i] = acc * (d / (d * d - w * w));
  }
}

hipError_t minres_scale_sum(MinresBufs& m, int splits, const double* D, long nD,
                            const int* mask, long nMask, hipStream_t st) {
  if (hipError_t e = check_bufs(m, "minres_scale_sum")) return e;
  GW_GUARD("minres_scale_sum", "part", (long)splits * m.kp * m.Kp - 1, m.n_part);
  GW_GUARD("minres_scale_sum", "V", (long)m.kp * m.Kp - 1, m.n_V);
  GW_GUARD("minres_scale_sum", "D", m.Kp - 1, nD);
  if (mask) GW_GUARD("minres_scale_sum", "mask", (m.kp - 1) / 16, nMask);
  GW_AUDIT_RETURN();
  const int bx = std::min((m.Kp + 255) / 256, 64);
  hipLaunchKernelGGL(k_minres_scale_sum, dim3(bx, m.kp), dim3(256), 0, st, m, splits, D, mask);
  return hipGetLastError();
}

// y = v + 4 sum_s part[s] for every element of every system: the matrix-vector
// product (1 - Pi(w)) v finished from the split-K partials of B_ov V^T.  One
// block row per system; with a mask, systems of converged 16-system blocks
// are skipped (their step is skipped too).
__global__ void k_minres_apply(MinresBufs m, int splitk, const int* mask) {
  const int j = blockIdx.y;
  if (mask && mask[j >> 4] == 0) return;
  const long slab = (long)m.kp * m.Np;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m.Np; p += gridDim.x * blockDim.x) {
    const long i = (long)j * m.Np + p;
    double av = 0.0;
    for (int s = 0; s < splitk; ++s) av += m.part[s * slab + i];
    m.y[i] = m.v[i] + 4.0 * av;
  }
}

hipError_t minres_apply(MinresBufs& m, int splitk, const int* mask, long nMask, hipStream_t st) {
  if (hipError_t e = check_bufs(m, "minres_apply")) return e;
  GW_GUARD("minres_apply", "part", (long)splitk * m.kp * m.Np - 1, m.n_part);
  if (mask) GW_GUARD("minres_apply", "mask", (m.kp - 1) / 16, nMask);
  GW_AUDIT_RETURN();
  const int bx = (m.Np + 255) / 256;
  hipLaunchKernelGGL(k_minres_apply, dim3(bx, m.kp), dim3(256), 0, st, m, splitk, mask);
  return hipGetLastError();
}

// One MINRES iteration for every unconverged system, given y = A v.  Each
// system counts its own iterations (S_ITERS), so the kernel depends on the
// global iteration only through its parity `par`: the systems still
// unconverged afterwards are counted in active[par] and flagged per 16-system
// block in blk[par]; the other slots (read after the previous iteration) are
// cleared for the next one.  This keeps the launch replayable from a graph.
__global__ __launch_bounds__(256) void k_minres_step(MinresBufs m, int par) {
  __shared__ double red[4];
  __shared__ double bc[5];
  const int j = blockIdx.x, t = threadIdx.x;
  const int nb = m.kp / 16;
  if (j == 0 && t == 0) m.active[par ^ 1] = 0;
  if (j == 0)
    for (int i = t; i < nb; i += 256) m.blk[(par ^ 1) * nb + i] = 0;
  double* sc = m.scal + j * 16;
  if (sc[S_DONE] != 0.0) return;
  const long o = (long)j * m.Np;
  const double beta = sc[S_BETA], oldb = sc[S_OLDB];
  const double itn = sc[S_ITERS] + 1.0;   // this system's iteration number
  // y = A v (- (beta/oldb) r1 from the second iteration on)
  const double c1 = (itn >= 2.0) ? beta / oldb : 0.0;
  double sa = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    double yv = m.y[o + p] - c1 * m.r1[o + p];
    m.y[o + p] = yv;
    sa += m.v[o + p] * yv;
  }
  const double alpha = block_sum(sa, red);
  double sb = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    double yv = m.y[o + p] - (alpha / beta) * m.r2[o + p];
    m.r1[o + p] = m.r2[o + p];
    m.r2[o + p] = yv;
    m.y[o + p] = yv;
    sb += yv * yv;
  }
  const double beta_new = sqrt(block_sum(sb, red));
  if (t == 0) {
    const double oldeps = sc[S_EPS];
    const double cs = sc[S_CS], sn = sc[S_SN], dbar = sc[S_DBAR];
    const double delta = cs * dbar + sn * alpha;
    const double gbar = sn * dbar - cs * alpha;
    const double epsln = sn * beta_new;
    const double dbar_n = -cs * beta_new;
    double gamma = sqrt(gbar * gbar + beta_new * beta_new);
    if (gamma < 1e-300) gamma = 1e-300;
    const double cs_n = gbar / gamma, sn_n = beta_new / gamma;
    const double phi = cs_n * sc[S_PHIBAR];
    const double phibar = sn_n * sc[S_PHIBAR];
    sc[S_OLDB] = beta;
    sc[S_BETA] = beta_new;
    sc[S_EPS] = epsln;
    sc[S_DBAR] = dbar_n;
    sc[S_CS] = cs_n;
    sc[S_SN] = sn_n;
    sc[S_PHIBAR] = phibar;
    sc[S_ITERS] = itn;
    // residual |b - A x| = phibar (the start vector is b - A x0); stop relative to |b|
    const double ratio = phibar / sc[S_BNORM];
    sc[S_RATIO] = ratio;
    const bool done = (ratio <= m.rtol[j]) || (beta_new <= 1e-300);
    if (done) sc[S_DONE] = 1.0;
    bc[0] = oldeps;
    bc[1] = delta;
    bc[2] = 1.0 / gamma;
    bc[3] = phi;
    bc[4] = done ? 1.0 : 0.0;
  }
  __syncthreads();
  const double oldeps = bc[0], delta = bc[1], ginv = bc[2], phi = bc[3];
  const bool done = bc[4] != 0.0;
  const double inv_b = (beta_new > 1e-300) ? 1.0 / beta_new : 0.0;
  for (int p = t; p < m.Np; p += 256) {
    double w1 = m.w2[o + p];
    double w2 = m.w[o + p];
    double wn = (m.v[o + p] - oldeps * w1 - delta * w2) * ginv;
    m.w2[o + p] = w2;
    m.w[o + p] = wn;
    m.x[o + p] += phi * wn;
    m.v[o + p] = done ? 0.0 : m.y[o + p] * inv_b;
  }
  if (t == 0 && !done) {
    atomicAdd(m.active + par, 1);
    m.blk[par * nb + j / 16] = 1;
  }
}

hipError_t minres_finish_step(MinresBufs& m, int par, hipStream_t st) {
  if (hipError_t e = check_bufs(m, "minres_step")) return e;
  GW_GUARD("minres_step", "blk", 2L * (m.kp / 16) - 1, m.n_blk);
  if (par != 0 && par != 1) return refuse("minres_step", "parity");
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_step, dim3(m.kp), dim3(256), 0, st, m, par);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Preconditioned MINRES (Paige and Saunders with a symmetric positive definite
// preconditioner M): the Lanczos vectors are built in the M^-1 inner product,
// z = M^-1 r supplies the next direction and beta = sqrt(r . z); the Givens
// recurrences are unchanged and phibar estimates |b - A x| in the M^-1 norm.
// Systems outside the preconditioned frequency window take z = r, which is
// the plain recurrence.

__device__ __forceinline__ bool is_pre(const MinresBufs& m, int j) {
  return m.pre != nullptr && m.preflag[j] != 0;
}

// z[p] of system j: the sum of the splitp slabs of r M^-1
__device__ __forceinline__ double pre_z(const MinresBufs& m, long i) {
  const long slab = (long)m.kp * m.Np;
  double z = 0.0;
  for (int s = 0; s < m.splitp; ++s) z += m.part[s * slab + i];
  return z;
}

// r1 = r2 = b - A x0 (or b); w = b (input of the first product); x = w2 = 0;
// |b| and |r| (the norms of unpreconditioned systems)
__global__ __launch_bounds__(256) void k_minres_pre_init_a(MinresBufs m, const double* rhs_base,
                                                           const int* rhs_idx, int use_y) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  if (j == 0) {
    if (t < 2) m.active[t] = 0;
    for (int i = t; i < 2 * (m.kp / 16); i += 256) m.blk[i] = 0;
  }
  const long o = (long)j * m.Np;
  const double* b = (j < m.k) ? rhs_base + (long)rhs_idx[j] * m.Np : nullptr;
  double s = 0.0, sb = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    const double bv = b ? b[p] : 0.0;
    const double rv = use_y ? bv - m.y[o + p] : bv;
    m.r1[o + p] = rv;
    m.r2[o + p] = rv;
    m.w[o + p] = bv;
    m.x[o + p] = 0.0;
    m.w2[o + p] = 0.0;
    s += rv * rv;
    sb += bv * bv;
  }
  const double rn = sqrt(block_sum(s, red));
  const double bn = sqrt(block_sum(sb, red));
  if (t == 0) {
    double* sc = m.scal + j * 16;
    sc[S_BETA1] = rn;
    sc[S_BNORM] = bn;
  }
}

// |b|_M^-1 = sqrt(b . b M^-1) for preconditioned systems
__global__ __launch_bounds__(256) void k_minres_pre_init_b(MinresBufs m) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  if (!is_pre(m, j)) return;
  const long o = (long)j * m.Np;
  double s = 0.0;
  for (int p = t; p < m.Np; p += 256) s += m.w[o + p] * pre_z(m, o + p);
  const double bn = sqrt(fmax(block_sum(s, red), 0.0));
  if (t == 0) m.scal[j * 16 + S_BNORM] = bn;
}

// beta1 = sqrt(r . z), v = z / beta1 (z = r M^-1, or r), w = 0, scalars
__global__ __launch_bounds__(256) void k_minres_pre_init_c(MinresBufs m) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  const long o = (long)j * m.Np;
  const bool pre = is_pre(m, j);
  double s = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    const double r = m.r1[o + p];
    const double z = pre ? pre_z(m, o + p) : r;
    m.y[o + p] = z;
    m.w[o + p] = 0.0;
    s += r * z;
  }
  const double beta1 = sqrt(fmax(block_sum(s, red), 0.0));
  const double inv = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
  for (int p = t; p < m.Np; p += 256) m.v[o + p] = m.y[o + p] * inv;
  if (t == 0) {
    double* sc = m.scal + j * 16;
    sc[S_BETA1] = beta1;
    sc[S_BETA] = beta1;
    sc[S_OLDB] = 0.0;
    sc[S_DBAR] = 0.0;
    sc[S_EPS] = 0.0;
    sc[S_PHIBAR] = beta1;
    sc[S_CS] = -1.0;
    sc[S_SN] = 0.0;
    sc[S_DONE] = (j < m.k && beta1 > 0.0) ? 0.0 : 1.0;
    sc[S_ITERS] = 0.0;
    sc[S_RATIO] = 0.0;
    sc[S_ALPHA] = 0.0;
  }
}

static hipError_t check_pre(const MinresBufs& m, const char* kn) {
  if (hipError_t e = check_bufs(m, kn)) return e;
  if (!m.pre || !m.preflag) return refuse(kn, "no preconditioner");
  if (m.splitp < 1) return refuse(kn, "splitp");
  GW_GUARD(kn, "part", (long)m.splitp * m.kp * m.Np - 1, m.n_part);
  return hipSuccess;
}

hipError_t minres_pre_init_a(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                             const int* host_idx, int n_rhs_rows, int use_y, hipStream_t st) {
  if (hipError_t e = check_pre(m, "minres_pre_init_a")) return e;
  GW_GUARD("minres_pre_init_a", "blk", 2L * (m.kp / 16) - 1, m.n_blk);
  for (int j = 0; j < m.k; ++j)
    if (host_idx[j] < 0 || host_idx[j] >= n_rhs_rows) return refuse("minres_pre_init_a", "rhs index");
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_pre_init_a, dim3(m.kp), dim3(256), 0, st, m, rhs_base, rhs_idx,
                     use_y);
  return hipGetLastError();
}

hipError_t minres_pre_init_b(MinresBufs& m, hipStream_t st) {
  if (hipError_t e = check_pre(m, "minres_pre_init_b")) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_pre_init_b, dim3(m.kp), dim3(256), 0, st, m);
  return hipGetLastError();
}

hipError_t minres_pre_init_c(MinresBufs& m, hipStream_t st) {
  if (hipError_t e = check_pre(m, "minres_pre_init_c")) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_pre_init_c, dim3(m.kp), dim3(256), 0, st, m);
  return hipGetLastError();
}

// Lanczos update, given y = A v: y -= (beta/oldb) r1 (second iteration on),
// alpha = v . y, y -= (alpha/beta) r2, r1 = r2, r2 = y.  (The other parity's
// block flags are still the mask of this iteration's preconditioner product;
// k_minres_pre_step_b clears them.)
__global__ __launch_bounds__(256) void k_minres_pre_step_a(MinresBufs m, int par) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  (void)par;
  double* sc = m.scal + j * 16;
  if (sc[S_DONE] != 0.0) return;
  const long o = (long)j * m.Np;
  const double beta = sc[S_BETA], oldb = sc[S_OLDB];
  const double itn = sc[S_ITERS] + 1.0;
  const double c1 = (itn >= 2.0) ? beta / oldb : 0.0;
  double sa = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    double yv = m.y[o + p] - c1 * m.r1[o + p];
    m.y[o + p] = yv;
    sa += m.v[o + p] * yv;
  }
  const double alpha = block_sum(sa, red);
  for (int p = t; p < m.Np; p += 256) {
    const double yv = m.y[o + p] - (alpha / beta) * m.r2[o + p];
    m.r1[o + p] = m.r2[o + p];
    m.r2[o + p] = yv;
  }
  if (t == 0) sc[S_ALPHA] = alpha;
}

// beta_new = sqrt(r2 . z), Givens rotation, w / x update, v = z / beta_new.
// Block 0 clears the other parity's counters as k_minres_step does.
__global__ __launch_bounds__(256) void k_minres_pre_step_b(MinresBufs m, int par) {
  __shared__ double red[4];
  __shared__ double bc[5];
  const int j = blockIdx.x, t = threadIdx.x;
  const int nb = m.kp / 16;
  if (j == 0 && t == 0) m.active[par ^ 1] = 0;
  if (j == 0)
    for (int i = t; i < nb; i += 256) m.blk[(par ^ 1) * nb + i] = 0;
  double* sc = m.scal + j * 16;
  if (sc[S_DONE] != 0.0) return;
  const long o = (long)j * m.Np;
  const bool pre = is_pre(m, j);
  double sb = 0.0;
  for (int p = t; p < m.Np; p += 256) {
    const double r = m.r2[o + p];
    const double z = pre ? pre_z(m, o + p) : r;
    m.y[o + p] = z;
    sb += r * z;
  }
  const double beta_new = sqrt(fmax(block_sum(sb, red), 0.0));
  if (t == 0) {
    const double beta = sc[S_BETA], alpha = sc[S_ALPHA];
    const double itn = sc[S_ITERS] + 1.0;
    const double oldeps = sc[S_EPS];
    const double cs = sc[S_CS], sn = sc[S_SN], dbar = sc[S_DBAR];
    const double delta = cs * dbar + sn * alpha;
    const double gbar = sn * dbar - cs * alpha;
    const double epsln = sn * beta_new;
    const double dbar_n = -cs * beta_new;
    double gamma = sqrt(gbar * gbar + beta_new * beta_new);
    if (gamma < 1e-300) gamma = 1e-300;
    const double cs_n = gbar / gamma, sn_n = beta_new / gamma;
    const double phi = cs_n * sc[S_PHIBAR];
    const double phibar = sn_n * sc[S_PHIBAR];
    sc[S_OLDB] = beta;
    sc[S_BETA] = beta_new;
    sc[S_EPS] = epsln;
    sc[S_DBAR] = dbar_n;
    sc[S_CS] = cs_n;
    sc[S_SN] = sn_n;
    sc[S_PHIBAR] = phibar;
    sc[S_ITERS] = itn;
    // phibar: |b - A x| in the M^-1 norm (plain norm for unpreconditioned
    // systems); the target is relative to |b| in the same norm
    const double ratio = phibar / sc[S_BNORM];
    sc[S_RATIO] = ratio;
    const bool done = (ratio <= m.rtol[j]) || (beta_new <= 1e-300);
    if (done) sc[S_DONE] = 1.0;
    bc[0] = oldeps;
    bc[1] = delta;
    bc[2] = 1.0 / gamma;
    bc[3] = phi;
    bc[4] = done ? 1.0 : 0.0;
  }
  __syncthreads();
  const double oldeps = bc[0], delta = bc[1], ginv = bc[2], phi = bc[3];
  const bool done = bc[4] != 0.0;
  const double inv_b = (beta_new > 1e-300) ? 1.0 / beta_new : 0.0;
  for (int p = t; p < m.Np; p += 256) {
    double w1 = m.w2[o + p];
    double w2 = m.w[o + p];
    double wn = (m.v[o + p] - oldeps * w1 - delta * w2) * ginv;
    m.w2[o + p] = w2;
    m.w[o + p] = wn;
    m.x[o + p] += phi * wn;
    m.v[o + p] = done ? 0.0 : m.y[o + p] * inv_b;
  }
  if (t == 0 && !done) {
    atomicAdd(m.active + par, 1);
    m.blk[par * nb + j / 16] = 1;
  }
}

hipError_t minres_pre_step_a(MinresBufs& m, int par, hipStream_t st) {
  if (hipError_t e = check_pre(m, "minres_pre_step_a")) return e;
  GW_GUARD("minres_pre_step_a", "blk", 2L * (m.kp / 16) - 1, m.n_blk);
  if (par != 0 && par != 1) return refuse("minres_pre_step_a", "parity");
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_pre_step_a, dim3(m.kp), dim3(256), 0, st, m, par);
  return hipGetLastError();
}

hipError_t minres_pre_step_b(MinresBufs& m, int par, hipStream_t st) {
  if (hipError_t e = check_pre(m, "minres_pre_step_b")) return e;
  GW_GUARD("minres_pre_step_b", "blk", 2L * (m.kp / 16) - 1, m.n_blk);
  if (par != 0 && par != 1) return refuse("minres_pre_step_b", "parity");
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_pre_step_b, dim3(m.kp), dim3(256), 0, st, m, par);
  return hipGetLastError();
}

// W^c = b.x - b.b and dW^c/dw = -4 sum of the derivative partials
__global__ __launch_bounds__(256) void k_minres_results(MinresBufs m, const double* rhs_base,
                                                        const int* rhs_idx, int nparts,
                                                        double* wc, double* dwc, int* conv) {
  __shared__ double red[4];
  const int j = blockIdx.x, t = threadIdx.x;
  const double* b = rhs_base + (long)rhs_idx[j] * m.Np;
  const long o = (long)j * m.Np;
  double s = 0.0;
  for (int p = t; p < m.Np; p += 256) s += b[p] * (m.x[o + p] - b[p]);
  const double bx = block_sum(s, red);
  double d = 0.0;
  for (int q = t; q < nparts; q += 256) d += m.part[(long)q * m.kp + j];
  const double dd = block_sum(d, red);
  if (t == 0) {
    wc[j] = bx;
    dwc[j] = -4.0 * dd;
    const double* sc = m.scal + j * 16;
    conv[j] = (sc[S_DONE] != 0.0) ? (int)sc[S_ITERS] : -(int)sc[S_ITERS] - 1;
  }
}

hipError_t minres_results(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                          int n_rhs_rows, int n_deriv_parts, double* wc, double* dwc, int* conv,
                          long n_out, hipStream_t st) {
  if (m.k <= 0) return hipSuccess;
  (void)n_rhs_rows;  // indices were checked by minres_init for this batch
  if (hipError_t e = check_bufs(m, "minres_results")) return e;
  GW_GUARD("minres_results", "part", (long)n_deriv_parts * m.kp - 1, m.n_part);
  GW_GUARD("minres_results", "outputs", m.k - 1, n_out);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_minres_results, dim3(m.k), dim3(256), 0, st, m, rhs_base, rhs_idx,
                     n_deriv_parts, wc, dwc, conv);
  return hipGetLastError();
}

}  // namespace gw
