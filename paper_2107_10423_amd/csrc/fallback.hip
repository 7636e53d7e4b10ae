// Dense fallback for residue systems that MINRES does not converge: the
// dielectric matrix 1 - Pi(w) is built explicitly (Pi build kernel with a
// signed scale) and solved by Gaussian elimination with partial pivoting.
// The paper switches to a Bunch-Kaufman factorization at this point; any
// stable dense solve of the same symmetric indefinite system gives the same x.
//
// Blocked right-looking LU (P A = L U) over a batch of systems, all padded to
// N_aux (a multiple of 128; the padding block of 1 - Pi is the identity, so
// the padded solution carries the true one unchanged).  Per 128-column panel:
//   k_lu_panel      the panel's column steps (pivot search over the rows
//                   below, swap inside the panel, multipliers, rank-1 update
//                   of the panel), one 1024-thread workgroup per system;
//   k_lu_swap_trsm  the panel's row swaps on every other column, and
//                   U12 = L11^-1 A12 right of the panel, one thread per column;
//   gemm_f64        A22 -= L21 U12 (MFMA, every system of the batch at once);
// then k_lu_solve applies the swaps to b and runs the two triangular solves,
// one workgroup per system with b in LDS (up to N_aux 6144; in place beyond).
#include "gw_internal.h"

namespace gw {

constexpr int LU_NB = 128;   // panel width (the trailing GEMM's tile)

__global__ __launch_bounds__(1024) void k_lu_panel(double* A, long ld, long sA, int n, int c0,
                                                   int* piv, long sP, int* info) {
  __shared__ double rv[1024];
  __shared__ int ri[1024];
  __shared__ int prow;
  A += (long)blockIdx.x * sA;
  piv += (long)blockIdx.x * sP;
  info += blockIdx.x;
  const int t = threadIdx.x;
  const int c1 = c0 + LU_NB;
  for (int j = c0; j < c1; ++j) {
    // pivot: the largest |A[r][j]| over rows r >= j (the lowest row on ties)
    double best = -1.0;
    int bi = j;
    for (int r = j + t; r < n; r += 1024) {
      const double v = fabs(A[(long)r * ld + j]);
      if (v > best) { best = v; bi = r; }
    }
    rv[t] = best;
    ri[t] = bi;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if (t < off && (rv[t + off] > rv[t] || (rv[t + off] == rv[t] && ri[t + off] < ri[t]))) {
        rv[t] = rv[t + off];
        ri[t] = ri[t + off];
      }
      __syncthreads();
    }
    if (t == 0) {
      prow = ri[0];
      piv[j] = ri[0];
      if (!(rv[0] > 0.0) && *info == 0) *info = j + 1;
    }
    __syncthreads();
    const int p = prow;
    if (p != j && t < LU_NB) {
      const long a = (long)j * ld + c0 + t, b = (long)p * ld + c0 + t;
      const double x = A[a];
      A[a] = A[b];
      A[b] = x;
    }
    __syncthreads();
    const double d = A[(long)j * ld + j];
    const double dinv = (d != 0.0) ? 1.0 / d : 0.0;
    for (int r = j + 1 + t; r < n; r += 1024) A[(long)r * ld + j] *= dinv;
    __syncthreads();
    // rank-1 update of the panel's columns right of j, rows below j
    const int w = c1 - 1 - j;
    if (w > 0) {
      const long cnt = (long)(n - j - 1) * w;
      for (long idx = t; idx < cnt; idx += 1024) {
        const int r = j + 1 + (int)(idx / w), col = j + 1 + (int)(idx % w);
        A[(long)r * ld + col] -= A[(long)r * ld + j] * A[(long)j * ld + col];
      }
    }
    __syncthreads();
  }
}

// One thread per column outside the panel: the panel's swaps in order, then
// (right of the panel) the unit-lower triangular solve with L11.
__global__ __launch_bounds__(256) void k_lu_swap_trsm(double* A, long ld, long sA, int n, int c0,
                                                      const int* piv, long sP) {
  A += (long)blockIdx.y * sA;
  piv += (long)blockIdx.y * sP;
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int c1 = c0 + LU_NB;
  if (col >= n || (col >= c0 && col < c1)) return;
  for (int j = c0; j < c1; ++j) {
    const int p = piv[j];
    if (p != j) {
      const double x = A[(long)j * ld + col];
      A[(long)j * ld + col] = A[(long)p * ld + col];
      A[(long)p * ld + col] = x;
    }
  }
  if (col < c1) return;
  for (int j = c0; j < c1; ++j) {
    const double x = A[(long)j * ld + col];
    for (int r = j + 1; r < c1; ++r) A[(long)r * ld + col] -= A[(long)r * ld + j] * x;
  }
}

// b <- P b, then L y = b (unit lower), then U x = y; b ends as x.  The vector
// is worked on in LDS when it fits (in_lds), else in place in b.
__global__ __launch_bounds__(1024) void k_lu_solve(const double* A, long ld, long sA, int n,
                                                   const int* piv, long sP, double* b, long sb,
                                                   int in_lds) {
  extern __shared__ double lds_x[];
  A += (long)blockIdx.x * sA;
  piv += (long)blockIdx.x * sP;
  b += (long)blockIdx.x * sb;
  const int t = threadIdx.x;
  double* xs = in_lds ? lds_x : b;
  if (in_lds)
    for (int i = t; i < n; i += 1024) xs[i] = b[i];
  __syncthreads();
  if (t == 0)
    for (int j = 0; j < n; ++j) {
      const int p = piv[j];
      if (p != j) {
        const double x = xs[j];
        xs[j] = xs[p];
        xs[p] = x;
      }
    }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double y = xs[j];
    for (int r = j + 1 + t; r < n; r += 1024) xs[r] -= A[(long)r * ld + j] * y;
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    const double d = A[(long)j * ld + j];
    const double x = (d != 0.0) ? xs[j] / d : 0.0;
    __syncthreads();   // every thread has read xs[j]
    if (t == 0) xs[j] = x;
    for (int r = t; r < j; r += 1024) xs[r] -= A[(long)r * ld + j] * x;
    __syncthreads();
  }
  if (in_lds)
    for (int i = t; i < n; i += 1024) b[i] = xs[i];
}

hipError_t dense_solve(double* A, long ldA, long sA, int n, double* b, long sb, int* piv,
                       long sP, int* info, int batch, long nA, long nb, long npiv, long ninfo,
                       hipStream_t st) {
  const char* kn = "dense_solve";
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (n % LU_NB != 0 || ldA < n || sA < (long)(n - 1) * ldA + n || sb < n || sP < n)
    return refuse(kn, "shape");
  GW_GUARD(kn, "A", (long)(batch - 1) * sA + (long)(n - 1) * ldA + n - 1, nA);
  GW_GUARD(kn, "b", (long)(batch - 1) * sb + n - 1, nb);
  GW_GUARD(kn, "piv", (long)(batch - 1) * sP + n - 1, npiv);
  GW_GUARD(kn, "info", batch - 1, ninfo);
  for (int c0 = 0; c0 < n; c0 += LU_NB) {
    if (audit_mode()) {
      audit_note();
      audit_note();
    } else {
      hipLaunchKernelGGL(k_lu_panel, dim3(batch), dim3(1024), 0, st, A, ldA, sA, n, c0, piv, sP,
                         info);
      hipLaunchKernelGGL(k_lu_swap_trsm, dim3((n + 255) / 256, batch), dim3(256), 0, st, A, ldA,
                         sA, n, c0, piv, sP);
      if (hipError_t e = hipGetLastError()) return e;
    }
    if (c0 + LU_NB < n) {   // A22 -= L21 U12 on 128 x 128 tiles, every system at once
      GemmArgs a{};
      a.A = A; a.lda = ldA; a.sA = sA;
      a.B = A; a.ldb = ldA; a.sB = sA;
      a.C = A; a.ldc = ldA; a.sC = sA;
      a.M = n - c0 - LU_NB; a.N = a.M; a.K = LU_NB;
      a.row0 = c0 + LU_NB; a.col0 = c0 + LU_NB; a.k0 = c0; a.kb0 = c0;
      a.map = MAP_FULL; a.tiles_m = a.M / 128; a.tiles_n = a.N / 128;
      a.n_tiles = a.tiles_m * a.tiles_n; a.batch = batch; a.splitk = 1;
      a.alpha = -1.0; a.beta = 1.0;
      a.nA = a.nB = a.nC = nA;
      if (hipError_t e = gemm_f64(a, 0, KC, KM, EPI_AXPBY, st)) return e;
    }
  }
  GW_AUDIT_RETURN();
  const int in_lds = (size_t)n * sizeof(double) <= 48 * 1024;
  hipLaunchKernelGGL(k_lu_solve, dim3(batch), dim3(1024), in_lds ? (size_t)n * sizeof(double) : 0,
                     st, A, ldA, sA, n, piv, sP, b, sb, in_lds);
  return hipGetLastError();
}

}  // namespace gw
