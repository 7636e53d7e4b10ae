// Dense fallback for residue systems that MINRES does not converge: the
// dielectric matrix 1 - Pi(w) is built explicitly (Pi build kernel with a
// signed scale) and solved by Gaussian elimination with partial pivoting.
// The paper switches to a Bunch-Kaufman factorization at this point; any
// stable dense solve of the same symmetric indefinite system gives the same x.
// One 1024-thread workgroup per system (blockIdx.x picks the system of a
// batch), so the systems of a batch are solved side by side on the CUs.
#include "gw_internal.h"

namespace gw {

__global__ __launch_bounds__(1024) void k_dense_solve(double* A, long ldA, long sA, int n,
                                                      double* b, long sb, int* info) {
  A += (long)blockIdx.x * sA;
  b += (long)blockIdx.x * sb;
  info += blockIdx.x;
  __shared__ double rv[1024];
  __shared__ int ri[1024];
  __shared__ double piv_inv;
  __shared__ int piv_row;
  const int t = threadIdx.x;
  for (int c = 0; c < n; ++c) {
    // pivot search in column c
    double best = -1.0;
    int bi = c;
    for (int i = c + t; i < n; i += 1024) {
      double v = fabs(A[(long)i * ldA + c]);
      if (v > best) { best = v; bi = i; }
    }
    rv[t] = best;
    ri[t] = bi;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if (t < off) {
        if (rv[t + off] > rv[t] || (rv[t + off] == rv[t] && ri[t + off] < ri[t])) {
          rv[t] = rv[t + off];
          ri[t] = ri[t + off];
        }
      }
      __syncthreads();
    }
    if (t == 0) {
      piv_row = ri[0];
      if (!(rv[0] > 0.0) && *info == 0) *info = c + 1;
    }
    __syncthreads();
    const int p = piv_row;
    if (p != c) {
      for (int j = t; j < n; j += 1024) {
        double a = A[(long)c * ldA + j];
        A[(long)c * ldA + j] = A[(long)p * ldA + j];
        A[(long)p * ldA + j] = a;
      }
      if (t == 0) {
        double a = b[c];
        b[c] = b[p];
        b[p] = a;
      }
    }
    __syncthreads();
    if (t == 0) {
      double d = A[(long)c * ldA + c];
      piv_inv = (d != 0.0) ? 1.0 / d : 0.0;
    }
    __syncthreads();
    // eliminate below: multipliers first, then the trailing update
    for (int i = c + 1 + t; i < n; i += 1024) A[(long)i * ldA + c] *= piv_inv;
    __syncthreads();
    const int w = n - c - 1;
    const long cnt = (long)w * w;
    for (long idx = t; idx < cnt; idx += 1024) {
      int i = c + 1 + (int)(idx / w), j = c + 1 + (int)(idx % w);
      A[(long)i * ldA + j] -= A[(long)i * ldA + c] * A[(long)c * ldA + j];
    }
    for (int i = c + 1 + t; i < n; i += 1024) b[i] -= A[(long)i * ldA + c] * b[c];
    __syncthreads();
  }
  // back substitution, one row at a time
  for (int i = n - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + t; j < n; j += 1024) s += A[(long)i * ldA + j] * b[j];
    rv[t] = s;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if (t < off) rv[t] += rv[t + off];
      __syncthreads();
    }
    if (t == 0) {
      double d = A[(long)i * ldA + i];
      b[i] = (d != 0.0) ? (b[i] - rv[0]) / d : 0.0;
    }
    __syncthreads();
  }
}

hipError_t dense_solve(double* A, long ldA, long sA, int n, double* b, long sb, int* info,
                       int batch, long nA, long nb, long ninfo, hipStream_t st) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (ldA < n || sA < (long)(n - 1) * ldA + n || sb < n)
    return refuse("dense_solve", "shape");
  GW_GUARD("dense_solve", "A", (long)(batch - 1) * sA + (long)(n - 1) * ldA + n - 1, nA);
  GW_GUARD("dense_solve", "b", (long)(batch - 1) * sb + n - 1, nb);
  GW_GUARD("dense_solve", "info", batch - 1, ninfo);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_dense_solve, dim3(batch), dim3(1024), 0, st, A, ldA, sA, n, b, sb, info);
  return hipGetLastError();
}

}  // namespace gw
