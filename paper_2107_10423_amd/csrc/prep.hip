// Small preparation kernels: transition energies, squared norms of the
// right-hand sides, and the real-frequency scale vector of the dense fallback.
#include "gw_internal.h"

namespace gw {

// D[i*n_virt + a] = eps[n_occ + a] - eps[i]; padding entries get a large
// value so that D/(D^2 - w^2) stays finite there (their B columns are 0).
__global__ void k_transition(const double* eps, int n_occ, int n_virt, int Kp, double* D) {
  const int Kov = n_occ * n_virt;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Kp; k += gridDim.x * blockDim.x) {
    if (k < Kov) {
      int i = k / n_virt, a = k % n_virt;
      D[k] = eps[n_occ + a] - eps[i];
    } else {
      D[k] = 1.0e6;
    }
  }
}

hipError_t transition_energies(const double* eps, int n_occ, int n_virt, int Kp, double* D,
                               long nEps, long nD, hipStream_t st) {
  GW_GUARD("transition", "eps", n_occ + n_virt - 1, nEps);
  GW_GUARD("transition", "D", Kp - 1, nD);
  GW_AUDIT_RETURN();
  int blocks = (Kp + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_transition, dim3(blocks), dim3(256), 0, st, eps, n_occ, n_virt, Kp, D);
  return hipGetLastError();
}

// bn[q] = |R[q][:]|^2, one wavefront per row
__global__ void k_row_norm2(const double* R, int nR, int Np, double* bn) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + wave;
  if (q >= nR) return;
  double s = 0.0;
  for (int c = lane; c < Np; c += 64) s += R[(long)q * Np + c] * R[(long)q * Np + c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) bn[q] = s;
}

hipError_t row_norm2(const double* R, int nR, int Np, double* bn, long nRext, long nBn,
                     hipStream_t st) {
  if (nR <= 0) return hipSuccess;
  GW_GUARD("row_norm2", "R", (long)nR * Np - 1, nRext);
  GW_GUARD("row_norm2", "bn", nR - 1, nBn);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_row_norm2, dim3((nR + 3) / 4), dim3(256), 0, st, R, nR, Np, bn);
  return hipGetLastError();
}

// s[k] = D_k/(D_k^2 - w^2) for k < Kov, 0 for the padding
__global__ void k_scale_real(const double* D, int Kov, int Kp, double w, double* s) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Kp; k += gridDim.x * blockDim.x) {
    double d = D[k];
    s[k] = (k < Kov) ? d / (d * d - w * w) : 0.0;
  }
}

hipError_t make_scale_real(const double* D, int Kov, int Kp, double w, double* s, long nD,
                           long nS, hipStream_t st) {
  GW_GUARD("scale_real", "D", Kp - 1, nD);
  GW_GUARD("scale_real", "s", Kp - 1, nS);
  if (Kov > Kp) return refuse("scale_real", "Kov > Kp");
  GW_AUDIT_RETURN();
  int blocks = (Kp + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_scale_real, dim3(blocks), dim3(256), 0, st, D, Kov, Kp, w, s);
  return hipGetLastError();
}

// b := rhs row (padded), used by the dense fallback
__global__ void k_copy_vec(const double* src, double* dst, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    dst[k] = src[k];
}

hipError_t copy_vec(const double* src, double* dst, int n, long nSrc, long nDst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  GW_GUARD("copy_vec", "src", n - 1, nSrc);
  GW_GUARD("copy_vec", "dst", n - 1, nDst);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_copy_vec, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace gw
