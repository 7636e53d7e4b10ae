// Small preparation kernels: transition energies, squared norms of the
// right-hand sides, and the real-frequency scale vector of the dense fallback.
#include "gw_internal.h"

namespace gw {

// Transition energies of every spin, stacked: spin s contributes
// D[k_s + i*n_virt_s + a] = eps_s[n_occ_s + a] - eps_s[i] with k_0 = 0 and
// k_1 = n_occ_0 * n_virt_0, eps_s = eps + s * n_mo.  Padding entries get a
// large value so that D/(D^2 - w^2) stays finite there (their B columns are 0).
__global__ void k_transition(const double* eps, int n_spin, int n_mo, int n_occ0, int n_occ1,
                             int Kp, double* D) {
  const int K0 = n_occ0 * (n_mo - n_occ0);
  const int K1 = n_spin > 1 ? n_occ1 * (n_mo - n_occ1) : 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Kp; k += gridDim.x * blockDim.x) {
    if (k < K0) {
      const int nv = n_mo - n_occ0, i = k / nv, a = k % nv;
      D[k] = eps[n_occ0 + a] - eps[i];
    } else if (k < K0 + K1) {
      const int nv = n_mo - n_occ1, i = (k - K0) / nv, a = (k - K0) % nv;
      D[k] = eps[n_mo + n_occ1 + a] - eps[n_mo + i];
    } else {
      D[k] = 1.0e6;
    }
  }
}

hipError_t transition_energies(const double* eps, int n_spin, int n_mo, const int* n_occ, int Kp,
                               double* D, long nEps, long nD, hipStream_t st) {
  if (n_spin < 1 || n_spin > 2) return refuse("transition", "n_spin");
  long K = 0;
  for (int s = 0; s < n_spin; ++s) {
    if (n_occ[s] < 1 || n_occ[s] >= n_mo) return refuse("transition", "n_occ");
    K += (long)n_occ[s] * (n_mo - n_occ[s]);
  }
  if (K > Kp) return refuse("transition", "K > Kp");
  GW_GUARD("transition", "eps", (long)n_spin * n_mo - 1, nEps);
  GW_GUARD("transition", "D", Kp - 1, nD);
  GW_AUDIT_RETURN();
  int blocks = (Kp + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_transition, dim3(blocks), dim3(256), 0, st, eps, n_spin, n_mo, n_occ[0],
                     n_spin > 1 ? n_occ[1] : 0, Kp, D);
  return hipGetLastError();
}

// x[k] *= f for k < n
__global__ void k_scale_inplace(double* x, long n, double f) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    x[k] *= f;
}

hipError_t scale_inplace(double* x, long n, double f, long nX, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  GW_GUARD("scale_inplace", "x", n - 1, nX);
  GW_AUDIT_RETURN();
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_scale_inplace, dim3((unsigned)blocks), dim3(256), 0, st, x, n, f);
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
