// Blocked Cholesky pieces for the dielectric matrices 1 - Pi(i xi_g) and the
// screened-interaction reduction.
//
// The matrix of grid point g is stored augmented: rows [0, Np) hold 1 - Pi
// (lower triangle), rows [Np, 2 Np) start as the identity.  A left-looking
// blocked Cholesky (panel width 128) run over the rows factors 1 - Pi = L L^T
// and, because the appended rows are treated like rows below the diagonal,
// leaves (L^-1 I)^T = L^-T in them (row Np + s holds column s of L^-1).
// Identity row s is untouched until the panel that contains column s, so each
// panel only carries the appended rows up to its own end, which makes the
// inverse cost N^3/3.  The screened interaction then needs
// b^T (1 - Pi)^-1 b = |L^-1 b|^2 for every b = (P|nm), one triangular GEMM
// with the squared-norm reduction in its epilogue.
#include <algorithm>

#include "gw_internal.h"

namespace gw {

constexpr int NB = 128;

// Factor the 128x128 diagonal block at (k, k) of every batch item, write L
// back (strict upper part zeroed) and write L^-1 to Linv[g][128][128].
//
// One 1024-thread workgroup per batch item; the block lives in registers.
// Thread (ti, tj) of a 32 x 32 grid holds L[ti + 32 a][tj + 32 b] and
// Y[ti + 32 a][tj + 32 b] for a, b = 0..3, where Y starts as the identity and
// is eliminated like rows appended below the block, so that it ends as L^-T
// (column s of L^-1 in row s).  Column j is published through LDS by the
// threads with tj = j mod 32 (double-buffered, one barrier per column); the
// owner of the diagonal element adds 1 / sqrt(L[j][j]).  Register blocks that
// cannot take part in column j (above or left of it, or upper-triangular) are
// skipped at compile time, which leaves 1/4 of the dense update work.
constexpr int CT = 32;       // thread grid edge
constexpr int CR = NB / CT;  // register block edge (4)

__global__ __launch_bounds__(1024) void k_chol_diag(double* A, long ldA, long sA, double* Linv,
                                                    int k, int* info) {
  __shared__ double colL[2][NB], colY[2][NB], rpiv[2];
  __shared__ double stage[NB][NB + 1];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  const int ti = t / CT, tj = t % CT;
  double* Ag = A + (long)g * sA + (long)k * ldA + k;

  double L[CR][CR], Y[CR][CR];
#pragma unroll
  for (int a = 0; a < CR; ++a)
#pragma unroll
    for (int b = 0; b < CR; ++b) {
      const int i = ti + CT * a, c = tj + CT * b;
      L[a][b] = (c <= i) ? Ag[(long)i * ldA + c] : 0.0;
      Y[a][b] = (c == i) ? 1.0 : 0.0;
    }

#pragma unroll
  for (int bj = 0; bj < CR; ++bj) {
#pragma unroll 1
    for (int jj = 0; jj < CT; ++jj) {
      const int j = CT * bj + jj;
      const int buf = jj & 1;
      if (tj == jj) {
#pragma unroll
        for (int a = 0; a < CR; ++a) {
          if (a >= bj) colL[buf][ti + CT * a] = L[a][bj];
          if (a <= bj) colY[buf][ti + CT * a] = Y[a][bj];
        }
        if (ti == jj) {
          double d = L[bj][bj];
          if (!(d > 0.0)) {  // not positive definite (or NaN): record, continue with 1
            if (info[g] == 0) info[g] = k + j + 1;
            d = 1.0;
          }
          const double piv = sqrt(d);
          rpiv[buf] = 1.0 / piv;
          L[bj][bj] = piv;
        }
      }
      __syncthreads();
      const double rp = rpiv[buf];
      double li[CR], lc[CR], ys[CR];
#pragma unroll
      for (int a = 0; a < CR; ++a) {
        li[a] = (a >= bj) ? colL[buf][ti + CT * a] * rp : 0.0;
        lc[a] = (a >= bj) ? colL[buf][tj + CT * a] * rp : 0.0;
        ys[a] = (a <= bj) ? colY[buf][ti + CT * a] * rp : 0.0;
      }
      if (tj == jj) {
#pragma unroll
        for (int a = 0; a < CR; ++a) {
          if (a >= bj && ti + CT * a > j) L[a][bj] = li[a];
          if (a <= bj) Y[a][bj] = ys[a];
        }
      }
      // trailing update of L: rows i > j, columns j < c <= i
#pragma unroll
      for (int a = bj; a < CR; ++a) {
        const bool row_ok = (a > bj) || (ti > jj);
#pragma unroll
        for (int b = bj; b <= a; ++b) {
          const bool col_ok = (b > bj) || (tj > jj);
          if (row_ok && col_ok) L[a][b] -= li[a] * lc[b];
        }
      }
      // appended rows: columns c > j of rows s <= j (rows s > j are still zero there)
#pragma unroll
      for (int a = 0; a <= bj; ++a)
#pragma unroll
        for (int b = bj; b < CR; ++b) {
          const bool col_ok = (b > bj) || (tj > jj);
          if (col_ok) Y[a][b] -= ys[a] * lc[b];
        }
    }
  }

#pragma unroll
  for (int a = 0; a < CR; ++a)
#pragma unroll
    for (int b = 0; b < CR; ++b) {
      const int i = ti + CT * a, c = tj + CT * b;
      Ag[(long)i * ldA + c] = (c <= i) ? L[a][b] : 0.0;
      stage[i][c] = Y[a][b];
    }
  __syncthreads();
  // Linv[i][c] = (L^-1)[i][c] = Y[c][i]
  double* Li = Linv + (long)g * NB * NB;
  for (int idx = t; idx < NB * NB; idx += 1024) {
    const int i = idx / NB, c = idx % NB;
    Li[idx] = (c <= i) ? stage[c][i] : 0.0;
  }
}

hipError_t chol_diag(double* A, long ldA, long sA, double* Linv, int k, int G, int* info,
                     long nA, long nLinv, long nInfo, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  GW_GUARD("chol_diag", "A", (long)(G - 1) * sA + (long)(k + NB - 1) * ldA + k + NB - 1, nA);
  GW_GUARD("chol_diag", "Linv", (long)G * NB * NB - 1, nLinv);
  GW_GUARD("chol_diag", "info", G - 1, nInfo);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_chol_diag, dim3(G), dim3(1024), 0, st, A, ldA, sA, Linv, k, info);
  return hipGetLastError();
}

// rows [row0, row0 + n) of every batch item <- e_0 .. e_{n-1} over columns [0, ncol)
__global__ void k_set_identity(double* A, long ldA, long sA, int row0, int n, int ncol) {
  const int g = blockIdx.y;
  const long cnt = (long)n * ncol;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < cnt;
       idx += (long)gridDim.x * blockDim.x) {
    int r = (int)(idx / ncol), c = (int)(idx % ncol);
    A[(long)g * sA + (long)(row0 + r) * ldA + c] = (r == c) ? 1.0 : 0.0;
  }
}

hipError_t set_identity_rows(double* A, long ldA, long sA, int row0, int n, int ncol, int G,
                             long nA, hipStream_t st) {
  const long cnt = (long)n * ncol;
  if (cnt <= 0 || G <= 0) return hipSuccess;
  GW_GUARD("set_identity", "A", (long)(G - 1) * sA + (long)(row0 + n - 1) * ldA + ncol - 1, nA);
  GW_AUDIT_RETURN();
  int blocks = (int)std::min<long>((cnt + 255) / 256, 1024);
  hipLaunchKernelGGL(k_set_identity, dim3(blocks, G), dim3(256), 0, st, A, ldA, sA, row0, n, ncol);
  return hipGetLastError();
}

// wtab[q][g0 + g] = sum_J part[g][J][q] - bnorm2[q] (bnorm2 null: no subtraction,
// the partials of the mixed contraction already are W^c)
__global__ void k_wc_from_parts(const double* part, long sPart, int nJ, int ldp,
                                const double* bnorm2, int nR, int Gtot, int g0, double* wtab) {
  const int g = blockIdx.y;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nR; q += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int J = 0; J < nJ; ++J) s += part[(long)g * sPart + (long)J * ldp + q];
    wtab[(long)q * Gtot + g0 + g] = bnorm2 ? s - bnorm2[q] : s;
  }
}

hipError_t wc_from_parts(const double* part, long sPart, int nJ, int ldp, const double* bnorm2,
                         int nR, int G, int Gtot, int g0, double* wtab, long nPart, long nBn,
                         long nW, hipStream_t st) {
  if (nR <= 0 || G <= 0) return hipSuccess;
  if (g0 + G > Gtot || ldp < nR) return refuse("wc_from_parts", "shape");
  GW_GUARD("wc_from_parts", "part", (long)(G - 1) * sPart + (long)(nJ - 1) * ldp + nR - 1, nPart);
  if (bnorm2) GW_GUARD("wc_from_parts", "bnorm2", nR - 1, nBn);
  GW_GUARD("wc_from_parts", "wtab", (long)(nR - 1) * Gtot + g0 + G - 1, nW);
  GW_AUDIT_RETURN();
  int blocks = std::min((nR + 255) / 256, 256);
  hipLaunchKernelGGL(k_wc_from_parts, dim3(blocks, G), dim3(256), 0, st, part, sPart, nJ, ldp,
                     bnorm2, nR, Gtot, g0, wtab);
  return hipGetLastError();
}

// Grouped form: item g of the batch is grid column g % grp of request g / grp
__global__ void k_wc_from_parts_tab(const double* part, long sPart, int nJ, int ldp,
                                    const double* const* bn_tab, int nR, int grp,
                                    double* const* wtab_tab) {
  const int g = blockIdx.y;
  const int r = g / grp, col = g % grp;
  const double* bn = bn_tab ? bn_tab[r] : nullptr;
  double* wtab = wtab_tab[r];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nR; q += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int J = 0; J < nJ; ++J) s += part[(long)g * sPart + (long)J * ldp + q];
    wtab[(long)q * grp + col] = bn ? s - bn[q] : s;
  }
}

hipError_t wc_from_parts_tab(const double* part, long sPart, int nJ, int ldp,
                             const double* const* bn_tab, int nR, int G, int grp,
                             double* const* wtab_tab, long nPart, long nBn, long nW,
                             hipStream_t st) {
  if (nR <= 0 || G <= 0) return hipSuccess;
  if (grp <= 0 || G % grp != 0 || ldp < nR || !wtab_tab) return refuse("wc_from_parts", "shape");
  GW_GUARD("wc_from_parts", "part", (long)(G - 1) * sPart + (long)(nJ - 1) * ldp + nR - 1, nPart);
  if (bn_tab) GW_GUARD("wc_from_parts", "bnorm2", nR - 1, nBn);
  GW_GUARD("wc_from_parts", "wtab", (long)(nR - 1) * grp + grp - 1, nW);
  GW_AUDIT_RETURN();
  int blocks = std::min((nR + 255) / 256, 256);
  hipLaunchKernelGGL(k_wc_from_parts_tab, dim3(blocks, G), dim3(256), 0, st, part, sPart, nJ, ldp,
                     bn_tab, nR, grp, wtab_tab);
  return hipGetLastError();
}

__global__ void k_fill_int(int* p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

hipError_t fill_int(int* p, int n, int v, long nP, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  GW_GUARD("fill_int", "p", n - 1, nP);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_fill_int, dim3(std::min((n + 255) / 256, 64)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// s[g][k] = D_k / (D_k^2 + xi_g^2) for k < Kov, 0 for the padding; s32 (if
// given) receives the same values rounded to FP32 for the mixed Pi builds
__global__ void k_scale_imag(const double* D, int Kov, int Kp, const double* xi, double* s,
                             float* s32) {
  const int g = blockIdx.y;
  const double x2 = xi[g] * xi[g];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Kp; k += gridDim.x * blockDim.x) {
    double d = D[k];
    const double v = (k < Kov) ? d / (d * d + x2) : 0.0;
    s[(long)g * Kp + k] = v;
    if (s32) s32[(long)g * Kp + k] = (float)v;
  }
}

hipError_t make_scale_imag(const double* D, int Kov, int Kp, const double* xi, int G, double* s,
                           float* s32, long nD, long nXi, long nS, long nS32, hipStream_t st) {
  if (G <= 0 || Kp <= 0) return hipSuccess;
  GW_GUARD("scale_imag", "D", Kp - 1, nD);
  GW_GUARD("scale_imag", "xi", G - 1, nXi);
  GW_GUARD("scale_imag", "s", (long)G * Kp - 1, nS);
  if (s32) GW_GUARD("scale_imag", "s32", (long)G * Kp - 1, nS32);
  if (Kov > Kp) return refuse("scale_imag", "Kov > Kp");
  GW_AUDIT_RETURN();
  int blocks = (Kp + 255) / 256;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_scale_imag, dim3(blocks, G), dim3(256), 0, st, D, Kov, Kp, xi, s, s32);
  return hipGetLastError();
}

// Grouped form: item g takes request g / grp's energies and real-column count
// and grid point xi[g % grp]
__global__ void k_scale_imag_tab(const double* const* D_tab, const int* Kov_tab, int Kp,
                                 const double* xi, int grp, double* s, float* s32) {
  const int g = blockIdx.y;
  const double* D = D_tab[g / grp];
  const int Kov = Kov_tab[g / grp];
  const double x = xi[g % grp];
  const double x2 = x * x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Kp; k += gridDim.x * blockDim.x) {
    double d = D[k];
    const double v = (k < Kov) ? d / (d * d + x2) : 0.0;
    s[(long)g * Kp + k] = v;
    if (s32) s32[(long)g * Kp + k] = (float)v;
  }
}

// nD: the smallest extent over the table's energy arrays
hipError_t make_scale_imag_tab(const double* const* D_tab, const int* Kov_tab, int Kp,
                               const double* xi, int grp, int G, double* s, float* s32,
                               long nD, long nXi, long nS, long nS32, hipStream_t st) {
  if (G <= 0 || Kp <= 0) return hipSuccess;
  if (grp <= 0 || G % grp != 0 || !D_tab || !Kov_tab) return refuse("scale_imag", "shape");
  GW_GUARD("scale_imag", "D", Kp - 1, nD);
  GW_GUARD("scale_imag", "xi", grp - 1, nXi);
  GW_GUARD("scale_imag", "s", (long)G * Kp - 1, nS);
  if (s32) GW_GUARD("scale_imag", "s32", (long)G * Kp - 1, nS32);
  GW_AUDIT_RETURN();
  int blocks = (Kp + 255) / 256;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_scale_imag_tab, dim3(blocks, G), dim3(256), 0, st, D_tab, Kov_tab, Kp, xi,
                     grp, s, s32);
  return hipGetLastError();
}

// Imaginary-axis part of Re Sigma^c and its omega-derivative for n states.
// sig_j = -(1/pi) sum_m sum_g W[r_j][m][g] z_g a/(a^2 + xi_g^2), a = omega_j - eps_m.
// The n_mo G terms of a state are split over QUAD_SLICES workgroups whose
// partial sums are added in a fixed order by a second small kernel.
constexpr int QUAD_SLICES = 16;

// Table rows hold ld >= G columns per m; with w0 the column G holds the static
// W^c_nm(0): the quadrature then takes W^c(i xi) - W^c(0) only, and the static
// part's integral int_0^inf a/(a^2 + xi^2) d xi = (pi/2) sgn(a) is added
// exactly (once per m, by the thread that visits g = 0).
__global__ __launch_bounds__(256) void k_sigma_quad_part(const double* wtab, int n_mo, int G,
                                                         int ld, int w0, const int* rowsel,
                                                         const int* rowspin,
                                                         const double* omega,
                                                         const double* eps, const double* xi,
                                                         const double* z, double* part) {
  __shared__ double rs[256], rd[256];
  const int j = blockIdx.x, sl = blockIdx.y, t = threadIdx.x;
  const int r = rowsel[j];
  if (rowspin) eps += (long)rowspin[r] * n_mo;
  const double w = omega[j];
  const double* W = wtab + (long)r * n_mo * ld;
  const long n = (long)n_mo * G;
  const long chunk = (n + QUAD_SLICES - 1) / QUAD_SLICES;
  const long lo = sl * chunk, hi = lo + chunk < n ? lo + chunk : n;
  const double half_pi = 1.57079632679489661923;
  double s = 0.0, d = 0.0;
  for (long idx = lo + t; idx < hi; idx += 256) {
    int m = (int)(idx / G), g = (int)(idx % G);
    double a = w - eps[m];
    double x2 = xi[g] * xi[g];
    double den = a * a + x2;
    double wv = W[(long)m * ld + g];
    if (w0) {
      const double ws = W[(long)m * ld + G];
      wv -= ws;
      if (g == 0) s += half_pi * (double)((a > 0.0) - (a < 0.0)) * ws;
    }
    double wz = wv * z[g];
    s += wz * a / den;
    d += wz * (x2 - a * a) / (den * den);
  }
  rs[t] = s;
  rd[t] = d;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      rs[t] += rs[t + off];
      rd[t] += rd[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[(long)(j * QUAD_SLICES + sl) * 2] = rs[0];
    part[(long)(j * QUAD_SLICES + sl) * 2 + 1] = rd[0];
  }
}

__global__ void k_sigma_quad_sum(const double* part, int n, double* sig, double* dsig) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0, d = 0.0;
  for (int sl = 0; sl < QUAD_SLICES; ++sl) {
    s += part[(long)(j * QUAD_SLICES + sl) * 2];
    d += part[(long)(j * QUAD_SLICES + sl) * 2 + 1];
  }
  const double inv_pi = 0.31830988618379067154;
  sig[j] = -inv_pi * s;
  dsig[j] = -inv_pi * d;
}

// A <- 2 I - A on the leading Np x Np block of every item (1 - Pi becomes
// 1 + Pi): the failure-handling test hook of the Cholesky
__global__ void k_reflect_unit(double* A, long ldA, long sA, int Np) {
  double* a = A + (long)blockIdx.y * sA;
  const long n = (long)Np * Np;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / Np), j = (int)(e % Np);
    double* x = a + (long)i * ldA + j;
    *x = (i == j ? 2.0 : 0.0) - *x;
  }
}

hipError_t reflect_unit(double* A, long ldA, long sA, int Np, int G, long nA, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  GW_GUARD("reflect_unit", "A", (long)(G - 1) * sA + (long)(Np - 1) * ldA + Np - 1, nA);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_reflect_unit, dim3(64, G), dim3(256), 0, st, A, ldA, sA, Np);
  return hipGetLastError();
}

hipError_t sigma_quad(const double* wtab, int n_mo, int G, int ld, int w0, const int* rowsel,
                      const int* rowspin, const double* omega, const double* eps,
                      const double* xi, const double* z, int n, double* sig, double* dsig,
                      double* part, int n_rows, long nW, long nPart, long nEps, long nXi,
                      long nZ, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (G < 1 || ld < G + (w0 ? 1 : 0)) return hipErrorInvalidValue;
  GW_GUARD("sigma_quad", "xi", G - 1, nXi);
  GW_GUARD("sigma_quad", "z", G - 1, nZ);
  // (row spins are 0 or 1, set by the context from validated row ids)
  GW_GUARD("sigma_quad", "eps", (rowspin ? 2L : 1L) * n_mo - 1, nEps);
  // row indices come from the context's validated state -> row map (< n_rows)
  GW_GUARD("sigma_quad", "wtab", (long)n_rows * n_mo * ld - 1, nW);
  GW_GUARD("sigma_quad", "partials", (long)n * QUAD_SLICES * 2 - 1, nPart);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_sigma_quad_part, dim3(n, QUAD_SLICES), dim3(256), 0, st, wtab, n_mo, G,
                     ld, w0, rowsel, rowspin, omega, eps, xi, z, part);
  hipLaunchKernelGGL(k_sigma_quad_sum, dim3((n + 63) / 64), dim3(64), 0, st, part, n, sig, dsig);
  return hipGetLastError();
}

}  // namespace gw
