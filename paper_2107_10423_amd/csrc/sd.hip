// Spectral-decomposition (Casida) route: the Hermitian RPA matrix, its
// eigendecomposition by block Jacobi, the pole strengths and the pole form of
// Sigma^c (Implementation - Spectral Decomposition; Theory - Spectral
// Decomposition).
//
// Matrix: M = (A - B)^1/2 (A + B) (A - B)^1/2 with A - B = diag(D) and
// A + B = diag(D) + 4 B_ov^T B_ov, i.e. M_ij = delta_ij D_i^2 +
// 4 sqrt(D_i D_j) (B_ov^T B_ov)_ij, M T = T Omega^2.  (Open-shell contexts
// hold both spins' transitions stacked and scaled by 1/sqrt(2), which turns
// the factor 4 into the 2 of the spin-block equations.)
//
// Eigensolver: two-sided block Jacobi over 32-wide column blocks.  A round
// pairs the nb blocks (circle method, nb - 1 rounds per sweep); each pair's
// 64 x 64 diagonal subproblem is diagonalised in LDS by cyclic Jacobi
// rotations (parallel ordering, 32 disjoint rotations at a time), and its
// 64 x 64 rotation is then applied to the pair's columns of M and of T and to
// the pair's rows of M.  Sweeps repeat until the off-diagonal norm is
// negligible.  Padding entries (index >= n) keep zero couplings, so no
// rotation ever mixes them with the real ones.
#include "gw_internal.h"

namespace gw {

#define JB 32
#define JP 64

// circle-method pairing of nb blocks (nb even): round r in [0, nb - 1), pair k
__device__ inline void rr_pair(int nb, int r, int k, int* I, int* J) {
  if (k == 0) {
    *I = nb - 1;
    *J = r;
  } else {
    *I = (r + k) % (nb - 1);
    *J = (r - k + (nb - 1)) % (nb - 1);
  }
}

__device__ inline long pair_index(int I, int J, int k) {
  return k < JB ? (long)I * JB + k : (long)J * JB + (k - JB);
}

// M from C = B_ov^T B_ov in place (n real transitions, ld >= Kp): padding
// rows and columns become 0, diagonal included.  A rotation between a real
// and a padding index then always has a zero coupling (the identity), and the
// subproblem's stopping test, relative to its diagonal, is not swamped by
// padding entries.
__global__ void k_casida_matrix(double* C, long ld, const double* D, int n, int Kp) {
  const long total = (long)Kp * Kp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / Kp), j = (int)(e % Kp);
    double* c = C + (long)i * ld + j;
    if (i < n && j < n) {
      const double v = 4.0 * sqrt(D[i] * D[j]) * *c;
      *c = i == j ? v + D[i] * D[i] : v;
    } else {
      *c = 0.0;
    }
  }
}

hipError_t casida_matrix(double* C, long ld, const double* D, int n, int Kp, long nC, long nD,
                         hipStream_t st) {
  if (n < 1 || n > Kp || ld < Kp) return refuse("casida_matrix", "shape");
  GW_GUARD("casida_matrix", "C", (long)(Kp - 1) * ld + Kp - 1, nC);
  GW_GUARD("casida_matrix", "D", n - 1, nD);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_casida_matrix, dim3(2048), dim3(256), 0, st, C, ld, D, n, Kp);
  return hipGetLastError();
}

// T = identity (Kp x Kp)
__global__ void k_identity(double* T, long ld, int Kp) {
  const long total = (long)Kp * Kp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / Kp), j = (int)(e % Kp);
    T[(long)i * ld + j] = i == j ? 1.0 : 0.0;
  }
}

hipError_t set_identity(double* T, long ld, int Kp, long nT, hipStream_t st) {
  GW_GUARD("set_identity", "T", (long)(Kp - 1) * ld + Kp - 1, nT);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_identity, dim3(2048), dim3(256), 0, st, T, ld, Kp);
  return hipGetLastError();
}

// Diagonalise the 64 x 64 subproblem of every block pair of round r and
// write its rotation V (S_new = V^T S V) to V[pair][64][64].
__global__ __launch_bounds__(256) void k_jacobi_sub(const double* M, long ld, int nb, int r,
                                                    double* Vout, int max_sweeps) {
  __shared__ double S[JP][JP + 1];
  __shared__ double V[JP][JP + 1];
  __shared__ double cs[JP / 2][2];
  __shared__ int pq[JP / 2][2];
  __shared__ double red[2][256];
  const int pair = blockIdx.x, t = threadIdx.x;
  int I, J;
  rr_pair(nb, r, pair, &I, &J);
  for (int e = t; e < JP * JP; e += 256) {
    const int i = e / JP, j = e % JP;
    S[i][j] = M[pair_index(I, J, i) * ld + pair_index(I, J, j)];
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // stop once the off-diagonal part is negligible against the diagonal
    double off = 0.0, dia = 0.0;
    for (int e = t; e < JP * JP; e += 256) {
      const int i = e / JP, j = e % JP;
      const double v = S[i][j] * S[i][j];
      if (i == j) dia += v;
      else off += v;
    }
    red[0][t] = off;
    red[1][t] = dia;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) {
        red[0][t] += red[0][t + h];
        red[1][t] += red[1][t + h];
      }
      __syncthreads();
    }
    const bool done = !(red[0][0] > 1e-32 * red[1][0]);
    __syncthreads();
    if (done) break;
    for (int rr = 0; rr < JP - 1; ++rr) {
      if (t < JP / 2) {
        int p, q;
        rr_pair(JP, rr, t, &p, &q);
        const double apq = S[p][q], app = S[p][p], aqq = S[q][q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          // symmetric 2 x 2 Schur decomposition (Golub and Van Loan)
          const double tau = (aqq - app) / (2.0 * apq);
          double tt;
          if (fabs(tau) > 1.0e150) tt = 0.5 / tau;
          else tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        pq[t][0] = p;
        pq[t][1] = q;
        cs[t][0] = c;
        cs[t][1] = s;
      }
      __syncthreads();
      // columns of S and of V: (S J)[:, p] = c S[:, p] - s S[:, q], (S J)[:, q] = s S[:, p] + c S[:, q]
      for (int e = t; e < JP * (JP / 2); e += 256) {
        const int k = e & (JP - 1), u = e >> 6;
        const int p = pq[u][0], q = pq[u][1];
        const double c = cs[u][0], s = cs[u][1];
        const double sp = S[k][p], sq = S[k][q];
        S[k][p] = c * sp - s * sq;
        S[k][q] = s * sp + c * sq;
        const double vp = V[k][p], vq = V[k][q];
        V[k][p] = c * vp - s * vq;
        V[k][q] = s * vp + c * vq;
      }
      __syncthreads();
      // rows of S
      for (int e = t; e < JP * (JP / 2); e += 256) {
        const int k = e & (JP - 1), u = e >> 6;
        const int p = pq[u][0], q = pq[u][1];
        const double c = cs[u][0], s = cs[u][1];
        const double sp = S[p][k], sq = S[q][k];
        S[p][k] = c * sp - s * sq;
        S[q][k] = s * sp + c * sq;
      }
      __syncthreads();
    }
  }
  double* out = Vout + (long)pair * JP * JP;
  for (int e = t; e < JP * JP; e += 256) out[e] = V[e / JP][e % JP];
}

// X[rows r0..r0+64)[pair columns] <- X[...][pair columns] V_pair, in place
__global__ __launch_bounds__(256) void k_jacobi_cols(double* X, long ld, int nb, int r,
                                                     const double* Vin) {
  __shared__ double Xs[JP][JP + 1];
  __shared__ double Vs[JP][JP + 1];
  const int r0 = blockIdx.x * JP, pair = blockIdx.y, t = threadIdx.x;
  int I, J;
  rr_pair(nb, r, pair, &I, &J);
  const double* V = Vin + (long)pair * JP * JP;
  for (int e = t; e < JP * JP; e += 256) {
    const int i = e / JP, j = e % JP;
    Xs[i][j] = X[(long)(r0 + i) * ld + pair_index(I, J, j)];
    Vs[i][j] = V[e];
  }
  __syncthreads();
  const int ti = t >> 4, tj = t & 15;
  double acc[4][4] = {};
  for (int k = 0; k < JP; ++k) {
    double a[4], b[4];
    for (int ii = 0; ii < 4; ++ii) a[ii] = Xs[4 * ti + ii][k];
    for (int jj = 0; jj < 4; ++jj) b[jj] = Vs[k][tj + 16 * jj];
    for (int ii = 0; ii < 4; ++ii)
      for (int jj = 0; jj < 4; ++jj) acc[ii][jj] += a[ii] * b[jj];
  }
  for (int ii = 0; ii < 4; ++ii)
    for (int jj = 0; jj < 4; ++jj)
      X[(long)(r0 + 4 * ti + ii) * ld + pair_index(I, J, tj + 16 * jj)] = acc[ii][jj];
}

// X[pair rows][cols c0..c0+64) <- V_pair^T X[pair rows][...], in place
__global__ __launch_bounds__(256) void k_jacobi_rows(double* X, long ld, int nb, int r,
                                                     const double* Vin) {
  __shared__ double Xs[JP][JP + 1];
  __shared__ double Vs[JP][JP + 1];
  const int c0 = blockIdx.x * JP, pair = blockIdx.y, t = threadIdx.x;
  int I, J;
  rr_pair(nb, r, pair, &I, &J);
  const double* V = Vin + (long)pair * JP * JP;
  for (int e = t; e < JP * JP; e += 256) {
    const int i = e / JP, j = e % JP;
    Xs[i][j] = X[pair_index(I, J, i) * ld + c0 + j];
    Vs[i][j] = V[e];
  }
  __syncthreads();
  const int ti = t >> 4, tj = t & 15;
  double acc[4][4] = {};
  for (int k = 0; k < JP; ++k) {
    double a[4], b[4];
    for (int ii = 0; ii < 4; ++ii) a[ii] = Vs[k][4 * ti + ii];   // V^T[i][k] = V[k][i]
    for (int jj = 0; jj < 4; ++jj) b[jj] = Xs[k][tj + 16 * jj];
    for (int ii = 0; ii < 4; ++ii)
      for (int jj = 0; jj < 4; ++jj) acc[ii][jj] += a[ii] * b[jj];
  }
  for (int ii = 0; ii < 4; ++ii)
    for (int jj = 0; jj < 4; ++jj)
      X[pair_index(I, J, 4 * ti + ii) * ld + c0 + tj + 16 * jj] = acc[ii][jj];
}

// One round r of block Jacobi on M (Kp x Kp) with eigenvector accumulation in T.
hipError_t jacobi_round(double* M, double* T, long ld, int Kp, int r, double* V, int max_sweeps,
                        long nM, long nT, long nV, hipStream_t st) {
  if (Kp < 2 * JB || Kp % JP != 0 || ld < Kp) return refuse("jacobi", "shape");
  const int nb = Kp / JB;
  if (r < 0 || r >= nb - 1) return refuse("jacobi", "round");
  GW_GUARD("jacobi", "M", (long)(Kp - 1) * ld + Kp - 1, nM);
  GW_GUARD("jacobi", "T", (long)(Kp - 1) * ld + Kp - 1, nT);
  GW_GUARD("jacobi", "V", (long)(nb / 2) * JP * JP - 1, nV);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_jacobi_sub, dim3(nb / 2), dim3(256), 0, st, M, ld, nb, r, V, max_sweeps);
  hipLaunchKernelGGL(k_jacobi_cols, dim3(Kp / JP, nb / 2), dim3(256), 0, st, M, ld, nb, r, V);
  hipLaunchKernelGGL(k_jacobi_rows, dim3(Kp / JP, nb / 2), dim3(256), 0, st, M, ld, nb, r, V);
  hipLaunchKernelGGL(k_jacobi_cols, dim3(Kp / JP, nb / 2), dim3(256), 0, st, T, ld, nb, r, V);
  return hipGetLastError();
}

// part[b] = (sum of squared off-diagonal, sum of squared diagonal) entries of
// the leading n x n block, over a grid-stride slice per block
__global__ void k_offnorm(const double* M, long ld, int n, double* part) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  const long total = (long)n * n;
  double off = 0.0, dia = 0.0;
  for (long e = blockIdx.x * 256L + t; e < total; e += (long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double v = M[(long)i * ld + j];
    if (i == j) dia += v * v;
    else off += v * v;
  }
  red[0][t] = off;
  red[1][t] = dia;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] += red[0][t + h];
      red[1][t] += red[1][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

hipError_t offnorm(const double* M, long ld, int n, double* part, int blocks, long nM,
                   long nPart, hipStream_t st) {
  if (n < 1 || blocks < 1) return refuse("offnorm", "shape");
  GW_GUARD("offnorm", "M", (long)(n - 1) * ld + n - 1, nM);
  GW_GUARD("offnorm", "part", 2L * blocks - 1, nPart);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_offnorm, dim3(blocks), dim3(256), 0, st, M, ld, n, part);
  return hipGetLastError();
}

// Omega[s] = sqrt(M[s][s]) (s < n)
__global__ void k_diag_sqrt(const double* M, long ld, int n, double* Omega) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) Omega[s] = sqrt(fmax(M[(long)s * ld + s], 0.0));
}

hipError_t diag_sqrt(const double* M, long ld, int n, double* Omega, long nM, long nO,
                     hipStream_t st) {
  GW_GUARD("diag_sqrt", "M", (long)(n - 1) * ld + n - 1, nM);
  GW_GUARD("diag_sqrt", "Omega", n - 1, nO);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_diag_sqrt, dim3((n + 255) / 256), dim3(256), 0, st, M, ld, n, Omega);
  return hipGetLastError();
}

// Y[q][k] *= 2 sqrt(D_k) for k < n (the factor of the pole strengths
// rho = 2 b^T B_ov D^1/2 T), 0 for the padding
__global__ void k_scale_cols(double* Y, long ld, int rows, const double* D, int n, int Kp) {
  const long total = (long)rows * Kp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e / Kp), k = (int)(e % Kp);
    double* y = Y + (long)q * ld + k;
    *y = k < n ? *y * 2.0 * sqrt(D[k]) : 0.0;
  }
}

hipError_t pole_scale(double* Y, long ld, int rows, const double* D, int n, int Kp, long nY,
                      long nD, hipStream_t st) {
  if (rows < 1) return hipSuccess;
  GW_GUARD("pole_scale", "Y", (long)(rows - 1) * ld + Kp - 1, nY);
  GW_GUARD("pole_scale", "D", n - 1, nD);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_scale_cols, dim3(2048), dim3(256), 0, st, Y, ld, rows, D, n, Kp);
  return hipGetLastError();
}

// Pole form of Re Sigma^c for entry j (row rowsel[j], frequency omega[j]):
// sum_m sum_s w2 / (omega - eps_m + Omega_s) over occupied m and
// w2 / (omega - eps_m - Omega_s) over virtual m, w2 = rho^2 / (2 Omega_s);
// 16 slices per entry, partial sums of Sigma and of its derivative.
__global__ __launch_bounds__(256) void k_sigma_sd_part(const double* rho, long ld, int n_mo,
                                                       int n, const int* rowsel,
                                                       const int* rowspin, int n_occ0,
                                                       int n_occ1, const double* omega,
                                                       const double* eps, const double* Omega,
                                                       double* part) {
  __shared__ double rs[256], rd[256];
  const int j = blockIdx.x, sl = blockIdx.y, t = threadIdx.x;
  const int r = rowsel[j];
  const int sp = rowspin ? rowspin[r] : 0;
  const int n_occ = sp ? n_occ1 : n_occ0;
  const double* e = eps + (long)sp * n_mo;
  const double w = omega[j];
  const long total = (long)n_mo * n;
  const long chunk = (total + 15) / 16;
  const long lo = sl * chunk, hi = lo + chunk < total ? lo + chunk : total;
  double s = 0.0, d = 0.0;
  for (long idx = lo + t; idx < hi; idx += 256) {
    const int m = (int)(idx / n), k = (int)(idx % n);
    const double x = rho[((long)r * n_mo + m) * ld + k];
    const double w2 = x * x / (2.0 * Omega[k]);
    const double den = m < n_occ ? w - e[m] + Omega[k] : w - e[m] - Omega[k];
    s += w2 / den;
    d -= w2 / (den * den);
  }
  rs[t] = s;
  rd[t] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      rs[t] += rs[t + h];
      rd[t] += rd[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[(long)(j * 16 + sl) * 2] = rs[0];
    part[(long)(j * 16 + sl) * 2 + 1] = rd[0];
  }
}

__global__ void k_sigma_sd_sum(const double* part, int cnt, double* sig, double* dsig) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  double s = 0.0, d = 0.0;
  for (int sl = 0; sl < 16; ++sl) {
    s += part[(long)(j * 16 + sl) * 2];
    d += part[(long)(j * 16 + sl) * 2 + 1];
  }
  sig[j] = s;
  dsig[j] = d;
}

hipError_t sigma_sd(const double* rho, long ld, int n_mo, int n, int n_rows, const int* rowsel,
                    const int* rowspin, int n_occ0, int n_occ1, const double* omega,
                    const double* eps, const double* Omega, int cnt, double* sig, double* dsig,
                    double* part, long nRho, long nEps, long nOmega, long nPart,
                    hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  if (n < 1 || ld < n) return refuse("sigma_sd", "shape");
  // row indices come from the context's validated state -> row map (< n_rows)
  GW_GUARD("sigma_sd", "rho", ((long)n_rows * n_mo - 1) * ld + n - 1, nRho);
  GW_GUARD("sigma_sd", "eps", (rowspin ? 2L : 1L) * n_mo - 1, nEps);
  GW_GUARD("sigma_sd", "Omega", n - 1, nOmega);
  GW_GUARD("sigma_sd", "partials", (long)cnt * 32 - 1, nPart);
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_sigma_sd_part, dim3(cnt, 16), dim3(256), 0, st, rho, ld, n_mo, n, rowsel,
                     rowspin, n_occ0, n_occ1, omega, eps, Omega, part);
  hipLaunchKernelGGL(k_sigma_sd_sum, dim3((cnt + 63) / 64), dim3(64), 0, st, part, cnt, sig, dsig);
  return hipGetLastError();
}

}  // namespace gw
