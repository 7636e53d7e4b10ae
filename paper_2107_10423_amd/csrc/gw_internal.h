// Internal declarations shared by the HIP translation units of libgw.
// Not part of the public C-ABI (see include/gw.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace gw {

// ---------------------------------------------------------------------------
// Launch guards.  Every kernel wrapper computes, on the host, the largest
// element index its launch can touch in each buffer and compares it with the
// buffer's extent (elements available from the pointer handed in); a launch
// that could leave a buffer is refused with hipErrorInvalidValue and the
// reason is kept in launch_error().  In audit mode the wrappers stop after
// the check and launch nothing (see include/gw_audit.h).
bool audit_mode();
void set_audit_mode(bool on);
const char* launch_error();
bool guard(const char* kernel, const char* buffer, long max_index, long extent);
hipError_t refuse(const char* kernel, const char* why);  // records why, returns an error
#define GW_GUARD(kernel, buffer, max_index, extent) \
  do {                                              \
    if (!::gw::guard(kernel, buffer, (long)(max_index), (long)(extent))) return hipErrorInvalidValue; \
  } while (0)
long audit_count();
void audit_note();
#define GW_AUDIT_RETURN()      \
  do {                         \
    if (::gw::audit_mode()) {  \
      ::gw::audit_note();      \
      return hipSuccess;       \
    }                          \
  } while (0)

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM.  C_tile = epilogue( sum_k A(i,k) * s(k) * B(j,k) ).
// Operand layouts: KC = row-major [row][k] (k contiguous), KM = [k][row].
enum OpLayout { KC = 0, KM = 1 };

enum Epilogue {
  EPI_ONE_PLUS_4 = 0,   // C = delta_ij + 4 acc           (1 - Pi(i xi) from B d B^T)
  EPI_AXPBY = 1,        // C = alpha acc + beta C
  EPI_RES_SCALE = 2,    // C = acc * D/(D^2 - w_row^2)    (MINRES: scaled B^T v, rows = systems)
  EPI_RES_DERIV = 3,    // part[colTile][row] = sum_col acc^2 * 2 D w/(D^2 - w^2)^2
  EPI_STORE = 4,        // C = acc (split-K partials)
  EPI_SQNORM = 5,       // part[colTile][row] = sum_col acc^2
};

enum TileMap {
  MAP_FULL = 0,   // every (I, J) tile, row tiles outer
  MAP_FULL_J = 2, // every (I, J) tile, column tiles outer (tiles sharing a B panel adjacent)
  MAP_LOWER = 1,  // tiles holding some element with row >= col (both offset by `diag_off`)
};

struct GemmArgs {
  const double* A; long lda; long sA;   // sA: batch stride (elements)
  const double* B; long ldb; long sB;
  const double* scale; long sS;         // per-k scale of B, or nullptr
  double* C; long ldc; long sC;
  int M, N, K;                          // M, N multiples of the tile; K multiple of 16
  int row0, col0;                       // offsets of the first A row / B row
  int k0, kb0;                          // k offsets of A and of B (and of the scale)
  int map;                              // TileMap
  int tiles_m, tiles_n;
  int n_tiles;                          // tiles per batch item
  int batch;
  int splitk;                           // >= 1; split s covers k in [s*K/splitk, (s+1)*K/splitk)
  int ktri;                             // B(j, k) = 0 for k > j: stop k at the tile's last B row
  int klo_from;                         // > 0: A rows r >= klo_from are zero for
                                        // k < r - klo_from; a row tile starting at r0
                                        // begins its k loop there (splitk 1 only)
  long sSplit;                          // C offset between split-K slabs
  int mrows;                            // rows >= mrows of each tile column are padding whose
                                        // MFMAs are skipped (0: every row is computed)
  const int* rowmask;                   // per 16-row block of A: 0 = rows known to be zero
                                        // whose outputs nobody reads: MFMAs skipped, and a
                                        // tile without a live block writes nothing
                                        // (nullptr: every block is computed)
  // Grouped launches (several requests' grid points in one launch): batch item b
  // belongs to request b / grp; a non-null table replaces the strided operand
  // base (A + b sA, B + b sB, C + b sC) by that request's pointer.  The host
  // then passes as nA / nB / nC the smallest extent over the table's pointers.
  const double* const* Atab;
  const double* const* Btab;
  double* const* Ctab;
  int grp;
  double alpha, beta;
  const double* Dvec;                   // transition energies (EPI_RES_*)
  const double* wrow;                   // per-row real frequency (EPI_RES_*)
  // extents (elements reachable from each pointer), checked before launch
  long nA, nB, nS, nC, nD, nW, nMask;
};

hipError_t gemm_f64(const GemmArgs& a, int tile_kind, int la, int lb, int epi, hipStream_t st);
// tile_kind 0: 128x128, 1: 128x64, 2: 64x128, 3: 64x64

// Mixed-precision Pi builds (write 1 - Pi lower tiles in FP64)
// nB: elements of each B copy, nS: of scale, nA: of the output
hipError_t pi_build_f32(const float* B32, long ld, const float* scale, long sS, double* A,
                        long ldA, long sA, int Np, int Kp, int G, long nB, long nS, long nA,
                        hipStream_t st);
hipError_t pi_build_bf16x3(const uint16_t* Bhi, const uint16_t* Blo, long ld, const float* B32,
                           const float* scale, long sS, double* A, long ldA, long sA, int Np,
                           int Kp, int G, long nB, long nS, long nA, hipStream_t st);
// Per-request operand tables of a grouped launch: item g of the batch reads the
// operands of request g / grp.  Null tables: the single-request operands.
struct OperandTabs {
  const float* const* B32;        // pi builds: FP32 copy of each request's B_ov
  const uint16_t* const* Bhi;     // pi builds: bf16 hi of each request's B_ov (lo follows
  const uint16_t* const* Blo;     //   in its own table)
  const uint16_t* const* Rh;      // mixed W^c: each request's split R (hi; lo at +nRR)
  int grp;
};
hipError_t pi_build_f32_tab(const OperandTabs& tb, long ld, const float* scale, long sS,
                            double* A, long ldA, long sA, int Np, int Kp, int G, long nB,
                            long nS, long nA, hipStream_t st);
hipError_t pi_build_bf16x3_tab(const OperandTabs& tb, long ld, const float* scale, long sS,
                               double* A, long ldA, long sA, int Np, int Kp, int G, long nB,
                               long nS, long nA, hipStream_t st);
// panels of W^c partial sums the contraction writes per grid point (its
// reduction sums this many: 128-wide panels, or 256-wide for large N_aux)
int wc_bf16x3_panels(int Np);
hipError_t wc_bf16x3_tab(const OperandTabs& tb, long nRR, long ldR, int Rp, const uint16_t* Fh,
                         const uint16_t* Fl, long sF, int Np, int G, double* part, long ldp,
                         long sP, long nR, long nF, long nP, hipStream_t st);
hipError_t split_bf16(const double* B, uint16_t* hi, uint16_t* lo, float* b32, long n, hipStream_t st);
// mixed W^c contraction: F = L^-1 - I split from X = L^-T (k-major), then
// part[g][J][q] = sum over panel J of (2 b + y) y with y = F b (BF16x3)
hipError_t split_linv(const double* X, long ldX, long sX, int Np, int G, uint16_t* Fh,
                      uint16_t* Fl, long sF, long nX, long nF, hipStream_t st);
hipError_t wc_bf16x3(const uint16_t* Rh, const uint16_t* Rl, long ldR, int Rp, const uint16_t* Fh,
                     const uint16_t* Fl, long sF, int Np, int G, double* part, long ldp, long sP,
                     long nR, long nF, long nP, hipStream_t st);

// Cholesky pieces
hipError_t chol_diag(double* A, long ldA, long sA, double* Linv, int k, int G, int* info,
                     long nA, long nLinv, long nInfo, hipStream_t st);
// test hook: A <- 2 I - A on the leading Np x Np block of G items
hipError_t reflect_unit(double* A, long ldA, long sA, int Np, int G, long nA, hipStream_t st);
// rows [row0, row0 + n) of every batch item <- identity rows e_0 .. e_{n-1}
// (columns [0, ncol))
hipError_t set_identity_rows(double* A, long ldA, long sA, int row0, int n, int ncol, int G,
                             long nA, hipStream_t st);
// wtab[q][g0 + g] = sum_J part[g][J][q] - bnorm2[q] for q < nR
hipError_t wc_from_parts(const double* part, long sPart, int nJ, int ldp, const double* bnorm2,
                         int nR, int G, int Gtot, int g0, double* wtab, long nPart, long nBn,
                         long nW, hipStream_t st);
// grouped form: item g writes column g % grp of request g / grp's table
// (wtab_tab, bn_tab: per-request pointers, bn_tab null for the mixed form)
hipError_t wc_from_parts_tab(const double* part, long sPart, int nJ, int ldp,
                             const double* const* bn_tab, int nR, int G, int grp,
                             double* const* wtab_tab, long nPart, long nBn, long nW,
                             hipStream_t st);
// fills n ints with v (graph-safe replacement for a memset)
hipError_t fill_int(int* p, int n, int v, long nP, hipStream_t st);

// prep
// stacked transition energies of n_spin (1 or 2) spins, eps [n_spin][n_mo]
hipError_t transition_energies(const double* eps, int n_spin, int n_mo, const int* n_occ, int Kp,
                               double* D, long nEps, long nD, hipStream_t st);
hipError_t scale_inplace(double* x, long n, double f, long nX, hipStream_t st);
hipError_t row_norm2(const double* R, int nR, int Np, double* bn, long nRext, long nBn,
                     hipStream_t st);
hipError_t make_scale_real(const double* D, int Kov, int Kp, double w, double* s, long nD,
                           long nS, hipStream_t st);
hipError_t copy_vec(const double* src, double* dst, int n, long nSrc, long nDst, hipStream_t st);
hipError_t make_scale_imag(const double* D, int Kov, int Kp, const double* xi, int G, double* s,
                           float* s32, long nD, long nXi, long nS, long nS32, hipStream_t st);
// grouped form: item g uses request g / grp's transition energies and its
// count Kov_tab[g / grp] of real columns, and grid point xi[g % grp]
hipError_t make_scale_imag_tab(const double* const* D_tab, const int* Kov_tab, int Kp,
                               const double* xi, int grp, int G, double* s, float* s32,
                               long nD, long nXi, long nS, long nS32, hipStream_t st);

// Sigma quadrature of n states: per state j, -(1/pi) sum_m sum_{g<G} W[row_j][m][g] z_g
// a/(a^2+xi^2) and its derivative, the table holding ld columns per m; w0 != 0: column G
// is W^c(0), whose part is integrated exactly.  part: scratch of n * 32 doubles (16
// slices, 2 sums)
// rowspin (nullable): spin of each table row; its levels are eps + rowspin[r] * n_mo
hipError_t sigma_quad(const double* wtab, int n_mo, int G, int ld, int w0, const int* rowsel,
                      const int* rowspin, const double* omega, const double* eps,
                      const double* xi, const double* z, int n, double* sig, double* dsig,
                      double* part, int n_rows, long nW, long nPart, long nEps, long nXi,
                      long nZ, hipStream_t st);

// Spectral-decomposition route (sd.hip)
hipError_t casida_matrix(double* C, long ld, const double* D, int n, int Kp, long nC, long nD,
                         hipStream_t st);
hipError_t set_identity(double* T, long ld, int Kp, long nT, hipStream_t st);
// one round r (0 <= r < Kp/32 - 1) of block Jacobi on M with T <- T V; V: Kp/64 * 64 * 64
hipError_t jacobi_round(double* M, double* T, long ld, int Kp, int r, double* V, int max_sweeps,
                        long nM, long nT, long nV, hipStream_t st);
hipError_t offnorm(const double* M, long ld, int n, double* part, int blocks, long nM,
                   long nPart, hipStream_t st);
hipError_t diag_sqrt(const double* M, long ld, int n, double* Omega, long nM, long nO,
                     hipStream_t st);
hipError_t pole_scale(double* Y, long ld, int rows, const double* D, int n, int Kp, long nY,
                      long nD, hipStream_t st);
hipError_t sigma_sd(const double* rho, long ld, int n_mo, int n, int n_rows, const int* rowsel,
                    const int* rowspin, int n_occ0, int n_occ1, const double* omega,
                    const double* eps, const double* Omega, int cnt, double* sig, double* dsig,
                    double* part, long nRho, long nEps, long nOmega, long nPart,
                    hipStream_t st);

// MINRES
struct MinresBufs {
  int k, kp, Np, Kp;       // systems, padded systems, padded aux, padded ov
  double *x, *w, *w2, *r1, *r2, *y, *v;     // [kp][Np] each
  double *scal;            // [kp][16] per-system scalars
  double *V;               // [kp][Kp] scaled B^T v
  double *part;            // split-K partials [splitk][kp][Np] (reused for deriv partials)
  double *x0;              // [kp][Np] starting guesses (0 for a cold start)
  double *omega;           // [kp] real frequencies
  double *rtol;            // [kp] per-system residual target relative to |b|
  int *active;             // [2] count of unconverged systems after odd / even iterations
  int *blk;                // [2][kp / 16] 1 where a block of 16 systems still has an
                           // unconverged one after an odd / even iteration
  long n_vec, n_scal, n_part, n_V, n_blk;   // extents in elements (per array)
  // preconditioning by M = 1 - Pi(0) (symmetric positive definite): systems
  // with preflag[j] != 0 run preconditioned MINRES; the product r M^-1 of all
  // systems arrives as splitp split-K slabs in part.  (Kernels read only
  // device data that a replayed graph sees current: the flags, not a
  // by-value threshold.)
  const double* pre;       // [Np][Np] M^-1, or nullptr (no system preconditioned)
  const int* preflag;      // [kp]
  int splitp;
};
// rhs_idx values must be < n_rhs_rows (rows of rhs_base, each Np long); the host
// passes the index array it uploaded so the guard can check it
// x0_j = v_j = warm_j ? xcache[rhs_idx_j] : 0 (then one operator pass gives y = A x0)
hipError_t minres_gather(MinresBufs& m, const double* xcache, const int* rhs_idx,
                         const int* host_idx, int n_rows, const int* warm, long n_cache,
                         hipStream_t st);
// start MINRES on b - A x0 (use_y: y holds A x0) with the stop test relative to |b|
hipError_t minres_init(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                       const int* host_idx, int n_rhs_rows, int use_y, hipStream_t st);
// x_j += x0_j, and xcache[rhs_idx_j] = x_j
hipError_t minres_finalize(MinresBufs& m, double* xcache, const int* rhs_idx,
                           const int* host_idx, int n_rows, long n_cache, hipStream_t st);
// V[j][ia] = D/(D^2 - w_j^2) * sum_s part[s][j][ia] (split partials of B_ov^T v);
// mask (nullable): per 16-system block, 0 where the block's systems are skipped
hipError_t minres_scale_sum(MinresBufs& m, int splits, const double* D, long nD,
                            const int* mask, long nMask, hipStream_t st);
// y = v + 4 sum_s part[s] (the operator applied to v), one block row per system;
// mask as for minres_scale_sum
hipError_t minres_apply(MinresBufs& m, int splitk, const int* mask, long nMask, hipStream_t st);
// one MINRES step per unconverged system; par = global iteration parity
hipError_t minres_finish_step(MinresBufs& m, int par, hipStream_t st);
// Preconditioned variants (m.pre set).  Start: pre_init_a (r = b - A x0, b kept
// in w), then the product b M^-1 into part, pre_init_b (|b|_M^-1), the product
// r M^-1, pre_init_c (beta1, v).  Iteration: apply, pre_step_a (Lanczos
// update of r1, r2), the product r2 M^-1, pre_step_b (beta, Givens, x).
hipError_t minres_pre_init_a(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                             const int* host_idx, int n_rhs_rows, int use_y, hipStream_t st);
hipError_t minres_pre_init_b(MinresBufs& m, hipStream_t st);
hipError_t minres_pre_init_c(MinresBufs& m, hipStream_t st);
hipError_t minres_pre_step_a(MinresBufs& m, int par, hipStream_t st);
hipError_t minres_pre_step_b(MinresBufs& m, int par, hipStream_t st);
hipError_t minres_results(MinresBufs& m, const double* rhs_base, const int* rhs_idx,
                          int n_rhs_rows, int n_deriv_parts, double* wc, double* dwc, int* conv,
                          long n_out, hipStream_t st);

// dense fallback: solve A_i x_i = b_i for `batch` systems (A_i = A + i sA, b_i =
// b + i sb, pivots piv + i sP, info[i]) by blocked LU with partial pivoting
// (A, b and piv overwritten; n a multiple of 128)
hipError_t dense_solve(double* A, long ldA, long sA, int n, double* b, long sb, int* piv,
                       long sP, int* info, int batch, long nA, long nb, long npiv, long ninfo,
                       hipStream_t st);

}  // namespace gw
