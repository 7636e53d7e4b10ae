// FP64 MFMA GEMM used by the Pi build, the blocked Cholesky of the augmented
// dielectric matrix and the MINRES matrix-vector products.
//
// Work tile: BM x BN outputs per 256-thread workgroup (4 wavefronts), staged
// through LDS in K-steps of 16 with double buffering; each wavefront owns
// TM x TN blocks of 16x16 and issues v_mfma_f64_16x16x4_f64.  Operands are
// either k-contiguous ([row][k]) or k-major ([k][row]) in HBM and keep that
// orientation in LDS (layouts below, chosen to be free of bank conflicts on
// the 64-bank LDS).  All extents handed to the kernel are padded to the tile,
// so the inner loop carries no bounds checks.
//
// Workgroups are swizzled so that each XCD (workgroups are dealt round-robin
// to the 8 XCDs) receives a contiguous range of the work list; with the batch
// index fastest (Pi build) the 64-128 grid points of one output tile run on
// one XCD at the same time and stream the same B rows through its L2.
#include "gw_internal.h"

namespace gw {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BK = 16;   // K-step of the default configurations

__device__ __forceinline__ int xcd_swizzle(int wid, int total) {
  const int nx = 8;
  int q = total / nx, r = total % nx;
  int x = wid % nx, l = wid / nx;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

template <int BM, int BN>
__device__ __forceinline__ void decode_tile(const GemmArgs& p, int tile, int& I, int& J) {
  if (p.map == MAP_FULL) {
    I = tile / p.tiles_n;
    J = tile % p.tiles_n;
    return;
  }
  if (p.map == MAP_FULL_J) {
    I = tile % p.tiles_m;
    J = tile / p.tiles_m;
    return;
  }
  // lower map: row tile I holds columns J <= ((I+1)*BM - 1) / BN
  int acc = 0;
  for (I = 0; I < p.tiles_m; ++I) {
    int cnt = ((I + 1) * BM - 1) / BN + 1;
    if (cnt > p.tiles_n) cnt = p.tiles_n;
    if (tile < acc + cnt) { J = tile - acc; return; }
    acc += cnt;
  }
  I = p.tiles_m; J = 0;  // unreachable when n_tiles is consistent
}

// LDS tiles.  k-contiguous operands keep [row][k] (16 doubles, 128 bytes a
// row) with the eight 16-byte chunks of a row XOR-permuted by the row pair;
// k-major operands keep [k][row] with the two 128-byte halves of each
// 32-double group swapped on rows k with bit 1 set.  Together with the
// K-step permutation below this keeps the staging stores and the fragment
// reads free of LDS bank conflicts (checked with SQ_LDS_BANK_CONFLICT on
// gfx950, whose 16-byte reads serve the four 16-lane groups of a wave
// together: their slot patterns may differ only in the low two slot bits).
template <int BR, int LAYOUT>
struct LdsTile {
  static_assert(BR % 32 == 0, "row tiles are multiples of 32");
  static constexpr int ELEMS = BR * BK;
};

__device__ __forceinline__ int kc_chunk(int row, int c) { return c ^ ((row >> 1) & 7); }
__device__ __forceinline__ int km_col(int k, int col) { return col ^ ((k & 2) << 3); }

// Fragment of one 16-row block for two of the four MFMAs of a K-step (half h
// = 0, 1).  The summation index inside a K-step is permuted identically for
// both operands: MFMA (h, e), lane group g = lane / 16 contracts over
// k = 2 g + 8 h + e, so a lane's two values form chunk g + 4 h of a
// k-contiguous row, and the four lane groups read chunks differing only in
// their low two bits.
template <int BR, int LAYOUT>
__device__ __forceinline__ d2 load_frag(const double* Xs, int row, int g, int h) {
  if (LAYOUT == KC) return *reinterpret_cast<const d2*>(Xs + row * BK + 2 * kc_chunk(row, g + 4 * h));
  const int k = 2 * g + 8 * h;
  d2 f;
  f.x = Xs[k * BR + km_col(k, row)];
  f.y = Xs[(k + 1) * BR + km_col(k + 1, row)];
  return f;
}

template <int BR, int LAYOUT, bool SCALED>
struct Stager {
  // number of 16-byte items per thread for a BR x BK tile
  static constexpr int NITEM = BR * BK / 2 / 256;
  d2 v[NITEM];
  __device__ __forceinline__ void load(const double* X, long ld, int r0, int kk0,
                                       const double* s, int t) {
#pragma unroll
    for (int u = 0; u < NITEM; ++u) {
      int q = t + 256 * u;
      if (LAYOUT == KC) {
        int row = q / (BK / 2), k = (q % (BK / 2)) * 2;
        v[u] = *reinterpret_cast<const d2*>(X + (long)(r0 + row) * ld + kk0 + k);
        if (SCALED) v[u] *= *reinterpret_cast<const d2*>(s + kk0 + k);
      } else {
        int k = q / (BR / 2), rp = (q % (BR / 2)) * 2;
        v[u] = *reinterpret_cast<const d2*>(X + (long)(kk0 + k) * ld + r0 + rp);
        if (SCALED) v[u] *= s[kk0 + k];
      }
    }
  }
  __device__ __forceinline__ void store(double* Xs, int t) {
#pragma unroll
    for (int u = 0; u < NITEM; ++u) {
      int q = t + 256 * u;
      if (LAYOUT == KC) {
        int row = q / (BK / 2), c = q % (BK / 2);
        *reinterpret_cast<d2*>(Xs + row * BK + 2 * kc_chunk(row, c)) = v[u];
      } else {
        int k = q / (BR / 2), rp = (q % (BR / 2)) * 2;
        *reinterpret_cast<d2*>(Xs + k * BR + km_col(k, rp)) = v[u];
      }
    }
  }
};

template <int WAVES_M, int TM, int TN, int LA, int LB, int EPI, bool SCALED, bool BATCH_FAST>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs p) {
  constexpr int WAVES_N = 4 / WAVES_M;
  constexpr int BM = WAVES_M * TM * 16;
  constexpr int BN = WAVES_N * TN * 16;
  constexpr int LA_N = LdsTile<BM, LA>::ELEMS;
  constexpr int LB_N = LdsTile<BN, LB>::ELEMS;
  __shared__ __attribute__((aligned(16))) double As[2 * LA_N];
  __shared__ __attribute__((aligned(16))) double Bs[2 * LB_N];
  __shared__ double red[WAVES_N][BM];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  const int total = p.n_tiles * p.batch * p.splitk;
  const int id = xcd_swizzle(blockIdx.x, total);
  int tile, b, split;
  if (BATCH_FAST) {
    b = id % p.batch;
    int rest = id / p.batch;
    split = rest % p.splitk;
    tile = rest / p.splitk;
  } else {
    tile = id % p.n_tiles;
    int rest = id / p.n_tiles;
    split = rest % p.splitk;
    b = rest / p.splitk;
  }
  int I, J;
  decode_tile<BM, BN>(p, tile, I, J);

  const double* A = p.Atab ? p.Atab[b / p.grp] : p.A + (long)b * p.sA;
  const double* Bm = p.Btab ? p.Btab[b / p.grp] : p.B + (long)b * p.sB;
  const double* S = SCALED ? p.scale + (long)b * p.sS : nullptr;
  const int arow0 = p.row0 + I * BM;
  const int brow0 = p.col0 + J * BN;

  int kchunk = ((p.K / BK + p.splitk - 1) / p.splitk) * BK;
  int kbeg = split * kchunk;
  int kend = kbeg + kchunk;
  if (kend > p.K) kend = p.K;
  if (p.ktri) {
    const int lim = p.col0 + (J + 1) * BN - p.kb0;
    if (kend > lim) kend = lim;
  }
  if (p.klo_from > 0) {
    const int r0 = p.row0 + I * BM - p.klo_from;
    if (r0 > kbeg) kbeg = (r0 / BK) * BK;
  }
  const int nk = kend > kbeg ? (kend - kbeg) / BK : 0;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // 16-row blocks of padding rows (systems beyond the batch) and blocks whose A
  // rows are known to be zero (converged systems) skip their MFMAs; a tile
  // with no live block at all returns before loading anything (its output
  // rows belong to systems that no longer read them)
  bool row_ok[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int r = I * BM + wm * TM * 16 + i * 16;
    row_ok[i] = (p.mrows <= 0 || r < p.mrows) && (!p.rowmask || p.rowmask[r >> 4] != 0);
  }
  if (p.rowmask) {
    bool live = false;
    for (int r = I * BM; r < I * BM + BM; r += 16)
      live |= (p.mrows <= 0 || r < p.mrows) && p.rowmask[r >> 4] != 0;
    if (!live) return;
  }

  Stager<BM, LA, false> sa;
  Stager<BN, LB, SCALED> sb;
  if (nk > 0) {
    sa.load(A, p.lda, arow0, p.k0 + kbeg, nullptr, t);
    sb.load(Bm, p.ldb, brow0, p.kb0 + kbeg, S, t);
    sa.store(As, t);
    sb.store(Bs, t);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      const int kstep = kbeg + (kt + 1) * BK;
      sa.load(A, p.lda, arow0, p.k0 + kstep, nullptr, t);
      sb.load(Bm, p.ldb, brow0, p.kb0 + kstep, S, t);
    }
    {
      const double* Ac = As + cur * LA_N;
      const double* Bc = Bs + cur * LB_N;
      const int g = lane >> 4;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        d2 av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = load_frag<BM, LA>(Ac, wm * TM * 16 + i * 16 + (lane & 15), g, h);
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = load_frag<BN, LB>(Bc, wn * TN * 16 + j * 16 + (lane & 15), g, h);
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
          for (int i = 0; i < TM; ++i)
            if (row_ok[i])
#pragma unroll
              for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][e], bv[j][e], acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) {
      sa.store(As + (cur ^ 1) * LA_N, t);
      sb.store(Bs + (cur ^ 1) * LB_N, t);
    }
    __syncthreads();
  }

  // Epilogue.  f64 16x16x4 output layout: lane l, register r holds
  // row (l / 16) + 4 r, column l % 16 of the 16x16 block.
  double* C = (p.Ctab ? p.Ctab[b / p.grp] : p.C + (long)b * p.sC) + (long)split * p.sSplit;
  if (EPI == EPI_RES_DERIV || EPI == EPI_SQNORM) {
    // per-row sum over this tile's columns of acc^2 (EPI_SQNORM) or of
    // acc^2 * 2 D w / (D^2 - w^2)^2 (EPI_RES_DERIV)
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lrow = wm * TM * 16 + i * 16 + (lane >> 4) + 4 * r;
        const double w = (EPI == EPI_RES_DERIV) ? p.wrow[arow0 + lrow] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const double u = acc[i][j][r];
          if (EPI == EPI_RES_DERIV) {
            const int gcol = brow0 + wn * TN * 16 + j * 16 + (lane & 15);
            const double D = p.Dvec[gcol];
            const double den = D * D - w * w;
            s += u * u * (2.0 * D * w / (den * den));
          } else {
            s += u * u;
          }
        }
        // reduce over the 16 lanes sharing this row
        for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
        if ((lane & 15) == 0) red[wn][lrow] = s;
      }
    }
    __syncthreads();
    if (t < BM) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < WAVES_N; ++q) s += red[q][t];
      C[(long)J * p.ldc + arow0 + t] = s;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int grow = arow0 + wm * TM * 16 + i * 16 + (lane >> 4) + 4 * r;
        const int gcol = brow0 + wn * TN * 16 + j * 16 + (lane & 15);
        double* c = C + (long)grow * p.ldc + gcol;
        const double v = acc[i][j][r];
        if (EPI == EPI_ONE_PLUS_4) {
          *c = (grow == gcol ? 1.0 : 0.0) + 4.0 * v;
        } else if (EPI == EPI_AXPBY) {
          *c = (p.beta == 0.0) ? p.alpha * v : p.alpha * v + p.beta * (*c);
        } else if (EPI == EPI_RES_SCALE) {
          const double w = p.wrow[grow];
          const double D = p.Dvec[gcol];
          *c = v * (D / (D * D - w * w));
        } else {
          *c = v;
        }
      }
    }
  }
}

template <int WAVES_M, int TM, int TN, int LA, int LB, int EPI, bool SCALED, bool BF>
static hipError_t launch(const GemmArgs& a, hipStream_t st) {
  const long total = (long)a.n_tiles * a.batch * a.splitk;
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL((k_gemm_f64<WAVES_M, TM, TN, LA, LB, EPI, SCALED, BF>),
                     dim3((unsigned)total), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Largest element index each operand of a launch can touch (see the kernel's
// index arithmetic above), checked against the extents carried in GemmArgs.
static hipError_t check_gemm(const GemmArgs& a, int tile_kind, int la, int lb, int epi) {
  const int BM = (tile_kind == 2 || tile_kind == 3) ? 64 : 128;
  const int BN = (tile_kind == 1 || tile_kind == 3) ? 64 : 128;
  const int KSTEP = BK;
  const char* kn = "gemm_f64";
  if (a.K <= 0 || a.K % KSTEP != 0 || a.tiles_m <= 0 || a.tiles_n <= 0 || a.batch <= 0 ||
      a.splitk <= 0 || a.row0 < 0 || a.col0 < 0 || a.k0 < 0 || a.kb0 < 0)
    return refuse(kn, "shape");
  long want = (a.map == MAP_FULL || a.map == MAP_FULL_J) ? (long)a.tiles_m * a.tiles_n : 0;
  if (a.map == MAP_LOWER)
    for (int I = 0; I < a.tiles_m; ++I) {
      int c = ((I + 1) * BM - 1) / BN + 1;
      want += c < a.tiles_n ? c : a.tiles_n;
    }
  if (want != a.n_tiles) return refuse(kn, "tile count");
  // 16-byte vector loads: even leading dimensions and offsets, aligned bases
  if ((a.lda | a.ldb | a.k0 | a.kb0 | a.row0 | a.col0) & 1)
    return refuse(kn, "odd leading dimension or offset");
  if (((uintptr_t)a.A | (uintptr_t)a.B) & 15)
    return refuse(kn, "operand pointer not 16-byte aligned");
  const long rmax = a.row0 + (long)a.tiles_m * BM - 1;
  const long cmax = a.col0 + (long)a.tiles_n * BN - 1;
  const long b1 = a.batch - 1;
  if ((a.Atab || a.Btab || a.Ctab) && (a.grp <= 0 || a.batch % a.grp != 0))
    return refuse(kn, "operand table group");
  // a table's pointers are checked one request at a time (item offset 0)
  const long bA = a.Atab ? 0 : b1, bB = a.Btab ? 0 : b1, bC = a.Ctab ? 0 : b1;
  long maxA = la == KC ? bA * a.sA + rmax * a.lda + a.k0 + a.K - 1
                       : bA * a.sA + (long)(a.k0 + a.K - 1) * a.lda + rmax;
  long maxB = lb == KC ? bB * a.sB + cmax * a.ldb + a.kb0 + a.K - 1
                       : bB * a.sB + (long)(a.kb0 + a.K - 1) * a.ldb + cmax;
  if (!guard(kn, "A", maxA, a.nA)) return hipErrorInvalidValue;
  if (!guard(kn, "B", maxB, a.nB)) return hipErrorInvalidValue;
  if (a.scale && !guard(kn, "scale", b1 * a.sS + a.kb0 + a.K - 1, a.nS)) return hipErrorInvalidValue;
  const bool per_tile = epi == EPI_RES_DERIV || epi == EPI_SQNORM;
  long maxC = bC * a.sC + (long)(a.splitk - 1) * a.sSplit +
              (per_tile ? (long)(a.tiles_n - 1) * a.ldc + rmax : rmax * a.ldc + cmax);
  if ((a.ktri || a.klo_from > 0) && a.splitk != 1) return refuse(kn, "triangular k limit with split-K");
  if (a.rowmask && !guard(kn, "rowmask", ((long)a.tiles_m * BM - 1) / 16, a.nMask))
    return hipErrorInvalidValue;
  if (!guard(kn, "C", maxC, a.nC)) return hipErrorInvalidValue;
  if (epi == EPI_RES_SCALE || epi == EPI_RES_DERIV) {
    if (!guard(kn, "D", cmax, a.nD)) return hipErrorInvalidValue;
    if (!guard(kn, "w", rmax, a.nW)) return hipErrorInvalidValue;
  }
  return hipSuccess;
}

// Instantiations used by the library.
// tile_kind: 0 = 128x128, 1 = 128x64, 2 = 64x128, 3 = 64x64.
hipError_t gemm_f64(const GemmArgs& a, int tile_kind, int la, int lb, int epi, hipStream_t st) {
  {
    hipError_t e = check_gemm(a, tile_kind, la, lb, epi);
    if (e != hipSuccess) return e;
  }
  const bool scaled = a.scale != nullptr;
  // Pi build: KC x KC, scaled, 1 + 4 acc, batch-fastest
  if (tile_kind == 0 && la == KC && lb == KC && epi == EPI_ONE_PLUS_4 && scaled)
    return launch<2, 4, 4, KC, KC, EPI_ONE_PLUS_4, true, true>(a, st);
  // Cholesky panel update (C -= L_left L_panel^T) and panel solve: KC x KC, axpby
  if (tile_kind == 0 && la == KC && lb == KC && epi == EPI_AXPBY && !scaled)
    return launch<2, 4, 4, KC, KC, EPI_AXPBY, false, false>(a, st);
  // MINRES first pass split over N_aux: partial X B, 64 x 64 tiles
  if (tile_kind == 3 && la == KC && lb == KM && epi == EPI_STORE && !scaled)
    return launch<2, 2, 2, KC, KM, EPI_STORE, false, false>(a, st);
  // MINRES: V = scale(X B) with X [sys][P] (KC) and B_ov [P][ia] (KM): 64 x 64 tiles
  if (tile_kind == 3 && la == KC && lb == KM && epi == EPI_RES_SCALE && !scaled)
    return launch<2, 2, 2, KC, KM, EPI_RES_SCALE, false, false>(a, st);
  if (tile_kind == 3 && la == KC && lb == KM && epi == EPI_RES_DERIV && !scaled)
    return launch<2, 2, 2, KC, KM, EPI_RES_DERIV, false, false>(a, st);
  // dense fallback LU: A22 -= L21 U12 (U12 rows k-major), 128 x 128 tiles, batched
  if (tile_kind == 0 && la == KC && lb == KM && epi == EPI_AXPBY && !scaled)
    return launch<2, 4, 4, KC, KM, EPI_AXPBY, false, false>(a, st);
  // MINRES operator passes on 128 x 128 tiles (batches of 128 systems and more)
  if (tile_kind == 0 && la == KC && lb == KM && epi == EPI_STORE && !scaled)
    return launch<2, 4, 4, KC, KM, EPI_STORE, false, false>(a, st);
  if (tile_kind == 0 && la == KC && lb == KM && epi == EPI_RES_SCALE && !scaled)
    return launch<2, 4, 4, KC, KM, EPI_RES_SCALE, false, false>(a, st);
  if (tile_kind == 0 && la == KC && lb == KM && epi == EPI_RES_DERIV && !scaled)
    return launch<2, 4, 4, KC, KM, EPI_RES_DERIV, false, false>(a, st);
  if (tile_kind == 0 && la == KC && lb == KC && epi == EPI_STORE && !scaled)
    return launch<2, 4, 4, KC, KC, EPI_STORE, false, false>(a, st);
  // MINRES: part[s][sys][P] = sum_ia V[sys][ia] B_ov[P][ia], split-K partials, 64 x 128 tiles
  if (tile_kind == 2 && la == KC && lb == KC && epi == EPI_STORE && !scaled)
    return launch<1, 4, 2, KC, KC, EPI_STORE, false, false>(a, st);
  // Cholesky panel solve and the preconditioner X X^T: short K or few tiles, so
  // 64 x 128 tiles for twice the workgroups of the 128 x 128 form
  if (tile_kind == 2 && la == KC && lb == KC && epi == EPI_AXPBY && !scaled)
    return launch<1, 4, 2, KC, KC, EPI_AXPBY, false, false>(a, st);
  // W^c reduction: |R^T Linv^T|^2 per row, Linv^T k-major, triangular k range;
  // grid point slowest so that the tiles reading one L^-T panel run together
  if (tile_kind == 0 && la == KC && lb == KM && epi == EPI_SQNORM && !scaled)
    return launch<2, 4, 4, KC, KM, EPI_SQNORM, false, false>(a, st);
  // Casida matrix: B_ov^T B_ov with both operands k-major (B_ov [P][ia])
  if (tile_kind == 0 && la == KM && lb == KM && epi == EPI_STORE && !scaled)
    return launch<2, 4, 4, KM, KM, EPI_STORE, false, false>(a, st);
  // generic full 128x128 store / axpby (tests, dense fallback build)
  if (tile_kind == 0 && la == KC && lb == KC && epi == EPI_STORE && scaled)
    return launch<2, 4, 4, KC, KC, EPI_STORE, true, false>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace gw
