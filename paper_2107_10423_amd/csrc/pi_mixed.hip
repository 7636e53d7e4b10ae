// Mixed-precision builds of the dielectric matrix 1 - Pi(i xi_g) =
// 1 + 4 B diag(s_g) B^T (lower tiles, written in FP64):
//
//  * FP32:   operands B and B s_g rounded to FP32, v_mfma_f32_16x16x4_f32,
//            FP32 accumulators flushed into FP64 every 512 k (split-K in
//            registers), so the long K = n_occ n_virt sum is finished in FP64.
//  * BF16x3: each operand x is split x = hi + lo with hi = bf16(x) and
//            lo = bf16(x - hi); the product is hi_a hi_b + hi_a lo_b + lo_a hi_b
//            (the lo lo term is below the split's own error), three
//            v_mfma_f32_16x16x32_bf16 per k-step, FP32 accumulation over the
//            whole K (the precision tests report the resulting error).  The
//            unscaled side B is split once per molecule and stored; the scaled
//            side B s_g is split on the fly per grid point (packed hardware
//            conversion) while it is staged into LDS.
//
// Tiles are 128 x 128 per 256-thread workgroup (2 x 2 wavefronts of 64 x 64),
// lower-triangular tile map, grid point index fastest and XCD-swizzled as in
// the FP64 kernel.
//
// The same BF16x3 products serve the optional mixed W^c contraction (end of
// this file).  There W^c = |L^-1 b|^2 - |b|^2 is evaluated as
// 2 b^T y + |y|^2 with y = (L^-1 - I) b: the difference of the two large norms
// is never formed, so the error of the low-precision products stays relative
// to W^c itself instead of to |b|^2.
#include "gw_internal.h"

namespace gw {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

constexpr int FLUSH_K = 512;

__device__ __forceinline__ int xcd_swizzle_m(int wid, int total) {
  const int nx = 8;
  int q = total / nx, r = total % nx;
  int x = wid % nx, l = wid / nx;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

__device__ __forceinline__ void lower_tile(int tile, int& I, int& J) {
  // tiles (I, J), J <= I, enumerated row by row
  I = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= tile) ++I;
  while (I * (I + 1) / 2 > tile) --I;
  J = tile - I * (I + 1) / 2;
}

// round-to-nearest-even float -> bf16 bits (inputs are finite)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

__global__ void k_split_bf16(const double* B, uint16_t* hi, uint16_t* lo, float* b32, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    float x = (float)B[i];
    unsigned short h = bf16_rne(x);
    float r = x - bf16_to_f(h);
    hi[i] = h;
    lo[i] = bf16_rne(r);
    if (b32) b32[i] = x;
  }
}

// b32 may be null (only the bf16 pair is wanted)
hipError_t split_bf16(const double* B, uint16_t* hi, uint16_t* lo, float* b32, long n,
                      hipStream_t st) {
  GW_AUDIT_RETURN();  // the arrays are allocated with n elements by the caller
  int blocks = (int)std::min<long>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_split_bf16, dim3(blocks), dim3(256), 0, st, B, hi, lo, b32, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 operands, f32 MFMA.  LDS holds [k][row] floats.

__global__ __launch_bounds__(256) void k_pi_f32(const float* B, long ld, const float* scale,
                                                long sS, double* A, long ldA, long sA, int T,
                                                int Kp, int G, OperandTabs tb) {
  constexpr int BKF = 16;
  __shared__ float As[2][BKF][128];
  __shared__ float Bs[2][BKF][128];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int total = T * (T + 1) / 2 * G;
  const int id = xcd_swizzle_m(blockIdx.x, total);
  const int g = id % G;
  int I, J;
  lower_tile(id / G, I, J);
  const float* S = scale + (long)g * sS;
  const int ar0 = I * 128, br0 = J * 128;
  if (tb.B32) B = tb.B32[g / tb.grp];

  f4 acc[4][4];
  d4 acc64[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // staging: 128 rows x 16 k floats = 512 float4; 2 per thread per operand
  float4 ra[2], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int q = t + 256 * u;
      int row = q >> 2, kq = (q & 3) * 4;
      ra[u] = *reinterpret_cast<const float4*>(B + (long)(ar0 + row) * ld + k0 + kq);
      float4 v = *reinterpret_cast<const float4*>(B + (long)(br0 + row) * ld + k0 + kq);
      const float4 sv = *reinterpret_cast<const float4*>(S + k0 + kq);
      v.x *= sv.x;
      v.y *= sv.y;
      v.z *= sv.z;
      v.w *= sv.w;
      rb[u] = v;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int q = t + 256 * u;
      int row = q >> 2, kq = (q & 3) * 4;
      As[buf][kq + 0][row] = ra[u].x;
      As[buf][kq + 1][row] = ra[u].y;
      As[buf][kq + 2][row] = ra[u].z;
      As[buf][kq + 3][row] = ra[u].w;
      Bs[buf][kq + 0][row] = rb[u].x;
      Bs[buf][kq + 1][row] = rb[u].y;
      Bs[buf][kq + 2][row] = rb[u].z;
      Bs[buf][kq + 3][row] = rb[u].w;
    }
  };
  const int nk = Kp / BKF;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BKF);
#pragma unroll
    for (int ks = 0; ks < BKF / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[cur][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (((kt + 1) * BKF) % FLUSH_K == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (kt + 1 < nk) lstore(cur ^ 1);
    __syncthreads();
  }
  // f32 16x16x4 output layout: lane l, register r -> row 4 (l / 16) + r, col l % 16
  double* Ag = A + (long)g * sA;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = ar0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        int col = br0 + wn * 64 + j * 16 + (lane & 15);
        Ag[(long)row * ldA + col] = (row == col ? 1.0 : 0.0) + 4.0 * acc64[i][j][r];
      }
}

static hipError_t check_pi(const char* kn, long ld, long sS, long ldA, long sA, int Np, int Kp,
                           int G, int bk, long nB, long nS, long nA) {
  if (Np % 128 != 0 || Kp % bk != 0 || ld < Kp || ld % 8 != 0 || sS % 4 != 0)
    return refuse(kn, "shape");
  GW_GUARD(kn, "B", (long)(Np - 1) * ld + Kp - 1, nB);
  GW_GUARD(kn, "scale", (long)(G - 1) * sS + Kp - 1, nS);
  GW_GUARD(kn, "A", (long)(G - 1) * sA + (long)(Np - 1) * ldA + Np - 1, nA);
  return hipSuccess;
}

static hipError_t launch_pi_f32(const float* B32, const OperandTabs& tb, long ld,
                                const float* scale, long sS, double* A, long ldA, long sA,
                                int Np, int Kp, int G, long nB, long nS, long nA, hipStream_t st) {
  const int T = Np / 128;
  const long total = (long)T * (T + 1) / 2 * G;
  if (total <= 0) return hipSuccess;
  if (tb.B32 && (tb.grp <= 0 || G % tb.grp != 0)) return refuse("pi_f32", "operand table group");
  if (hipError_t e = check_pi("pi_f32", ld, sS, ldA, sA, Np, Kp, G, 16, nB, nS, nA)) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_pi_f32, dim3((unsigned)total), dim3(256), 0, st, B32, ld, scale, sS, A, ldA,
                     sA, T, Kp, G, tb);
  return hipGetLastError();
}

hipError_t pi_build_f32(const float* B32, long ld, const float* scale, long sS, double* A,
                        long ldA, long sA, int Np, int Kp, int G, long nB, long nS, long nA,
                        hipStream_t st) {
  return launch_pi_f32(B32, OperandTabs{}, ld, scale, sS, A, ldA, sA, Np, Kp, G, nB, nS, nA, st);
}

// nB: the smallest extent over the table's B copies
hipError_t pi_build_f32_tab(const OperandTabs& tb, long ld, const float* scale, long sS,
                            double* A, long ldA, long sA, int Np, int Kp, int G, long nB,
                            long nS, long nA, hipStream_t st) {
  if (!tb.B32) return refuse("pi_f32", "missing operand table");
  return launch_pi_f32(nullptr, tb, ld, scale, sS, A, ldA, sA, Np, Kp, G, nB, nS, nA, st);
}

// ---------------------------------------------------------------------------
// BF16x3.  LDS holds each 128 x 32 bf16 operand slab chunk-major in 16-byte
// slots: chunk q (k = 8 q .. 8 q + 7) of row r sits in slot
// 128 q + 16 (r / 16) + 4 (r % 4) + ((r % 16) / 4 XOR q).  Staging stores (4
// lanes per row for the pre-split side, 8 lanes per row for the FP32 side,
// so that global loads stay coalesced) then spread over all LDS banks.  For
// the operand reads, the 16 MFMA rows of a block are taken in the permuted
// order pi(p) = 4 (p % 4) + p / 4, which makes lane l (p = l % 16, chunk
// g = l / 16) read slot 128 g + (p XOR g): again free of bank conflicts.  The
// permutation is undone when the accumulators are written.  (All three
// patterns were checked with the SQ_LDS_BANK_CONFLICT counter on gfx950.)

constexpr int BKB = 32;
constexpr int SLAB = 128 * BKB;  // bf16 elements of one operand slab

__device__ __forceinline__ int lds_slot(int row, int ch) {
  return 8 * (ch * 128 + (row >> 4) * 16 + 4 * (row & 3) + (((row & 15) >> 2) ^ ch));
}
// physical row (within a 16-row block) of MFMA row p
__device__ __forceinline__ int mfma_row(int p) { return 4 * (p & 3) + (p >> 2); }

// Staging of one 32-wide K-step: the unscaled side is loaded pre-split
// (bf16 hi and lo, one 16-byte chunk per item, 2 items per thread); the scaled
// side is loaded as FP32 (4 values per item, 4 items per thread) with its
// scales, and multiplied and split into hi/lo when it is written to LDS.
// Item maps: A item q -> row q / 4, chunk q % 4; B item q -> row q / 8, chunk
// (q % 8) / 2, half q % 2.
__device__ __forceinline__ void a_item(int q, int& row, int& ch) {
  row = q >> 2;
  ch = q & 3;
}
__device__ __forceinline__ void b_item(int q, int& row, int& ch, int& half) {
  row = q >> 3;
  ch = (q & 7) >> 1;
  half = q & 1;
}

__device__ __forceinline__ void bf_gload(const uint16_t* Bhi, const uint16_t* Blo,
                                         const float* B32, const float* S, long ld, int ar0,
                                         int br0, int k0, int t, u32x4 (&rah)[2],
                                         u32x4 (&ral)[2], f32x4 (&rb)[4], f32x4 (&rs)[4]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int row, ch;
    a_item(t + 256 * u, row, ch);
    rah[u] = *reinterpret_cast<const u32x4*>(Bhi + (long)(ar0 + row) * ld + k0 + 8 * ch);
    ral[u] = *reinterpret_cast<const u32x4*>(Blo + (long)(ar0 + row) * ld + k0 + 8 * ch);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int row, ch, half;
    b_item(t + 256 * u, row, ch, half);
    const int k = k0 + 8 * ch + 4 * half;
    rb[u] = *reinterpret_cast<const f32x4*>(B32 + (long)(br0 + row) * ld + k);
    rs[u] = *reinterpret_cast<const f32x4*>(S + k);
  }
}

// x = hi + lo for two values at once: hi = bf16(x) and lo = bf16(x - hi), both
// rounded to nearest even by the packed conversion; returns the packed pairs
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned& hi, unsigned& lo) {
  f32x2 x;
  x.x = x0;
  x.y = x1;
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf2));
  f32x2 h;
  h.x = __uint_as_float(hi << 16);
  h.y = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(x - h, bf2));
}

__device__ __forceinline__ void bf_lstore(uint16_t* Ah, uint16_t* Al, uint16_t* Bh,
                                          uint16_t* Bl, int t, const u32x4 (&rah)[2],
                                          const u32x4 (&ral)[2], const f32x4 (&rb)[4],
                                          const f32x4 (&rs)[4]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int row, ch;
    a_item(t + 256 * u, row, ch);
    *reinterpret_cast<u32x4*>(&Ah[lds_slot(row, ch)]) = rah[u];
    *reinterpret_cast<u32x4*>(&Al[lds_slot(row, ch)]) = ral[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int row, ch, half;
    b_item(t + 256 * u, row, ch, half);
    unsigned h01, l01, h23, l23;
    const f32x4 v = rb[u] * rs[u];
    split_pair(v.x, v.y, h01, l01);
    split_pair(v.z, v.w, h23, l23);
    u32x2 hv, lv;
    hv.x = h01;
    hv.y = h23;
    lv.x = l01;
    lv.y = l23;
    *reinterpret_cast<u32x2*>(&Bh[lds_slot(row, ch) + 4 * half]) = hv;
    *reinterpret_cast<u32x2*>(&Bl[lds_slot(row, ch) + 4 * half]) = lv;
  }
}

// One K-step of the 64 x 64 wave tile: 4 x 4 blocks, three bf16 MFMAs each
// (lo x hi, hi x lo, hi x hi; the lo x lo term is below the split's error).
// Operand fragments: lane l reads MFMA row l % 16 (physical row
// mfma_row(l % 16) of the block), k = 8 (l / 16) .. +7.  The A fragments are
// read first, then the B fragments one block column at a time with its 12
// MFMAs, so that only 8 B-fragment registers are live at once.
__device__ __forceinline__ void bf_mfma_step(const uint16_t* Ah, const uint16_t* Al,
                                                  const uint16_t* Bh, const uint16_t* Bl,
                                                  int lane, int wm, int wn, f4 (&acc)[4][4]) {
  const int ko = 8 * ((lane >> 4) * 128 + ((lane & 15) ^ (lane >> 4)));
  s8 ah[4], al[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = ko + (wm * 4 + i) * 128;
    ah[i] = *reinterpret_cast<const s8*>(&Ah[o]);
    al[i] = *reinterpret_cast<const s8*>(&Al[o]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = ko + (wn * 4 + j) * 128;
    const s8 bh = *reinterpret_cast<const s8*>(&Bh[o]);
    const s8 bl = *reinterpret_cast<const s8*>(&Bl[o]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          __builtin_bit_cast(bf8, al[i]), __builtin_bit_cast(bf8, bh), acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          __builtin_bit_cast(bf8, ah[i]), __builtin_bit_cast(bf8, bl), acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          __builtin_bit_cast(bf8, ah[i]), __builtin_bit_cast(bf8, bh), acc[i][j], 0, 0, 0);
    }
  }
}

// 128 x 128 tile per workgroup (2 x 2 waves of 64 x 64), FP32 accumulation
// over the whole K.  One LDS slab set (32 KB): a K-step issues its MFMAs from
// LDS, then loads the next slabs into registers, waits at a barrier until
// every wave has read its fragments, stores the slabs and waits again.  No
// staging register is live across the MFMAs, so the kernel takes 144 VGPRs
// and three workgroups share a CU, covering each other's load latency and
// barriers (5.36 ms at (H2O)10, against 5.8 ms for a double-buffered form
// that loads a K-step ahead at 197 VGPRs and two workgroups per CU).
__global__ __launch_bounds__(256) void k_pi_bf16x3(const uint16_t* Bhi, const uint16_t* Blo,
                                                   long ld, const float* B32,
                                                   const float* scale, long sS, double* A,
                                                   long ldA, long sA, int T, int Kp, int G,
                                                   OperandTabs tb) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Al[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[1][SLAB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int total = T * (T + 1) / 2 * G;
  const int id = xcd_swizzle_m(blockIdx.x, total);
  const int g = id % G;
  int I, J;
  lower_tile(id / G, I, J);
  const float* S = scale + (long)g * sS;
  const int ar0 = I * 128, br0 = J * 128;
  if (tb.Bhi) {
    Bhi = tb.Bhi[g / tb.grp];
    Blo = tb.Blo[g / tb.grp];
    B32 = tb.B32[g / tb.grp];
  }

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // A side: 128 rows x 32 k bf16 = 512 chunks of 8 (16 B) per array -> 2 per thread
  // B side: 128 rows x 32 k fp32 = 1024 float4 -> 4 per thread
  u32x4 rah[2], ral[2];
  f32x4 rb[4], rs[4];
  const int nk = Kp / BKB;
  bf_gload(Bhi, Blo, B32, S, ld, ar0, br0, 0, t, rah, ral, rb, rs);
  bf_lstore(Ah[0], Al[0], Bh[0], Bl[0], t, rah, ral, rb, rs);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    bf_mfma_step(Ah[0], Al[0], Bh[0], Bl[0], lane, wm, wn, acc);
    // loads after the MFMAs (the scheduling barrier keeps them there, out of
    // the fragment registers' live range); the last K-step reloads its own
    // slab, so that loads and stores stay unconditional
    __builtin_amdgcn_sched_barrier(0);
    const int knext = (kt + 1 < nk ? kt + 1 : kt) * BKB;
    bf_gload(Bhi, Blo, B32, S, ld, ar0, br0, knext, t, rah, ral, rb, rs);
    __syncthreads();   // every wave has read its fragments of this K-step
    bf_lstore(Ah[0], Al[0], Bh[0], Bl[0], t, rah, ral, rb, rs);
    __syncthreads();   // the next K-step's slabs are in place
  }
  double* Ag = A + (long)g * sA;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // accumulator element (4 (l / 16) + r, l % 16) of the MFMA block
        const int row = ar0 + wm * 64 + i * 16 + mfma_row(4 * (lane >> 4) + r);
        const int col = br0 + wn * 64 + j * 16 + mfma_row(lane & 15);
        Ag[(long)row * ldA + col] = (row == col ? 1.0 : 0.0) + 4.0 * (double)acc[i][j][r];
      }
}

// Tile set of the wide Pi build, in 128-row blocks (nb = Np / 128).  A
// workgroup computes the four blocks (r[0..1], c[0..1]) and stores those whose
// bit 2 rh + ch of mask is set.  Even nb: the lower 256 x 256 tiles (I, J),
// J <= I (rows 2I, 2I + 1 against columns 2J, 2J + 1), the block above the
// diagonal of a diagonal tile not stored.  Odd nb, where the last block row
// L = nb - 1 would pad its tiles to 256 rows: first the strictly lower tiles of
// the nb - 1 paired blocks; then, for each pair T, rows {2T + 1, L} against
// columns {2T, 2T + 1} (the lower half of the diagonal tile plus two blocks
// of row L); then the diagonal blocks left over, (2T, 2T) and (L, L), two per
// workgroup (rows {d1, d2} against columns {d1, d2}, the two diagonal blocks
// stored).  Each block of the lower triangle is stored by exactly one
// workgroup; at nb = 27 ((H2O)30) that is 98 workgroups per grid point
// against 105 tiles of 256.
struct WideTile {
  int r[2], c[2];
  unsigned mask;
};

__host__ __device__ inline int wide_tile_count(int nb) {
  const int P = nb / 2;
  if (nb % 2 == 0) return P * (P + 1) / 2;
  return P * (P - 1) / 2 + P + (P + 2) / 2;
}

__device__ inline WideTile wide_tile(int p, int nb) {
  WideTile w;
  const int P = nb / 2, L = nb - 1;
  int I, J;
  if (nb % 2 == 0) {
    lower_tile(p, I, J);
    w.r[0] = 2 * I; w.r[1] = 2 * I + 1;
    w.c[0] = 2 * J; w.c[1] = 2 * J + 1;
    w.mask = I == J ? 0xDu : 0xFu;   // (2I, 2I + 1) lies above the diagonal
    return w;
  }
  const int n_off = P * (P - 1) / 2;
  if (p < n_off) {
    lower_tile(p, I, J);
    ++I;                             // strictly lower: J < I
    w.r[0] = 2 * I; w.r[1] = 2 * I + 1;
    w.c[0] = 2 * J; w.c[1] = 2 * J + 1;
    w.mask = 0xFu;
  } else if (p < n_off + P) {
    const int T = p - n_off;
    w.r[0] = 2 * T + 1; w.r[1] = L;
    w.c[0] = 2 * T; w.c[1] = 2 * T + 1;
    w.mask = 0xFu;
  } else {
    const int q = p - n_off - P;     // diagonal blocks 2q and 2q + 1 of (0, 2, .., 2P - 2, L)
    const int d1 = 2 * q < P ? 4 * q : L;
    const bool two = 2 * q + 1 <= P;
    const int d2 = !two ? d1 : (2 * q + 1 < P ? 4 * q + 2 : L);
    w.r[0] = d1; w.r[1] = d2;
    w.c[0] = d1; w.c[1] = d2;
    w.mask = two ? 0x9u : 0x1u;      // (d1, d1) and (d2, d2)
  }
  return w;
}

// Wide form for large N_aux: 256 x 256 tiles per 512-thread workgroup (eight
// wavefronts, each 128 x 64: 8 x 4 blocks of three bf16 MFMAs, the B
// fragments of its four block columns held while the A block rows stream
// through) with a double-buffered LDS (128 KB) and one barrier per K-step:
// after the barrier the staged slabs of step k+1 are split and stored into the
// other buffer and the loads of step k+2 are issued, in one basic block with
// the MFMAs of step k so that the scheduler interleaves them.  Per flop it stages half of the global bytes and 7/8 of the LDS bytes
// of a 256 x 128 tile, and half of the scaled side's split work of the
// 128 x 128 form.  At up to 256 VGPRs one workgroup (two wavefronts per SIMD)
// holds a CU.  The workgroup's two 128-row halves on each side are the
// blocks of its WideTile (above); a wavefront (128 x 64, within one block
// pair) whose block is not in the tile's store mask still computes (which
// keeps the K-step one basic block) but stores nothing.  Same K order and
// products as the 128 x 128 form, so the results are identical bit for bit.
__global__ __launch_bounds__(512) void k_pi_bf16x3_wide(const uint16_t* Bhi, const uint16_t* Blo,
                                                        long ld, const float* B32,
                                                        const float* scale, long sS, double* A,
                                                        long ldA, long sA, int Np, int Kp,
                                                        int G, OperandTabs tb) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[2][2][SLAB];   // [buffer][128-row half]
  __shared__ __attribute__((aligned(16))) uint16_t Al[2][2][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[2][2][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[2][2][SLAB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int nb = Np / 128;
  const int id = xcd_swizzle_m(blockIdx.x, wide_tile_count(nb) * G);
  const int g = id % G;
  const WideTile wt = wide_tile(id / G, nb);
  const float* S = scale + (long)g * sS;
  if (tb.Bhi) {
    Bhi = tb.Bhi[g / tb.grp];
    Blo = tb.Blo[g / tb.grp];
    B32 = tb.B32[g / tb.grp];
  }
  // first global row of each 128-row half (every block lies below Np)
  const long arow[2] = {128L * wt.r[0], 128L * wt.r[1]};
  const long brow[2] = {128L * wt.c[0], 128L * wt.c[1]};
  const int wr0 = 128 * wt.r[wm], wc0 = 128 * wt.c[wn >> 1] + 64 * (wn & 1);
  const bool live = (wt.mask >> (2 * wm + (wn >> 1))) & 1u;
  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // staging, per thread: pre-split side 256 rows x 4 chunks per array = 2
  // items; scaled side 256 rows x 8 float4 = 4 items
  u32x4 rah[2], ral[2];
  f32x4 rb[4], rs[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 512 * u, row, ch);   // row >> 7 == u
      const long gr = arow[u] + (row & 127);
      rah[u] = *reinterpret_cast<const u32x4*>(Bhi + gr * ld + k0 + 8 * ch);
      ral[u] = *reinterpret_cast<const u32x4*>(Blo + gr * ld + k0 + 8 * ch);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int row, ch, half;
      b_item(t + 512 * u, row, ch, half);   // row >> 7 == u >> 1
      const int k = k0 + 8 * ch + 4 * half;
      const long gr = brow[u >> 1] + (row & 127);
      rb[u] = *reinterpret_cast<const f32x4*>(B32 + gr * ld + k);
      rs[u] = *reinterpret_cast<const f32x4*>(S + k);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 512 * u, row, ch);
      const int sl = lds_slot(row & 127, ch);
      *reinterpret_cast<u32x4*>(&Ah[buf][row >> 7][sl]) = rah[u];
      *reinterpret_cast<u32x4*>(&Al[buf][row >> 7][sl]) = ral[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int row, ch, half;
      b_item(t + 512 * u, row, ch, half);
      unsigned h01, l01, h23, l23;
      const f32x4 v = rb[u] * rs[u];
      split_pair(v.x, v.y, h01, l01);
      split_pair(v.z, v.w, h23, l23);
      u32x2 hv, lv;
      hv.x = h01;
      hv.y = h23;
      lv.x = l01;
      lv.y = l23;
      const int sl = lds_slot(row & 127, ch) + 4 * half;
      *reinterpret_cast<u32x2*>(&Bh[buf][row >> 7][sl]) = hv;
      *reinterpret_cast<u32x2*>(&Bl[buf][row >> 7][sl]) = lv;
    }
  };
  const int nk = Kp / BKB;
  gload(0);
  lstore(0);
  gload(nk > 1 ? BKB : 0);
  const int ko = 8 * ((lane >> 4) * 128 + ((lane & 15) ^ (lane >> 4)));
  const int bhalf = wn >> 1, bq = (wn & 1) * 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    __syncthreads();   // step kt's slabs are in place; nobody reads buffer cur ^ 1 any more
    // one basic block per K-step (no branches), so that the scheduler weaves
    // the next step's split, stores and loads into this step's MFMA stream:
    // the B fragments of this step, the slabs of step kt + 1 into the other
    // buffer (the last step's store goes to a buffer nobody reads again), the
    // loads of step kt + 2, then the MFMAs (wavefronts with no live block
    // compute too and store nothing)
    s8 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = ko + (bq + j) * 128;
      bh[j] = *reinterpret_cast<const s8*>(&Bh[cur][bhalf][o]);
      bl[j] = *reinterpret_cast<const s8*>(&Bl[cur][bhalf][o]);
    }
    lstore(cur ^ 1);
    gload((kt + 2 < nk ? kt + 2 : nk - 1) * BKB);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int o = ko + i * 128;
      const s8 ah = *reinterpret_cast<const s8*>(&Ah[cur][wm][o]);
      const s8 al = *reinterpret_cast<const s8*>(&Al[cur][wm][o]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, al), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bl[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
      }
    }
  }
  if (!live) return;
  double* Ag = A + (long)g * sA;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr0 + i * 16 + mfma_row(4 * (lane >> 4) + r);
        const int col = wc0 + j * 16 + mfma_row(lane & 15);
        Ag[(long)row * ldA + col] = (row == col ? 1.0 : 0.0) + 4.0 * (double)acc[i][j][r];
      }
}

// N_aux (padded) from which the wide form is used: measured faster from the
// (H2O)20 shape up; at (H2O)10 the two forms tie (15 wide tile pairs per grid
// point leave the last round of workgroups short of the CUs)
constexpr int WIDE_FROM = 2048;

static hipError_t launch_pi_bf16x3(const uint16_t* Bhi, const uint16_t* Blo, const float* B32,
                                   const OperandTabs& tb, long ld, const float* scale, long sS,
                                   double* A, long ldA, long sA, int Np, int Kp, int G, long nB,
                                   long nS, long nA, hipStream_t st) {
  const int T = Np / 128;
  const long total = (long)T * (T + 1) / 2 * G;
  if (total <= 0) return hipSuccess;
  if (tb.Bhi && (tb.grp <= 0 || G % tb.grp != 0 || !tb.Blo || !tb.B32))
    return refuse("pi_bf16x3", "operand table group");
  if (hipError_t e = check_pi("pi_bf16x3", ld, sS, ldA, sA, Np, Kp, G, BKB, nB, nS, nA)) return e;
  if (Np >= WIDE_FROM) {
    const long wtotal = (long)wide_tile_count(T) * G;
    if (wtotal > 0x7fffffffL) return refuse("pi_bf16x3", "grid too large");
    GW_AUDIT_RETURN();
    hipLaunchKernelGGL(k_pi_bf16x3_wide, dim3((unsigned)wtotal), dim3(512), 0, st, Bhi, Blo, ld,
                       B32, scale, sS, A, ldA, sA, Np, Kp, G, tb);
    return hipGetLastError();
  }
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_pi_bf16x3, dim3((unsigned)total), dim3(256), 0, st, Bhi, Blo, ld, B32, scale,
                     sS, A, ldA, sA, T, Kp, G, tb);
  return hipGetLastError();
}

hipError_t pi_build_bf16x3(const uint16_t* Bhi, const uint16_t* Blo, long ld, const float* B32,
                           const float* scale, long sS, double* A, long ldA, long sA, int Np,
                           int Kp, int G, long nB, long nS, long nA, hipStream_t st) {
  return launch_pi_bf16x3(Bhi, Blo, B32, OperandTabs{}, ld, scale, sS, A, ldA, sA, Np, Kp, G, nB,
                          nS, nA, st);
}

// nB: the smallest extent over the table's B copies
hipError_t pi_build_bf16x3_tab(const OperandTabs& tb, long ld, const float* scale, long sS,
                               double* A, long ldA, long sA, int Np, int Kp, int G, long nB,
                               long nS, long nA, hipStream_t st) {
  if (!tb.Bhi) return refuse("pi_bf16x3", "missing operand table");
  return launch_pi_bf16x3(nullptr, nullptr, nullptr, tb, ld, scale, sS, A, ldA, sA, Np, Kp, G, nB,
                          nS, nA, st);
}

// ---------------------------------------------------------------------------
// Mixed W^c contraction.
//
// k_split_linv: F = L^-1 - I of each grid point, from X = L^-T held k-major
// (X[k][p] = (L^-1)[p][k]; row k of the work buffer's appended block), written
// row-major [p][k] (k contiguous, zero for k > p) as a bf16 hi/lo pair, 64 x 64
// tiles transposed through LDS.

__global__ __launch_bounds__(256) void k_split_linv(const double* X, long ldX, long sX, int Np,
                                                    uint16_t* Fh, uint16_t* Fl, long sF) {
  __shared__ float T[64][65];
  const int nt = Np / 64;
  const int kt = blockIdx.x / nt, pt = blockIdx.x % nt;
  const int g = blockIdx.y;
  const int t = threadIdx.x;
  const double* Xg = X + (long)g * sX;
  if (kt <= pt) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = (t >> 4) + 16 * u, pp = (t & 15) * 4;
      const int k = kt * 64 + kk;
      const double* src = Xg + (long)k * ldX + pt * 64 + pp;
      const d2 v0 = *reinterpret_cast<const d2*>(src);
      const d2 v1 = *reinterpret_cast<const d2*>(src + 2);
      const double v[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = pt * 64 + pp + e;
        T[kk][pp + e] = k > p ? 0.f : (float)(k == p ? v[e] - 1.0 : v[e]);
      }
    }
  }
  __syncthreads();
  // thread -> row p = pt*64 + t/4, 16 k values from kt*64 + 16 (t%4)
  const int pr = t >> 2, kq = (t & 3) * 16;
  unsigned h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x0 = kt <= pt ? T[kq + 2 * e][pr] : 0.f;
    const float x1 = kt <= pt ? T[kq + 2 * e + 1][pr] : 0.f;
    split_pair(x0, x1, h[e], l[e]);
  }
  const long o = (long)g * sF + (long)(pt * 64 + pr) * Np + kt * 64 + kq;
  u32x4* dh = reinterpret_cast<u32x4*>(Fh + o);
  u32x4* dl = reinterpret_cast<u32x4*>(Fl + o);
  dh[0] = u32x4{h[0], h[1], h[2], h[3]};
  dh[1] = u32x4{h[4], h[5], h[6], h[7]};
  dl[0] = u32x4{l[0], l[1], l[2], l[3]};
  dl[1] = u32x4{l[4], l[5], l[6], l[7]};
}

hipError_t split_linv(const double* X, long ldX, long sX, int Np, int G, uint16_t* Fh,
                      uint16_t* Fl, long sF, long nX, long nF, hipStream_t st) {
  const char* kn = "split_linv";
  if (G <= 0) return hipSuccess;
  if (Np % 128 != 0 || ldX < Np || (ldX & 1) || (sX & 1) || sF < (long)Np * Np || sF % 8 != 0)
    return refuse(kn, "shape");
  GW_GUARD(kn, "X", (long)(G - 1) * sX + (long)(Np - 1) * ldX + Np - 1, nX);
  GW_GUARD(kn, "F", (long)(G - 1) * sF + (long)Np * Np - 1, nF);
  GW_AUDIT_RETURN();
  const int nt = Np / 64;
  hipLaunchKernelGGL(k_split_linv, dim3(nt * nt, G), dim3(256), 0, st, X, ldX, sX, Np, Fh, Fl, sF);
  return hipGetLastError();
}

// k_wc_bf16x3: for every grid point g, row q of R (b = (P|nm) of one
// (state, m) pair) and 128-wide column panel J of the auxiliary index,
//   part[g][J][q] = sum_{p in J} (2 b_p + y_p) y_p,   y = F_g b,
// with the BF16x3 products and LDS layout of the Pi build.  F_g[p][k] is zero
// for k > p, so panel J contracts k < 128 (J + 1) only.  b_p at the output
// positions is re-read from the split R (hi + lo): the same values the last
// K-steps of the tile have just staged, so the reads hit the cache.
//
// Tile order: blocks of 8 grid points (each XCD receives a contiguous range of
// the order, i.e. about one such block), then the panel J, then groups of 16
// row tiles, and inside a group of 16 x 8 tiles the grid point fastest.  The
// 128 workgroups an XCD holds at a time (four per CU) then read 16 R panels
// and 8 F panels, shared by 8 and 16 of them through that XCD's L2, instead
// of one F panel and 128 distinct R panels (which stream the whole of R from
// outside L2 for every grid point and panel).
//
// The K-loop is the Pi build's (one LDS slab set, 34 KB with the reduction
// buffer; loads after the MFMAs; two barriers per K-step).  At 126 VGPRs four
// workgroups share a CU: 1.25 ms at (H2O)10, against 1.46 ms for the
// double-buffered form with loads a K-step ahead (two workgroups per CU).
__global__ __launch_bounds__(256, 4) void k_wc_bf16x3(const uint16_t* Rh, const uint16_t* Rl,
                                                   long ldR, const uint16_t* Fh,
                                                   const uint16_t* Fl, long sF, int Np,
                                                   double* part, long ldp, long sP, int TM,
                                                   int TN, int G, OperandTabs tb, long nRR) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Al[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[1][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[1][SLAB];
  __shared__ double red[2][128];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int total = TM * TN * G;
  const int id = xcd_swizzle_m(blockIdx.x, total);
  // every block of 8 grid points but the last is full, and likewise every
  // group of 16 row tiles of a panel, so block offsets are plain products
  const int gb = id / (8 * TN * TM);
  const int gs = min(8, G - 8 * gb);
  const int rem = id - gb * 8 * TN * TM;
  const int J = rem / (gs * TM);
  const int rem2 = rem % (gs * TM);
  const int r16 = rem2 % (16 * gs);
  const int I = 16 * (rem2 / (16 * gs)) + r16 / gs;
  const int g = 8 * gb + r16 % gs;
  if (tb.Rh) {
    Rh = tb.Rh[g / tb.grp];
    Rl = Rh + nRR;
  }
  const uint16_t* Fhg = Fh + (long)g * sF;
  const uint16_t* Flg = Fl + (long)g * sF;
  const int ar0 = I * 128, br0 = J * 128;
  const int nk = (br0 + 128) / BKB;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // both sides pre-split: 128 rows x 32 k bf16 = 512 chunks of 16 B per array,
  // 2 per thread
  u32x4 rah[2], ral[2], rbh[2], rbl[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 256 * u, row, ch);
      const long oa = (long)(ar0 + row) * ldR + k0 + 8 * ch;
      const long ob = (long)(br0 + row) * Np + k0 + 8 * ch;
      rah[u] = *reinterpret_cast<const u32x4*>(Rh + oa);
      ral[u] = *reinterpret_cast<const u32x4*>(Rl + oa);
      rbh[u] = *reinterpret_cast<const u32x4*>(Fhg + ob);
      rbl[u] = *reinterpret_cast<const u32x4*>(Flg + ob);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 256 * u, row, ch);
      const int s = lds_slot(row, ch);
      *reinterpret_cast<u32x4*>(&Ah[buf][s]) = rah[u];
      *reinterpret_cast<u32x4*>(&Al[buf][s]) = ral[u];
      *reinterpret_cast<u32x4*>(&Bh[buf][s]) = rbh[u];
      *reinterpret_cast<u32x4*>(&Bl[buf][s]) = rbl[u];
    }
  };
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    bf_mfma_step(Ah[0], Al[0], Bh[0], Bl[0], lane, wm, wn, acc);
    __builtin_amdgcn_sched_barrier(0);
    gload((kt + 1 < nk ? kt + 1 : kt) * BKB);   // unconditional, as in the Pi build
    __syncthreads();   // every wave has read its fragments of this K-step
    lstore(0);
    __syncthreads();   // the next K-step's slabs are in place
  }
  // accumulator element (4 (l / 16) + r, l % 16) of block (i, j): R row
  // ar0 + wm 64 + 16 i + mfma_row(4 (l / 16) + r), column br0 + wn 64 + 16 j +
  // mfma_row(l % 16); the 16 lanes of one l / 16 group share the row
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lrow = wm * 64 + i * 16 + mfma_row(4 * (lane >> 4) + r);
      const long ro = (long)(ar0 + lrow) * ldR;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = br0 + wn * 64 + j * 16 + mfma_row(lane & 15);
        const double b = (double)bf16_to_f(Rh[ro + col]) + (double)bf16_to_f(Rl[ro + col]);
        const double y = (double)acc[i][j][r];
        s += (2.0 * b + y) * y;
      }
      for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
      if ((lane & 15) == 0) red[wn][lrow] = s;
    }
  __syncthreads();
  if (t < 128) part[(long)g * sP + (long)J * ldp + ar0 + t] = red[0][t] + red[1][t];
}

// Wide form for large N_aux: 256 x 256 tiles (256 rows of R, a 256-wide panel
// J of F) on 512-thread workgroups, eight wavefronts of 128 x 64, with the
// double-buffered LDS and single-block K-step of the wide Pi build (both
// operands arrive pre-split, so the stores are plain copies).  Panel J covers
// p in [256 J - o, 256 J - o + 256) with o = 128 when N_aux / 128 is odd (else
// 0), so that the panels end at N_aux: the half panel an odd count leaves
// falls at p < 0, where K is 128 long, instead of past N_aux, where K is
// N_aux long.  K runs over k < min(256 J - o + 256, N_aux) (F is zero for
// k > p, so each y_p has its full sum).  part[g][J][q] holds the panel sums
// (J < ceil(N_aux / 256)).  Order: blocks of 8 grid points, then the panel,
// then groups of 4 row tiles, grid point fastest, so the 32 workgroups an
// XCD holds share 4 R tiles and 8 F panels through its L2.  Rows past the
// padded R and columns outside [0, N_aux) are clamped on load and neither
// stored nor summed.
__global__ __launch_bounds__(512) void k_wc_bf16x3_wide(const uint16_t* Rh, const uint16_t* Rl,
                                                        long ldR, const uint16_t* Fh,
                                                        const uint16_t* Fl, long sF, int Np,
                                                        int Rp, double* part, long ldp, long sP,
                                                        int TM, int TN, int G, OperandTabs tb,
                                                        long nRR) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[2][2][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Al[2][2][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[2][2][SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[2][2][SLAB];
  __shared__ double red[4][256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int id = xcd_swizzle_m(blockIdx.x, TM * TN * G);
  const int gb = id / (8 * TN * TM);
  const int gs = min(8, G - 8 * gb);
  const int rem = id - gb * 8 * TN * TM;
  const int J = rem / (gs * TM);
  const int rem2 = rem % (gs * TM);
  const int r4 = rem2 % (4 * gs);
  const int I = 4 * (rem2 / (4 * gs)) + r4 / gs;
  const int g = 8 * gb + r4 % gs;
  if (tb.Rh) {
    Rh = tb.Rh[g / tb.grp];
    Rl = Rh + nRR;
  }
  const uint16_t* Fhg = Fh + (long)g * sF;
  const uint16_t* Flg = Fl + (long)g * sF;
  const int ar0 = I * 256, br0 = J * 256 - ((Np >> 7) & 1) * 128;
  const int nk = min(br0 + 256, Np) / BKB;
  const bool live = br0 + wn * 64 >= 0 && br0 + wn * 64 < Np && ar0 + wm * 128 < Rp;
  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // 256 rows x 4 chunks per array and operand: 2 items per thread
  u32x4 rah[2], ral[2], rbh[2], rbl[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 512 * u, row, ch);
      const long oa = (long)min(ar0 + row, Rp - 1) * ldR + k0 + 8 * ch;
      const long ob = (long)min(max(br0 + row, 0), Np - 1) * Np + k0 + 8 * ch;
      rah[u] = *reinterpret_cast<const u32x4*>(Rh + oa);
      ral[u] = *reinterpret_cast<const u32x4*>(Rl + oa);
      rbh[u] = *reinterpret_cast<const u32x4*>(Fhg + ob);
      rbl[u] = *reinterpret_cast<const u32x4*>(Flg + ob);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int row, ch;
      a_item(t + 512 * u, row, ch);
      const int sl = lds_slot(row & 127, ch);
      *reinterpret_cast<u32x4*>(&Ah[buf][row >> 7][sl]) = rah[u];
      *reinterpret_cast<u32x4*>(&Al[buf][row >> 7][sl]) = ral[u];
      *reinterpret_cast<u32x4*>(&Bh[buf][row >> 7][sl]) = rbh[u];
      *reinterpret_cast<u32x4*>(&Bl[buf][row >> 7][sl]) = rbl[u];
    }
  };
  gload(0);
  lstore(0);
  gload(nk > 1 ? BKB : 0);
  const int ko = 8 * ((lane >> 4) * 128 + ((lane & 15) ^ (lane >> 4)));
  const int bhalf = wn >> 1, bq = (wn & 1) * 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    __syncthreads();   // step kt's slabs are in place; nobody reads buffer cur ^ 1 any more
    s8 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = ko + (bq + j) * 128;
      bh[j] = *reinterpret_cast<const s8*>(&Bh[cur][bhalf][o]);
      bl[j] = *reinterpret_cast<const s8*>(&Bl[cur][bhalf][o]);
    }
    lstore(cur ^ 1);   // the last step's store goes to a buffer nobody reads again
    gload((kt + 2 < nk ? kt + 2 : nk - 1) * BKB);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int o = ko + i * 128;
      const s8 ah = *reinterpret_cast<const s8*>(&Ah[cur][wm][o]);
      const s8 al = *reinterpret_cast<const s8*>(&Al[cur][wm][o]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, al), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bl[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
      }
    }
  }
  // per row, the sum over this wavefront's 64 columns (p < N_aux) of
  // (2 b_p + y_p) y_p, then over the four wavefronts of the row half
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lrow = wm * 128 + i * 16 + mfma_row(4 * (lane >> 4) + r);
      const long ro = (long)min(ar0 + lrow, Rp - 1) * ldR;
      double sum = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = br0 + wn * 64 + j * 16 + mfma_row(lane & 15);
        if (live && col < Np) {   // live: the wavefront's 64 columns lie in [0, Np)
          const double b = (double)bf16_to_f(Rh[ro + col]) + (double)bf16_to_f(Rl[ro + col]);
          const double y = (double)acc[i][j][r];
          sum += (2.0 * b + y) * y;
        }
      }
      for (int off = 8; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 16);
      if ((lane & 15) == 0) red[wn][lrow] = sum;
    }
  __syncthreads();
  if (t < 256 && ar0 + t < Rp)
    part[(long)g * sP + (long)J * ldp + ar0 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// Panels of the W^c partial sums the contraction writes per grid point
// (128 wide, or 256 wide for the wide form); the reduction sums this many.
int wc_bf16x3_panels(int Np) { return Np >= WIDE_FROM ? (Np + 255) / 256 : Np / 128; }

static hipError_t launch_wc_bf16x3(const uint16_t* Rh, const uint16_t* Rl, const OperandTabs& tb,
                                   long nRR, long ldR, int Rp, const uint16_t* Fh,
                                   const uint16_t* Fl, long sF, int Np, int G, double* part,
                                   long ldp, long sP, long nR, long nF, long nP, hipStream_t st) {
  const char* kn = "wc_bf16x3";
  const long total = (long)(Rp / 128) * (Np / 128) * G;
  if (G <= 0 || Rp <= 0) return hipSuccess;
  if (Rp % 128 != 0 || Np % 128 != 0 || ldR < Np || ldR % 8 != 0 || sF < (long)Np * Np ||
      sF % 8 != 0 || ldp < Rp || total > 0x7fffffffL)
    return refuse(kn, "shape");
  if (tb.Rh && (tb.grp <= 0 || G % tb.grp != 0 || nRR % 8 != 0 || nRR < (long)(Rp - 1) * ldR + Np))
    return refuse(kn, "operand table group");
  if (((uintptr_t)Rh | (uintptr_t)Rl | (uintptr_t)Fh | (uintptr_t)Fl) & 15)
    return refuse(kn, "operand pointer not 16-byte aligned");
  GW_GUARD(kn, "R", (long)(Rp - 1) * ldR + Np - 1, nR);
  GW_GUARD(kn, "F", (long)(G - 1) * sF + (long)(Np - 1) * Np + Np - 1, nF);
  GW_GUARD(kn, "part", (long)(G - 1) * sP + (long)(Np / 128 - 1) * ldp + Rp - 1, nP);
  GW_AUDIT_RETURN();
  if (Np >= WIDE_FROM) {
    const int TM = (Rp + 255) / 256, TN = (Np + 255) / 256;
    const long wtotal = (long)TM * TN * G;
    if (wtotal > 0x7fffffffL) return refuse(kn, "grid too large");
    hipLaunchKernelGGL(k_wc_bf16x3_wide, dim3((unsigned)wtotal), dim3(512), 0, st, Rh, Rl, ldR, Fh,
                       Fl, sF, Np, Rp, part, ldp, sP, TM, TN, G, tb, nRR);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_wc_bf16x3, dim3((unsigned)total), dim3(256), 0, st, Rh, Rl, ldR, Fh, Fl, sF,
                     Np, part, ldp, sP, Rp / 128, Np / 128, G, tb, nRR);
  return hipGetLastError();
}

hipError_t wc_bf16x3(const uint16_t* Rh, const uint16_t* Rl, long ldR, int Rp, const uint16_t* Fh,
                     const uint16_t* Fl, long sF, int Np, int G, double* part, long ldp, long sP,
                     long nR, long nF, long nP, hipStream_t st) {
  return launch_wc_bf16x3(Rh, Rl, OperandTabs{}, 0, ldR, Rp, Fh, Fl, sF, Np, G, part, ldp, sP, nR,
                          nF, nP, st);
}

// each table entry Rh holds the hi half and, nRR elements further, the lo half;
// nR: the smallest extent of either half over the table
hipError_t wc_bf16x3_tab(const OperandTabs& tb, long nRR, long ldR, int Rp, const uint16_t* Fh,
                         const uint16_t* Fl, long sF, int Np, int G, double* part, long ldp,
                         long sP, long nR, long nF, long nP, hipStream_t st) {
  if (!tb.Rh) return refuse("wc_bf16x3", "missing operand table");
  return launch_wc_bf16x3(nullptr, nullptr, tb, nRR, ldR, Rp, Fh, Fl, sF, Np, G, part, ldp, sP, nR,
                          nF, nP, st);
}

}  // namespace gw
