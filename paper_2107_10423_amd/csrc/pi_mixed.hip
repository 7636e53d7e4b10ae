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
//            whole K (the FP64 flush variant costs the occupancy of a second
//            workgroup per CU; the accuracy difference is reported by the
//            precision tests).  The unscaled side B is split once per molecule
//            and stored; the scaled side B s_g is split on the fly per grid point
//            while it is staged into LDS.
//
// Tiles are 128 x 128 per 256-thread workgroup (2 x 2 wavefronts of 64 x 64),
// lower-triangular tile map, grid point index fastest and XCD-swizzled as in
// the FP64 kernel.
#include "gw_internal.h"

namespace gw {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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
    b32[i] = x;
  }
}

hipError_t split_bf16(const double* B, uint16_t* hi, uint16_t* lo, float* b32, long n,
                      hipStream_t st) {
  GW_AUDIT_RETURN();  // all four arrays are allocated with n elements by the caller
  int blocks = (int)std::min<long>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_split_bf16, dim3(blocks), dim3(256), 0, st, B, hi, lo, b32, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 operands, f32 MFMA.  LDS holds [k][row] floats.

__global__ __launch_bounds__(256) void k_pi_f32(const float* B, long ld, const double* scale,
                                                long sS, double* A, long ldA, long sA, int T,
                                                int Kp, int G) {
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
  const double* S = scale + (long)g * sS;
  const int ar0 = I * 128, br0 = J * 128;

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
      double2 s01 = *reinterpret_cast<const double2*>(S + k0 + kq);
      double2 s23 = *reinterpret_cast<const double2*>(S + k0 + kq + 2);
      v.x *= (float)s01.x;
      v.y *= (float)s01.y;
      v.z *= (float)s23.x;
      v.w *= (float)s23.y;
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

hipError_t pi_build_f32(const float* B32, long ld, const double* scale, long sS, double* A,
                        long ldA, long sA, int Np, int Kp, int G, long nB, long nS, long nA,
                        hipStream_t st) {
  const int T = Np / 128;
  const long total = (long)T * (T + 1) / 2 * G;
  if (total <= 0) return hipSuccess;
  if (hipError_t e = check_pi("pi_f32", ld, sS, ldA, sA, Np, Kp, G, 16, nB, nS, nA)) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_pi_f32, dim3((unsigned)total), dim3(256), 0, st, B32, ld, scale, sS, A, ldA,
                     sA, T, Kp, G);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16x3.  LDS holds [row][k] bf16 (k contiguous, 32 per K-step) with a pad,
// so an MFMA operand (8 consecutive k of one row) is one 16-byte read.

constexpr int BKB = 32;
constexpr int LROW = BKB + 8;  // padded row length in bf16 elements

// Staging of one 32-wide K-step: the unscaled side is loaded pre-split
// (bf16 hi and lo, 2 x 16 B per thread each); the scaled side is loaded as
// FP32 (4 x 16 B per thread), multiplied by the grid point's scale and split
// into hi/lo while it is written to LDS.
__device__ __forceinline__ void bf_gload(const uint16_t* Bhi, const uint16_t* Blo,
                                         const float* B32, const double* S, long ld, int ar0,
                                         int br0, int k0, int t, u32x4 (&rah)[2],
                                         u32x4 (&ral)[2], f32x4 (&rb)[4]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int q = t + 256 * u;
    int row = q >> 2, kq = (q & 3) * 8;
    rah[u] = *reinterpret_cast<const u32x4*>(Bhi + (long)(ar0 + row) * ld + k0 + kq);
    ral[u] = *reinterpret_cast<const u32x4*>(Blo + (long)(ar0 + row) * ld + k0 + kq);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int q = t + 256 * u;
    int row = q >> 3, kq = (q & 7) * 4;
    f32x4 v = *reinterpret_cast<const f32x4*>(B32 + (long)(br0 + row) * ld + k0 + kq);
    double2 s01 = *reinterpret_cast<const double2*>(S + k0 + kq);
    double2 s23 = *reinterpret_cast<const double2*>(S + k0 + kq + 2);
    v.x *= (float)s01.x;
    v.y *= (float)s01.y;
    v.z *= (float)s23.x;
    v.w *= (float)s23.y;
    rb[u] = v;
  }
}

__device__ __forceinline__ void bf_lstore(uint16_t* Ah, uint16_t* Al, uint16_t* Bh,
                                          uint16_t* Bl, int t, const u32x4 (&rah)[2],
                                          const u32x4 (&ral)[2], const f32x4 (&rb)[4]) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int q = t + 256 * u;
    int row = q >> 2, kq = (q & 3) * 8;
    *reinterpret_cast<u32x4*>(&Ah[row * LROW + kq]) = rah[u];
    *reinterpret_cast<u32x4*>(&Al[row * LROW + kq]) = ral[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int q = t + 256 * u;
    int row = q >> 3, kq = (q & 7) * 4;
    const float x0 = rb[u].x, x1 = rb[u].y, x2 = rb[u].z, x3 = rb[u].w;
    const unsigned short h0 = bf16_rne(x0), h1 = bf16_rne(x1), h2 = bf16_rne(x2),
                         h3 = bf16_rne(x3);
    const unsigned short l0 = bf16_rne(x0 - bf16_to_f(h0)), l1 = bf16_rne(x1 - bf16_to_f(h1)),
                         l2 = bf16_rne(x2 - bf16_to_f(h2)), l3 = bf16_rne(x3 - bf16_to_f(h3));
    u32x2 hv, lv;
    hv.x = (unsigned)h0 | ((unsigned)h1 << 16);
    hv.y = (unsigned)h2 | ((unsigned)h3 << 16);
    lv.x = (unsigned)l0 | ((unsigned)l1 << 16);
    lv.y = (unsigned)l2 | ((unsigned)l3 << 16);
    *reinterpret_cast<u32x2*>(&Bh[row * LROW + kq]) = hv;
    *reinterpret_cast<u32x2*>(&Bl[row * LROW + kq]) = lv;
  }
}

template <bool FLUSH64>
__global__ __launch_bounds__(256) void k_pi_bf16x3(const uint16_t* Bhi, const uint16_t* Blo,
                                                   long ld, const float* B32,
                                                   const double* scale, long sS, double* A,
                                                   long ldA, long sA, int T, int Kp, int G) {
  __shared__ __attribute__((aligned(16))) uint16_t Ah[2][128 * LROW];
  __shared__ __attribute__((aligned(16))) uint16_t Al[2][128 * LROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[2][128 * LROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[2][128 * LROW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int total = T * (T + 1) / 2 * G;
  const int id = xcd_swizzle_m(blockIdx.x, total);
  const int g = id % G;
  int I, J;
  lower_tile(id / G, I, J);
  const double* S = scale + (long)g * sS;
  const int ar0 = I * 128, br0 = J * 128;

  f4 acc[4][4];
  d4 acc64[FLUSH64 ? 4 : 1][FLUSH64 ? 4 : 1];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < (FLUSH64 ? 4 : 1); ++i)
#pragma unroll
    for (int j = 0; j < (FLUSH64 ? 4 : 1); ++j) acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // A side: 128 rows x 32 k bf16 = 512 chunks of 8 (16 B) per array -> 2 per thread
  // B side: 128 rows x 32 k fp32 = 1024 float4 -> 4 per thread
  u32x4 rah[2], ral[2];
  f32x4 rb[4];
  const int nk = Kp / BKB;
  bf_gload(Bhi, Blo, B32, S, ld, ar0, br0, 0, t, rah, ral, rb);
  bf_lstore(Ah[0], Al[0], Bh[0], Bl[0], t, rah, ral, rb);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) bf_gload(Bhi, Blo, B32, S, ld, ar0, br0, (kt + 1) * BKB, t, rah, ral, rb);
    // operand fragments: lane l reads row l % 16, k = 8 (l / 16) .. +7
    const int ko = 8 * (lane >> 4);
    s8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * 64 + i * 16 + (lane & 15);
      ah[i] = *reinterpret_cast<const s8*>(&Ah[cur][row * LROW + ko]);
      al[i] = *reinterpret_cast<const s8*>(&Al[cur][row * LROW + ko]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = wn * 64 + j * 16 + (lane & 15);
      bh[j] = *reinterpret_cast<const s8*>(&Bh[cur][row * LROW + ko]);
      bl[j] = *reinterpret_cast<const s8*>(&Bl[cur][row * LROW + ko]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, al[i]), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah[i]), __builtin_bit_cast(bf8, bl[j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, ah[i]), __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
      }
    if (FLUSH64 && (((kt + 1) * BKB) % FLUSH_K == 0 || kt + 1 == nk)) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[FLUSH64 ? i : 0][FLUSH64 ? j : 0][r] += (double)acc[i][j][r];
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (kt + 1 < nk) bf_lstore(Ah[cur ^ 1], Al[cur ^ 1], Bh[cur ^ 1], Bl[cur ^ 1], t, rah, ral, rb);
    __syncthreads();
  }
  double* Ag = A + (long)g * sA;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = ar0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        int col = br0 + wn * 64 + j * 16 + (lane & 15);
        const double v = FLUSH64 ? acc64[FLUSH64 ? i : 0][FLUSH64 ? j : 0][r] : (double)acc[i][j][r];
        Ag[(long)row * ldA + col] = (row == col ? 1.0 : 0.0) + 4.0 * v;
      }
}

hipError_t pi_build_bf16x3(const uint16_t* Bhi, const uint16_t* Blo, long ld, const float* B32,
                           const double* scale, long sS, double* A, long ldA, long sA, int Np,
                           int Kp, int G, long nB, long nS, long nA, hipStream_t st) {
  const int T = Np / 128;
  const long total = (long)T * (T + 1) / 2 * G;
  if (total <= 0) return hipSuccess;
  if (hipError_t e = check_pi("pi_bf16x3", ld, sS, ldA, sA, Np, Kp, G, BKB, nB, nS, nA)) return e;
  GW_AUDIT_RETURN();
  hipLaunchKernelGGL(k_pi_bf16x3<false>, dim3((unsigned)total), dim3(256), 0, st, Bhi, Blo, ld, B32, scale,
                     sS, A, ldA, sA, T, Kp, G);
  return hipGetLastError();
}

}  // namespace gw
