// Lower-precision dense gradient paths for the precision study: the product
// D~_X T D~_Y on FP32 or BF16 matrix cores with FP32 accumulation, and split
// refinement.  The distance operand is generated from indices as in the FP64
// path (csrc/dense.hip).
//
//   F32:        operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32
//               accumulation over the whole K; A = T D~_Y kept in FP32.
//   BF16:       operands rounded to BF16, v_mfma_f32_16x16x32_bf16, FP32
//               accumulation over the whole K; A rounded to BF16 as the
//               second product's operand.
//   *_SPLIT:    each operand x = x_hi + x_lo (x_hi = round(x), x_lo =
//               round(x - x_hi)); the products hi*hi and hi*lo + lo*hi are
//               accumulated in FP32 over chunks of k (4 for FP32: one
//               instruction; 256 for BF16) and the chunk sums are added in
//               FP64; A kept in FP64.
// A-priori bound for FP32 accumulation over K terms of non-negative products:
// |dB| <= gamma_K |D~| |T| |D~| with gamma_K = K u / (1 - K u).
//
// The BF16 paths run as two matrix-core GEMMs on BF16 copies made once per
// call (T, D~_Y and D~_X rounded, split into hi/lo for *_SPLIT), padded with
// zeros to whole tiles so the K loop needs no bounds:
//   A^T = D~_Y T^T   (A operand D~_Y, B operand T: both have K contiguous)
//   B   = D~_X A     (A operand D~_X, B operand A^T), epilogue writes G.
// Block tiles double-buffered through LDS (256 x 256 with 8 waves of
// 64 x 128; the split path 128 x 128 with waves of 32 x 64, as its three
// products per pair and the FP64 chunk sums need the registers).
#include "common.h"
#include "runtime.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum { LP_F32 = 0, LP_BF16 = 1, LP_F32_SPLIT = 2, LP_BF16_SPLIT = 3 };

constexpr int BM = 64, BN = 64, BK = 32, KC = 256;

template <int MODE>
struct LpTraits;
template <>
struct LpTraits<LP_F32> {
  static constexpr bool split = false, bf16 = false;
};
template <>
struct LpTraits<LP_BF16> {
  static constexpr bool split = false, bf16 = true;
};
template <>
struct LpTraits<LP_F32_SPLIT> {
  static constexpr bool split = true, bf16 = false;
};
template <>
struct LpTraits<LP_BF16_SPLIT> {
  static constexpr bool split = true, bf16 = true;
};

GW_DEV float hi_f32(double x) { return (float)x; }
GW_DEV float lo_f32(double x) { return (float)(x - (double)(float)x); }
GW_DEV __bf16 hi_bf16(double x) { return (__bf16)(float)x; }
GW_DEV __bf16 lo_bf16(double x) { return (__bf16)(float)(x - (double)(float)(__bf16)(float)x); }

GW_DEV double dist_pow(int a, int b, int kd) {
  const int d = a > b ? a - b : b - a;
  return gwk::ipow((double)d, kd);
}

// C[M x N] = A[M x K] * B[K x N]; exactly one of A, B is the distance matrix
// |i-j|^kd.  SYN_B: A from memory (MemT, lda), B = D.  !SYN_B: A = D, B from
// memory.  If G != null the epilogue writes G = (c1 + c2) - s2 * C (FP64), else
// C is written to Cf (FP32) or Cd (FP64, split modes).
template <int MODE, bool SYN_B, typename MemT>
__global__ __launch_bounds__(256) void k_dense_lp(const MemT* __restrict__ Xmem, int64_t ldx,
                                                   int M, int N, int K, int kd,
                                                   float* __restrict__ Cf,
                                                   double* __restrict__ Cd, int64_t ldc,
                                                   const double* __restrict__ c1,
                                                   const double* __restrict__ c2, double s2,
                                                   double* __restrict__ G, int64_t ldG) {
  using Tr = LpTraits<MODE>;
  __shared__ MemT Xs[SYN_B ? BM : BK][SYN_B ? BK + 1 : BN + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int li = lane & 15, lq = lane >> 4;
  f4 acc[2][2], accx[2][2];
  double dacc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      accx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          dacc[i][j][v] += (double)acc[i][j][v] + (double)accx[i][j][v];
        acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        accx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    if (SYN_B) {
      // 64 rows x 32 k: thread t loads row t/4, k (t%4)*8 .. +8
      const int r = t >> 2, kk = (t & 3) * 8;
      const int gm = m0 + r;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gk = k0 + kk + u;
        Xs[r][kk + u] = (gm < M && gk < K) ? Xmem[(int64_t)gm * ldx + gk] : (MemT)0;
      }
    } else {
      // 32 k x 64 cols: thread t loads row t/8, cols (t%8)*8 .. +8
      const int r = t >> 3, cc = (t & 7) * 8;
      const int gk = k0 + r;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gn = n0 + cc + u;
        Xs[r][cc + u] = (gk < K && gn < N) ? Xmem[(int64_t)gk * ldx + gn] : (MemT)0;
      }
    }
    __syncthreads();
    if (!Tr::bf16) {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        const int kg = k0 + ks + lq;
        float ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int row = wm + i * 16 + li;
          const double a = SYN_B ? (double)Xs[row][ks + lq] : dist_pow(m0 + row, kg, kd);
          ah[i] = hi_f32(a);
          al[i] = lo_f32(a);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn + j * 16 + li;
          const double b = SYN_B ? dist_pow(n0 + col, kg, kd) : (double)Xs[ks + lq][col];
          bh[j] = hi_f32(b);
          bl[j] = lo_f32(b);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[i], bh[j], acc[i][j], 0, 0, 0);
            if (Tr::split) {
              accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[i], bl[j], accx[i][j], 0, 0, 0);
              accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[i], bh[j], accx[i][j], 0, 0, 0);
            }
          }
        if (Tr::split) flush();  // FP32 chunk of one instruction (4 k)
      }
    } else {
      // one 16x16x32 step: lane holds k = 8 * (lane / 16) + e, e < 8
      bf8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + i * 16 + li;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int kl = 8 * lq + e;
          const double a = SYN_B ? (double)Xs[row][kl] : dist_pow(m0 + row, k0 + kl, kd);
          ah[i][e] = hi_bf16(a);
          al[i][e] = lo_bf16(a);
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wn + j * 16 + li;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int kl = 8 * lq + e;
          const double b = SYN_B ? dist_pow(n0 + col, k0 + kl, kd) : (double)Xs[kl][col];
          bh[j][e] = hi_bf16(b);
          bl[j][e] = lo_bf16(b);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          if (Tr::split) {
            accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], accx[i][j], 0, 0, 0);
            accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], accx[i][j], 0, 0, 0);
          }
        }
    }
    if (Tr::split && Tr::bf16 && ((k0 + BK) % KC == 0)) flush();
  }
  if (Tr::split) flush();
  // FP32 16x16 accumulator layout: slot v of a lane holds row 4 * (lane / 16) + v
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + i * 16 + 4 * lq + v;
        const int gn = n0 + wn + j * 16 + li;
        if (gm < M && gn < N) {
          const double x = Tr::split ? dacc[i][j][v] : (double)acc[i][j][v];
          if (G) {
            G[(int64_t)gm * ldG + gn] = (c1[gm] + c2[gn]) - s2 * x;
          } else if (Tr::split) {
            Cd[(int64_t)gm * ldc + gn] = x;
          } else {
            Cf[(int64_t)gm * ldc + gn] = (float)x;
          }
        }
      }
}

// ---------------------------------------------------------------- BF16 GEMMs
__host__ __device__ inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
constexpr int GB_K = 64, GB_PAD = 8;  // K per stage, LDS row padding (bf16 elements)

// BF16 copies (hi, and lo if lo != null) of a row-major FP64 matrix
// src[rows x cols] into dst[rp x kp] (ld kp), zero outside the matrix.
__global__ __launch_bounds__(256) void k_to_bf16(const double* __restrict__ src, int64_t lds,
                                                  int rows, int cols, __bf16* __restrict__ hi,
                                                  __bf16* __restrict__ lo, int64_t rp, int64_t kp) {
  const int64_t c8 = (int64_t)blockIdx.x * 256 + threadIdx.x;  // 8-element chunk
  const int64_t nchunks = rp * (kp / 8);
  if (c8 >= nchunks) return;
  const int64_t r = c8 / (kp / 8), c0 = (c8 - r * (kp / 8)) * 8;
  bf8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const double x = (r < rows && c0 + e < cols) ? src[r * lds + c0 + e] : 0.0;
    h[e] = hi_bf16(x);
    l[e] = lo_bf16(x);
  }
  *reinterpret_cast<bf8*>(hi + r * kp + c0) = h;
  if (lo) *reinterpret_cast<bf8*>(lo + r * kp + c0) = l;
}

// BF16 copies of the integer distance matrix |i - j|^k (n x n) into
// dst[rp x kp], zero outside it.
__global__ __launch_bounds__(256) void k_dist_bf16(int n, int kd, __bf16* __restrict__ hi,
                                                    __bf16* __restrict__ lo, int64_t rp,
                                                    int64_t kp) {
  const int64_t c8 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nchunks = rp * (kp / 8);
  if (c8 >= nchunks) return;
  const int64_t r = c8 / (kp / 8), c0 = (c8 - r * (kp / 8)) * 8;
  bf8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t c = c0 + e;
    const double x = (r < n && c < n) ? dist_pow((int)r, (int)c, kd) : 0.0;
    h[e] = hi_bf16(x);
    l[e] = lo_bf16(x);
  }
  *reinterpret_cast<bf8*>(hi + r * kp + c0) = h;
  if (lo) *reinterpret_cast<bf8*>(lo + r * kp + c0) = l;
}

// C = A Bt^T over k in [0, kp): A [>= grid rows][lda], Bt [>= grid cols][ldb],
// BF16, row-major with K contiguous; kp a multiple of GB_K, lda and ldb of 8,
// rows of A and Bt allocated (and zero) up to whole block tiles.
//   OUT 0: C[m][n] to BF16 hi (and lo) at O[m * ldo + n] for m < Mo, n < No
//          (the padded range: zero rows and columns give zeros);
//   OUT 1: G[m][n] = (c1[m] + c2[n]) - s2 C for m < M, n < N (FP64).
// Plain: 128 x 128 block tiles, 2 x 2 waves of 64 x 64 (4 x 4 MFMA tiles of
// 16 x 16); split: 64 x 64 block tiles, waves of 32 x 32, products hi*hi and
// hi*lo + lo*hi in FP32 over KC = 256 k, chunk sums in FP64.
// Tile shapes: the plain path runs 256 x 256 block tiles with 8 waves of
// 64 x 128 (fewer LDS reads per matrix-core operation); the split path 128 x 128
// block tiles with 8 waves of 32 x 64.
template <bool SPLIT>
struct GemmShape;
template <>
struct GemmShape<false> {
  static constexpr int BM = 256, BN = 256, WGM = 4, WGN = 2, NTH = 512;
};
template <>
struct GemmShape<true> {
  static constexpr int BM = 128, BN = 128, WGM = 4, WGN = 2, NTH = 512;
};

template <bool SPLIT, int OUT>
__global__ __launch_bounds__(GemmShape<SPLIT>::NTH) void k_gemm_bt(
    const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al, int64_t lda,
    const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int64_t ldb, int kp, int Mo,
    int No, __bf16* __restrict__ Oh, __bf16* __restrict__ Ol, int64_t ldo,
    const double* __restrict__ c1, const double* __restrict__ c2, double s2,
    double* __restrict__ G, int64_t ldG) {
  using S = GemmShape<SPLIT>;
  constexpr int BM = S::BM, BN = S::BN, NTH = S::NTH;
  constexpr int WM = BM / S::WGM, WN = BN / S::WGN;  // wave tile
  constexpr int NTM = WM / 16, NTN = WN / 16;         // MFMA tiles per wave
  constexpr int NMAT = SPLIT ? 2 : 1;                 // hi (and lo) of each operand
  constexpr int LDK = GB_K + GB_PAD;
  constexpr int CHA = BM * GB_K / 8 / NTH, CHB = BN * GB_K / 8 / NTH;  // 16-byte chunks per thread
  __shared__ __bf16 As[2][NMAT][BM][LDK];
  __shared__ __bf16 Bs[2][NMAT][BN][LDK];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave / S::WGN) * WM, wn = (wave % S::WGN) * WN;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int li = lane & 15, lq = lane >> 4;
  f4 acc[NTM][NTN], accx[SPLIT ? NTM : 1][SPLIT ? NTN : 1];
  double dacc[SPLIT ? NTM : 1][SPLIT ? NTN : 1][4];
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int j = 0; j < NTN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (SPLIT) {
#pragma unroll
    for (int i = 0; i < NTM; ++i)
#pragma unroll
      for (int j = 0; j < NTN; ++j) {
        accx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
      }
  }
  // global -> registers -> LDS, 16-byte chunks: chunk c = t + NTH u of a tile
  // is row c / 8, k (c % 8) * 8
  bf8 ra[NMAT][CHA], rb[NMAT][CHB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < CHA; ++u) {
      const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 8;
      ra[0][u] = *reinterpret_cast<const bf8*>(Ah + (m0 + r) * lda + k0 + kc);
      if constexpr (SPLIT) ra[1][u] = *reinterpret_cast<const bf8*>(Al + (m0 + r) * lda + k0 + kc);
    }
#pragma unroll
    for (int u = 0; u < CHB; ++u) {
      const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 8;
      rb[0][u] = *reinterpret_cast<const bf8*>(Bh + (n0 + r) * ldb + k0 + kc);
      if constexpr (SPLIT) rb[1][u] = *reinterpret_cast<const bf8*>(Bl + (n0 + r) * ldb + k0 + kc);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int mt = 0; mt < NMAT; ++mt) {
#pragma unroll
      for (int u = 0; u < CHA; ++u) {
        const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 8;
        *reinterpret_cast<bf8*>(&As[buf][mt][r][kc]) = ra[mt][u];
      }
#pragma unroll
      for (int u = 0; u < CHB; ++u) {
        const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 8;
        *reinterpret_cast<bf8*>(&Bs[buf][mt][r][kc]) = rb[mt][u];
      }
    }
  };
  auto flush = [&]() {
    if constexpr (SPLIT) {
#pragma unroll
      for (int i = 0; i < NTM; ++i)
#pragma unroll
        for (int j = 0; j < NTN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            dacc[i][j][v] += (double)acc[i][j][v] + (double)accx[i][j][v];
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          accx[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < GB_K; ks += 32) {
      bf8 fa[NMAT][NTM], fb[NMAT][NTN];
#pragma unroll
      for (int mt = 0; mt < NMAT; ++mt) {
#pragma unroll
        for (int i = 0; i < NTM; ++i)
          fa[mt][i] = *reinterpret_cast<const bf8*>(&As[buf][mt][wm + 16 * i + li][ks + 8 * lq]);
#pragma unroll
        for (int j = 0; j < NTN; ++j)
          fb[mt][j] = *reinterpret_cast<const bf8*>(&Bs[buf][mt][wn + 16 * j + li][ks + 8 * lq]);
      }
#pragma unroll
      for (int i = 0; i < NTM; ++i)
#pragma unroll
        for (int j = 0; j < NTN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[0][j], acc[i][j], 0, 0, 0);
          if constexpr (SPLIT) {
            accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[1][j], accx[i][j], 0, 0, 0);
            accx[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[0][j], accx[i][j], 0, 0, 0);
          }
        }
    }
  };
  const int nk = kp / GB_K;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) gload((kt + 1) * GB_K);
    compute(kt & 1);
    if (SPLIT && ((kt + 1) * GB_K) % KC == 0) flush();
    if (kt + 1 < nk) lstore((kt + 1) & 1);
    __syncthreads();
  }
  flush();
  // FP32 16x16 accumulator layout: slot v of a lane holds row 4 * (lane / 16) + v;
  // with G, the constant terms of the lane's rows and columns are all
  // requested before the stores
  double c1v[OUT ? NTM : 1][4], c2v[OUT ? NTN : 1];
  if constexpr (OUT != 0) {
#pragma unroll
    for (int i = 0; i < NTM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        c1v[i][v] = c1[min(m0 + wm + i * 16 + 4 * lq + v, (int64_t)Mo - 1)];
#pragma unroll
    for (int j = 0; j < NTN; ++j) c2v[j] = c2[min(n0 + wn + j * 16 + li, (int64_t)No - 1)];
  }
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int j = 0; j < NTN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm + i * 16 + 4 * lq + v;
        const int64_t gn = n0 + wn + j * 16 + li;
        double x;
        if constexpr (SPLIT) x = dacc[i][j][v];
        else x = (double)acc[i][j][v];
        if constexpr (OUT == 0) {
          if (gm < Mo && gn < No) {
            Oh[gm * ldo + gn] = hi_bf16(x);
            if constexpr (SPLIT) Ol[gm * ldo + gn] = lo_bf16(x);
          }
        } else {
          if (gm < Mo && gn < No) G[gm * ldG + gn] = (c1v[i][v] + c2v[j]) - s2 * x;
        }
      }
}

// FP32 operands on the FP32 matrix cores: the same two products as the BF16
// path on 128 x 128 block tiles of 8 waves (v_mfma_f32_16x16x4f32: a lane
// holds one operand element, row lane % 16, k = lane / 16), FP32 accumulation
// over the whole K; A^T stays FP32.  OUT as in k_gemm_bt (0: FP32 output, 1: G).
template <int OUT>
__global__ __launch_bounds__(512) void k_gemm_bt_f32(const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ Bt, int64_t ldb,
                                                      int kp, int Mo, int No,
                                                      float* __restrict__ O, int64_t ldo,
                                                      const double* __restrict__ c1,
                                                      const double* __restrict__ c2, double s2,
                                                      double* __restrict__ G, int64_t ldG) {
  // 4 x 2 waves of 32 x 64 (64 accumulator registers: 4 waves per SIMD)
  constexpr int BM = 128, NTH = 512, WTM = 32, WTN = 64, NTI = WTM / 16, NTJ = WTN / 16;
  constexpr int BK = 32, LDK = BK + 4;                        // K per stage; LDS row padding
  constexpr int CH = BM * BK / 4 / NTH;                        // 16-byte chunks per thread
  typedef float fl4 __attribute__((ext_vector_type(4)));
  __shared__ float As[2][BM][LDK];
  __shared__ float Bs[2][BM][LDK];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * WTM, wn = (wave & 1) * WTN;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BM;
  const int li = lane & 15, lq = lane >> 4;
  f4 acc[NTI][NTJ];
#pragma unroll
  for (int i = 0; i < NTI; ++i)
#pragma unroll
    for (int j = 0; j < NTJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  fl4 ra[CH], rb[CH];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 4;
      ra[u] = *reinterpret_cast<const fl4*>(A + (m0 + r) * lda + k0 + kc);
      rb[u] = *reinterpret_cast<const fl4*>(Bt + (n0 + r) * ldb + k0 + kc);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int c = t + NTH * u, r = c >> 3, kc = (c & 7) * 4;
      *reinterpret_cast<fl4*>(&As[buf][r][kc]) = ra[u];
      *reinterpret_cast<fl4*>(&Bs[buf][r][kc]) = rb[u];
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float fa[NTI], fb[NTJ];
#pragma unroll
      for (int i = 0; i < NTI; ++i) fa[i] = As[buf][wm + 16 * i + li][ks + lq];
#pragma unroll
      for (int j = 0; j < NTJ; ++j) fb[j] = Bs[buf][wn + 16 * j + li][ks + lq];
#pragma unroll
      for (int i = 0; i < NTI; ++i)
#pragma unroll
        for (int j = 0; j < NTJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  };
  const int nk = kp / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) gload((kt + 1) * BK);
    compute(kt & 1);
    if (kt + 1 < nk) lstore((kt + 1) & 1);
    __syncthreads();
  }
  // with G, the constant terms of the lane's rows and columns are all
  // requested before the stores
  double c1v[OUT ? NTI : 1][4], c2v[OUT ? NTJ : 1];
  if constexpr (OUT != 0) {
#pragma unroll
    for (int i = 0; i < NTI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        c1v[i][v] = c1[min(m0 + wm + i * 16 + 4 * lq + v, (int64_t)Mo - 1)];
#pragma unroll
    for (int j = 0; j < NTJ; ++j) c2v[j] = c2[min(n0 + wn + j * 16 + li, (int64_t)No - 1)];
  }
#pragma unroll
  for (int i = 0; i < NTI; ++i)
#pragma unroll
    for (int j = 0; j < NTJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm + i * 16 + 4 * lq + v;
        const int64_t gn = n0 + wn + j * 16 + li;
        if (gm < Mo && gn < No) {
          if constexpr (OUT == 0) O[gm * ldo + gn] = acc[i][j][v];
          else G[gm * ldG + gn] = (c1v[i][v] + c2v[j]) - s2 * (double)acc[i][j][v];
        }
      }
}

// FP32 copies of a row-major FP64 matrix, or of |i - j|^k (src null: n x n),
// into dst[rp x kp], zero outside.
__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ src, int64_t lds,
                                                 int rows, int cols, int kd,
                                                 float* __restrict__ dst, int64_t rp, int64_t kp) {
  const int64_t c4 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c4 >= rp * (kp / 4)) return;
  const int64_t r = c4 / (kp / 4), c0 = (c4 - r * (kp / 4)) * 4;
  typedef float fl4 __attribute__((ext_vector_type(4)));
  fl4 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t c = c0 + e;
    double x = 0.0;
    if (r < rows && c < cols) x = src ? src[r * lds + c] : dist_pow((int)r, (int)c, kd);
    v[e] = (float)x;
  }
  *reinterpret_cast<fl4*>(dst + r * kp + c0) = v;
}

gw_status run_f32(int M, int N, int kx, int ky, const double* T, int64_t ldT, double* G,
                  int64_t ldG, const double* c1, const double* c2, double s2, float* w,
                  hipStream_t s) {
  const int64_t Mp = round_up(M, 128), Np = round_up(N, 128);
  const int64_t kN = round_up(N, 32), kM = round_up(M, 32);
  float* tf = w;              // T       [Mp][kN]
  float* dy = tf + Mp * kN;   // D~_Y    [Np][kN]
  float* dx = dy + Np * kN;   // D~_X    [Mp][kM]
  float* at = dx + Mp * kM;   // A^T     [Np][Mp]
  auto blocks = [](int64_t elems) { return (unsigned)((elems / 4 + 255) / 256); };
  k_to_f32<<<blocks(Mp * kN), 256, 0, s>>>(T, ldT, M, N, 0, tf, Mp, kN);
  k_to_f32<<<blocks(Np * kN), 256, 0, s>>>(nullptr, 0, N, N, ky, dy, Np, kN);
  k_to_f32<<<blocks(Mp * kM), 256, 0, s>>>(nullptr, 0, M, M, kx, dx, Mp, kM);
  k_gemm_bt_f32<0><<<dim3((unsigned)(Mp / 128), (unsigned)(Np / 128)), 512, 0, s>>>(
      dy, kN, tf, kN, (int)kN, (int)Np, (int)Mp, at, Mp, nullptr, nullptr, 0.0, nullptr, 0);
  k_gemm_bt_f32<1><<<dim3((unsigned)(Np / 128), (unsigned)(Mp / 128)), 512, 0, s>>>(
      dx, kM, at, Mp, (int)kM, M, N, nullptr, 0, c1, c2, s2, G, ldG);
  return gwr::last_launch_status();
}

size_t f32_ws_floats(int64_t M, int64_t N) {
  const int64_t Mp = round_up(M, 128), Np = round_up(N, 128);
  const int64_t kN = round_up(N, 32), kM = round_up(M, 32);
  return (size_t)(Mp * kN + Np * kN + Mp * kM + Np * Mp);
}

struct Bf16Layout {
  int64_t Mp, Np, kN, kM;  // padded rows (block tiles) and K extents
  size_t t, dy, dx, at;    // elements of each BF16 copy
};

Bf16Layout bf16_layout(int64_t M, int64_t N, bool split) {
  const int64_t BMx = split ? GemmShape<true>::BM : GemmShape<false>::BM;
  Bf16Layout L;
  L.Mp = round_up(M, BMx);
  L.Np = round_up(N, BMx);
  L.kN = round_up(N, GB_K);
  L.kM = round_up(M, GB_K);
  L.t = (size_t)L.Mp * L.kN;   // T        [Mp][kN]
  L.dy = (size_t)L.Np * L.kN;  // D~_Y     [Np][kN]
  L.dx = (size_t)L.Mp * L.kM;  // D~_X     [Mp][kM]
  L.at = (size_t)L.Np * L.Mp;  // A^T      [Np][Mp]
  return L;
}

template <bool SPLIT>
gw_status run_bf16(int M, int N, int kx, int ky, const double* T, int64_t ldT, double* G,
                   int64_t ldG, const double* c1, const double* c2, double s2, __bf16* w,
                   hipStream_t s) {
  const Bf16Layout L = bf16_layout(M, N, SPLIT);
  const int nm = SPLIT ? 2 : 1;
  __bf16* th = w;
  __bf16* tl = SPLIT ? th + L.t : nullptr;
  __bf16* dyh = w + nm * L.t;
  __bf16* dyl = SPLIT ? dyh + L.dy : nullptr;
  __bf16* dxh = dyh + nm * L.dy;
  __bf16* dxl = SPLIT ? dxh + L.dx : nullptr;
  __bf16* ath = dxh + nm * L.dx;
  __bf16* atl = SPLIT ? ath + L.at : nullptr;
  auto blocks = [](size_t elems) { return (unsigned)((elems / 8 + 255) / 256); };
  k_to_bf16<<<blocks(L.t), 256, 0, s>>>(T, ldT, M, N, th, tl, L.Mp, L.kN);
  k_dist_bf16<<<blocks(L.dy), 256, 0, s>>>(N, ky, dyh, dyl, L.Np, L.kN);
  k_dist_bf16<<<blocks(L.dx), 256, 0, s>>>(M, kx, dxh, dxl, L.Mp, L.kM);
  using S = GemmShape<SPLIT>;
  // A^T = D~_Y T^T: rows n < Np, columns m < Mp (the padding comes out zero)
  k_gemm_bt<SPLIT, 0><<<dim3((unsigned)(L.Mp / S::BN), (unsigned)(L.Np / S::BM)), S::NTH, 0, s>>>(
      dyh, dyl, L.kN, th, tl, L.kN, (int)L.kN, (int)L.Np, (int)L.Mp, ath, atl, L.Mp, nullptr,
      nullptr, 0.0, nullptr, 0);
  // B = D~_X A, G = c1 + c2 - s2 B
  k_gemm_bt<SPLIT, 1><<<dim3((unsigned)(L.Np / S::BN), (unsigned)(L.Mp / S::BM)), S::NTH, 0, s>>>(
      dxh, dxl, L.kM, ath, atl, L.Mp, (int)L.kM, M, N, nullptr, nullptr, 0, c1, c2, s2, G, ldG);
  return gwr::last_launch_status();
}

template <int MODE>
gw_status run_lp(int M, int N, int kx, int ky, const double* T, int64_t ldT, double* G,
                 int64_t ldG, const double* c1, const double* c2, double s2, void* Abuf,
                 hipStream_t s) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
  if (LpTraits<MODE>::split) {
    double* A = static_cast<double*>(Abuf);
    k_dense_lp<MODE, true, double><<<grid, 256, 0, s>>>(T, ldT, M, N, N, ky, nullptr, A, N,
                                                        nullptr, nullptr, 0.0, nullptr, 0);
    k_dense_lp<MODE, false, double><<<grid, 256, 0, s>>>(A, N, M, N, M, kx, nullptr, nullptr, 0,
                                                         c1, c2, s2, G, ldG);
  } else {
    float* A = static_cast<float*>(Abuf);
    k_dense_lp<MODE, true, double><<<grid, 256, 0, s>>>(T, ldT, M, N, N, ky, A, nullptr, N,
                                                        nullptr, nullptr, 0.0, nullptr, 0);
    k_dense_lp<MODE, false, float><<<grid, 256, 0, s>>>(A, N, M, N, M, kx, nullptr, nullptr, 0,
                                                        c1, c2, s2, G, ldG);
  }
  return gwr::last_launch_status();
}

bool split_path(int path) {
  return path == GW_PATH_DENSE_F32_SPLIT || path == GW_PATH_DENSE_BF16_SPLIT;
}

}  // namespace

namespace gwl {

size_t dense_lp_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y, int path) {
  gwr::Arena a{nullptr, 0, 0};
  if (path == GW_PATH_DENSE_BF16 || path == GW_PATH_DENSE_BF16_SPLIT) {
    const bool split = path == GW_PATH_DENSE_BF16_SPLIT;
    const Bf16Layout L = bf16_layout(X.n(), Y.n(), split);
    a.take<__bf16>((split ? 2 : 1) * (L.t + L.dy + L.dx + L.at));
  } else if (split_path(path)) {
    a.take<double>((size_t)X.n() * Y.n());
  } else {
    a.take<float>(f32_ws_floats(X.n(), Y.n()));
  }
  return a.used;
}

gw_status dense_lp(const gwr::Grid& X, const gwr::Grid& Y, const double* T, int64_t ldT,
                   double* G, int64_t ldG, int path, gwr::Arena& ws, hipStream_t s,
                   const double* c1, const double* c2) {
  const int M = (int)X.n(), N = (int)Y.n();
  const double s2 = 2.0 * (X.hk() * Y.hk());
  gwr::ProfScope ps(gwr::kFamDense, s);
  if (path == GW_PATH_DENSE_BF16 || path == GW_PATH_DENSE_BF16_SPLIT) {
    const bool split = path == GW_PATH_DENSE_BF16_SPLIT;
    const Bf16Layout L = bf16_layout(M, N, split);
    __bf16* w = ws.take<__bf16>((split ? 2 : 1) * (L.t + L.dy + L.dx + L.at));
    return split ? run_bf16<true>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, w, s)
                 : run_bf16<false>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, w, s);
  }
  if (path == GW_PATH_DENSE_F32) {
    float* w = ws.take<float>(f32_ws_floats(M, N));
    return run_f32(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, w, s);
  }
  void* A = (void*)ws.take<double>((size_t)M * N);
  switch (path) {
    case GW_PATH_DENSE_F32_SPLIT:
      return run_lp<LP_F32_SPLIT>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, A, s);
  }
  return GW_EUNSUPPORTED;
}

}  // namespace gwl
