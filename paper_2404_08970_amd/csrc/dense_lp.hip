// Lower-precision dense gradient paths for the precision study: the product
// D~_X T D~_Y on FP32 or BF16 matrix cores with FP32 accumulation, and split
// refinement.  The distance operand is generated from indices as in the FP64
// path (csrc/dense.hip).
//
//   F32:        operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32
//               accumulation over the whole K; A = T D~_Y kept in FP32.
//   BF16:       operands rounded to BF16, v_mfma_f32_16x16x32_bf16, FP32
//               accumulation over the whole K; A kept in FP32.
//   *_SPLIT:    each operand x = x_hi + x_lo (x_hi = round(x), x_lo =
//               round(x - x_hi)); the products hi*hi and hi*lo + lo*hi are
//               accumulated in FP32 over chunks of k (4 for FP32: one
//               instruction; 256 for BF16) and the chunk sums are added in
//               FP64; A kept in FP64.
// A-priori bound for FP32 accumulation over K terms of non-negative products:
// |dB| <= gamma_K |D~| |T| |D~| with gamma_K = K u / (1 - K u).
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
  if (split_path(path))
    a.take<double>((size_t)X.n() * Y.n());
  else
    a.take<float>((size_t)X.n() * Y.n());
  return a.used;
}

gw_status dense_lp(const gwr::Grid& X, const gwr::Grid& Y, const double* T, int64_t ldT,
                   double* G, int64_t ldG, int path, gwr::Arena& ws, hipStream_t s,
                   const double* c1, const double* c2) {
  const int M = (int)X.n(), N = (int)Y.n();
  const double s2 = 2.0 * (X.hk() * Y.hk());
  void* A = split_path(path) ? (void*)ws.take<double>((size_t)M * N)
                             : (void*)ws.take<float>((size_t)M * N);
  gwr::ProfScope ps(gwr::kFamDense, s);
  switch (path) {
    case GW_PATH_DENSE_F32:
      return run_lp<LP_F32>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, A, s);
    case GW_PATH_DENSE_BF16:
      return run_lp<LP_BF16>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, A, s);
    case GW_PATH_DENSE_F32_SPLIT:
      return run_lp<LP_F32_SPLIT>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, A, s);
    case GW_PATH_DENSE_BF16_SPLIT:
      return run_lp<LP_BF16_SPLIT>(M, N, X.k1d(), Y.k1d(), T, ldT, G, ldG, c1, c2, s2, A, s);
  }
  return GW_EUNSUPPORTED;
}

}  // namespace gwl
