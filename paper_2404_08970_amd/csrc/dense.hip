// Dense ("original", O(N^3)) gradient on matrix cores: G = c1 1^T + 1 c2^T -
// 2 h_X^k h_Y^k D~_X T D~_Y, as two GEMMs (Sec. 2, the decomposition after
// Eq. (gradient entry); Sec. 5 calls this the original computation).  The
// integer distance operand is generated from its indices inside the kernel,
// so only T and the intermediate A = T D~_Y move through memory.
//
// FP64 path: v_mfma_f64_16x16x4f64.  Lower-precision paths (FP32, BF16 and
// their split refinements) live in dense_lp.hip.
#include "common.h"
#include "runtime.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int DM = 128, DK = 16;  // block tile DM x DM, DK of K per stage
constexpr int NTHR = 512;           // 4 x 2 waves of 32 x 64
constexpr int WTM = 32, WTN = 64, NTI = WTM / 16, NTJ = WTN / 16;

// C = op(A) * op(B) where exactly one operand is the distance matrix
// |i-j|^kd generated from indices.
//   SYN_B: C[M x N] = A[M x K] (memory, lda) * D[K x N]  (D[k][n] = |k-n|^kd)
//   !SYN_B: C[M x N] = D[M x K] (D[m][k] = |m-k|^kd) * B[K x N] (memory, ldb)
// Epilogue: if c1 != null, C = (c1[m] + c2[n]) - s2 * acc; else C = acc.
// The memory operand goes through LDS in two buffers: the next tile is loaded
// into registers while the current one feeds the matrix cores, then stored
// into the other buffer (one barrier per stage).  The distance operand of a
// stage is formed from its indices (integers, exact below 2^53) once per block, into LDS
// beside it, instead of by every wave that reads it.
// 128 x 128 block tiles of 8 waves (32 x 64 each) keep the accumulators in
// 64 registers, so two blocks share a CU.  KD is the distance exponent (the
// powers unroll into KD - 1 multiplications).
template <bool SYN_B, int KD>
__global__ __launch_bounds__(NTHR) void k_dense_f64(const double* __restrict__ Amem, int64_t lda,
                                                     int M, int N, int K,
                                                     double* __restrict__ C, int64_t ldc,
                                                     const double* __restrict__ c1,
                                                     const double* __restrict__ c2, double s2) {
  // SYN_B: A tiles [DM rows][DK k]; else B tiles [DK k][DM cols].  Rows are
  // padded so that a wave's 64 operand reads (16 rows or columns x 4 k) fall
  // at most two to a pair of LDS banks: DK + 2 for the row-operand layout,
  // DM + 8 for the column-operand layout
  constexpr int PA = DK + 2, PB = DM + 8;
  constexpr int R0 = SYN_B ? DM : DK, R1 = SYN_B ? PA : PB;
  constexpr int PER = DM * DK / NTHR;  // memory-operand entries per thread and stage
  __shared__ double Ms[2][R0][R1];
  __shared__ double Ds[2][SYN_B ? DK : DM][SYN_B ? PB : PA];  // distance tile
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * WTM, wn = (wave & 1) * WTN;  // wave tile origin in block
  const int m0 = blockIdx.y * DM, n0 = blockIdx.x * DM;
  const int li = lane & 15, lk = lane >> 4;  // operand lane mapping
  d4 acc[NTI][NTJ];
#pragma unroll
  for (int i = 0; i < NTI; ++i)
#pragma unroll
    for (int j = 0; j < NTJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // thread t's entries of a stage: SYN_B row t/4, k (t%4)*PER + u; else k row
  // t/32, columns (t%32)*PER + u (zero outside the matrix)
  const int lr = SYN_B ? t >> 2 : t >> 5, lc = SYN_B ? (t & 3) * PER : (t & 31) * PER;
  double rv[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int gr = SYN_B ? m0 + lr : k0 + lr;         // row of the memory operand
      const int gc = SYN_B ? k0 + lc + u : n0 + lc + u;  // its column
      const bool in = SYN_B ? (gr < M && gc < K) : (gr < K && gc < N);
      rv[u] = in ? Amem[(int64_t)gr * lda + gc] : 0.0;
    }
  };
  auto lstore = [&](int buf, int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) Ms[buf][lr][lc + u] = rv[u];
    // the distance tile of the stage: SYN_B D[k][n], else D[m][k]
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t * PER + u;
      const int r = SYN_B ? e / DM : e / DK, c = SYN_B ? e % DM : e % DK;
      const int i = SYN_B ? k0 + r : m0 + r, j = SYN_B ? n0 + c : k0 + c;
      const double d = (double)(i > j ? i - j : j - i);
      double dk = d;
#pragma unroll
      for (int e = 1; e < KD; ++e) dk *= d;
      Ds[buf][r][c] = dk;
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < DK; ks += 4) {
      double a[NTI], b[NTJ];
#pragma unroll
      for (int i = 0; i < NTI; ++i) {
        const int row = wm + i * 16 + li;
        a[i] = SYN_B ? Ms[buf][row][ks + lk] : Ds[buf][row][ks + lk];
      }
#pragma unroll
      for (int j = 0; j < NTJ; ++j) {
        const int col = wn + j * 16 + li;
        b[j] = SYN_B ? Ds[buf][ks + lk][col] : Ms[buf][ks + lk][col];
      }
#pragma unroll
      for (int i = 0; i < NTI; ++i)
#pragma unroll
        for (int j = 0; j < NTJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  const int nk = (K + DK - 1) / DK;
  gload(0);
  lstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) gload((kt + 1) * DK);
    compute(kt & 1);
    if (kt + 1 < nk) lstore((kt + 1) & 1, (kt + 1) * DK);
    __syncthreads();
  }
  // store: for the FP64 16x16x4 instruction, accumulator slot v of a lane holds
  // row 4 * v + lane / 16 and column lane % 16 of its 16 x 16 block; the
  // constant terms of the lane's rows and columns are all requested first
  double c1v[NTI][4], c2v[NTJ];
  if (c1) {
#pragma unroll
    for (int i = 0; i < NTI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) c1v[i][v] = c1[min(m0 + wm + i * 16 + 4 * v + lk, M - 1)];
#pragma unroll
    for (int j = 0; j < NTJ; ++j) c2v[j] = c2[min(n0 + wn + j * 16 + li, N - 1)];
  }
#pragma unroll
  for (int i = 0; i < NTI; ++i)
#pragma unroll
    for (int j = 0; j < NTJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + i * 16 + 4 * v + lk;
        const int gn = n0 + wn + j * 16 + li;
        if (gm < M && gn < N) {
          const double x = acc[i][j][v];
          C[(int64_t)gm * ldc + gn] = c1 ? (c1v[i][v] + c2v[j]) - s2 * x : x;
        }
      }
}

}  // namespace

namespace gwl {

gw_status dense_lp(const gwr::Grid& X, const gwr::Grid& Y, const double* T, int64_t ldT,
                   double* G, int64_t ldG, int path, gwr::Arena& ws, hipStream_t s,
                   const double* c1, const double* c2);
size_t dense_lp_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y, int path);

size_t dense_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y, int path) {
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(X.n());
  a.take<double>(Y.n());
  if (path == GW_PATH_DENSE_F64) {
    a.take<double>((size_t)X.n() * Y.n());
    return a.used;
  }
  return a.used + dense_lp_ws_bytes(X, Y, path);
}

gw_status dense(const gwr::Grid& X, const gwr::Grid& Y, const double* p, const double* q,
                const double* T, int64_t ldT, double* G, int64_t ldG, int path, gwr::Arena& ws,
                hipStream_t s, const double* c1_pre, const double* c2_pre) {
  if (X.ndim != 1 || Y.ndim != 1) return GW_EUNSUPPORTED;
  const int M = (int)X.n(), N = (int)Y.n();
  double* c1 = ws.take<double>(M);
  double* c2 = ws.take<double>(N);
  gw_status st = resolve_const_terms(X, p, c1_pre, &c1, Y, q, c2_pre, &c2, s);
  if (st != GW_OK) return st;
  const double s2 = 2.0 * (X.hk() * Y.hk());
  if (path != GW_PATH_DENSE_F64) return dense_lp(X, Y, T, ldT, G, ldG, path, ws, s, c1, c2);
  double* A = ws.take<double>((size_t)M * N);
  gwr::ProfScope ps(gwr::kFamDense, s);
  dim3 grid((N + DM - 1) / DM, (M + DM - 1) / DM);
  // A = T D~_Y
  switch (Y.k1d()) {
    case 1: k_dense_f64<true, 1><<<grid, NTHR, 0, s>>>(T, ldT, M, N, N, A, N, nullptr, nullptr, 0.0); break;
    case 2: k_dense_f64<true, 2><<<grid, NTHR, 0, s>>>(T, ldT, M, N, N, A, N, nullptr, nullptr, 0.0); break;
    case 3: k_dense_f64<true, 3><<<grid, NTHR, 0, s>>>(T, ldT, M, N, N, A, N, nullptr, nullptr, 0.0); break;
    case 4: k_dense_f64<true, 4><<<grid, NTHR, 0, s>>>(T, ldT, M, N, N, A, N, nullptr, nullptr, 0.0); break;
    default: return GW_EUNSUPPORTED;
  }
  // B = D~_X A, G = (c1 + c2) - s2 B
  switch (X.k1d()) {
    case 1: k_dense_f64<false, 1><<<grid, NTHR, 0, s>>>(A, N, M, N, M, G, ldG, c1, c2, s2); break;
    case 2: k_dense_f64<false, 2><<<grid, NTHR, 0, s>>>(A, N, M, N, M, G, ldG, c1, c2, s2); break;
    case 3: k_dense_f64<false, 3><<<grid, NTHR, 0, s>>>(A, N, M, N, M, G, ldG, c1, c2, s2); break;
    case 4: k_dense_f64<false, 4><<<grid, NTHR, 0, s>>>(A, N, M, N, M, G, ldG, c1, c2, s2); break;
    default: return GW_EUNSUPPORTED;
  }
  return gwr::last_launch_status();
}

}  // namespace gwl
