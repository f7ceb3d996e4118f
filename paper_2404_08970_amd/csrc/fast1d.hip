// FAST gradient for 1D x 1D grids: B = D~_X T D~_Y by the Pascal recursion
// (Sec. 3, Eq. (Dx), Eq. (1d y), Eq. (1d recursive relation)), then
// G = c1 1^T + 1 c2^T - 2 h_X^k h_Y^k B.
//
// The M x N matrix is cut into 64 x 64 tiles.  Every tile needs, besides its
// own entries, the recursion state that the rest of its rows and columns
// carry into it.  Those states are sums with non-negative weights, so they are
// exchanged as Pascal-form moments and never as the cancelling polynomial
// expansion of (i - j)^k:
//   P1  one read of T: per tile, the row moments sum_q w^r T_iq of each tile
//       row (w = distance to the tile's right / left edge) and the column
//       moments of each tile column;
//   P2  scans of those moments across tiles (state advanced over a tile of
//       width w by the Pascal matrix C(r,s) w^{r-s}): the row carries of T,
//       the column carries of T, and the row carries of the column-carry
//       vectors (these give the column carries of A = T D~_Y, since the
//       column moments of A are the column moments of T times D~_Y);
//   P3  second read of T: in-tile row sweep with row carries gives the tile of
//       A exactly, in-tile column sweep with A's column carries gives the tile
//       of B; the epilogue writes G.
// HBM traffic: two reads of T, one write of G, plus O(MN (kx+ky)/64) of
// moments.
#include "common.h"
#include "runtime.h"

namespace {

constexpr int TS = 64;   // tile edge
constexpr int LDS_STRIDE = TS + 1;

// Workspace layout (doubles):
//   rowmom [2][nJ][ky+1][M]   row moments, then (in place) row carries
//   colmom [2][nI][kx+1][N]   column moments, then column carries
//   augmom [2*nI*(kx+1)][nJ][2][ky+1]  tile moments of the column-carry vectors,
//                                       then (in place) their row carries
struct Layout {
  int64_t M, N;
  int nI, nJ, kx, ky;
  size_t rowmom, colmom, augmom;  // element counts
};

Layout make_layout(int64_t M, int64_t N, int kx, int ky) {
  Layout L;
  L.M = M;
  L.N = N;
  L.kx = kx;
  L.ky = ky;
  L.nI = (int)((M + TS - 1) / TS);
  L.nJ = (int)((N + TS - 1) / TS);
  L.rowmom = (size_t)2 * L.nJ * (ky + 1) * M;
  L.colmom = (size_t)2 * L.nI * (kx + 1) * N;
  L.augmom = (size_t)2 * L.nI * (kx + 1) * L.nJ * 2 * (ky + 1);
  return L;
}

// ---------------------------------------------------------------- P1 moments
template <int KX, int KY>
__global__ __launch_bounds__(256) void k_p1_moments(const double* __restrict__ T, int64_t ldT,
                                                     int M, int N, int nI, int nJ,
                                                     double* __restrict__ rowmom,
                                                     double* __restrict__ colmom) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  __shared__ double X[TS][LDS_STRIDE];
  __shared__ double part[4][TS][2 * KM];
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  const int js = I * TS, qs = J * TS;
  const int h = min(TS, M - js), w = min(TS, N - qs);
  {
    const int c = t & (TS - 1);
    for (int r = t >> 6; r < TS; r += 4)
      X[r][c] = (r < h && c < w) ? T[(int64_t)(js + r) * ldT + qs + c] : 0.0;
  }
  __syncthreads();
  const int grp = t >> 6, line = t & (TS - 1);
  if (grp < 2) {
    // row moments of tile row `line` over columns [32 grp, 32 grp + 32)
    double pre[KY + 1], suf[KY + 1];
#pragma unroll
    for (int r = 0; r <= KY; ++r) pre[r] = suf[r] = 0.0;
    for (int cc = 32 * grp; cc < 32 * grp + 32; ++cc) {
      const double x = X[line][cc];
      const double wp = (double)(w - cc), wsu = (double)(cc + 1);
      double pp = 1.0, ps = 1.0;
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        pre[r] = fma(pp, x, pre[r]);
        suf[r] = fma(ps, x, suf[r]);
        pp *= wp;
        ps *= wsu;
      }
    }
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      part[grp][line][r] = pre[r];
      part[grp][line][KM + r] = suf[r];
    }
  } else {
    const int g2 = grp - 2;
    double pre[KX + 1], suf[KX + 1];
#pragma unroll
    for (int r = 0; r <= KX; ++r) pre[r] = suf[r] = 0.0;
    for (int rr = 32 * g2; rr < 32 * g2 + 32; ++rr) {
      const double x = X[rr][line];
      const double wp = (double)(h - rr), wsu = (double)(rr + 1);
      double pp = 1.0, ps = 1.0;
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        pre[r] = fma(pp, x, pre[r]);
        suf[r] = fma(ps, x, suf[r]);
        pp *= wp;
        ps *= wsu;
      }
    }
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      part[grp][line][r] = pre[r];
      part[grp][line][KM + r] = suf[r];
    }
  }
  __syncthreads();
  if (t < TS) {
    if (t < h) {
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        rowmom[((size_t)(0 * nJ + J) * (KY + 1) + r) * M + js + t] = part[0][t][r] + part[1][t][r];
        rowmom[((size_t)(1 * nJ + J) * (KY + 1) + r) * M + js + t] =
            part[0][t][KM + r] + part[1][t][KM + r];
      }
    }
  } else if (t < 2 * TS) {
    const int c = t - TS;
    if (c < w) {
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        colmom[((size_t)(0 * nI + I) * (KX + 1) + r) * N + qs + c] = part[2][c][r] + part[3][c][r];
        colmom[((size_t)(1 * nI + I) * (KX + 1) + r) * N + qs + c] =
            part[2][c][KM + r] + part[3][c][KM + r];
      }
    }
  }
}

// In-place exclusive scan of the moments of one line across its tiles.
// base[(dir * ntiles + t) * (K+1) + r) * stride]; prefix from the left, suffix
// from the right; the state is advanced over the width of the tile it passes.
template <int K>
__device__ void scan_line(double* base, size_t stride, int ntiles, int64_t extent) {
  double st[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) st[r] = 0.0;
  for (int tt = 0; tt < ntiles; ++tt) {
    double* p = base + (size_t)tt * (K + 1) * stride;
    double tmp[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      tmp[r] = p[r * stride];
      p[r * stride] = st[r];
    }
    const double wd = (double)min<int64_t>(TS, extent - (int64_t)tt * TS);
    gwk::pascal_shift<K>(st, wd);
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] += tmp[r];
  }
#pragma unroll
  for (int r = 0; r <= K; ++r) st[r] = 0.0;
  double* sbase = base + (size_t)ntiles * (K + 1) * stride;
  for (int tt = ntiles - 1; tt >= 0; --tt) {
    double* p = sbase + (size_t)tt * (K + 1) * stride;
    double tmp[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      tmp[r] = p[r * stride];
      p[r * stride] = st[r];
    }
    const double wd = (double)min<int64_t>(TS, extent - (int64_t)tt * TS);
    gwk::pascal_shift<K>(st, wd);
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] += tmp[r];
  }
}

// ------------------------------------------- P2a/b: row and column carries of T
template <int KX, int KY>
__global__ __launch_bounds__(256) void k_p2_scan(int M, int N, int nI, int nJ,
                                                  double* __restrict__ rowmom,
                                                  double* __restrict__ colmom) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < M) {
    scan_line<KY>(rowmom + idx, (size_t)M, nJ, N);
  } else if (idx < (int64_t)M + N) {
    scan_line<KX>(colmom + (idx - M), (size_t)N, nI, M);
  }
}

// ------------------- P2c: tile moments of the column-carry vectors (one wave each)
template <int KX, int KY>
__global__ __launch_bounds__(64) void k_p2c_moments(int N, int nI, int nJ,
                                                     const double* __restrict__ colmom,
                                                     double* __restrict__ augmom) {
  const int J = blockIdx.x;
  const int v = blockIdx.y;  // (dirC * nI + I) * (KX+1) + r, matches colmom's vector order
  const int c = threadIdx.x;
  const int qs = J * TS;
  const int w = min(TS, N - qs);
  const double x = c < w ? colmom[(size_t)v * N + qs + c] : 0.0;
  const double wp = (double)(w - c), wsu = (double)(c + 1);
  double pp = 1.0, ps = 1.0;
  double* out = augmom + ((size_t)v * nJ + J) * 2 * (KY + 1);
#pragma unroll
  for (int r = 0; r <= KY; ++r) {
    const double a = gwk::wave_sum(pp * x);
    const double b = gwk::wave_sum(ps * x);
    if (c == 0) {
      out[r] = a;
      out[(KY + 1) + r] = b;
    }
    pp *= wp;
    ps *= wsu;
  }
}

// augmom layout per vector: [nJ][2][KY+1]; scan prefix over J, suffix over J.
template <int KX, int KY>
__global__ __launch_bounds__(64) void k_p2c_scan(int N, int nvec, int nJ,
                                                  double* __restrict__ augmom) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * nvec) return;
  const int v = idx >> 1, dir = idx & 1;
  double* base = augmom + (size_t)v * nJ * 2 * (KY + 1) + dir * (KY + 1);
  const size_t step = 2 * (KY + 1);
  double st[KY + 1];
#pragma unroll
  for (int r = 0; r <= KY; ++r) st[r] = 0.0;
  for (int s = 0; s < nJ; ++s) {
    const int J = dir == 0 ? s : nJ - 1 - s;
    double* p = base + (size_t)J * step;
    double tmp[KY + 1];
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      tmp[r] = p[r];
      p[r] = st[r];
    }
    const double wd = (double)min(TS, N - J * TS);
    gwk::pascal_shift<KY>(st, wd);
#pragma unroll
    for (int r = 0; r <= KY; ++r) st[r] += tmp[r];
  }
}

// Sweep one line of length L held in LDS with stride `xs` from x, writing
// D~ x (including the carried-in states) to y.  Both directions run in one
// loop (independent recursions) to expose instruction-level parallelism.
template <int K>
__device__ void sweep_both(const double* x, double* y, int xs, int L, double (&a)[K + 1],
                           double (&b)[K + 1]) {
  for (int s = 0; s < L; ++s) {
    const int cp = s, cs = L - 1 - s;
    const double xp = x[cp * xs], xq = x[cs * xs];
    const double op = a[K], oq = b[K];
    gwk::pascal_step<K>(a, xp);
    gwk::pascal_step<K>(b, xq);
    if (cp < cs) {
      y[cp * xs] = op;
      y[cs * xs] = oq;
    } else if (cp == cs) {
      y[cp * xs] = op + oq;
    } else {
      y[cp * xs] += op;
      y[cs * xs] += oq;
    }
  }
}

// ---------------------------------------------------------- P3: tile sweeps
template <int KX, int KY>
__global__ __launch_bounds__(128) void k_p3_tile(const double* __restrict__ T, int64_t ldT, int M,
                                                  int N, int nI, int nJ,
                                                  const double* __restrict__ rowmom,
                                                  const double* __restrict__ colmom,
                                                  const double* __restrict__ augmom,
                                                  const double* __restrict__ c1,
                                                  const double* __restrict__ c2, double s2,
                                                  double* __restrict__ G, int64_t ldG) {
  __shared__ double X[TS][LDS_STRIDE];
  __shared__ double Y[TS][LDS_STRIDE];
  __shared__ double Vin[2][KX + 1][TS];
  __shared__ double Vout[2][KX + 1][TS];
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  const int js = I * TS, qs = J * TS;
  const int h = min(TS, M - js), w = min(TS, N - qs);
  {
    const int c = t & (TS - 1);
    for (int r = t >> 6; r < TS; r += 2)
      X[r][c] = (r < h && c < w) ? T[(int64_t)(js + r) * ldT + qs + c] : 0.0;
    for (int v = t >> 6; v < 2 * (KX + 1); v += 2) {
      const int dirC = v / (KX + 1), r = v % (KX + 1);
      Vin[dirC][r][c] = c < w ? colmom[((size_t)(dirC * nI + I) * (KX + 1) + r) * N + qs + c] : 0.0;
    }
  }
  __syncthreads();
  if (t < TS) {
    if (t < h) {
      double a[KY + 1], b[KY + 1];
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        a[r] = rowmom[((size_t)(0 * nJ + J) * (KY + 1) + r) * M + js + t];
        b[r] = rowmom[((size_t)(1 * nJ + J) * (KY + 1) + r) * M + js + t];
      }
      sweep_both<KY>(&X[t][0], &Y[t][0], 1, w, a, b);
    }
  } else if (t - TS < 2 * (KX + 1)) {
    const int v = t - TS;
    const int dirC = v / (KX + 1), r = v % (KX + 1);
    const int vidx = (dirC * nI + I) * (KX + 1) + r;
    const double* cor = augmom + ((size_t)vidx * nJ + J) * 2 * (KY + 1);
    double a[KY + 1], b[KY + 1];
#pragma unroll
    for (int rr = 0; rr <= KY; ++rr) {
      a[rr] = cor[rr];
      b[rr] = cor[(KY + 1) + rr];
    }
    sweep_both<KY>(&Vin[dirC][r][0], &Vout[dirC][r][0], 1, w, a, b);
  }
  __syncthreads();
  if (t < w) {
    double a[KX + 1], b[KX + 1];
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      a[r] = Vout[0][r][t];
      b[r] = Vout[1][r][t];
    }
    sweep_both<KX>(&Y[0][t], &X[0][t], LDS_STRIDE, h, a, b);
  }
  __syncthreads();
  {
    const int c = t & (TS - 1);
    if (c < w) {
      const double c2v = c2[qs + c];
      for (int r = t >> 6; r < h; r += 2)
        G[(int64_t)(js + r) * ldG + qs + c] = (c1[js + r] + c2v) - s2 * X[r][c];
    }
  }
}

template <int KX, int KY>
gw_status run_fast1d(const Layout& L, const double* T, int64_t ldT, double* G, int64_t ldG,
                     const double* c1, const double* c2, double s2, double* rowmom,
                     double* colmom, double* augmom, hipStream_t s) {
  const int M = (int)L.M, N = (int)L.N;
  {
    gwr::ProfScope ps(gwr::kFamFastCarry, s);
    k_p1_moments<KX, KY><<<dim3(L.nJ, L.nI), 256, 0, s>>>(T, ldT, M, N, L.nI, L.nJ, rowmom, colmom);
    const int64_t lines = (int64_t)M + N;
    k_p2_scan<KX, KY><<<(unsigned)((lines + 255) / 256), 256, 0, s>>>(M, N, L.nI, L.nJ, rowmom, colmom);
    const int nvec = 2 * L.nI * (KX + 1);
    k_p2c_moments<KX, KY><<<dim3(L.nJ, nvec), 64, 0, s>>>(N, L.nI, L.nJ, colmom, augmom);
    k_p2c_scan<KX, KY><<<(2 * nvec + 63) / 64, 64, 0, s>>>(N, nvec, L.nJ, augmom);
  }
  {
    gwr::ProfScope ps(gwr::kFamFastMain, s);
    k_p3_tile<KX, KY><<<dim3(L.nJ, L.nI), 128, 0, s>>>(T, ldT, M, N, L.nI, L.nJ, rowmom, colmom,
                                                       augmom, c1, c2, s2, G, ldG);
  }
  return gwr::last_launch_status();
}

template <int KX>
gw_status dispatch_ky(int ky, const Layout& L, const double* T, int64_t ldT, double* G,
                      int64_t ldG, const double* c1, const double* c2, double s2, double* rm,
                      double* cm, double* am, hipStream_t s) {
  switch (ky) {
    case 1: return run_fast1d<KX, 1>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 2: return run_fast1d<KX, 2>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 3: return run_fast1d<KX, 3>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 4: return run_fast1d<KX, 4>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
  }
  return GW_EUNSUPPORTED;
}

}  // namespace

namespace gwl {

size_t fast1d_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y) {
  Layout L = make_layout(X.n(), Y.n(), X.k1d(), Y.k1d());
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(L.rowmom);
  a.take<double>(L.colmom);
  a.take<double>(L.augmom);
  a.take<double>(X.n());
  a.take<double>(Y.n());
  return a.used;
}

gw_status fast1d(const gwr::Grid& X, const gwr::Grid& Y, const double* p, const double* q,
                 const double* T, int64_t ldT, double* G, int64_t ldG, gwr::Arena& ws,
                 hipStream_t s, const double* c1_pre, const double* c2_pre) {
  Layout L = make_layout(X.n(), Y.n(), X.k1d(), Y.k1d());
  double* rm = ws.take<double>(L.rowmom);
  double* cm = ws.take<double>(L.colmom);
  double* am = ws.take<double>(L.augmom);
  double* c1 = ws.take<double>(X.n());
  double* c2 = ws.take<double>(Y.n());
  gw_status st;
  if (c1_pre) {
    c1 = const_cast<double*>(c1_pre);
  } else if ((st = const_term(X, p, c1, s)) != GW_OK) {
    return st;
  }
  if (c2_pre) {
    c2 = const_cast<double*>(c2_pre);
  } else if ((st = const_term(Y, q, c2, s)) != GW_OK) {
    return st;
  }
  const double s2 = 2.0 * (X.hk() * Y.hk());
  switch (L.kx) {
    case 1: return dispatch_ky<1>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 2: return dispatch_ky<2>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 3: return dispatch_ky<3>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
    case 4: return dispatch_ky<4>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, s);
  }
  return GW_EUNSUPPORTED;
}

}  // namespace gwl
