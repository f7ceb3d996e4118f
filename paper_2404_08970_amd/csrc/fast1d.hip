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

// A line segment of SEG consecutive entries held in registers.
constexpr int SEG = 16;
constexpr int NSEG = TS / SEG;

// Prefix summary at the segment's end and suffix summary at its start - 1 of
// x[0..SEG) (zero state on entry): pre_r = sum_c (SEG - c)^r x_c,
// suf_r = sum_c (c + 1)^r x_c.  The weights are compile-time integers.
template <int K>
GW_DEV void seg_summaries(const double (&x)[SEG], double (&pre)[K + 1], double (&suf)[K + 1]) {
#pragma unroll
  for (int r = 0; r <= K; ++r) pre[r] = suf[r] = 0.0;
#pragma unroll
  for (int c = 0; c < SEG; ++c) {
    double wp = 1.0, ws = 1.0;
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      pre[r] = fma(wp, x[c], pre[r]);
      suf[r] = fma(ws, x[c], suf[r]);
      wp *= (double)(SEG - c);
      ws *= (double)(c + 1);
    }
  }
}

// out[c] = a_K(c) + b_K(c) over the segment, starting from prefix state `a`
// (at the segment's first entry) and suffix state `b` (at its last entry).
template <int K>
GW_DEV void seg_sweep(const double (&x)[SEG], double (&a)[K + 1], double (&b)[K + 1],
                      double (&out)[SEG]) {
#pragma unroll
  for (int c = 0; c < SEG; ++c) {
    out[c] = a[K];
    gwk::pascal_step<K>(a, x[c]);
  }
#pragma unroll
  for (int c = SEG - 1; c >= 0; --c) {
    out[c] += b[K];
    gwk::pascal_step<K>(b, x[c]);
  }
}

// ---------------------------------------------------------------- P1 moments
// Block of 256 threads per 64 x 64 tile: thread (line, seg) sums a 16-entry
// segment of its row (for row moments) and of its column (column moments);
// the 4 segment summaries of a line are combined with Pascal shifts.  Entries
// beyond the matrix are zero, so every tile is handled at its nominal size.
template <int KX, int KY>
__global__ __launch_bounds__(256) void k_p1_moments(const double* __restrict__ T, int64_t ldT,
                                                     int M, int N, int nI, int nJ,
                                                     double* __restrict__ rowmom,
                                                     double* __restrict__ colmom) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  __shared__ double X[TS][LDS_STRIDE];
  __shared__ double part[2][NSEG][TS][2 * KM];
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  const int js = I * TS, qs = J * TS;
  const int h = min(TS, M - js), w = min(TS, N - qs);
  const int line = t & (TS - 1), seg = t >> 6;
  {
    // column segment straight from global memory (lanes = columns)
    double x[SEG];
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
      const int r = seg * SEG + i;
      x[i] = (r < h && line < w) ? T[(int64_t)(js + r) * ldT + qs + line] : 0.0;
      X[r][line] = x[i];
    }
    double pre[KX + 1], suf[KX + 1];
    seg_summaries<KX>(x, pre, suf);
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      part[1][seg][line][r] = pre[r];
      part[1][seg][line][KM + r] = suf[r];
    }
  }
  __syncthreads();
  {
    double x[SEG];
#pragma unroll
    for (int c = 0; c < SEG; ++c) x[c] = X[line][seg * SEG + c];
    double pre[KY + 1], suf[KY + 1];
    seg_summaries<KY>(x, pre, suf);
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      part[0][seg][line][r] = pre[r];
      part[0][seg][line][KM + r] = suf[r];
    }
  }
  __syncthreads();
  // combine: prefix at the tile end = sum_s P(16 (3 - s)) pre_s; suffix at
  // the tile start - 1 = sum_s P(16 s) suf_s.  Threads 0..63 rows, 64..127 columns.
  if (t < TS) {
    if (t < h) {
      double a[KY + 1], b[KY + 1];
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        a[r] = part[0][0][t][r];
        b[r] = part[0][NSEG - 1][t][KM + r];
      }
#pragma unroll
      for (int sg = 1; sg < NSEG; ++sg) {
        gwk::pascal_shift<KY>(a, (double)SEG);
        gwk::pascal_shift<KY>(b, (double)SEG);
#pragma unroll
        for (int r = 0; r <= KY; ++r) {
          a[r] += part[0][sg][t][r];
          b[r] += part[0][NSEG - 1 - sg][t][KM + r];
        }
      }
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        rowmom[((size_t)(0 * nJ + J) * (KY + 1) + r) * M + js + t] = a[r];
        rowmom[((size_t)(1 * nJ + J) * (KY + 1) + r) * M + js + t] = b[r];
      }
    }
  } else if (t < 2 * TS) {
    const int c = t - TS;
    if (c < w) {
      double a[KX + 1], b[KX + 1];
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        a[r] = part[1][0][c][r];
        b[r] = part[1][NSEG - 1][c][KM + r];
      }
#pragma unroll
      for (int sg = 1; sg < NSEG; ++sg) {
        gwk::pascal_shift<KX>(a, (double)SEG);
        gwk::pascal_shift<KX>(b, (double)SEG);
#pragma unroll
        for (int r = 0; r <= KX; ++r) {
          a[r] += part[1][sg][c][r];
          b[r] += part[1][NSEG - 1 - sg][c][KM + r];
        }
      }
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        colmom[((size_t)(0 * nI + I) * (KX + 1) + r) * N + qs + c] = a[r];
        colmom[((size_t)(1 * nI + I) * (KX + 1) + r) * N + qs + c] = b[r];
      }
    }
  }
}

// In-place exclusive scan of the moments of one line across its tiles.
// base[(dir * ntiles + t) * (K+1) + r) * stride]; prefix from the left, suffix
// from the right; the state is advanced over the width of the tile it passes.
// Loads are issued PF tiles ahead of the recurrence.
template <int K>
__device__ void scan_line(double* base, size_t stride, int ntiles, int64_t extent) {
  constexpr int PF = 8;
  for (int dir = 0; dir < 2; ++dir) {
    double* db = base + (size_t)dir * ntiles * (K + 1) * stride;
    double st[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] = 0.0;
    for (int s0 = 0; s0 < ntiles; s0 += PF) {
      double buf[PF][K + 1];
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int s = s0 + u;
        const int tt = dir == 0 ? s : ntiles - 1 - s;
        if (s < ntiles) {
#pragma unroll
          for (int r = 0; r <= K; ++r) buf[u][r] = db[((size_t)tt * (K + 1) + r) * stride];
        }
      }
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int s = s0 + u;
        if (s < ntiles) {
          const int tt = dir == 0 ? s : ntiles - 1 - s;
#pragma unroll
          for (int r = 0; r <= K; ++r) db[((size_t)tt * (K + 1) + r) * stride] = st[r];
          const double wd = (double)min<int64_t>(TS, extent - (int64_t)tt * TS);
          gwk::pascal_shift<K>(st, wd);
#pragma unroll
          for (int r = 0; r <= K; ++r) st[r] += buf[u][r];
        }
      }
    }
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

// ------------- P2c: row carries of the column-carry vectors, one block per vector
// Thread J computes the moments of its tile of the vector; two threads then
// scan the tiles (prefix, suffix) out of LDS.  Output layout per vector:
// [nJ][2][KY+1] (prefix state at the tile's first column, suffix state at its
// last column).
template <int KX, int KY>
__global__ __launch_bounds__(256) void k_p2c(int N, int nJ, const double* __restrict__ colmom,
                                              double* __restrict__ augmom) {
  extern __shared__ double mom[];  // [nJ][2][KY+1]
  const int v = blockIdx.x;        // (dirC * nI + I) * (KX+1) + r, colmom's vector order
  const double* vec = colmom + (size_t)v * N;
  for (int J = threadIdx.x; J < nJ; J += blockDim.x) {
    const int qs = J * TS;
    const int w = min(TS, N - qs);
    double pre[KY + 1], suf[KY + 1];
#pragma unroll
    for (int r = 0; r <= KY; ++r) pre[r] = suf[r] = 0.0;
    for (int c = 0; c < w; ++c) {
      const double x = vec[qs + c];
      double wp = 1.0, wsu = 1.0;
      const double dp = (double)(w - c), ds = (double)(c + 1);
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        pre[r] = fma(wp, x, pre[r]);
        suf[r] = fma(wsu, x, suf[r]);
        wp *= dp;
        wsu *= ds;
      }
    }
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      mom[(J * 2 + 0) * (KY + 1) + r] = pre[r];
      mom[(J * 2 + 1) * (KY + 1) + r] = suf[r];
    }
  }
  __syncthreads();
  const int dir = threadIdx.x;
  if (dir >= 2) return;
  double* out = augmom + (size_t)v * nJ * 2 * (KY + 1);
  double st[KY + 1];
#pragma unroll
  for (int r = 0; r <= KY; ++r) st[r] = 0.0;
  for (int s = 0; s < nJ; ++s) {
    const int J = dir == 0 ? s : nJ - 1 - s;
#pragma unroll
    for (int r = 0; r <= KY; ++r) out[(J * 2 + dir) * (KY + 1) + r] = st[r];
    const double wd = (double)min(TS, N - J * TS);
    gwk::pascal_shift<KY>(st, wd);
#pragma unroll
    for (int r = 0; r <= KY; ++r) st[r] += mom[(J * 2 + dir) * (KY + 1) + r];
  }
}

// ---------------------------------------------------------- P3: tile sweeps
// 320 threads: (line, seg) for 64 lines x 4 segments of 16, plus one wave for
// the 2(KX+1) column-carry vectors (x 4 segments).  Row phase: each thread
// loads its segment into registers, publishes segment summaries, combines the
// summaries of the segments to its left/right with the tile's carries, sweeps
// its segment and writes A in place.  Column phase: the same along columns
// with A's column carries; results go from registers to G with the epilogue.
template <int KX, int KY>
__global__ __launch_bounds__(320) void k_p3_tile(const double* __restrict__ T, int64_t ldT, int M,
                                                  int N, int nI, int nJ,
                                                  const double* __restrict__ rowmom,
                                                  const double* __restrict__ colmom,
                                                  const double* __restrict__ augmom,
                                                  const double* __restrict__ c1,
                                                  const double* __restrict__ c2, double s2,
                                                  double* __restrict__ G, int64_t ldG) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  constexpr int NAUG = 2 * (KX + 1);
  __shared__ double X[TS][LDS_STRIDE];
  __shared__ double V[NAUG][TS];                   // column-carry vectors, then A's column carries
  __shared__ double sums[2][NSEG][TS + NAUG][KM];  // [pre/suf][seg][line][r]
  const int J = blockIdx.x, I = blockIdx.y, t = threadIdx.x;
  const int js = I * TS, qs = J * TS;
  const int h = min(TS, M - js), w = min(TS, N - qs);
  const int lane = t & (TS - 1), wv = t >> 6;
  // ---- load T tile (zero padded) and the column-carry vector slices
  for (int r = wv; r < TS; r += 5)
    X[r][lane] = (r < h && lane < w) ? T[(int64_t)(js + r) * ldT + qs + lane] : 0.0;
  if (wv == 4) {
    for (int v = 0; v < NAUG; ++v) {
      const int dirC = v / (KX + 1), r = v % (KX + 1);
      V[v][lane] = lane < w ? colmom[((size_t)(dirC * nI + I) * (KX + 1) + r) * N + qs + lane] : 0.0;
    }
  }
  __syncthreads();
  // ---- row phase: line = tile row (wv < 4) or column-carry vector (wv == 4)
  const bool is_row = wv < 4;
  const int seg = is_row ? wv : (lane & 3);
  const int line = is_row ? lane : (TS + (lane >> 2));  // index into sums
  const bool active = is_row ? true : ((lane >> 2) < NAUG);
  double x[SEG];
  if (active) {
    const double* src = is_row ? &X[lane][0] : &V[lane >> 2][0];
#pragma unroll
    for (int c = 0; c < SEG; ++c) x[c] = src[seg * SEG + c];
    double pre[KY + 1], suf[KY + 1];
    seg_summaries<KY>(x, pre, suf);
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      sums[0][seg][line][r] = pre[r];
      sums[1][seg][line][r] = suf[r];
    }
  }
  __syncthreads();
  double out[SEG];
  if (active) {
    double a[KY + 1], b[KY + 1];
    if (is_row) {
      const bool real = lane < h;
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        a[r] = real ? rowmom[((size_t)(0 * nJ + J) * (KY + 1) + r) * M + js + lane] : 0.0;
        b[r] = real ? rowmom[((size_t)(1 * nJ + J) * (KY + 1) + r) * M + js + lane] : 0.0;
      }
    } else {
      const int v = lane >> 2;
      const int dirC = v / (KX + 1), rr = v % (KX + 1);
      const int vidx = (dirC * nI + I) * (KX + 1) + rr;
      const double* cor = augmom + ((size_t)vidx * nJ + J) * 2 * (KY + 1);
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        a[r] = cor[r];
        b[r] = cor[(KY + 1) + r];
      }
    }
    // prefix state entering the segment: carries over segments 0..seg-1
    for (int sg = 0; sg < seg; ++sg) {
      gwk::pascal_shift<KY>(a, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KY; ++r) a[r] += sums[0][sg][line][r];
    }
    // suffix state entering from the right: segments NSEG-1 .. seg+1
    for (int sg = NSEG - 1; sg > seg; --sg) {
      gwk::pascal_shift<KY>(b, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KY; ++r) b[r] += sums[1][sg][line][r];
    }
    seg_sweep<KY>(x, a, b, out);
  }
  __syncthreads();  // everyone has read X / V
  if (active) {
    double* dst = is_row ? &X[lane][0] : &V[lane >> 2][0];
#pragma unroll
    for (int c = 0; c < SEG; ++c) dst[seg * SEG + c] = out[c];
  }
  __syncthreads();
  // ---- column phase: 4 waves, (column = lane, segment of rows = wv)
  if (wv < 4) {
#pragma unroll
    for (int i = 0; i < SEG; ++i) x[i] = X[wv * SEG + i][lane];
    double pre[KX + 1], suf[KX + 1];
    seg_summaries<KX>(x, pre, suf);
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      sums[0][wv][lane][r] = pre[r];
      sums[1][wv][lane][r] = suf[r];
    }
  }
  __syncthreads();
  if (wv < 4) {
    double a[KX + 1], b[KX + 1];
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      a[r] = V[r][lane];             // A's column carry from above (from Cpre)
      b[r] = V[(KX + 1) + r][lane];  // from below (from Csuf)
    }
    for (int sg = 0; sg < wv; ++sg) {
      gwk::pascal_shift<KX>(a, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KX; ++r) a[r] += sums[0][sg][lane][r];
    }
    for (int sg = NSEG - 1; sg > wv; --sg) {
      gwk::pascal_shift<KX>(b, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KX; ++r) b[r] += sums[1][sg][lane][r];
    }
    seg_sweep<KX>(x, a, b, out);
    if (lane < w) {
      const double c2v = c2[qs + lane];
#pragma unroll
      for (int i = 0; i < SEG; ++i) {
        const int r = wv * SEG + i;
        if (r < h) G[(int64_t)(js + r) * ldG + qs + lane] = (c1[js + r] + c2v) - s2 * out[i];
      }
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
    const size_t shm = (size_t)L.nJ * 2 * (KY + 1) * sizeof(double);
    k_p2c<KX, KY><<<nvec, 256, shm, s>>>(N, L.nJ, colmom, augmom);
  }
  {
    gwr::ProfScope ps(gwr::kFamFastMain, s);
    k_p3_tile<KX, KY><<<dim3(L.nJ, L.nI), 320, 0, s>>>(T, ldT, M, N, L.nI, L.nJ, rowmom, colmom,
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
