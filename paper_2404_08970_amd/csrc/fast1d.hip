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
#include <hip/hip_ext.h>
#include "common.h"
#include "runtime.h"

namespace {

constexpr int TS = 64;   // tile edge
constexpr int LDS_STRIDE = TS + 1;

// Workspace layout (doubles):
//   rowmom [2][nJ][ky+1][M]   row moments, then (in place) row carries
//   colmom [2][nI][kx+1][N]   column moments, then column carries
//   acarry [2][nI][kx+1][N]   column carries of A = T D~_Y (D~_Y applied to
//                             the column carries of T)
struct Layout {
  int64_t M, N;
  int nI, nJ, kx, ky;
  size_t rowmom, colmom, acarry;  // element counts
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
  L.acarry = L.colmom;
  return L;
}

// A line segment of SEG consecutive entries held in registers.
constexpr int SEG = 16;
constexpr int NSEG = TS / SEG;

// Prefix summary at the segment's end and suffix summary at its start - 1 of
// x[0..L) (zero state on entry): pre_r = sum_c (L - c)^r x_c,
// suf_r = sum_c (c + 1)^r x_c.  The weights are compile-time integers.
template <int K, int L>
GW_DEV void seg_summaries(const double (&x)[L], double (&pre)[K + 1], double (&suf)[K + 1]) {
#pragma unroll
  for (int r = 0; r <= K; ++r) pre[r] = suf[r] = 0.0;
#pragma unroll
  for (int c = 0; c < L; ++c) {
    double wp = 1.0, ws = 1.0;
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      pre[r] = fma(wp, x[c], pre[r]);
      suf[r] = fma(ws, x[c], suf[r]);
      wp *= (double)(L - c);
      ws *= (double)(c + 1);
    }
  }
}

// out[c] = a_K(c) + b_K(c) over the segment, starting from prefix state `a`
// (at the segment's first entry) and suffix state `b` (at its last entry).
template <int K, int L>
GW_DEV void seg_sweep(const double (&x)[L], double (&a)[K + 1], double (&b)[K + 1],
                      double (&out)[L]) {
#pragma unroll
  for (int c = 0; c < L; ++c) {
    out[c] = a[K];
    gwk::pascal_step<K>(a, x[c]);
  }
#pragma unroll
  for (int c = L - 1; c >= 0; --c) {
    out[c] += b[K];
    gwk::pascal_step<K>(b, x[c]);
  }
}

// Combine the NSEG segment summaries of one line (LDS layout part[seg][line][*],
// prefix in [0..K], suffix in [KM..KM+K]) into the line's tile moments:
// prefix at the tile end = sum_s P(SEG (NSEG-1-s)) pre_s, suffix at the tile
// start - 1 = sum_s P(SEG s) suf_s.
template <int K, int KM, int LINES>
GW_DEV void combine_segments(const double (*part)[LINES][2 * KM], int line, double (&a)[K + 1],
                             double (&b)[K + 1]) {
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    a[r] = part[0][line][r];
    b[r] = part[NSEG - 1][line][KM + r];
  }
#pragma unroll
  for (int sg = 1; sg < NSEG; ++sg) {
    gwk::pascal_shift<K>(a, (double)SEG);
    gwk::pascal_shift<K>(b, (double)SEG);
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      a[r] += part[sg][line][r];
      b[r] += part[NSEG - 1 - sg][line][KM + r];
    }
  }
}

// ---------------------------------------------------------------- P1 moments
constexpr int P1_DEPTH = 2;  // tiles in flight per block (3 measured no faster)

// Persistent blocks of 256 threads walk the tiles; thread (line, seg) holds a
// 16-entry column segment of the tile in registers (loaded one tile ahead),
// sums it for the column moments, and sums a row segment (through LDS) for
// the row moments.  Entries beyond the matrix are zero, so every tile is
// handled at its nominal size.  The segment summaries reuse the tile's LDS
// once every thread has read its row segment (one LDS buffer per block: more
// resident blocks).
template <int KX, int KY>
__global__ __launch_bounds__(256) void k_p1_moments(const double* __restrict__ T, int64_t ldT,
                                                     int M, int N, int nI, int nJ,
                                                     double* __restrict__ rowmom,
                                                     double* __restrict__ colmom) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  constexpr int XW = TS * LDS_STRIDE, PW = 2 * NSEG * TS * 2 * KM;
  __shared__ double lds1[XW > PW ? XW : PW];
  auto X = reinterpret_cast<double (*)[LDS_STRIDE]>(lds1);          // the tile
  auto part = reinterpret_cast<double (*)[NSEG][TS][2 * KM]>(lds1);  // then the summaries
  // seg is the wave index: kept in a scalar register, so row addresses are scalar
  const int t = threadIdx.x, lane = t & (TS - 1), seg = __builtin_amdgcn_readfirstlane(t >> 6);
  const int ntiles = nI * nJ;
  // P1_DEPTH tiles in flight: the tile processed now was requested P1_DEPTH
  // tiles ago.
  double pf3[P1_DEPTH][SEG];
  auto load_tile = [&](double (&pf)[SEG], int tile) {
    const int I = tile / nJ, J = tile - (tile / nJ) * nJ;
    const int col = min(J * TS + lane, N - 1);
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
      const int row = min(I * TS + seg * SEG + i, M - 1);
      pf[i] = T[(int64_t)row * ldT + col];
    }
  };
  const int stride = gridDim.x;
  // tile_in >= ntiles: a pass over the last tile whose stores are dropped, so
  // that both bodies of the loop run on every iteration
  auto body = [&](double (&pf)[SEG], int tile_in) {
    const bool live = tile_in < ntiles;
    const int tile = min(tile_in, ntiles - 1);
    const int I = tile / nJ, J = tile - I * nJ;
    const int js = I * TS, qs = J * TS;
    const int h = min(TS, M - js), w = min(TS, N - qs);
    double x[SEG];
#pragma unroll
    for (int i = 0; i < SEG; ++i) x[i] = (seg * SEG + i < h && lane < w) ? pf[i] : 0.0;
    load_tile(pf, min(tile + P1_DEPTH * stride, ntiles - 1));
    double cpre[KX + 1], csuf[KX + 1], rpre[KY + 1], rsuf[KY + 1];
    seg_summaries<KX>(x, cpre, csuf);
#pragma unroll
    for (int i = 0; i < SEG; ++i) X[seg * SEG + i][lane] = x[i];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < SEG; ++c) x[c] = X[lane][seg * SEG + c];
    seg_summaries<KY>(x, rpre, rsuf);
    __syncthreads();  // every row segment has been read: the summaries take the LDS
#pragma unroll
    for (int r = 0; r <= KY; ++r) {
      part[0][seg][lane][r] = rpre[r];
      part[0][seg][lane][KM + r] = rsuf[r];
    }
#pragma unroll
    for (int r = 0; r <= KX; ++r) {
      part[1][seg][lane][r] = cpre[r];
      part[1][seg][lane][KM + r] = csuf[r];
    }
    __syncthreads();
    // wave 0 writes the row moments of the tile's rows, wave 1 the column
    // moments of its columns; every wave issues the same KM x 2 stores (the
    // others and the unused ones dropped by the buffer range check), so no
    // branch surrounds a store
    {
      double a[KM], b[KM];
#pragma unroll
      for (int r = 0; r < KM; ++r) a[r] = b[r] = 0.0;
      bool ok = false;
      if (seg == 0) {
        double ra[KY + 1], rb[KY + 1];
        combine_segments<KY, KM, TS>(part[0], lane, ra, rb);
#pragma unroll
        for (int r = 0; r <= KY; ++r) {
          a[r] = ra[r];
          b[r] = rb[r];
        }
        ok = live && lane < h;
      } else if (seg == 1) {
        double ca[KX + 1], cb[KX + 1];
        combine_segments<KX, KM, TS>(part[1], lane, ca, cb);
#pragma unroll
        for (int r = 0; r <= KX; ++r) {
          a[r] = ca[r];
          b[r] = cb[r];
        }
        ok = live && lane < w;
      }
#pragma unroll
      for (int r = 0; r < KM; ++r) {
        // moment row (direction, tile, r) of the wave's array, at the tile's first line
        const double* pa;
        const double* pb;
        bool okr;
        if (seg == 0) {
          okr = ok && r <= KY;
          const int rr = min(r, KY);
          pa = rowmom + ((size_t)(0 * nJ + J) * (KY + 1) + rr) * M + js;
          pb = rowmom + ((size_t)(1 * nJ + J) * (KY + 1) + rr) * M + js;
        } else {
          okr = seg == 1 && ok && r <= KX;
          const int rr = min(r, KX);
          pa = colmom + ((size_t)(0 * nI + I) * (KX + 1) + rr) * N + qs;
          pb = colmom + ((size_t)(1 * nI + I) * (KX + 1) + rr) * N + qs;
        }
        const int off = okr ? lane * 8 : gwk::kOffDrop;
        gwk::buffer_store_f64(a[r], gwk::buffer_rsrc(pa), off);
        gwk::buffer_store_f64(b[r], gwk::buffer_rsrc(pb), off);
      }
    }
    __syncthreads();
  };
  int tile = blockIdx.x;
  if (tile < ntiles) {
    // the prologue issues the same memory operations between the
    // prefetches as a loop iteration (its stores dropped, at distinct and
    // non-adjacent offsets so that none is merged with another), so the waits
    // for a prefetched tile do not also cover the stores that follow it
#pragma unroll
    for (int d = 0; d < P1_DEPTH; ++d) {
      load_tile(pf3[d], min(tile + d * stride, ntiles - 1));
#pragma unroll
      for (int u = 0; u < 2 * KM; ++u)
        gwk::buffer_store_f64(0.0, gwk::buffer_rsrc(rowmom), gwk::kOffDrop + 64 * u);
    }
  }
  for (; tile < ntiles; tile += P1_DEPTH * stride) {
#pragma unroll
    for (int d = 0; d < P1_DEPTH; ++d) body(pf3[d], tile + d * stride);
  }
}

// In-place exclusive scans of the moments of 64 lines across their tiles
// (layout base[((dir * ntiles + tile) * (K+1) + r) * stride + line]): prefix
// from the left (dir 0), suffix from the right (dir 1); the state is advanced
// over the width of each tile it passes.  The tiles of a line are cut into
// CH chunks, one thread per (line, chunk): each thread folds its chunk
// into an aggregate, the aggregates of the earlier chunks (shifted over the
// chunks between) give the thread's incoming state, and a second pass over
// the chunk writes the exclusive states.  A block takes LN lines x CH chunks.
// With at least SCAN_ONE_THREAD_LINES lines the scan runs one thread per line
// (one read and one write of the moments, which then stream at about the
// copy rate); with fewer lines, one thread per line would leave most CUs idle,
// so chunked threads share a line at the price of a second read.
constexpr int64_t SCAN_ONE_THREAD_LINES = 32768;
constexpr int SCAN_MAXCH = 16;

GW_DEV int tile_width(int tt, int64_t extent) {
  const int64_t w = extent - (int64_t)tt * TS;
  return w < TS ? (int)w : TS;
}

template <int K, int LN, int CH>
GW_DEV void scan_lines(double* base, size_t stride, int line, bool valid, int ntiles,
                       int64_t extent, double (*agg)[CH][LN][K + 1], double (*span)[CH], int ln,
                       int ch) {
  constexpr int PF = 8;  // tiles loaded ahead of the recurrence
  const int cs = (ntiles + CH - 1) / CH;
  const int s0 = ch * cs, s1 = min(ntiles, s0 + cs);
  // Loads are unconditional (the tile index clamped into this chunk), so all
  // PF tiles are in flight at once; entries past the chunk are zeroed after.
  auto load = [&](const double* db, double (&buf)[PF][K + 1], int sb, int dir) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int sidx = min(sb + u, s1 - 1);
      const int tt = dir == 0 ? sidx : ntiles - 1 - sidx;
#pragma unroll
      for (int r = 0; r <= K; ++r) buf[u][r] = db[((size_t)tt * (K + 1) + r) * stride];
    }
#pragma unroll
    for (int u = 0; u < PF; ++u)
      if (!(valid && sb + u < s1)) {
#pragma unroll
        for (int r = 0; r <= K; ++r) buf[u][r] = 0.0;
      }
  };
  // pass 1: chunk aggregates and spans in both directions
#pragma unroll
  for (int dir = 0; dir < 2 && CH > 1; ++dir) {
    const double* db = base + (size_t)dir * ntiles * (K + 1) * stride + line;
    double st[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] = 0.0;
    int width = 0;
    for (int sb = s0; sb < s1; sb += PF) {
      double buf[PF][K + 1];
      load(db, buf, sb, dir);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int sidx = sb + u;
        if (sidx < s1) {
          const int tt = dir == 0 ? sidx : ntiles - 1 - sidx;
          const int wd = tile_width(tt, extent);
          gwk::pascal_shift<K>(st, (double)wd);
#pragma unroll
          for (int r = 0; r <= K; ++r) st[r] += buf[u][r];
          width += wd;
        }
      }
    }
#pragma unroll
    for (int r = 0; r <= K; ++r) agg[dir][ch][ln][r] = st[r];
    if (ln == 0) span[dir][ch] = (double)width;
  }
  if (CH > 1) __syncthreads();
  // pass 2: incoming state from the earlier chunks, then exclusive states
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    double* db = base + (size_t)dir * ntiles * (K + 1) * stride + line;
    double st[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] = 0.0;
    for (int c = 0; c < ch; ++c) {
      gwk::pascal_shift<K>(st, span[dir][c]);
#pragma unroll
      for (int r = 0; r <= K; ++r) st[r] += agg[dir][c][ln][r];
    }
    for (int sb = s0; sb < s1; sb += PF) {
      double buf[PF][K + 1];
      load(db, buf, sb, dir);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int sidx = sb + u;
        if (sidx < s1) {
          const int tt = dir == 0 ? sidx : ntiles - 1 - sidx;
          if (valid) {
#pragma unroll
            for (int r = 0; r <= K; ++r) db[((size_t)tt * (K + 1) + r) * stride] = st[r];
          }
          gwk::pascal_shift<K>(st, (double)tile_width(tt, extent));
#pragma unroll
          for (int r = 0; r <= K; ++r) st[r] += buf[u][r];
        }
      }
    }
  }
}

// ------------------------------------------- P2a/b: row and column carries of T
// Blocks [0, ceil(M/64)) scan the row moments of 64 rows each, the rest the
// column moments of 64 columns each.
template <int KX, int KY, int LN, int CH>
__global__ __launch_bounds__(LN * CH) void k_p2_scan(int M, int N, int nI, int nJ,
                                                              double* __restrict__ rowmom,
                                                              double* __restrict__ colmom) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  __shared__ double agg[2][CH][LN][KM];
  __shared__ double span[2][CH];
  const int ln = threadIdx.x % LN, ch = threadIdx.x / LN;
  const int rblocks = (M + LN - 1) / LN;
  if ((int)blockIdx.x < rblocks) {
    const int line = blockIdx.x * LN + ln;
    scan_lines<KY, LN, CH>(rowmom, (size_t)M, min(line, M - 1), line < M, nJ, N,
                           reinterpret_cast<double (*)[CH][LN][KY + 1]>(&agg[0][0][0][0]),
                       span, ln, ch);
  } else {
    const int line = (blockIdx.x - rblocks) * LN + ln;
    scan_lines<KX, LN, CH>(colmom, (size_t)N, min(line, N - 1), line < N, nI, M,
                           reinterpret_cast<double (*)[CH][LN][KX + 1]>(&agg[0][0][0][0]),
                       span, ln, ch);
  }
}

// ------------- P2c: column carries of A = T D~_Y, one block per vector.
// A's column carries at the top (bottom) of tile-row I are D~_Y applied to the
// column carries of T, vectors of length N (one per direction, tile-row and
// moment order), zero-padded to nJ full tiles.  The vector is processed in
// rounds of 64 tiles (4096 entries) staged through LDS with coalesced loads
// and stores; thread (tile tl, segment seg) works on 16 entries.
//   pass A  segment summaries -> tile moments (prefix at the tile end, suffix
//           at its start - 1);
//   scan    exclusive scans of the tile moments over the tiles: each thread
//           folds a run of consecutive tiles, a shuffle scan inside each wave
//           and the totals of the earlier waves combine the runs (shift over
//           the span between them), and each thread writes the exclusive
//           states of its run;
//   pass B  each segment is swept with its tile's carries advanced over the
//           segments before (after) it, and the output leaves through LDS.
constexpr int P2C_TILES = 64;                       // tiles per round
constexpr int P2C_ROUND = P2C_TILES * TS;           // entries per round
constexpr int P2C_STG = P2C_ROUND + P2C_ROUND / SEG;  // one pad double per segment

GW_DEV int stg_index(int i) { return i + (i >> 4); }

// KEEP: rounds whose entries stay in registers between the passes (the
// vector is then read once); 0 re-reads it in pass B.
template <int KX, int KY, int KEEP>
__global__ __launch_bounds__(256) void k_p2c(int N, int nJ, const double* __restrict__ colmom,
                                              double* __restrict__ acarry) {
  constexpr int K = KY, KM = KY + 1;
  extern __shared__ double mom[];  // [2][nJ][KM]: tile moments, then exclusive carries
  __shared__ double stg[P2C_STG];
  __shared__ double part[NSEG][P2C_TILES][2 * KM];
  const int v = blockIdx.x;
  const double* vec = colmom + (size_t)v * N;
  double* out = acarry + (size_t)v * N;
  const int t = threadIdx.x, tl = t >> 2, seg = t & 3;
  const int nround = (nJ + P2C_TILES - 1) / P2C_TILES;
  const int sb = tl * TS + seg * SEG;  // segment start within a round
  auto stage_in = [&](int e0) {
    double v[P2C_ROUND / 256];  // all loads issued before any is used (indices clamped)
#pragma unroll
    for (int c = 0; c < P2C_ROUND / 256; ++c) v[c] = vec[min(e0 + t + 256 * c, N - 1)];
#pragma unroll
    for (int c = 0; c < P2C_ROUND / 256; ++c) {
      const int i = t + 256 * c;
      stg[stg_index(i)] = e0 + i < N ? v[c] : 0.0;
    }
  };
  auto summaries = [&](double (&x)[SEG]) {
#pragma unroll
    for (int c = 0; c < SEG; ++c) x[c] = stg[stg_index(sb + c)];
    double pre[K + 1], suf[K + 1];
    seg_summaries<K>(x, pre, suf);
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      part[seg][tl][r] = pre[r];
      part[seg][tl][KM + r] = suf[r];
    }
  };
  double keep[KEEP > 0 ? KEEP : 1][SEG];
  // pass A: tile moments
  for (int rd = 0; rd < nround; ++rd) {
    __syncthreads();
    stage_in(rd * P2C_ROUND);
    __syncthreads();
    double x[SEG];
    summaries(x);
    if constexpr (KEEP > 0) {
#pragma unroll
      for (int k = 0; k < KEEP; ++k)
        if (k == rd) {
#pragma unroll
          for (int c = 0; c < SEG; ++c) keep[k][c] = x[c];
        }
    }
    __syncthreads();
    const int J = rd * P2C_TILES + tl;
    if (seg == 0 && J < nJ) {
      double a[K + 1], b[K + 1];
      combine_segments<K, KM, P2C_TILES>(part, tl, a, b);
#pragma unroll
      for (int r = 0; r <= K; ++r) {
        mom[(0 * nJ + J) * KM + r] = a[r];
        mom[(1 * nJ + J) * KM + r] = b[r];
      }
    }
  }
  // scans over the tiles; their buffers live in the staging area
  const int run = (nJ + 255) / 256;  // tiles per thread
  double* hs = stg;                  // [256][KM] inclusive states, then [4][KM] wave totals
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    __syncthreads();
    double agg[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) agg[r] = 0.0;
    for (int u = 0; u < run; ++u) {
      const int pos = t * run + u;
      if (pos < nJ) {
        const int J = dir == 0 ? pos : nJ - 1 - pos;
        gwk::pascal_shift<K>(agg, (double)TS);
#pragma unroll
        for (int r = 0; r <= K; ++r) agg[r] += mom[(dir * nJ + J) * KM + r];
      }
    }
    // inclusive scan of the run states: inside each wave by shuffles (the
    // state from lane - d is shifted over the d runs between), then the totals
    // of the earlier waves, each shifted from its wave's end to this run's end
    const int lane = t & 63, wv = t >> 6;
    for (int d = 1; d < 64; d <<= 1) {
      double o[K + 1];
#pragma unroll
      for (int r = 0; r <= K; ++r) o[r] = __shfl_up(agg[r], d, 64);
      if (lane >= d) {
        gwk::pascal_shift<K>(o, (double)TS * run * d);
#pragma unroll
        for (int r = 0; r <= K; ++r) agg[r] += o[r];
      }
    }
    double* wtot = hs + 256 * KM;  // [4][KM]: the waves' totals
    if (lane == 63) {
#pragma unroll
      for (int r = 0; r <= K; ++r) wtot[wv * KM + r] = agg[r];
    }
    __syncthreads();
    for (int w = 0; w < wv; ++w) {
      double o[K + 1];
#pragma unroll
      for (int r = 0; r <= K; ++r) o[r] = wtot[w * KM + r];
      gwk::pascal_shift<K>(o, (double)TS * run * (t - 64 * w - 63));
#pragma unroll
      for (int r = 0; r <= K; ++r) agg[r] += o[r];
    }
#pragma unroll
    for (int r = 0; r <= K; ++r) hs[t * KM + r] = agg[r];
    __syncthreads();
    double st[K + 1];  // exclusive: the inclusive state of the run before
#pragma unroll
    for (int r = 0; r <= K; ++r) st[r] = t > 0 ? hs[(t - 1) * KM + r] : 0.0;
    for (int u = 0; u < run; ++u) {
      const int pos = t * run + u;
      if (pos < nJ) {
        const int J = dir == 0 ? pos : nJ - 1 - pos;
        double m[K + 1];
#pragma unroll
        for (int r = 0; r <= K; ++r) {
          m[r] = mom[(dir * nJ + J) * KM + r];
          mom[(dir * nJ + J) * KM + r] = st[r];
        }
        gwk::pascal_shift<K>(st, (double)TS);
#pragma unroll
        for (int r = 0; r <= K; ++r) st[r] += m[r];
      }
    }
  }
  // pass B: in-tile sweeps with the tile carries
  for (int rd = 0; rd < nround; ++rd) {
    const int e0 = rd * P2C_ROUND;
    double x[SEG];
    __syncthreads();
    if constexpr (KEEP > 0) {
#pragma unroll
      for (int k = 0; k < KEEP; ++k)
        if (k == rd) {
#pragma unroll
          for (int c = 0; c < SEG; ++c) x[c] = keep[k][c];
        }
      double pre[K + 1], suf[K + 1];
      seg_summaries<K>(x, pre, suf);
#pragma unroll
      for (int r = 0; r <= K; ++r) {
        part[seg][tl][r] = pre[r];
        part[seg][tl][KM + r] = suf[r];
      }
    } else {
      stage_in(e0);
      __syncthreads();
      summaries(x);
    }
    __syncthreads();
    const int J = rd * P2C_TILES + tl;
    if (J < nJ) {
      double a[K + 1], b[K + 1];
#pragma unroll
      for (int r = 0; r <= K; ++r) {
        a[r] = mom[(0 * nJ + J) * KM + r];
        b[r] = mom[(1 * nJ + J) * KM + r];
      }
      for (int sg = 0; sg < seg; ++sg) {
        gwk::pascal_shift<K>(a, (double)SEG);
#pragma unroll
        for (int r = 0; r <= K; ++r) a[r] += part[sg][tl][r];
      }
      for (int sg = NSEG - 1; sg > seg; --sg) {
        gwk::pascal_shift<K>(b, (double)SEG);
#pragma unroll
        for (int r = 0; r <= K; ++r) b[r] += part[sg][tl][KM + r];
      }
      double o[SEG];
      seg_sweep<K>(x, a, b, o);
      // each thread rewrites only its own segment of the staging area
#pragma unroll
      for (int c = 0; c < SEG; ++c) stg[stg_index(sb + c)] = o[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < P2C_ROUND / 256; ++c) {
      const int i = t + 256 * c;
      const int p = e0 + i;
      if (p < N) out[p] = stg[stg_index(i)];
    }
  }
}

// ---------------------------------------------------------- P3: tile sweeps
// Persistent blocks of 256 threads walk the tiles, the next tile's T already
// in registers.  Row phase: thread (row = lane, seg = wave) sweeps a 16-entry
// row segment; segment summaries pass through LDS and are combined with the
// tile's row carries, and A overwrites T in LDS.  Column phase: thread
// (column = lane, seg = wave) does the same along the column with A's column
// carries, and writes G = (c1 + c2) - s2 B from registers (non-temporal
// stores: G is streamed out, not read back by this gradient).  With FG the
// fused GW feature term is applied on the way out:
// G = ea ((c1 + c2) - s2 B) + eb (fa_i - fb_p)^2.
template <int KX, int KY, bool FG>
__global__ __launch_bounds__(256) void k_p3_tile(const double* __restrict__ T, int64_t ldT, int M,
                                                  int N, int nI, int nJ,
                                                  const double* __restrict__ rowmom,
                                                  const double* __restrict__ acarry,
                                                  const double* __restrict__ c1,
                                                  const double* __restrict__ c2, double s2,
                                                  double* __restrict__ G, int64_t ldG,
                                                  gwr::Epilogue epi) {
  constexpr int KM = (KX > KY ? KX : KY) + 1;
  __shared__ double X[TS][LDS_STRIDE];
  __shared__ double sums[2][NSEG][TS][KM];  // [pre/suf][seg][line][r]
  // seg is the wave index: kept in a scalar register, so row addresses are scalar
  const int t = threadIdx.x, lane = t & (TS - 1), seg = __builtin_amdgcn_readfirstlane(t >> 6);
  const int ntiles = nI * nJ;
  double pf[SEG];  // the next tile, requested while this one is processed
  auto load_tile = [&](double (&dst)[SEG], int tile) {
    const int I = tile / nJ, J = tile - (tile / nJ) * nJ;
    const int col = min(J * TS + lane, N - 1);
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
      const int row = min(I * TS + seg * SEG + i, M - 1);
      dst[i] = T[(int64_t)row * ldT + col];
    }
  };
  const int stride = gridDim.x;
  auto body = [&](int tile) {
    const int I = tile / nJ, J = tile - I * nJ;
    const int js = I * TS, qs = J * TS;
    const int h = min(TS, M - js), w = min(TS, N - qs);
    // carries for this tile: row carries of the thread's row, A's column
    // carries of its column, and c2 of its column (used after the barriers).
    // They are requested before the next tile: loads complete in issue order,
    // so waiting for them then leaves the next tile's loads in flight.
    double ra[KY + 1], rb[KY + 1], ca[KX + 1], cb[KX + 1];
    const double c2v = c2[min(qs + lane, N - 1)];
    double fbv = 0.0;
    if constexpr (FG) fbv = epi.fb[min(qs + lane, N - 1)];
    {
      const int row = min(js + lane, M - 1);
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        ra[r] = rowmom[((size_t)(0 * nJ + J) * (KY + 1) + r) * M + row];
        rb[r] = rowmom[((size_t)(1 * nJ + J) * (KY + 1) + r) * M + row];
      }
      const int col = min(qs + lane, N - 1);
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        ca[r] = acarry[((size_t)(0 * nI + I) * (KX + 1) + r) * N + col];
        cb[r] = acarry[((size_t)(1 * nI + I) * (KX + 1) + r) * N + col];
      }
    }
    // the tile goes to LDS straight from the prefetch registers, which then
    // take the next tile (the same registers in every iteration)
#pragma unroll
    for (int i = 0; i < SEG; ++i) X[seg * SEG + i][lane] = (seg * SEG + i < h && lane < w) ? pf[i] : 0.0;
    // the next tile's loads are issued at raised wave priority, so they go
    // out ahead of the other resident waves' sweeps (in-kernel wave priority
    // only; every stream keeps the default priority)
    __builtin_amdgcn_s_setprio(3);
    load_tile(pf, min(tile + stride, ntiles - 1));
    __builtin_amdgcn_s_setprio(0);
    if (lane >= h) {  // rows past the matrix carry nothing
#pragma unroll
      for (int r = 0; r <= KY; ++r) ra[r] = rb[r] = 0.0;
    }
    double x[SEG];
    __syncthreads();
    // ---- row phase
#pragma unroll
    for (int c = 0; c < SEG; ++c) x[c] = X[lane][seg * SEG + c];
    {
      double pre[KY + 1], suf[KY + 1];
      seg_summaries<KY>(x, pre, suf);
#pragma unroll
      for (int r = 0; r <= KY; ++r) {
        sums[0][seg][lane][r] = pre[r];
        sums[1][seg][lane][r] = suf[r];
      }
    }
    __syncthreads();
    double out[SEG];
    {
      for (int sg = 0; sg < seg; ++sg) {
        gwk::pascal_shift<KY>(ra, (double)SEG);
#pragma unroll
        for (int r = 0; r <= KY; ++r) ra[r] += sums[0][sg][lane][r];
      }
      for (int sg = NSEG - 1; sg > seg; --sg) {
        gwk::pascal_shift<KY>(rb, (double)SEG);
#pragma unroll
        for (int r = 0; r <= KY; ++r) rb[r] += sums[1][sg][lane][r];
      }
      seg_sweep<KY>(x, ra, rb, out);
#pragma unroll
      for (int c = 0; c < SEG; ++c) X[lane][seg * SEG + c] = out[c];
    }
    __syncthreads();
    // ---- column phase
#pragma unroll
    for (int i = 0; i < SEG; ++i) x[i] = X[seg * SEG + i][lane];
    {
      double pre[KX + 1], suf[KX + 1];
      seg_summaries<KX>(x, pre, suf);
#pragma unroll
      for (int r = 0; r <= KX; ++r) {
        sums[0][seg][lane][r] = pre[r];
        sums[1][seg][lane][r] = suf[r];
      }
    }
    __syncthreads();
    for (int sg = 0; sg < seg; ++sg) {
      gwk::pascal_shift<KX>(ca, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KX; ++r) ca[r] += sums[0][sg][lane][r];
    }
    for (int sg = NSEG - 1; sg > seg; --sg) {
      gwk::pascal_shift<KX>(cb, (double)SEG);
#pragma unroll
      for (int r = 0; r <= KX; ++r) cb[r] += sums[1][sg][lane][r];
    }
    seg_sweep<KX>(x, ca, cb, out);
    // every lane stores (rows and columns past the matrix are dropped by the
    // buffer range check): no branch around the stores
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
      const int r = seg * SEG + i;  // wave-uniform
      const int row = min(js + r, M - 1);
      double v = (c1[row] + c2v) - s2 * out[i];
      if constexpr (FG) {
        const double d = epi.fa[row] - fbv;
        v = fma(epi.a, v, epi.b * (d * d));
      }
      gwk::buffer_store_f64<2>(v, gwk::buffer_rsrc(G + (int64_t)row * ldG + qs),
                            (r < h && lane < w) ? lane * 8 : gwk::kOffDrop);
    }
    __syncthreads();
  };
  if ((int)blockIdx.x < ntiles) {
    load_tile(pf, blockIdx.x);
    // as many (dropped) stores after the first prefetch as a tile issues after
    // its prefetch, so the wait for a prefetched tile never covers the stores
    // (distinct, non-adjacent offsets: identical stores would be merged into
    // one, adjacent ones into wider stores)
#pragma unroll
    for (int u = 0; u < SEG; ++u) gwk::buffer_store_f64(0.0, gwk::buffer_rsrc(G), gwk::kOffDrop + 64 * u);
  }
  for (int tile = blockIdx.x; tile < ntiles; tile += stride) body(tile);
}

int cu_count() {
  static const int ncu = [] {  // thread-safe one-time initialisation
    int dev = 0, n = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      n = prop.multiProcessorCount;
    return n > 0 ? n : 256;
  }();
  return ncu;
}

// Persistent grid: as many blocks as are resident at once (occupancy of the
// kernel on this device), at most one per tile.
template <class K>
int persistent_blocks(K kernel, int ntiles) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int g = cu_count() * per_cu;
  return ntiles < g ? ntiles : g;
}

template <int KX, int KY>
gw_status run_fast1d(const Layout& L, const double* T, int64_t ldT, double* G, int64_t ldG,
                     const double* c1, const double* c2, double s2, double* rowmom,
                     double* colmom, double* acarry, const gwr::Epilogue* epi, gwr::SideJoin& sj,
                     hipStream_t s) {
  const int M = (int)L.M, N = (int)L.N;
  const int ntiles = L.nI * L.nJ;
  {
    gwr::ProfScope ps(gwr::kFamFastCarry, s);
    k_p1_moments<KX, KY><<<persistent_blocks(k_p1_moments<KX, KY>, ntiles), 256, 0, s>>>(T, ldT, M, N, L.nI, L.nJ, rowmom, colmom);
    auto sblocks = [&](int ln) { return (unsigned)((M + ln - 1) / ln + (N + ln - 1) / ln); };
    const int64_t lines = (int64_t)M + N;
    if (lines >= SCAN_ONE_THREAD_LINES)
      k_p2_scan<KX, KY, 64, 1><<<sblocks(64), 64, 0, s>>>(M, N, L.nI, L.nJ, rowmom, colmom);
    else if (lines >= SCAN_ONE_THREAD_LINES / 2)
      k_p2_scan<KX, KY, 32, 8><<<sblocks(32), 256, 0, s>>>(M, N, L.nI, L.nJ, rowmom, colmom);
    else
      k_p2_scan<KX, KY, 16, SCAN_MAXCH><<<sblocks(16), 16 * SCAN_MAXCH, 0, s>>>(M, N, L.nI, L.nJ,
                                                                               rowmom, colmom);
    const int nvec = 2 * L.nI * (KX + 1);
    const size_t shm = (size_t)L.nJ * 2 * (KY + 1) * sizeof(double);
    if (L.nJ <= 4 * P2C_TILES) {
      k_p2c<KX, KY, 4><<<nvec, 256, shm, s>>>(N, L.nJ, colmom, acarry);
    } else {
      // dynamic LDS above the default limit
      if (gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_p2c<KX, KY, 0>), shm) != GW_OK)
        return GW_EDEVICE;
      k_p2c<KX, KY, 0><<<nvec, 256, shm, s>>>(N, L.nJ, colmom, acarry);
    }
  }
  // the constant terms (maybe on a side stream) are read from here on
  if (sj.join() != GW_OK) return GW_EDEVICE;
  {
    gwr::ProfDispatch pd(gwr::kFamFastMain);
    if (epi)
      hipExtLaunchKernelGGL(k_p3_tile<KX, KY, true>,
                            dim3(persistent_blocks(k_p3_tile<KX, KY, true>, ntiles)), dim3(256), 0,
                            s, pd.b, pd.e, 0, T, ldT, M, N, L.nI, L.nJ, rowmom, acarry, c1, c2, s2,
                            G, ldG, *epi);
    else
      hipExtLaunchKernelGGL(k_p3_tile<KX, KY, false>,
                            dim3(persistent_blocks(k_p3_tile<KX, KY, false>, ntiles)), dim3(256),
                            0, s, pd.b, pd.e, 0, T, ldT, M, N, L.nI, L.nJ, rowmom, acarry, c1, c2,
                            s2, G, ldG, gwr::Epilogue{});
  }
  return gwr::last_launch_status();
}

template <int KX>
gw_status dispatch_ky(int ky, const Layout& L, const double* T, int64_t ldT, double* G,
                      int64_t ldG, const double* c1, const double* c2, double s2, double* rm,
                      double* cm, double* am, const gwr::Epilogue* epi, gwr::SideJoin& sj,
                      hipStream_t s) {
  switch (ky) {
    case 1: return run_fast1d<KX, 1>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 2: return run_fast1d<KX, 2>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 3: return run_fast1d<KX, 3>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 4: return run_fast1d<KX, 4>(L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
  }
  return GW_EUNSUPPORTED;
}

// ------------------------------------------------ image operator (2D rows)
// For 2D grids whose image fits one 64 x 64 or 96 x 96 tile: each row of `in`
// is an H x W image (zero padded to the tile) and receives
//   sum_t coef_t  D_H^{o mh_t} X D_W^{o mw_t}   (D^{o0} = J, the diagonal included),
// the Kronecker expansion of Sec. 3.1 applied to one image.  A block owns one
// row: thread (line, seg) applies the recursion to one segment of a line (16
// entries of a 64-point line, 12 of a 96-point one), with the carries of the
// other segments combined through LDS (as the tile sweep does), first along
// the image rows (exponent mw), the result staged in LDS, then along the image
// columns (exponent mh), summed over the terms in registers.  The thread keeps
// its row segment of the image in registers for every term.
constexpr int IMG_MAX = 96;  // longest image side of the LDS image operator

struct ImgTerms {
  int n;
  int coef[GW_KMAX + 1], mh[GW_KMAX + 1], mw[GW_KMAX + 1];
};

// An image of up to ITS x ITS points: thread (lane, seg) holds segment seg
// (ITS / NS entries) of line `lane`; NS ITS threads.  64-point images take 4
// segments of 16, 96-point ones 8 of 12 (fewer registers per thread).
template <int ITS>
struct ImgShape {
  static constexpr int NS = ITS == 64 ? 4 : 8, SL = ITS / NS, NT = NS * ITS;
};

template <int K, int ITS>
GW_DEV void img_line(const double (&x)[ImgShape<ITS>::SL], double (&out)[ImgShape<ITS>::SL],
                     double (*sums)[ImgShape<ITS>::NS][ITS][GW_KMAX + 1], int lane, int seg) {
  constexpr int NS = ImgShape<ITS>::NS, SL = ImgShape<ITS>::SL;
  double pre[K + 1], suf[K + 1];
  seg_summaries<K>(x, pre, suf);
#pragma unroll
  for (int r = 0; r <= K; ++r) {
    sums[0][seg][lane][r] = pre[r];
    sums[1][seg][lane][r] = suf[r];
  }
  __syncthreads();
  double a[K + 1], b[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) a[r] = b[r] = 0.0;
  for (int sg = 0; sg < seg; ++sg) {
    gwk::pascal_shift<K>(a, (double)SL);
#pragma unroll
    for (int r = 0; r <= K; ++r) a[r] += sums[0][sg][lane][r];
  }
  for (int sg = NS - 1; sg > seg; --sg) {
    gwk::pascal_shift<K>(b, (double)SL);
#pragma unroll
    for (int r = 0; r <= K; ++r) b[r] += sums[1][sg][lane][r];
  }
  seg_sweep<K>(x, a, b, out);
  if constexpr (K == 0) {  // J: the entry itself belongs to the line sum
#pragma unroll
    for (int c = 0; c < SL; ++c) out[c] += x[c];
  }
  __syncthreads();  // the summaries are read before the next line pass writes them
}

template <int ITS>
GW_DEV void img_line_m(int m, const double (&x)[ImgShape<ITS>::SL],
                       double (&out)[ImgShape<ITS>::SL],
                       double (*sums)[ImgShape<ITS>::NS][ITS][GW_KMAX + 1], int lane, int seg) {
  switch (m) {
    case 0: img_line<0, ITS>(x, out, sums, lane, seg); break;
    case 1: img_line<1, ITS>(x, out, sums, lane, seg); break;
    case 2: img_line<2, ITS>(x, out, sums, lane, seg); break;
    case 3: img_line<3, ITS>(x, out, sums, lane, seg); break;
    default: img_line<4, ITS>(x, out, sums, lane, seg); break;
  }
}

template <int ITS>
__global__ __launch_bounds__(ImgShape<ITS>::NT) void k_img_rowop(const double* __restrict__ in,
                                                       int64_t ldi, int H, int W, ImgTerms terms,
                                                       double* __restrict__ out, int64_t ldo) {
  constexpr int NT = ImgShape<ITS>::NT, NS = ImgShape<ITS>::NS, SL = ImgShape<ITS>::SL;
  __shared__ double Y[ITS][ITS + 1];
  __shared__ double sums[2][NS][ITS][GW_KMAX + 1];
  __shared__ double vec[4][ITS];  // row sums, column sums, D^m (row sums), (column sums) D^m
  const int t = threadIdx.x, lane = t % ITS;
  // with 64-point lines a segment is a wave: keep its index in a scalar register
  const int seg = ITS == 64 ? __builtin_amdgcn_readfirstlane(t >> 6) : t / ITS;
  const int64_t row = blockIdx.x;
  const double* src = in + row * ldi;
  // the image into LDS (zero padded to the tile; consecutive threads read
  // consecutive entries of an image row), then the thread's row segment: image
  // row `lane`, columns seg*SL + c
  {
    // all loads issued before any is used (indices clamped into the image)
    constexpr int PER = ITS * ITS / NT;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + NT * u, r = e / ITS, c = e % ITS;
      v[u] = src[min(r, H - 1) * W + min(c, W - 1)];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + NT * u, r = e / ITS, c = e % ITS;
      Y[r][c] = (r < H && c < W) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  double xr[SL];
#pragma unroll
  for (int c = 0; c < SL; ++c) xr[c] = Y[lane][seg * SL + c];
  double acc[SL];
#pragma unroll
  for (int i = 0; i < SL; ++i) acc[i] = 0.0;
  double o[SL], x[SL];
  // Terms with a J factor act on the image's line sums only:
  //   D_H^{o m} X J = (D^{o m} X 1) 1^T,   J X D_W^{o m} = 1 (1^T X D^{o m}).
  // Row and column sums first (segments, then the segments in order).
  {
    double rp = 0.0;
#pragma unroll
    for (int c = 0; c < SL; ++c) rp += xr[c];
    sums[0][seg][lane][0] = rp;
    double cp = 0.0;
#pragma unroll
    for (int i = 0; i < SL; ++i) cp += Y[seg * SL + i][lane];
    sums[1][seg][lane][0] = cp;
    __syncthreads();
    if (seg < 2) {
      double v = sums[seg][0][lane][0];
#pragma unroll
      for (int sg = 1; sg < NS; ++sg) v += sums[seg][sg][lane][0];
      vec[seg][lane] = v;
    }
    __syncthreads();
  }
  for (int tm = 0; tm < terms.n; ++tm) {
    const int mh = terms.mh[tm], mw = terms.mw[tm];
    const double cf = (double)terms.coef[tm];
    if (mw == 0 || mh == 0) {
      // one line operator on a vector of line sums: vec[2] = D^{mh} rowsums
      // (mw = 0), vec[3] = colsums D^{mw} (mh = 0); then broadcast
      const int m = mw == 0 ? mh : mw;
      const int which = mw == 0 ? 0 : 1;
      {
        // output `lane`: thread (lane, seg) sums the segment's SL sums, the
        // segments are added in order
        double v = 0.0;
#pragma unroll
        for (int jj = 0; jj < SL; ++jj) {
          const int j = seg * SL + jj;
          const int d = lane > j ? lane - j : j - lane;
          double w = 1.0;
          for (int u = 0; u < m; ++u) w *= (double)d;
          v = fma(w, vec[which][j], v);
        }
        sums[0][seg][lane][0] = v;
      }
      __syncthreads();
      if (seg == 0) {
        double v = sums[0][0][lane][0];
#pragma unroll
        for (int sg = 1; sg < NS; ++sg) v += sums[0][sg][lane][0];
        vec[2 + which][lane] = v;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < SL; ++i)
        acc[i] = fma(cf, which == 0 ? vec[2][seg * SL + i] : vec[3][lane], acc[i]);
      __syncthreads();  // vec[2 + which] is rewritten by the next such term
      continue;
    }
    // cross terms: along the image rows: Y[r][.] = (row r) D_W^{o mw}
    img_line_m<ITS>(mw, xr, o, sums, lane, seg);
#pragma unroll
    for (int c = 0; c < SL; ++c) Y[lane][seg * SL + c] = o[c];
    __syncthreads();
    // along the image columns: column `lane`, rows seg*SL + i
#pragma unroll
    for (int i = 0; i < SL; ++i) x[i] = Y[seg * SL + i][lane];
    img_line_m<ITS>(mh, x, o, sums, lane, seg);
#pragma unroll
    for (int i = 0; i < SL; ++i) acc[i] = fma(cf, o[i], acc[i]);
  }
  double* dst = out + row * ldo;
#pragma unroll
  for (int i = 0; i < SL; ++i) {
    const int r = seg * SL + i;
    if (r < H && lane < W) dst[r * W + lane] = acc[i];
  }
}

// ------------------------------------------------ 3D image operator
// For 3D grids with every axis of at most SEG points: each row of `in` is a
// Z x H x W array receiving sum_t coef_t (A_z^{a_t} (x) A_r^{b_t} (x) A_c^{c_t}) x,
// A^{e} = [|i-j|^e] (A^0 = J), one multinomial term per (a, b, c) (squared
// Euclidean: the three squared axes).  One block per row: the array and one
// temporary in LDS (line stride W + 1); a thread per line loads the line (at
// most SEG entries) into registers, applies the recursion of one segment with
// zero carries and writes the line back (the second pass in place: the lines
// of a pass are disjoint); the last axis' results are summed over the terms in
// registers.
struct Img3Terms {
  int n;
  int coef[15], ez[15], eh[15], ew[15];
};

template <int K>
GW_DEV void line16(const double (&x)[SEG], double (&out)[SEG]) {
  double a[K + 1], b[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) a[r] = b[r] = 0.0;
  seg_sweep<K>(x, a, b, out);
  if constexpr (K == 0) {  // J: the entry itself belongs to the line sum
#pragma unroll
    for (int c = 0; c < SEG; ++c) out[c] += x[c];
  }
}

GW_DEV void line16_m(int m, const double (&x)[SEG], double (&out)[SEG]) {
  switch (m) {
    case 0: line16<0>(x, out); break;
    case 1: line16<1>(x, out); break;
    case 2: line16<2>(x, out); break;
    case 3: line16<3>(x, out); break;
    default: line16<4>(x, out); break;
  }
}

constexpr int I3_NT = 256;

__global__ __launch_bounds__(I3_NT) void k_img3_rowop(const double* __restrict__ in, int64_t ldi,
                                                      int Z, int H, int W, Img3Terms terms,
                                                      double* __restrict__ out, int64_t ldo) {
  extern __shared__ double l3[];
  const int Wp = W + 1, hwp = H * Wp, np = Z * hwp, hw = H * W, n = Z * hw;
  double* xs = l3;
  double* t1 = l3 + np;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const double* src = in + row * ldi;
  for (int e = tid; e < n; e += I3_NT) {
    const int z = e / hw, rem = e - z * hw, r = rem / W, c = rem - r * W;
    xs[z * hwp + r * Wp + c] = src[e];
  }
  // the Z-line (r, c) = tid of the last pass is the thread's output (hw <= I3_NT)
  double acc[SEG];
#pragma unroll
  for (int i = 0; i < SEG; ++i) acc[i] = 0.0;
  double x[SEG], o[SEG];
  __syncthreads();
  for (int tm = 0; tm < terms.n; ++tm) {
    // along W: the Z*H lines (z, r), contiguous
    for (int l = tid; l < Z * H; l += I3_NT) {
      const int base = (l / H) * hwp + (l % H) * Wp;
#pragma unroll
      for (int c = 0; c < SEG; ++c) x[c] = c < W ? xs[base + c] : 0.0;
      line16_m(terms.ew[tm], x, o);
#pragma unroll
      for (int c = 0; c < SEG; ++c)
        if (c < W) t1[base + c] = o[c];
    }
    __syncthreads();
    // along H: the Z*W lines (z, c), stride W + 1
    for (int l = tid; l < Z * W; l += I3_NT) {
      const int base = (l / W) * hwp + (l % W);
#pragma unroll
      for (int r = 0; r < SEG; ++r) x[r] = r < H ? t1[base + r * Wp] : 0.0;
      line16_m(terms.eh[tm], x, o);
#pragma unroll
      for (int r = 0; r < SEG; ++r)
        if (r < H) t1[base + r * Wp] = o[r];
    }
    __syncthreads();
    // along Z: the H*W lines (r, c), stride H (W + 1), summed over the terms
    if (tid < hw) {
      const int base = (tid / W) * Wp + (tid % W);
#pragma unroll
      for (int z = 0; z < SEG; ++z) x[z] = z < Z ? t1[base + z * hwp] : 0.0;
      line16_m(terms.ez[tm], x, o);
      const double cf = (double)terms.coef[tm];
#pragma unroll
      for (int z = 0; z < SEG; ++z) acc[z] = fma(cf, o[z], acc[z]);
    }
    __syncthreads();  // t1 is rewritten by the next term
  }
  if (tid < hw) {
    double* dst = out + row * ldo;
#pragma unroll
    for (int z = 0; z < SEG; ++z)
      if (z < Z) dst[z * hw + tid] = acc[z];
  }
}

}  // namespace

namespace gwl {

size_t fast1d_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y) {
  Layout L = make_layout(X.n(), Y.n(), X.k1d(), Y.k1d());
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(L.rowmom);
  a.take<double>(L.colmom);
  a.take<double>(L.acarry);
  a.take<double>(X.n());
  a.take<double>(Y.n());
  return a.used;
}

gw_status fast1d(const gwr::Grid& X, const gwr::Grid& Y, const double* p, const double* q,
                 const double* T, int64_t ldT, double* G, int64_t ldG, gwr::Arena& ws,
                 hipStream_t s, const double* c1_pre, const double* c2_pre,
                 const gwr::Epilogue* epi) {
  Layout L = make_layout(X.n(), Y.n(), X.k1d(), Y.k1d());
  double* rm = ws.take<double>(L.rowmom);
  double* cm = ws.take<double>(L.colmom);
  double* am = ws.take<double>(L.acarry);
  double* c1 = ws.take<double>(X.n());
  double* c2 = ws.take<double>(Y.n());
  // the constant terms need only p and q: on a side stream they run beside
  // the moment and carry passes, joined before the tile pass reads them
  gwr::SideJoin sj{(!c1_pre || !c2_pre) ? gwr::side_take(s) : nullptr, s};
  gw_status st =
      resolve_const_terms(X, p, c1_pre, &c1, Y, q, c2_pre, &c2, sj.ss ? sj.ss->side : s);
  if (st != GW_OK) return st;
  const double s2 = 2.0 * (X.hk() * Y.hk());
  switch (L.kx) {
    case 1: return dispatch_ky<1>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 2: return dispatch_ky<2>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 3: return dispatch_ky<3>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
    case 4: return dispatch_ky<4>(L.ky, L, T, ldT, G, ldG, c1, c2, s2, rm, cm, am, epi, sj, s);
  }
  return GW_EUNSUPPORTED;
}

// The image operator on every row of `in` for a 2D grid of at most
// IMG_MAX x IMG_MAX points (GW_EUNSUPPORTED otherwise): 64-point tiles up to
// 64 x 64 (256 threads), 96-point tiles above (768 threads).
gw_status img_rowop(const double* in, int64_t ldi, int64_t rows, const gwr::Grid& g,
                    double* out, int64_t ldo, hipStream_t s) {
  if (g.ndim != 2 || g.H > IMG_MAX || g.W > IMG_MAX) return GW_EUNSUPPORTED;
  ImgTerms tm{};
  if (g.metric == GW_METRIC_SQEUCLID) {
    tm.n = 2;
    tm.coef[0] = 1; tm.mh[0] = 2; tm.mw[0] = 0;
    tm.coef[1] = 1; tm.mh[1] = 0; tm.mw[1] = 2;
  } else {
    tm.n = g.k + 1;
    int cb = 1;  // C(k, r)
    for (int r = 0; r <= g.k; ++r) {
      tm.coef[r] = cb;
      tm.mh[r] = g.k - r;
      tm.mw[r] = r;
      cb = cb * (g.k - r) / (r + 1);
    }
  }
  if (g.H <= TS && g.W <= TS)
    k_img_rowop<TS><<<(unsigned)rows, ImgShape<TS>::NT, 0, s>>>(in, ldi, (int)g.H, (int)g.W, tm,
                                                                out, ldo);
  else
    k_img_rowop<IMG_MAX><<<(unsigned)rows, ImgShape<IMG_MAX>::NT, 0, s>>>(in, ldi, (int)g.H,
                                                                          (int)g.W, tm, out, ldo);
  return gwr::last_launch_status();
}

// The 3D grid operator on every row of `in`, for arrays whose axes have at
// most 16 points (GW_EUNSUPPORTED otherwise).
gw_status img3_rowop(const double* in, int64_t ldi, int64_t rows, const gwr::Grid& g,
                     double* out, int64_t ldo, hipStream_t s) {
  if (g.ndim != 3 || g.Z > SEG || g.H > SEG || g.W > SEG) return GW_EUNSUPPORTED;
  Img3Terms tm{};
  if (g.metric == GW_METRIC_SQEUCLID) {
    tm.n = 3;
    for (int ax = 0; ax < 3; ++ax) {
      tm.coef[ax] = 1;
      tm.ez[ax] = ax == 0 ? 2 : 0;
      tm.eh[ax] = ax == 1 ? 2 : 0;
      tm.ew[ax] = ax == 2 ? 2 : 0;
    }
  } else {
    int fact[GW_KMAX + 1];
    fact[0] = 1;
    for (int u = 1; u <= g.k; ++u) fact[u] = fact[u - 1] * u;
    for (int a = 0; a <= g.k; ++a)
      for (int b = 0; a + b <= g.k; ++b) {
        tm.coef[tm.n] = fact[g.k] / (fact[a] * fact[b] * fact[g.k - a - b]);
        tm.ez[tm.n] = a;
        tm.eh[tm.n] = b;
        tm.ew[tm.n] = g.k - a - b;
        ++tm.n;
      }
  }
  const size_t shm = 2 * (size_t)(g.Z * g.H * (g.W + 1)) * sizeof(double);
  // dynamic LDS above the default
  if (gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_img3_rowop), 160 * 1024) != GW_OK)
    return GW_EDEVICE;
  k_img3_rowop<<<(unsigned)rows, I3_NT, shm, s>>>(in, ldi, (int)g.Z, (int)g.H, (int)g.W, tm, out,
                                                  ldo);
  return gwr::last_launch_status();
}

}  // namespace gwl
