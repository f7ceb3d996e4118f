// Constant terms and the FAST gradient for grids that are not both 1D.
//
// Constant terms c = (D o D) w are evaluated directly, O(n^2) per vector, as
// the paper does once per solve (Sec. 2, "computed once").
//
// 2D grids (Sec. 3.1): the grid operator is a sum of Kronecker products of 1D
// operators on the image axes, D^ = sum_r C(k,r) D_1^{o(k-r)} (x) D_1^{o r}
// (Eq. (2D kronecker)), with D_1^{o0} = J; SQEUCLID is D^{o2} (x) J + J (x) D^{o2}.
//
// Separable path (SQEUCLID, and (l1)^1): every term carries a J factor on one
// image axis, so J is applied first as a sum.  For T viewed as a 4-index
// tensor T[(a,b),(a',b')], B = D^_X T D^_Y is the sum of four broadcasts of
// small matrices S R S, where R are the two-axis marginals of T
// (R1[a][a'] = sum_{b,b'} T, R2[a][b'] = sum_{b,a'} T, R3[b][a'] = sum_{a,b'} T,
// R4[b][b'] = sum_{a,a'} T) and S = [|i-j|^m] on the short axes.  One read of
// T and one write of G.
//
// Generic path (any 1D/2D combination, any k): the grid operator of Y is
// applied to every row of T as an image (all Kronecker terms), the result is
// transposed, the operator of X is applied to its rows, and the final
// transpose writes G with the constant terms.
#include "common.h"
#include "runtime.h"

namespace {

constexpr int NT = 256;

// ------------------------------------------------------------ constant terms
// c[i] = hk^2 * sum_j (d_ij)^2 w_j, d_ij the integer distance of the grid.
// A block of 1024 threads owns 64 outputs; its 16 waves split j into 16
// contiguous ranges and their partial sums are added in wave order.
constexpr int CT_GROUPS = 16;

// Separable form of the same constant term for 2D grids: D^2 / hk^2 is a sum
// of non-negative terms coef_t |dr|^er_t |dc|^ec_t (squared Euclidean:
// dr^4 + 2 dr^2 dc^2 + dc^4; (L1)^k: sum_m C(2k, m) |dr|^m |dc|^(2k-m)), so
// c[(ri, ci)] = hk^2 sum_t coef_t sum_rj |ri - rj|^er_t Z_t[rj][ci] with
// Z_t[rj][ci] = sum_cj |ci - cj|^ec_t w[rj][cj]: O(N (H + W)) work instead of
// O(N^2).  A block owns image column ci: the image of w and tables of the
// powers are staged in LDS, a thread per (term, image row) builds Z_t (summed
// over cj in order) and then its share of c, and the terms are added in order.
struct SepConst {
  int nt;  // number of terms (<= 9)
  int er[9], ec[9];
  double coef[9];
};
constexpr int CS_MAXT = 9;

size_t const_sep_lds(int H, int W, int nt) {
  return ((size_t)H * (W + 1) + (size_t)nt * (3 * H + W)) * sizeof(double);
}

__global__ __launch_bounds__(256) void k_const_sep(SepConst sc, int H, int W, double hk2,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ c) {
  extern __shared__ double sh[];
  const int nt = sc.nt;
  double* img = sh;                       // [H][W + 1] (padded rows)
  double* z = img + (int64_t)H * (W + 1);  // [nt][H]  Z_t[rj] of this block's column
  double* part = z + nt * H;              // [nt][H]  per-term sums of each row ri
  double* pwr = part + nt * H;            // [nt][H]  d^er_t, d < H
  double* pwc = pwr + nt * H;             // [nt][W]  d^ec_t, d < W
  const int ci = blockIdx.x, n = H * W, tid = threadIdx.x;
  // the image of w, loads issued 8 at a time before they are stored
  for (int p0 = 0; p0 < n; p0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = w[min(p0 + tid + u * 256, n - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = p0 + tid + u * 256;
      if (p < n) img[(p / W) * (W + 1) + p % W] = v[u];
    }
  }
  for (int x = tid; x < nt * H; x += 256) pwr[x] = gwk::ipow((double)(x % H), sc.er[x / H]);
  for (int x = tid; x < nt * W; x += 256) pwc[x] = gwk::ipow((double)(x % W), sc.ec[x / W]);
  __syncthreads();
  // Z_t[rj] = sum_cj |ci - cj|^ec_t w[rj][cj], summed over cj in order
  for (int x = tid; x < nt * H; x += 256) {
    const int t = x / H, rj = x % H;
    const double* pw = pwc + t * W;
    const double* row = img + rj * (W + 1);
    double acc = 0.0;
    for (int cj = 0; cj < W; ++cj) acc = fma(pw[abs(ci - cj)], row[cj], acc);
    z[x] = acc;
  }
  __syncthreads();
  // per term: sum_rj |ri - rj|^er_t Z_t[rj]
  for (int x = tid; x < nt * H; x += 256) {
    const int t = x / H, ri = x % H;
    const double* pw = pwr + t * H;
    const double* zt = z + t * H;
    double st = 0.0;
    for (int rj = 0; rj < H; ++rj) st = fma(pw[abs(ri - rj)], zt[rj], st);
    part[x] = st;
  }
  __syncthreads();
  for (int ri = tid; ri < H; ri += 256) {
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s = fma(sc.coef[t], part[t * H + ri], s);
    c[(int64_t)ri * W + ci] = hk2 * s;
  }
}

__global__ __launch_bounds__(1024) void k_const_term(int metric, int k, int H, int W, double hk,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ c) {
  __shared__ double part[CT_GROUPS][64];
  const int n = H * W;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (i < n) {
    const int ri = i / W, ci = i % W;
    const int chunk = (n + CT_GROUPS - 1) / CT_GROUPS;
    const int j0 = grp * chunk, j1 = min(n, j0 + chunk);
    int rj = j0 / W, cj = j0 % W;
    for (int j = j0; j < j1; ++j) {
      const int dr = abs(ri - rj), dc = abs(ci - cj);
      double d;
      if (metric == GW_METRIC_SQEUCLID) {
        d = (double)(dr * dr + dc * dc);
      } else {
        const double e = (double)(dr + dc);
        d = e;
        for (int u = 1; u < k; ++u) d *= e;
      }
      const double D = hk * d;
      acc = fma(D * D, w[j], acc);
      if (++cj == W) {
        cj = 0;
        ++rj;
      }
    }
  }
  part[grp][lane] = acc;
  __syncthreads();
  if (grp == 0 && i < n) {
    double s = part[0][lane];
#pragma unroll
    for (int g = 1; g < CT_GROUPS; ++g) s += part[g][lane];
    c[i] = s;
  }
}

// 3D grids: c_i = sum_j (hk d(i,j))^2 w_j directly, d the (l1)^k or squared
// Euclidean distance of the (z, r, c) coordinates.  A block of 1024 threads
// owns CT3_OUT outputs (lane) and splits j over 64 groups; w passes through
// LDS in chunks, each chunk split into 64 contiguous group ranges; a group's
// partial runs over its ranges in chunk order and the groups' partials are
// added in group order.
constexpr int CT3_OUT = 16, CT3_GRP = 64, CT3_CHUNK = 8192;
__global__ __launch_bounds__(1024) void k_const_term3(int metric, int k, int Z, int H, int W,
                                                       double hk, const double* __restrict__ w,
                                                       double* __restrict__ c) {
  __shared__ double wc[CT3_CHUNK];
  __shared__ double part[CT3_GRP][CT3_OUT];
  const int hw = H * W, n = Z * hw;
  const int lane = threadIdx.x & (CT3_OUT - 1), grp = threadIdx.x / CT3_OUT;
  const int i = blockIdx.x * CT3_OUT + lane;
  const int ii = min(i, n - 1);
  const int zi = ii / hw, ri = (ii % hw) / W, ci = ii % W;
  double acc = 0.0;
  for (int j0 = 0; j0 < n; j0 += CT3_CHUNK) {
    const int len = min(CT3_CHUNK, n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < len; e += 1024) wc[e] = w[j0 + e];
    __syncthreads();
    const int glen = (len + CT3_GRP - 1) / CT3_GRP;
    const int a0 = grp * glen, a1 = min(len, a0 + glen);
    if (a0 < a1) {
      const int j = j0 + a0;
      int zj = j / hw, rj = (j % hw) / W, cj = j % W;
      for (int a = a0; a < a1; ++a) {
        const int dz = abs(zi - zj), dr = abs(ri - rj), dc = abs(ci - cj);
        double d;
        if (metric == GW_METRIC_SQEUCLID) {
          d = (double)(dz * dz + dr * dr + dc * dc);
        } else {
          const double e = (double)(dz + dr + dc);
          d = e;
          for (int u = 1; u < k; ++u) d *= e;
        }
        const double D = hk * d;
        acc = fma(D * D, wc[a], acc);
        if (++cj == W) {
          cj = 0;
          if (++rj == H) {
            rj = 0;
            ++zj;
          }
        }
      }
    }
  }
  part[grp][lane] = acc;
  __syncthreads();
  if (grp == 0 && i < n) {
    double s = part[0][lane];
    for (int g = 1; g < CT3_GRP; ++g) s += part[g][lane];
    c[i] = s;
  }
}

// 1D grids: c = hk^2 [|i-j|^{2k}] w by the recursion with exponent K2 = 2k,
// one block per vector (up to two vectors per launch: blockIdx.x selects the
// job).  Thread t owns entries [16 t, 16 t + 16).  Segment summaries (prefix
// state at the segment end, suffix state at its start - 1) are scanned along
// the block in each direction: a shuffle scan inside each wave, then every
// thread folds the totals of the waves before it, always shifting a state over
// the span it crosses (all weights non-negative).  Each thread then sweeps its
// segment with its carries.  n <= 16 NT.
constexpr int C1_SEG = 16;

struct ConstJob {
  int n;
  double hk2;
  const double* w;
  double* c;
};

template <int K2>
GW_DEV void shfl_state(const double (&v)[K2 + 1], double (&o)[K2 + 1], int src) {
#pragma unroll
  for (int r = 0; r <= K2; ++r) o[r] = __shfl(v[r], src, 64);
}

template <int K2, int NT>
__global__ __launch_bounds__(NT) void k_const_1d(ConstJob j0, ConstJob j1) {
  constexpr int NW = NT / 64;
  __shared__ double wtot[2][NW][K2 + 1];
  const ConstJob jb = blockIdx.x == 0 ? j0 : j1;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double x[C1_SEG];
#pragma unroll
  for (int e = 0; e < C1_SEG; ++e) {
    const int i = t * C1_SEG + e;
    x[e] = i < jb.n ? jb.w[i] : 0.0;
  }
  double pre[K2 + 1], suf[K2 + 1];
#pragma unroll
  for (int r = 0; r <= K2; ++r) pre[r] = suf[r] = 0.0;
#pragma unroll
  for (int e = 0; e < C1_SEG; ++e) {
    double wp = 1.0, ws = 1.0;
#pragma unroll
    for (int r = 0; r <= K2; ++r) {
      pre[r] = fma(wp, x[e], pre[r]);
      suf[r] = fma(ws, x[e], suf[r]);
      wp *= (double)(C1_SEG - e);
      ws *= (double)(e + 1);
    }
  }
  // inclusive scans in scan order: dir 0 left to right, dir 1 right to left
  double inc[2][K2 + 1];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int pos = dir == 0 ? lane : 63 - lane;  // position in the wave, scan order
    double v[K2 + 1];
#pragma unroll
    for (int r = 0; r <= K2; ++r) v[r] = dir == 0 ? pre[r] : suf[r];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      double o[K2 + 1];
      shfl_state<K2>(v, o, dir == 0 ? lane - d : lane + d);
      if (pos >= d) {
        gwk::pascal_shift<K2>(o, (double)(C1_SEG * d));
#pragma unroll
        for (int r = 0; r <= K2; ++r) v[r] += o[r];
      }
    }
    const int wpos = dir == 0 ? wv : NW - 1 - wv;  // wave position, scan order
    if (pos == 63) {
#pragma unroll
      for (int r = 0; r <= K2; ++r) wtot[dir][wpos][r] = v[r];
    }
#pragma unroll
    for (int r = 0; r <= K2; ++r) inc[dir][r] = v[r];
  }
  __syncthreads();
  double a[K2 + 1], b[K2 + 1];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int pos = dir == 0 ? lane : 63 - lane;
    const int wpos = dir == 0 ? wv : NW - 1 - wv;
    // state at the end of the previous waves (scan order)
    double acc[K2 + 1];
#pragma unroll
    for (int r = 0; r <= K2; ++r) acc[r] = 0.0;
    for (int w2 = 0; w2 < wpos; ++w2) {
      gwk::pascal_shift<K2>(acc, (double)(64 * C1_SEG));
#pragma unroll
      for (int r = 0; r <= K2; ++r) acc[r] += wtot[dir][w2][r];
    }
    // exclusive state of this thread: the inclusive value of the previous
    // position in the wave, plus the earlier waves shifted up to this segment
    double ex[K2 + 1];
    shfl_state<K2>(inc[dir], ex, dir == 0 ? lane - 1 : lane + 1);
    gwk::pascal_shift<K2>(acc, (double)(C1_SEG * pos));
#pragma unroll
    for (int r = 0; r <= K2; ++r) {
      const double e = pos > 0 ? ex[r] : 0.0;
      if (dir == 0) a[r] = e + acc[r];
      else b[r] = e + acc[r];
    }
  }
  double out[C1_SEG];
#pragma unroll
  for (int e = 0; e < C1_SEG; ++e) {
    out[e] = a[K2];
    gwk::pascal_step<K2>(a, x[e]);
  }
#pragma unroll
  for (int e = C1_SEG - 1; e >= 0; --e) {
    out[e] += b[K2];
    gwk::pascal_step<K2>(b, x[e]);
  }
#pragma unroll
  for (int e = 0; e < C1_SEG; ++e) {
    const int i = t * C1_SEG + e;
    if (i < jb.n) jb.c[i] = jb.hk2 * out[e];
  }
}

template <int K2>
void launch_const_1d(int nblocks, int nmax, ConstJob j0, ConstJob j1, hipStream_t s) {
  if (nmax <= 256 * C1_SEG) k_const_1d<K2, 256><<<nblocks, 256, 0, s>>>(j0, j1);
  else k_const_1d<K2, 1024><<<nblocks, 1024, 0, s>>>(j0, j1);
}

// ---------------------------------------------------------------- transpose
// out[j][i] = in[i][j] (rows x cols input); with epilogue when c1 != null:
// out[j][i] = (c1[j] + c2[i]) - s2 * in[i][j].
__global__ __launch_bounds__(NT) void k_transpose(const double* __restrict__ in, int64_t ldi,
                                                   int64_t rows, int64_t cols,
                                                   double* __restrict__ out, int64_t ldo,
                                                   const double* __restrict__ c1,
                                                   const double* __restrict__ c2, double s2) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, c = c0 + tx;
    tile[y][tx] = (r < rows && c < cols) ? in[r * ldi + c] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t orow = c0 + y, ocol = r0 + tx;  // out[orow][ocol] = in[ocol][orow]
    if (orow < cols && ocol < rows) {
      const double v = tile[tx][y];
      out[orow * ldo + ocol] = c1 ? (c1[orow] + c2[ocol]) - s2 * v : v;
    }
  }
}

// ------------------------------------------------ 1D operator on a strided line
// y[i*ys] (+)= coef * sum_j |i-j|^m x[j*xs] for i < L, via the recursion; m = 0
// means J (total sum).  Sequential, one thread per line.
template <int K>
__device__ void line_apply(const double* x, int64_t xs, double* y, int64_t ys, int64_t L,
                           double coef, bool accumulate) {
  double a[K + 1], b[K + 1];
#pragma unroll
  for (int r = 0; r <= K; ++r) a[r] = b[r] = 0.0;
  // suffix pass writes, prefix pass adds
  for (int64_t i = L - 1; i >= 0; --i) {
    const double v = coef * b[K];
    y[i * ys] = accumulate ? y[i * ys] + v : v;
    gwk::pascal_step<K>(b, x[i * xs]);
  }
  for (int64_t i = 0; i < L; ++i) {
    y[i * ys] += coef * a[K];
    gwk::pascal_step<K>(a, x[i * xs]);
  }
}

__device__ void line_sum(const double* x, int64_t xs, double* y, int64_t ys, int64_t L,
                         double coef, bool accumulate) {
  double s = 0.0;
  for (int64_t i = 0; i < L; ++i) s += x[i * xs];
  s *= coef;
  for (int64_t i = 0; i < L; ++i) y[i * ys] = accumulate ? y[i * ys] + s : s;
}

__device__ void line_op(int m, const double* x, int64_t xs, double* y, int64_t ys, int64_t L,
                        double coef, bool acc) {
  switch (m) {
    case 0: line_sum(x, xs, y, ys, L, coef, acc); break;
    case 1: line_apply<1>(x, xs, y, ys, L, coef, acc); break;
    case 2: line_apply<2>(x, xs, y, ys, L, coef, acc); break;
    case 3: line_apply<3>(x, xs, y, ys, L, coef, acc); break;
    case 4: line_apply<4>(x, xs, y, ys, L, coef, acc); break;
  }
}

// ------------------------------------------- 1D operator on rows, one wave each
// y = D^m x for every row x of `in` (a 1D grid of unit spacing, m >= 1), with
// the recursion of Sec. 3, Eq. (1d recursive relation) cut into pieces.  A
// row is taken in chunks of 64 runs of LE entries, one run per lane.  The
// recursion is linear in (state, entry), so the state after a run is the
// state carried in, advanced LE positions with no entry (pascal_shift), plus
// the state the run's own entries build from zero: the lanes' own states
// combine by a scan over the wave and the chunks by a carry.  The suffix half
// (entries to the right) runs first, from the last chunk down, keeping the
// carry that enters each chunk in LDS; the prefix half then runs from the
// first chunk up, and each entry of y = prefix + suffix is written once.
constexpr int LE = 8;                            // entries per lane and chunk
constexpr int LCH = 64 * LE;                     // entries per chunk
constexpr int LMAXCH = (65535 + LCH - 1) / LCH;  // chunks of the longest axis
constexpr int LWAVES = 4;                        // rows per block

// Inclusive scan of run states over the wave: towards higher lanes (UP, the
// prefix half) or towards lower lanes (the suffix half).
template <int K, bool UP>
__device__ void wave_scan_runs(double (&a)[K + 1], int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double n[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) n[r] = UP ? __shfl_up(a[r], d, 64) : __shfl_down(a[r], d, 64);
    gwk::pascal_shift<K>(n, (double)(d * LE));
    if (UP ? lane >= d : lane + d < 64) {
#pragma unroll
      for (int r = 0; r <= K; ++r) a[r] += n[r];
    }
  }
}

template <int K>
__global__ __launch_bounds__(64 * LWAVES) void k_line_rows(const double* __restrict__ in,
                                                            int64_t ldi, int64_t rows, int64_t W,
                                                            double* __restrict__ out, int64_t ldo) {
  __shared__ double buf[LWAVES][LCH + 64];         // a chunk; run l at l * (LE + 1)
  __shared__ double carry[LWAVES][LMAXCH][K + 1];  // suffix state entering each chunk
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * LWAVES + wv;
  const bool live = row < rows;  // every wave runs the loops: the barriers are block-wide
  const double* x = in + (live ? row : 0) * ldi;
  const int nch = (int)((W + LCH - 1) / LCH);
  double* b = buf[wv];
  auto load = [&](int c, double (&v)[LE]) {
    const int64_t c0 = (int64_t)c * LCH;
#pragma unroll
    for (int e = 0; e < LE; ++e) {
      const int i = e * 64 + lane;
      const int64_t j = c0 + i;
      b[i + i / LE] = (live && j < W) ? x[j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < LE; ++e) v[e] = b[lane * (LE + 1) + e];
    __syncthreads();
  };
  double v[LE];
  double cs[K + 1];  // suffix state entering the current chunk from the right
#pragma unroll
  for (int r = 0; r <= K; ++r) cs[r] = 0.0;
  for (int c = nch - 1;; --c) {
    if (lane == 0)
#pragma unroll
      for (int r = 0; r <= K; ++r) carry[wv][c][r] = cs[r];
    if (c == 0) break;
    load(c, v);
    double s[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) s[r] = 0.0;
#pragma unroll
    for (int e = LE - 1; e >= 0; --e) gwk::pascal_step<K>(s, v[e]);
    wave_scan_runs<K, false>(s, lane);
    gwk::pascal_shift<K>(cs, (double)LCH);
#pragma unroll
    for (int r = 0; r <= K; ++r) cs[r] += __shfl(s[r], 0, 64);
  }
  __syncthreads();
  double cp[K + 1];  // prefix state entering the current chunk from the left
#pragma unroll
  for (int r = 0; r <= K; ++r) cp[r] = 0.0;
  for (int c = 0; c < nch; ++c) {
    load(c, v);
    double p[K + 1], s[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) p[r] = s[r] = 0.0;
#pragma unroll
    for (int e = 0; e < LE; ++e) gwk::pascal_step<K>(p, v[e]);
#pragma unroll
    for (int e = LE - 1; e >= 0; --e) gwk::pascal_step<K>(s, v[e]);
    wave_scan_runs<K, true>(p, lane);
    wave_scan_runs<K, false>(s, lane);
    // states entering this lane's run: the lanes before it in the chunk plus
    // the chunk's carry, advanced over the runs in between
    double pn[K + 1], sn[K + 1], tot[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      const double pl = __shfl_up(p[r], 1, 64), sl = __shfl_down(s[r], 1, 64);
      pn[r] = lane > 0 ? pl : 0.0;
      sn[r] = lane < 63 ? sl : 0.0;
      tot[r] = __shfl(p[r], 63, 64);
    }
    double ca[K + 1], cb[K + 1];
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      ca[r] = cp[r];
      cb[r] = carry[wv][c][r];
    }
    gwk::pascal_shift<K>(ca, (double)(lane * LE));
    gwk::pascal_shift<K>(cb, (double)((63 - lane) * LE));
#pragma unroll
    for (int r = 0; r <= K; ++r) {
      pn[r] += ca[r];
      sn[r] += cb[r];
    }
    gwk::pascal_shift<K>(cp, (double)LCH);
#pragma unroll
    for (int r = 0; r <= K; ++r) cp[r] += tot[r];
    double yv[LE];
#pragma unroll
    for (int e = 0; e < LE; ++e) {
      yv[e] = pn[K];
      gwk::pascal_step<K>(pn, v[e]);
    }
#pragma unroll
    for (int e = LE - 1; e >= 0; --e) {
      yv[e] += sn[K];
      gwk::pascal_step<K>(sn, v[e]);
    }
#pragma unroll
    for (int e = 0; e < LE; ++e) b[lane * (LE + 1) + e] = yv[e];
    __syncthreads();
    const int64_t c0 = (int64_t)c * LCH;
    if (live) {
      double* y = out + row * ldo;
#pragma unroll
      for (int e = 0; e < LE; ++e) {
        const int i = e * 64 + lane;
        const int64_t j = c0 + i;
        if (j < W) y[j] = b[i + i / LE];
      }
    }
    __syncthreads();
  }
}

template <int K>
void launch_line_rows(const double* in, int64_t ldi, int64_t rows, int64_t W, double* out,
                      int64_t ldo, hipStream_t s) {
  if (rows <= 0 || W <= 0) return;
  const unsigned nb = (unsigned)((rows + LWAVES - 1) / LWAVES);
  k_line_rows<K><<<nb, 64 * LWAVES, 0, s>>>(in, ldi, rows, W, out, ldo);
}

// y = D^m x on every row (1D grid, unit spacing), m in [1, GW_KMAX].
void line_rows(int m, const double* in, int64_t ldi, int64_t rows, int64_t W, double* out,
               int64_t ldo, hipStream_t s) {
  switch (m) {
    case 1: launch_line_rows<1>(in, ldi, rows, W, out, ldo, s); break;
    case 2: launch_line_rows<2>(in, ldi, rows, W, out, ldo, s); break;
    case 3: launch_line_rows<3>(in, ldi, rows, W, out, ldo, s); break;
    default: launch_line_rows<4>(in, ldi, rows, W, out, ldo, s); break;
  }
}

// Apply the (unscaled) grid operator to each row of `in` (rows x n,
// n = Z*H*W) treating the row as a Z x H x W array (2D and 3D grids); one
// block per row.  `tmp` (and `tmp2` for 3D) are rows x n scratch.
__global__ __launch_bounds__(NT) void k_rowop(const double* __restrict__ in, int64_t ldi,
                                               int64_t rows, int ndim, int k, int metric,
                                               int64_t Z, int64_t H, int64_t W,
                                               double* __restrict__ out, int64_t ldo,
                                               double* __restrict__ tmp,
                                               double* __restrict__ tmp2) {
  const int64_t row = blockIdx.x;
  const double* x = in + row * ldi;
  double* y = out + row * ldo;
  const int64_t hw = H * W;
  double* t = tmp + row * (Z * hw);
  const int tid = threadIdx.x;
  if (ndim == 3) {
    // (l1)^k: (dz + dr + dc)^k = sum over a + b + c = k of k!/(a! b! c!) dz^a dr^b dc^c,
    // one Kronecker term per (a, b, c); SQEUCLID: the three squared axes
    constexpr int MAXT = (GW_KMAX + 1) * (GW_KMAX + 2) / 2;
    int nterms = 0;
    int coefs[MAXT], mz[MAXT], mh[MAXT], mw[MAXT];
    if (metric == GW_METRIC_SQEUCLID) {
      for (int ax = 0; ax < 3; ++ax) {
        coefs[ax] = 1;
        mz[ax] = ax == 0 ? 2 : 0;
        mh[ax] = ax == 1 ? 2 : 0;
        mw[ax] = ax == 2 ? 2 : 0;
      }
      nterms = 3;
    } else {
      int fact[GW_KMAX + 1];
      fact[0] = 1;
      for (int u = 1; u <= k; ++u) fact[u] = fact[u - 1] * u;
      for (int a = 0; a <= k; ++a)
        for (int b = 0; a + b <= k; ++b) {
          coefs[nterms] = fact[k] / (fact[a] * fact[b] * fact[k - a - b]);
          mz[nterms] = a;
          mh[nterms] = b;
          mw[nterms] = k - a - b;
          ++nterms;
        }
    }
    double* t2 = tmp2 + row * (Z * hw);
    for (int term = 0; term < nterms; ++term) {
      // along W: the Z*H lines of length W
      for (int64_t l = tid; l < Z * H; l += NT)
        line_op(mw[term], x + l * W, 1, t + l * W, 1, W, 1.0, false);
      __syncthreads();
      // along H: the Z*W lines of stride W
      for (int64_t l = tid; l < Z * W; l += NT) {
        const int64_t off = (l / W) * hw + l % W;
        line_op(mh[term], t + off, W, t2 + off, W, H, 1.0, false);
      }
      __syncthreads();
      // along Z: the H*W lines of stride H*W, accumulated into y
      for (int64_t e = tid; e < hw; e += NT)
        line_op(mz[term], t2 + e, hw, y + e, hw, Z, (double)coefs[term], term > 0);
      __syncthreads();
    }
    return;
  }
  int nterms;
  int coefs[GW_KMAX + 1], mh[GW_KMAX + 1], mw[GW_KMAX + 1];
  if (metric == GW_METRIC_SQEUCLID) {
    nterms = 2;
    coefs[0] = 1; mh[0] = 2; mw[0] = 0;
    coefs[1] = 1; mh[1] = 0; mw[1] = 2;
  } else {
    nterms = k + 1;
    int cb = 1;
    for (int r = 0; r <= k; ++r) {
      coefs[r] = cb;
      mh[r] = k - r;
      mw[r] = r;
      cb = cb * (k - r) / (r + 1);
    }
  }
  for (int term = 0; term < nterms; ++term) {
    // along W (image rows): t = x D^{o mw}
    for (int64_t a = tid; a < H; a += NT) line_op(mw[term], x + a * W, 1, t + a * W, 1, W, 1.0, false);
    __syncthreads();
    // along H (image columns): y (+)= coef D^{o mh} t
    for (int64_t b = tid; b < W; b += NT)
      line_op(mh[term], t + b, W, y + b, W, H, (double)coefs[term], term > 0);
    __syncthreads();
  }
}

// ------------------------------------------------------------ separable path
struct SepGrid {
  int64_t H, W;
  int m;             // exponent of the non-J factor
  double alpha;      // coefficient of D_H^{m} (x) J
  double beta;       // coefficient of J (x) D_W^{m}
};

// U[i][a'] = sum_{b'} T[i][(a',b')], V[i][b'] = sum_{a'} T[i][(a',b')]; one
// block per row of T, row staged in LDS (loads issued 8 at a time before they
// are stored).  Each line sum of the image is split into four quarters summed
// by four adjacent lanes and combined in a fixed order.
constexpr int RR_Q = 4;
__global__ __launch_bounds__(NT) void k_sep_rowreduce(const double* __restrict__ T, int64_t ldT,
                                                       int64_t M, int64_t H2, int64_t W2,
                                                       double* __restrict__ U,
                                                       double* __restrict__ V) {
  extern __shared__ double img[];
  const int64_t i = blockIdx.x;
  const int n2 = (int)(H2 * W2), h2 = (int)H2, w2 = (int)W2;
  const int t = threadIdx.x;
  const double* row = T + i * ldT;
  for (int p0 = 0; p0 < n2; p0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = row[min(p0 + t + u * NT, n2 - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + t + u * NT < n2) img[p0 + t + u * NT] = v[u];
  }
  __syncthreads();
  // row sums of the image: four adjacent lanes per image row
  const int q = t & (RR_Q - 1);
  const int qlen = (w2 + RR_Q - 1) / RR_Q;
  for (int a0 = 0; a0 < h2; a0 += NT / RR_Q) {
    const int a = a0 + t / RR_Q;
    double s = 0.0;
    if (a < h2) {
      const int b0 = q * qlen, b1 = min(w2, b0 + qlen);
      for (int b = b0; b < b1; ++b) s += img[a * w2 + b];
    }
    const double s1 = __shfl_xor(s, 1);
    const double s2 = __shfl_xor(s, 2);
    const double s3 = __shfl_xor(s, 3);
    // lane q = 0 holds quarter 0; fixed order (q0 + q1) + (q2 + q3)
    if (q == 0 && a < h2) U[i * H2 + a] = (s + s1) + (s2 + s3);
  }
  // column sums: four adjacent lanes per image column, a quarter of the rows each
  const int hlen = (h2 + RR_Q - 1) / RR_Q;
  for (int b0 = 0; b0 < w2; b0 += NT / RR_Q) {
    const int b = b0 + t / RR_Q;
    double s = 0.0;
    if (b < w2) {
      const int a0 = q * hlen, a1 = min(h2, a0 + hlen);
      for (int a = a0; a < a1; ++a) s += img[a * w2 + b];
    }
    const double s1 = __shfl_xor(s, 1);
    const double s2 = __shfl_xor(s, 2);
    const double s3 = __shfl_xor(s, 3);
    if (q == 0 && b < w2) V[i * W2 + b] = (s + s1) + (s2 + s3);
  }
}

// R1[a][a'] = sum_b U[(a,b)][a'], R2[a][b'] = sum_b V[(a,b)][b'],
// R3[b][a'] = sum_a U[(a,b)][a'], R4[b][b'] = sum_a V[(a,b)][b'].
__global__ __launch_bounds__(NT) void k_sep_colreduce(const double* __restrict__ U,
                                                       const double* __restrict__ V, int64_t H1,
                                                       int64_t W1, int64_t H2, int64_t W2,
                                                       double* __restrict__ R1,
                                                       double* __restrict__ R2,
                                                       double* __restrict__ R3,
                                                       double* __restrict__ R4) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t n1 = H1 * H2, n2 = H1 * W2, n3 = W1 * H2, n4 = W1 * W2;
  if (idx < n1) {
    const int64_t a = idx / H2, ap = idx % H2;
    double s = 0.0;
#pragma unroll 8
    for (int64_t b = 0; b < W1; ++b) s += U[(a * W1 + b) * H2 + ap];
    R1[idx] = s;
  } else if (idx < n1 + n2) {
    const int64_t j = idx - n1, a = j / W2, bp = j % W2;
    double s = 0.0;
#pragma unroll 8
    for (int64_t b = 0; b < W1; ++b) s += V[(a * W1 + b) * W2 + bp];
    R2[j] = s;
  } else if (idx < n1 + n2 + n3) {
    const int64_t j = idx - n1 - n2, b = j / H2, ap = j % H2;
    double s = 0.0;
#pragma unroll 8
    for (int64_t a = 0; a < H1; ++a) s += U[(a * W1 + b) * H2 + ap];
    R3[j] = s;
  } else if (idx < n1 + n2 + n3 + n4) {
    const int64_t j = idx - n1 - n2 - n3, b = j / W2, bp = j % W2;
    double s = 0.0;
#pragma unroll 8
    for (int64_t a = 0; a < H1; ++a) s += V[(a * W1 + b) * W2 + bp];
    R4[j] = s;
  }
}

// Q = S_x R S_y for the four small matrices (S = |i-j|^m, dense, short axes),
// scaled by the Kronecker coefficients.  Two launches, each covering all four
// terms: P = S_x R with one block per (term, column of R), then Q = P S_y with
// one block per (term, row of P); the line (at most `line` entries, dynamic
// LDS) is staged once and every thread reads it as a broadcast.
struct SepTerms {
  const double* in[4];
  double* out[4];
  int nx[4], ny[4];
  int first[5];  // first block of each term (cumulative line counts)
  int m;         // exponent of S on this side
  double coef[4];
};
constexpr int SEP_LINE = 128;  // threads of the product kernels

GW_DEV int sep_term(const SepTerms& st) {
  int t = 0;
  while (t < 3 && (int)blockIdx.x >= st.first[t + 1]) ++t;
  return t;
}

__global__ __launch_bounds__(SEP_LINE) void k_sep_left(SepTerms st) {
  extern __shared__ double col[];
  const int t = sep_term(st);
  const int j = blockIdx.x - st.first[t], nx = st.nx[t], ny = st.ny[t];
  const double* R = st.in[t];
  for (int i = threadIdx.x; i < nx; i += SEP_LINE) col[i] = R[(int64_t)i * ny + j];
  __syncthreads();
  for (int i = threadIdx.x; i < nx; i += SEP_LINE) {
    double s = 0.0;
    for (int l = 0; l < nx; ++l) {
      const double d = gwk::ipow((double)(i > l ? i - l : l - i), st.m);
      s = fma(d, col[l], s);
    }
    st.out[t][(int64_t)i * ny + j] = s;
  }
}

__global__ __launch_bounds__(SEP_LINE) void k_sep_right(SepTerms st) {
  extern __shared__ double rowv[];
  const int t = sep_term(st);
  const int i = blockIdx.x - st.first[t], ny = st.ny[t];
  const double* P = st.in[t] + (int64_t)i * ny;
  for (int j = threadIdx.x; j < ny; j += SEP_LINE) rowv[j] = P[j];
  __syncthreads();
  for (int j = threadIdx.x; j < ny; j += SEP_LINE) {
    double s = 0.0;
    for (int l = 0; l < ny; ++l) {
      const double d = gwk::ipow((double)(j > l ? j - l : l - j), st.m);
      s = fma(rowv[l], d, s);
    }
    st.out[t][(int64_t)i * ny + j] = st.coef[t] * s;
  }
}

// G[(a,b)][(a',b')] = (c1 + c2) - s2 (Q1[a][a'] + Q2[a][b'] + Q3[b][a'] + Q4[b][b'])
__global__ __launch_bounds__(NT) void k_sep_write(int64_t H1, int64_t W1, int64_t H2, int64_t W2,
                                                   const double* __restrict__ Q1,
                                                   const double* __restrict__ Q2,
                                                   const double* __restrict__ Q3,
                                                   const double* __restrict__ Q4,
                                                   const double* __restrict__ c1,
                                                   const double* __restrict__ c2, double s2,
                                                   double* __restrict__ G, int64_t ldG,
                                                   gwr::Epilogue epi) {
  const int64_t i = blockIdx.x;
  const int64_t a = i / W1, b = i % W1;
  const double c1v = c1[i];
  const bool fg = epi.fa != nullptr;  // fused GW feature term (uniform)
  const double fai = fg ? epi.fa[i] : 0.0;
  const int w2 = (int)W2, h2 = (int)H2;
  auto put = [&](int ap, int bp, double q2, double q4) {
    const int64_t p = (int64_t)ap * W2 + bp;
    const double Bv = ((Q1[a * H2 + ap] + q2) + Q3[b * H2 + ap]) + q4;
    double v = (c1v + c2[p]) - s2 * Bv;
    if (fg) {
      const double d = fai - epi.fb[p];
      v = fma(epi.a, v, epi.b * (d * d));
    }
    G[i * ldG + p] = v;
  };
  if (w2 <= NT) {
    // NT / W2 image rows per pass: thread t takes column t % W2 of row t / W2
    const int rpp = NT / w2, bp = threadIdx.x % w2, ar = threadIdx.x / w2;
    if (ar < rpp) {
      const double q2 = Q2[a * W2 + bp], q4 = Q4[b * W2 + bp];
      for (int ap = ar; ap < h2; ap += rpp) put(ap, bp, q2, q4);
    }
  } else {
    for (int bp = threadIdx.x; bp < w2; bp += NT) {
      const double q2 = Q2[a * W2 + bp], q4 = Q4[b * W2 + bp];
      for (int ap = 0; ap < h2; ++ap) put(ap, bp, q2, q4);
    }
  }
}

bool separable(const gwr::Grid& g, SepGrid* s) {
  if (g.ndim != 2) return false;
  if (g.metric == GW_METRIC_SQEUCLID) {
    *s = SepGrid{g.H, g.W, 2, 1.0, 1.0};
    return true;
  }
  if (g.k == 1) {
    *s = SepGrid{g.H, g.W, 1, 1.0, 1.0};
    return true;
  }
  return false;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// --------------------------------------------------- axis-separable path
// Grids whose distance is a sum of per-axis terms, d(i, j) = sum_a |x_a(i) -
// x_a(j)|^m (1D: one axis, m = k; 2D/3D squared Euclidean: m = 2; 2D/3D
// (l1)^1: m = 1), so D = sum_a J (x) .. (x) D_a^{om} (x) .. (x) J (the
// Kronecker expansion of Sec. 3.1 without cross terms).  Then
//   (D_X T D_Y)[i][p] = sum_{u, v} Q_uv[x_u(i)][y_v(p)],
//   Q_uv = D_u^{om} R_uv D_v^{om},  R_uv[x][y] = sum of T over the rows with
//   x_u = x and the columns with y_v = y,
// so T is reduced once to small matrices, the 1D operators act on those, and
// the write pass gathers one value per axis pair.  Used for 3D grids and for
// mixed 1D/2D pairs; 1D x 1D and 2D x 2D have their own paths.
struct AxGrid {
  int na;             // number of axes (leading axis first)
  int n[3];           // extents
  int64_t stride[3];  // flat-index strides
  int m;              // exponent of every per-axis term
};
constexpr int AX_MAXP = 9;  // axis pairs

struct AxPlan {
  AxGrid x, y;
  int offy[3];               // offset of Y axis v in a row of U (sum of the Y extents before it)
  int sy;                    // sum of the Y extents
  const double* U;           // M x sy row sums (T itself when Y has one axis)
  int64_t ldU;
  const double* R[AX_MAXP];  // R_uv, nx_u x ny_v, leading dimension ldR (a view of U
  int64_t ldR[AX_MAXP];      // when X has one axis)
  double* Rw[AX_MAXP];       // where k_ax_colreduce writes R_uv
  double* P[AX_MAXP];        // D_u R_uv
  double* Q[AX_MAXP];        // P_uv D_v
  int first_left[AX_MAXP + 1], first_right[AX_MAXP + 1];  // thread ranges of the line kernels
  int first_elem[AX_MAXP + 1];  // cumulative nx_u ny_v: entry ranges of the dense kernels
};

GW_DEV int ax_coord(const AxGrid& g, int a, int64_t flat) {
  return (int)((flat / g.stride[a]) % g.n[a]);
}

// Row sums for a Y grid of two or three axes, seen as Zy x H x W (Zy = 1 in
// 2D): U[i][offy_v + y] = sum over the columns p of row i with y_v(p) = y.
// One block per row, the row staged in LDS; the plane P[r][c] = sum_z row is
// formed first (a thread per (r, c)), the H and W sums come from P, and the
// slab sums over z (3D) are split into `qs` contiguous parts added in order.
__global__ __launch_bounds__(NT) void k_ax_rowreduce(const double* __restrict__ T, int64_t ldT,
                                                      int N, AxGrid ay, int qs,
                                                      double* __restrict__ U, int sy) {
  extern __shared__ double lds[];
  const int na = ay.na;
  const int Zy = na == 3 ? ay.n[0] : 1, H = ay.n[na - 2], W = ay.n[na - 1], hw = H * W;
  double* row = lds;
  double* P = lds + N;
  double* part = P + hw;
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
  const double* src = T + i * ldT;
  for (int p0 = 0; p0 < N; p0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[min(p0 + t + u * NT, N - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + t + u * NT < N) row[p0 + t + u * NT] = v[u];
  }
  __syncthreads();
  for (int rc = t; rc < hw; rc += NT) {
    double acc = row[rc];
    for (int z = 1; z < Zy; ++z) acc += row[z * hw + rc];
    P[rc] = acc;
  }
  if (na == 3) {
    const int len = (hw + qs - 1) / qs;
    for (int w = t; w < Zy * qs; w += NT) {
      const int z = w / qs, q = w - z * qs;
      const int e0 = q * len, e1 = min(hw, e0 + len);
      double acc = 0.0;
      for (int e = e0; e < e1; ++e) acc += row[z * hw + e];
      part[w] = acc;
    }
  }
  __syncthreads();
  double* out = U + i * sy;
  const int offH = na == 3 ? Zy : 0, offW = offH + H;
  for (int r = t; r < H; r += NT) {
    double acc = P[r * W];
    for (int c = 1; c < W; ++c) acc += P[r * W + c];
    out[offH + r] = acc;
  }
  for (int c = t; c < W; c += NT) {
    double acc = P[c];
    for (int r = 1; r < H; ++r) acc += P[r * W + c];
    out[offW + c] = acc;
  }
  if (na == 3) {
    for (int z = t; z < Zy; z += NT) {
      double acc = part[z * qs];
      for (int q = 1; q < qs; ++q) acc += part[z * qs + q];
      out[z] = acc;
    }
  }
}

// R_uv[x][y] = sum over the rows i with x_u(i) = x of U[i][offy_v + y]; one
// block per (pair, x).  With nv < NT each sum is split into NT / nv parts
// (rows in index order within a part) added in part order.
__global__ __launch_bounds__(NT) void k_ax_colreduce(AxPlan pl, int M) {
  __shared__ double part[NT];
  int b = blockIdx.x, pr = 0;
  while (b >= pl.first_right[pr + 1] - pl.first_right[pr]) {
    b -= pl.first_right[pr + 1] - pl.first_right[pr];
    ++pr;
  }
  const int u = pr / pl.y.na, v = pr % pl.y.na, x = b;
  const int nv = pl.y.n[v], nu = pl.x.n[u];
  const int su = (int)pl.x.stride[u];
  const int cnt = M / nu;
  const int K = nv >= NT ? 1 : NT / nv;
  const int len = (cnt + K - 1) / K;
  const int t = threadIdx.x;
  const double* Ub = pl.U + pl.offy[v];
  for (int y0 = 0; y0 < nv; y0 += NT) {
    const int y = y0 + t % min(nv, NT), k = t / min(nv, NT);
    double acc = 0.0;
    if (k < K && y < nv) {
      const int o0 = k * len, o1 = min(cnt, o0 + len);
      int lo = o0 % su;
      int64_t i = (int64_t)(o0 / su) * (su * nu) + (int64_t)x * su + lo;
      for (int o = o0; o < o1; ++o) {
        acc += Ub[i * pl.ldU + y];
        ++i;
        if (++lo == su) {
          lo = 0;
          i += (int64_t)su * (nu - 1);
        }
      }
    }
    if (K > 1) {
      part[t] = acc;
      __syncthreads();
      if (t < nv) {
        double r = part[t];
        for (int kk = 1; kk < K; ++kk) r += part[kk * nv + t];
        pl.Rw[pr][(int64_t)x * nv + t] = r;
      }
      __syncthreads();
    } else if (y < nv) {
      pl.Rw[pr][(int64_t)x * nv + y] = acc;
    }
  }
}

// P_uv = D_u^{om} R_uv: one thread per (pair, column y), the recursion along x.
__global__ __launch_bounds__(NT) void k_ax_left(AxPlan pl) {
  const int tid = blockIdx.x * NT + threadIdx.x;
  const int npairs = pl.x.na * pl.y.na;
  if (tid >= pl.first_left[npairs]) return;
  int pr = 0;
  while (tid >= pl.first_left[pr + 1]) ++pr;
  const int u = pr / pl.y.na, v = pr % pl.y.na;
  const int y = tid - pl.first_left[pr], nv = pl.y.n[v];
  line_op(pl.x.m, pl.R[pr] + y, pl.ldR[pr], pl.P[pr] + y, nv, pl.x.n[u], 1.0, false);
}

// Short axes: the same products densely, one thread per entry of P (or Q).
GW_DEV double small_pow(int d, int e) {
  double v = 1.0;
  for (int u = 0; u < e; ++u) v *= (double)d;
  return v;
}

GW_DEV int ax_pair_of(const AxPlan& pl, int e) {
  int pr = 0;
  while (e >= pl.first_elem[pr + 1]) ++pr;
  return pr;
}

__global__ __launch_bounds__(NT) void k_ax_left_dense(AxPlan pl) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= pl.first_elem[pl.x.na * pl.y.na]) return;
  const int pr = ax_pair_of(pl, e), u = pr / pl.y.na, v = pr % pl.y.na;
  const int nv = pl.y.n[v], nu = pl.x.n[u], r = e - pl.first_elem[pr];
  const int x = r / nv, y = r - x * nv;
  const double* R = pl.R[pr] + y;
  const int64_t ld = pl.ldR[pr];
  double s = 0.0;
#pragma unroll 4
  for (int l = 0; l < nu; ++l) s = fma(small_pow(abs(x - l), pl.x.m), R[l * ld], s);
  pl.P[pr][r] = s;
}

__global__ __launch_bounds__(NT) void k_ax_right_dense(AxPlan pl) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= pl.first_elem[pl.x.na * pl.y.na]) return;
  const int pr = ax_pair_of(pl, e), v = pr % pl.y.na;
  const int nv = pl.y.n[v], r = e - pl.first_elem[pr];
  const int x = r / nv, y = r - x * nv;
  const double* Pr = pl.P[pr] + (int64_t)x * nv;
  double s = 0.0;
#pragma unroll 4
  for (int l = 0; l < nv; ++l) s = fma(Pr[l], small_pow(abs(l - y), pl.y.m), s);
  pl.Q[pr][r] = s;
}

// Q_uv = P_uv D_v^{om}: one thread per (pair, row x), the recursion along y.
__global__ __launch_bounds__(NT) void k_ax_right(AxPlan pl) {
  const int tid = blockIdx.x * NT + threadIdx.x;
  const int npairs = pl.x.na * pl.y.na;
  if (tid >= pl.first_right[npairs]) return;
  int pr = 0;
  while (tid >= pl.first_right[pr + 1]) ++pr;
  const int v = pr % pl.y.na;
  const int x = tid - pl.first_right[pr], nv = pl.y.n[v];
  line_op(pl.y.m, pl.P[pr] + (int64_t)x * nv, 1, pl.Q[pr] + (int64_t)x * nv, 1, nv, 1.0, false);
}

// G[i][p] = (c1_i + c2_p) - s2 sum_v V_v[y_v(p)], V_v[y] = sum_u Q_uv[x_u(i)][y]
// (u, v in axis order); V in LDS, one block per row, the column coordinates
// stepped in mixed radix.  With epi.fa the fused GW feature term follows.
template <int NA>
__global__ __launch_bounds__(NT) void k_ax_write(AxPlan pl, int N, const double* __restrict__ c1,
                                                  const double* __restrict__ c2, double s2,
                                                  double* __restrict__ G, int64_t ldG,
                                                  gwr::Epilogue epi) {
  extern __shared__ double V[];
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NA; ++v) {
    const int nv = pl.y.n[v];
    for (int y = t; y < nv; y += NT) {
      double acc = 0.0;
      for (int u = 0; u < pl.x.na; ++u)
        acc += pl.Q[u * NA + v][(int64_t)ax_coord(pl.x, u, i) * nv + y];
      V[pl.offy[v] + y] = acc;
    }
  }
  __syncthreads();
  const double c1v = c1[i];
  const bool fg = epi.fa != nullptr;
  const double fai = fg ? epi.fa[i] : 0.0;
  // mixed-radix digits (last axis fastest) of the thread's first column and
  // of the step NT; the leading digit is unbounded
  int d[3] = {0, 0, 0}, st[3] = {0, 0, 0};
  {
    int a = t, b = NT;
#pragma unroll
    for (int v = NA - 1; v >= 1; --v) {
      d[v] = a % pl.y.n[v];
      a /= pl.y.n[v];
      st[v] = b % pl.y.n[v];
      b /= pl.y.n[v];
    }
    d[0] = a;
    st[0] = b;
  }
  double* grow = G + i * ldG;
  const int o1 = pl.offy[1], o2 = pl.offy[2];
  for (int p = t; p < N; p += NT) {
    double B = V[d[0]];
    if constexpr (NA > 1) B += V[o1 + d[1]];
    if constexpr (NA > 2) B += V[o2 + d[2]];
    double val = (c1v + c2[p]) - s2 * B;
    if (fg) {
      const double df = fai - epi.fb[p];
      val = fma(epi.a, val, epi.b * (df * df));
    }
    grow[p] = val;
    // advance by NT: each digit and step digit is below its extent, so one
    // subtraction and a carry of at most one per axis
    int carry = 0;
#pragma unroll
    for (int v = NA - 1; v >= 1; --v) {
      d[v] += st[v] + carry;
      carry = d[v] >= pl.y.n[v] ? 1 : 0;
      if (carry) d[v] -= pl.y.n[v];
    }
    d[0] += st[0] + carry;
  }
}


// One launch for up to two 1D vectors of the same exponent (job 1 may be
// empty: nblocks = 1).
bool const_1d_ok(const gwr::Grid& g) { return g.ndim == 1 && g.n() <= (int64_t)1024 * C1_SEG; }

gw_status launch_const_jobs(int k1d, int nblocks, int nmax, ConstJob j0, ConstJob j1,
                            hipStream_t s) {
  switch (k1d) {
    case 1: launch_const_1d<2>(nblocks, nmax, j0, j1, s); break;
    case 2: launch_const_1d<4>(nblocks, nmax, j0, j1, s); break;
    case 3: launch_const_1d<6>(nblocks, nmax, j0, j1, s); break;
    case 4: launch_const_1d<8>(nblocks, nmax, j0, j1, s); break;
    default: return GW_EUNSUPPORTED;
  }
  return gwr::last_launch_status();
}

ConstJob job_of(const gwr::Grid& g, const double* w, double* c) {
  const double hk = g.hk();
  return ConstJob{(int)g.n(), hk * hk, w, c};
}

}  // namespace

namespace gwl {

gw_status const_term(const gwr::Grid& g, const double* w, double* c, hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  const int64_t n = g.n();
  if (const_1d_ok(g)) {
    const ConstJob j = job_of(g, w, c);
    return launch_const_jobs(g.k1d(), 1, (int)n, j, j, s);
  }
  if (g.ndim == 2) {
    SepConst sc{};
    if (g.metric == GW_METRIC_SQEUCLID) {
      sc.nt = 3;
      const int er[3] = {4, 2, 0}, ec[3] = {0, 2, 4};
      const double cf[3] = {1.0, 2.0, 1.0};
      for (int t = 0; t < 3; ++t) {
        sc.er[t] = er[t];
        sc.ec[t] = ec[t];
        sc.coef[t] = cf[t];
      }
    } else if (2 * g.k + 1 <= CS_MAXT) {
      sc.nt = 2 * g.k + 1;
      double binom = 1.0;  // C(2k, m)
      for (int m = 0; m <= 2 * g.k; ++m) {
        sc.er[m] = m;
        sc.ec[m] = 2 * g.k - m;
        sc.coef[m] = binom;
        binom = binom * (double)(2 * g.k - m) / (double)(m + 1);
      }
    }
    const size_t shm = const_sep_lds((int)g.H, (int)g.W, sc.nt);
    if (sc.nt > 0 && shm <= 160 * 1024) {
      // dynamic LDS above the default
      if (shm > 64 * 1024 &&
          gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_const_sep), shm) != GW_OK)
        return GW_EDEVICE;
      const double hk = g.hk();
      k_const_sep<<<(unsigned)g.W, 256, shm, s>>>(sc, (int)g.H, (int)g.W, hk * hk, w, c);
      return gwr::last_launch_status();
    }
  }
  if (g.ndim == 3) {
    k_const_term3<<<(unsigned)((n + CT3_OUT - 1) / CT3_OUT), 1024, 0, s>>>(
        g.metric, g.k, (int)g.Z, (int)g.H, (int)g.W, g.hk(), w, c);
  } else
    k_const_term<<<(unsigned)((n + 63) / 64), 1024, 0, s>>>(g.metric, g.k, (int)g.H, (int)g.W,
                                                            g.hk(), w, c);
  return gwr::last_launch_status();
}

gw_status const_terms(const gwr::Grid& X, const double* p, double* c1, const gwr::Grid& Y,
                      const double* q, double* c2, hipStream_t s) {
  if (const_1d_ok(X) && const_1d_ok(Y) && X.k1d() == Y.k1d()) {
    gwr::ProfScope ps(gwr::kFamOther, s);
    const int nmax = (int)(X.n() > Y.n() ? X.n() : Y.n());
    return launch_const_jobs(X.k1d(), 2, nmax, job_of(X, p, c1), job_of(Y, q, c2), s);
  }
  gw_status st = const_term(X, p, c1, s);
  return st != GW_OK ? st : const_term(Y, q, c2, s);
}

gw_status resolve_const_terms(const gwr::Grid& X, const double* p, const double* c1_pre,
                              double** c1, const gwr::Grid& Y, const double* q,
                              const double* c2_pre, double** c2, hipStream_t s) {
  if (!c1_pre && !c2_pre) return const_terms(X, p, *c1, Y, q, *c2, s);
  gw_status st = GW_OK;
  if (c1_pre) *c1 = const_cast<double*>(c1_pre);
  else st = const_term(X, p, *c1, s);
  if (st != GW_OK) return st;
  if (c2_pre) *c2 = const_cast<double*>(c2_pre);
  else st = const_term(Y, q, *c2, s);
  return st;
}

bool axis_separable(const gwr::Grid& g, AxGrid* a) {
  *a = AxGrid{};
  if (g.ndim == 1) {
    a->na = 1;
    a->n[0] = (int)g.W;
    a->stride[0] = 1;
    a->m = g.k1d();
    return true;
  }
  if (g.metric == GW_METRIC_SQEUCLID) a->m = 2;
  else if (g.k == 1) a->m = 1;
  else return false;
  if (g.ndim == 2) {
    a->na = 2;
    a->n[0] = (int)g.H;
    a->n[1] = (int)g.W;
    a->stride[0] = g.W;
    a->stride[1] = 1;
  } else {
    a->na = 3;
    a->n[0] = (int)g.Z;
    a->n[1] = (int)g.H;
    a->n[2] = (int)g.W;
    a->stride[0] = g.H * g.W;
    a->stride[1] = g.W;
    a->stride[2] = 1;
  }
  return true;
}

int ax_extent_sum(const AxGrid& a) {
  int s = 0;
  for (int v = 0; v < a.na; ++v) s += a.n[v];
  return s;
}

// parts per slab sum of the row reduction (3D Y): enough work items for the block
int ax_parts(const AxGrid& ay) {
  if (ay.na != 3) return 1;
  const int q = NT / ay.n[0];
  return q < 1 ? 1 : (q > 16 ? 16 : q);
}

size_t ax_row_lds(int64_t N, const AxGrid& ay) {
  const int64_t hw = (int64_t)ay.n[ay.na - 2] * ay.n[ay.na - 1];
  const int64_t zs = ay.na == 3 ? (int64_t)ay.n[0] * ax_parts(ay) : 0;
  return (size_t)(N + hw + zs) * sizeof(double);
}

int64_t ax_pair_elems(const AxGrid& ax, const AxGrid& ay) {
  int64_t t = 0;
  for (int u = 0; u < ax.na; ++u)
    for (int v = 0; v < ay.na; ++v) t += (int64_t)ax.n[u] * ay.n[v];
  return t;
}

// The axis-separable path serves 3D grids and mixed 1D/2D pairs whose two
// distances are sums of per-axis terms, when its LDS stages fit.
bool ax_path(const gwr::Grid& X, const gwr::Grid& Y, AxGrid* ax, AxGrid* ay) {
  if (X.ndim == Y.ndim && X.ndim < 3) return false;
  if (!axis_separable(X, ax) || !axis_separable(Y, ay)) return false;
  if (ay->na > 1 && ax_row_lds(Y.n(), *ay) > 160 * 1024) return false;
  if ((size_t)ax_extent_sum(*ay) * sizeof(double) > 160 * 1024) return false;
  return true;
}

size_t fast_generic_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y) {
  const int64_t M = X.n(), N = Y.n();
  gwr::Arena a{nullptr, 0, 0};
  SepGrid sx, sy;
  if (separable(X, &sx) && separable(Y, &sy)) {
    a.take<double>(M * Y.H);
    a.take<double>(M * Y.W);
    for (int t = 0; t < 3; ++t) {  // R, P, Q sets
      a.take<double>(X.H * Y.H);
      a.take<double>(X.H * Y.W);
      a.take<double>(X.W * Y.H);
      a.take<double>(X.W * Y.W);
    }
  } else if (AxGrid ax, ay; ax_path(X, Y, &ax, &ay)) {
    if (ay.na > 1) a.take<double>((size_t)M * ax_extent_sum(ay));
    const int64_t pe = ax_pair_elems(ax, ay);
    if (ax.na > 1) a.take<double>(pe);
    a.take<double>(pe);
    a.take<double>(pe);
  } else {
    a.take<double>((size_t)M * N);
    a.take<double>((size_t)M * N);
    a.take<double>((size_t)M * N);
    if (X.ndim == 3 || Y.ndim == 3) a.take<double>((size_t)M * N);
  }
  a.take<double>(M);
  a.take<double>(N);
  return a.used;
}

gw_status fast_generic(const gwr::Grid& X, const gwr::Grid& Y, const double* p,
                       const double* q, const double* T, int64_t ldT, double* G, int64_t ldG,
                       gwr::Arena& ws, hipStream_t s, const double* c1_pre,
                       const double* c2_pre, const gwr::Epilogue* epi) {
  const int64_t M = X.n(), N = Y.n();
  SepGrid sx, sy;
  const bool sep = separable(X, &sx) && separable(Y, &sy);
  double *U = nullptr, *V = nullptr, *R[4] = {}, *P[4] = {}, *Q[4] = {};
  double *A = nullptr, *At = nullptr, *tmp = nullptr, *tmp2 = nullptr;
  AxGrid ax{}, ay{};
  const bool axp = !sep && ax_path(X, Y, &ax, &ay);
  double *aU = nullptr, *aR = nullptr, *aP = nullptr, *aQ = nullptr;
  if (sep) {
    U = ws.take<double>(M * Y.H);
    V = ws.take<double>(M * Y.W);
    double** sets[3] = {R, P, Q};
    for (int t = 0; t < 3; ++t) {
      sets[t][0] = ws.take<double>(X.H * Y.H);
      sets[t][1] = ws.take<double>(X.H * Y.W);
      sets[t][2] = ws.take<double>(X.W * Y.H);
      sets[t][3] = ws.take<double>(X.W * Y.W);
    }
  } else if (axp) {
    if (ay.na > 1) aU = ws.take<double>((size_t)M * ax_extent_sum(ay));
    const int64_t pe = ax_pair_elems(ax, ay);
    if (ax.na > 1) aR = ws.take<double>(pe);
    aP = ws.take<double>(pe);
    aQ = ws.take<double>(pe);
  } else {
    A = ws.take<double>((size_t)M * N);
    At = ws.take<double>((size_t)M * N);
    tmp = ws.take<double>((size_t)M * N);
    if (X.ndim == 3 || Y.ndim == 3) tmp2 = ws.take<double>((size_t)M * N);
  }
  double* c1 = ws.take<double>(M);
  double* c2 = ws.take<double>(N);
  // the constant terms need only p and q: on a side stream they run beside
  // the reductions and products, joined before the kernel that writes G
  gwr::SideJoin sj{(!c1_pre || !c2_pre) ? gwr::side_take(s) : nullptr, s};
  gw_status st =
      resolve_const_terms(X, p, c1_pre, &c1, Y, q, c2_pre, &c2, sj.ss ? sj.ss->side : s);
  if (st != GW_OK) return st;
  const double s2 = 2.0 * (X.hk() * Y.hk());
  gwr::ProfScope ps(gwr::kFam2D, s);
  if (sep) {
    const size_t shm = (size_t)N * sizeof(double);
    if (shm > 160 * 1024) return GW_EUNSUPPORTED;
    if (gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_sep_rowreduce), 160 * 1024) != GW_OK)
      return GW_EDEVICE;
    k_sep_rowreduce<<<(unsigned)M, NT, shm, s>>>(T, ldT, M, Y.H, Y.W, U, V);
    const int64_t ntot = X.H * Y.H + X.H * Y.W + X.W * Y.H + X.W * Y.W;
    k_sep_colreduce<<<blocks_for(ntot), NT, 0, s>>>(U, V, X.H, X.W, Y.H, Y.W, R[0], R[1], R[2], R[3]);
    // term t: (x axis, y axis) = (H,H), (H,W), (W,H), (W,W)
    const int64_t nx[4] = {X.H, X.H, X.W, X.W};
    const int64_t ny[4] = {Y.H, Y.W, Y.H, Y.W};
    const double cx[4] = {sx.alpha, sx.alpha, sx.beta, sx.beta};
    const double cy[4] = {sy.alpha, sy.beta, sy.alpha, sy.beta};
    SepTerms lt{}, rt{};
    lt.first[0] = rt.first[0] = 0;
    int64_t lmax = 1, rmax = 1;  // longest line of each launch
    for (int t = 0; t < 4; ++t) {
      lmax = nx[t] > lmax ? nx[t] : lmax;
      rmax = ny[t] > rmax ? ny[t] : rmax;
      lt.in[t] = R[t];
      lt.out[t] = P[t];
      rt.in[t] = P[t];
      rt.out[t] = Q[t];
      lt.nx[t] = rt.nx[t] = (int)nx[t];
      lt.ny[t] = rt.ny[t] = (int)ny[t];
      lt.first[t + 1] = lt.first[t] + (int)ny[t];  // a block per column of R
      rt.first[t + 1] = rt.first[t] + (int)nx[t];  // a block per row of P
      rt.coef[t] = cx[t] * cy[t];
    }
    lt.m = sx.m;
    rt.m = sy.m;
    const size_t lsh = (size_t)lmax * sizeof(double), rsh = (size_t)rmax * sizeof(double);
    if (lsh > 160 * 1024 || rsh > 160 * 1024) return GW_EUNSUPPORTED;
    // dynamic LDS above the default
    if (lsh > 64 * 1024 &&
        gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_sep_left), lsh) != GW_OK)
      return GW_EDEVICE;
    if (rsh > 64 * 1024 &&
        gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_sep_right), rsh) != GW_OK)
      return GW_EDEVICE;
    k_sep_left<<<(unsigned)lt.first[4], SEP_LINE, lsh, s>>>(lt);
    k_sep_right<<<(unsigned)rt.first[4], SEP_LINE, rsh, s>>>(rt);
    if (sj.join() != GW_OK) return GW_EDEVICE;
    k_sep_write<<<(unsigned)M, NT, 0, s>>>(X.H, X.W, Y.H, Y.W, Q[0], Q[1], Q[2], Q[3], c1, c2,
                                           s2, G, ldG, epi ? *epi : gwr::Epilogue{});
    return gwr::last_launch_status();
  }
  if (axp) {
    AxPlan pl{};
    pl.x = ax;
    pl.y = ay;
    int off = 0;
    for (int v = 0; v < ay.na; ++v) {
      pl.offy[v] = off;
      off += ay.n[v];
    }
    pl.sy = off;
    if (ay.na == 1) {  // one axis: the row sums are T itself
      pl.U = T;
      pl.ldU = ldT;
    } else {
      const int qs = ax_parts(ay);
      const size_t shm = ax_row_lds(N, ay);
      if (gwr::allow_dyn_lds(reinterpret_cast<const void*>(&k_ax_rowreduce), 160 * 1024) !=
          GW_OK)
        return GW_EDEVICE;
      k_ax_rowreduce<<<(unsigned)M, NT, shm, s>>>(T, ldT, (int)N, ay, qs, aU, off);
      pl.U = aU;
      pl.ldU = off;
    }
    int64_t roff = 0;
    for (int u = 0; u < ax.na; ++u)
      for (int v = 0; v < ay.na; ++v) {
        const int pr = u * ay.na + v;
        if (ax.na == 1) {  // one axis: R_0v is a view of U
          pl.R[pr] = pl.U + pl.offy[v];
          pl.ldR[pr] = pl.ldU;
        } else {
          pl.Rw[pr] = aR + roff;
          pl.R[pr] = pl.Rw[pr];
          pl.ldR[pr] = ay.n[v];
        }
        pl.P[pr] = aP + roff;
        pl.Q[pr] = aQ + roff;
        roff += (int64_t)ax.n[u] * ay.n[v];
        pl.first_left[pr + 1] = pl.first_left[pr] + ay.n[v];
        pl.first_right[pr + 1] = pl.first_right[pr] + ax.n[u];
        pl.first_elem[pr + 1] = pl.first_elem[pr] + ax.n[u] * ay.n[v];
      }
    const int npairs = ax.na * ay.na;
    if (ax.na > 1) k_ax_colreduce<<<(unsigned)pl.first_right[npairs], NT, 0, s>>>(pl, (int)M);
    // dense products on axes of up to 64 points, the recursion on longer ones
    int lx = 0, ly = 0;
    for (int u = 0; u < ax.na; ++u) lx = ax.n[u] > lx ? ax.n[u] : lx;
    for (int v = 0; v < ay.na; ++v) ly = ay.n[v] > ly ? ay.n[v] : ly;
    if (lx <= 64) k_ax_left_dense<<<blocks_for(roff), NT, 0, s>>>(pl);
    else k_ax_left<<<blocks_for(pl.first_left[npairs]), NT, 0, s>>>(pl);
    if (ly <= 64) k_ax_right_dense<<<blocks_for(roff), NT, 0, s>>>(pl);
    else k_ax_right<<<blocks_for(pl.first_right[npairs]), NT, 0, s>>>(pl);
    const size_t wsh = (size_t)pl.sy * sizeof(double);
    const gwr::Epilogue e = epi ? *epi : gwr::Epilogue{};
    {  // dynamic LDS above the default
      const void* fns[3] = {reinterpret_cast<const void*>(&k_ax_write<1>),
                            reinterpret_cast<const void*>(&k_ax_write<2>),
                            reinterpret_cast<const void*>(&k_ax_write<3>)};
      for (const void* fn : fns)
        if (gwr::allow_dyn_lds(fn, 160 * 1024) != GW_OK) return GW_EDEVICE;
    }
    if (sj.join() != GW_OK) return GW_EDEVICE;
    switch (ay.na) {
      case 1: k_ax_write<1><<<(unsigned)M, NT, wsh, s>>>(pl, (int)N, c1, c2, s2, G, ldG, e); break;
      case 2: k_ax_write<2><<<(unsigned)M, NT, wsh, s>>>(pl, (int)N, c1, c2, s2, G, ldG, e); break;
      default: k_ax_write<3><<<(unsigned)M, NT, wsh, s>>>(pl, (int)N, c1, c2, s2, G, ldG, e); break;
    }
    return gwr::last_launch_status();
  }
  // generic: A = T D^_Y (rows), At = A^T, Bt = At D^_X (rows), G = epilogue(Bt^T)
  // 1D sides: one wave per row; images of up to 96 x 96 points (3D: 16 per axis): the LDS
  // kernels, one block per row; larger ones: k_rowop
  if (Y.ndim == 1)
    line_rows(Y.metric == GW_METRIC_SQEUCLID ? 2 : Y.k, T, ldT, M, N, A, N, s);
  else if (gwl::img_rowop(T, ldT, M, Y, A, N, s) == GW_EUNSUPPORTED &&
           gwl::img3_rowop(T, ldT, M, Y, A, N, s) == GW_EUNSUPPORTED)
    k_rowop<<<(unsigned)M, NT, 0, s>>>(T, ldT, M, Y.ndim, Y.k, Y.metric, Y.Z, Y.H, Y.W, A, N, tmp,
                                       tmp2);
  dim3 tg1((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
  k_transpose<<<tg1, NT, 0, s>>>(A, N, M, N, At, M, nullptr, nullptr, 0.0);
  if (X.ndim == 1)
    line_rows(X.metric == GW_METRIC_SQEUCLID ? 2 : X.k, At, M, N, M, A, M, s);
  else if (gwl::img_rowop(At, M, N, X, A, M, s) == GW_EUNSUPPORTED &&
           gwl::img3_rowop(At, M, N, X, A, M, s) == GW_EUNSUPPORTED)
    k_rowop<<<(unsigned)N, NT, 0, s>>>(At, M, N, X.ndim, X.k, X.metric, X.Z, X.H, X.W, A, M, tmp,
                                       tmp2);
  dim3 tg2((unsigned)((M + 31) / 32), (unsigned)((N + 31) / 32));
  if (sj.join() != GW_OK) return GW_EDEVICE;
  k_transpose<<<tg2, NT, 0, s>>>(A, M, N, M, G, ldG, c1, c2, s2);
  if (epi) return fgw_blend(G, ldG, M, N, epi->fa, epi->fb, epi->a, epi->b, s);
  return gwr::last_launch_status();
}

}  // namespace gwl
