// Unbalanced GW (Remark, Entropic algorithm for UGW).  Each step solves
//   min_{T >= 0} <G(Th) + g(Th), T> + m(Th) (rho KL(T1|u) + rho KL(T^T 1|v) + eps KL(T|u (x) v))
// with G(Th) the half gradient at Th's own marginals (the FAST paths), then
// rescales the plan's mass.  The Remark leaves the scalar g(Th) and the
// solver of this sub-problem to the UGW work it cites; taken from there:
//   g(Th) = rho <log(a/u), a> + rho <log(b/v), b> + eps <log(Th/(u (x) v)), Th>,
//   f = -tau e LSE_p((g_p - C_ip)/e + ln v_p),  g = -tau e LSE_i((f_i - C_ip)/e + ln u_i),
//   tau = rho / (rho + eps), e = m(Th) eps,  T = exp((f + g - C)/e) u (x) v,
//   T <- sqrt(m(Th) / m(T)) T,  T^0 = u (x) v / sqrt(m(u) m(v)).
// The scalars of a step (m, the shift g(Th), e, tau, the rescale factor) stay
// in device memory, so a solve needs no host synchronisation.
//
// Kernels: rows of up to 8192 entries take one pass over C per iteration (a
// block per band of rows updates f and keeps the band's column sums, a small
// merge sets g; described above k_uot_fused).  Longer rows take two: the row
// update is one block per row (each thread holds its entries of the row,
// block max then block sum of the exponentials); the column update runs an
// online log-sum-exp over row chunks (a block per 64 columns x chunk, 16 waves
// splitting the chunk) and merges the chunks per column in order.  Every
// reduction has a fixed order.
#include "common.h"
#include "expx.h"
#include "runtime.h"

namespace {

struct UgwScal {
  double m;       // m(Th)
  double shift;   // g(Th), added to every cost entry
  double e;       // m(Th) eps
  double tau;     // rho / (rho + eps)
  double factor;  // mass rescale of the last plan
  double mu, mv;  // m(u), m(v)
  double pad;
};

constexpr int UR_NT = 1024;                  // row update threads
constexpr int UC_COLS = 64, UC_WAVES = 16;   // column update block shape
constexpr int UC_MAX_CHUNKS = 64;

// Fixed-order block reductions (butterfly inside a wave, waves in order).
template <int NTH>
GW_DEV double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NTH / 64; ++w) r = fmax(r, red[w]);
  return r;
}

template <int NTH>
GW_DEV double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NTH / 64; ++w) r += red[w];
  return r;
}

// (m, s) pairs of a log-sum-exp: the value is m + log(s); m = -inf is empty.
GW_DEV void lse_merge(double& m, double& s, double m2, double s2) {
  const double mx = fmax(m, m2);
  if (mx == -INFINITY) return;
  s = s * exp(m - mx) + s2 * exp(m2 - mx);
  m = mx;
}

__global__ __launch_bounds__(256) void k_uot_logs(const double* __restrict__ u,
                                                  const double* __restrict__ v, int M, int N,
                                                  double* __restrict__ lu,
                                                  double* __restrict__ lv, double* __restrict__ f,
                                                  double* __restrict__ g, int zero) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < M) {
    lu[i] = u[i] > 0.0 ? log(u[i]) : -INFINITY;
    if (zero) f[i] = 0.0;
  }
  if (i < N) {
    lv[i] = v[i] > 0.0 ? log(v[i]) : -INFINITY;
    if (zero) g[i] = 0.0;
  }
}

__global__ void k_uot_set(UgwScal* sc, double shift, double e, double tau) {
  if (threadIdx.x != 0) return;
  sc->m = 1.0;
  sc->shift = shift;
  sc->e = e;
  sc->tau = tau;
  sc->factor = 1.0;
}

// f_i = -tau e LSE_p((g_p - C_ip - shift)/e + ln v_p): one block per row.
template <int NTH, int EPT>
__global__ __launch_bounds__(NTH) void k_uot_row(const double* __restrict__ C, int64_t ldC,
                                                 int N, const double* __restrict__ g,
                                                 const double* __restrict__ lv,
                                                 const UgwScal* __restrict__ sc,
                                                 double* __restrict__ f) {
  __shared__ double red[NTH / 64];
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
  const double* row = C + i * ldC;
  const double shift = sc->shift, ie = 1.0 / sc->e;
  double z[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int p = t + k * NTH, pc = min(p, N - 1);
    const double zz = (g[pc] - row[pc] - shift) * ie + lv[pc];
    z[k] = p < N ? zz : -INFINITY;
  }
  double mx = z[0];
#pragma unroll
  for (int k = 1; k < EPT; ++k) mx = fmax(mx, z[k]);
  mx = block_max<NTH>(mx, red);
  double s = 0.0;
  if (mx != -INFINITY) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) s += exp(z[k] - mx);
  }
  s = block_sum<NTH>(s, red);
  if (t == 0) {
    const double L = mx == -INFINITY ? -INFINITY : mx + log(s);
    f[i] = -sc->tau * sc->e * L;
  }
}

// ---- one pass per iteration, rows of up to 8192 entries
// With b_p = (g_p - shift)/e + ln v_p and z_ip = b_p - C_ip/e the row update
// is f_i = -tau e (m_i + ln s_i), m_i = max_p z_ip, s_i = sum_p exp(z_ip - m_i).
// The column update needs exp((f_i - C_ip - shift)/e + ln u_i)
//   = exp(z_ip - m_i) exp(lam_i) exp(-b_p),  lam_i = m_i + (f_i - shift)/e + ln u_i,
// so the row's own exponentials feed the column sums.  A column with v_p = 0
// is left out of the row maxima and sums and takes b_p = (g_p - shift)/e for
// its exponentials (its g_p is still defined by the column update).  The
// merge adds the bands in order and sets g_p = -tau e (ln S_p - b_p) with the
// b_p of the pass, S_p = sum_i exp(z_ip - m_i + lam_i).
//
// Two kinds of pass.  The exact pass reduces each row's maximum and keeps the
// band's column sums as (mantissa, binary exponent) pairs (a column's largest
// term can lie far below every row maximum).  The shifted pass (rows of up to
// 4096 entries, after the first iteration of a call, when the moves of g
// allow it) takes m_i = a_i + D+ instead of the maximum, a_i the previous
// pass's bound of the row's log-sum-exp and D+ the largest move up of b_p
// over the columns in the rows since then, and keeps plain doubles in a frame
// 2^kq_p per column.  After the previous merge,
//   sum_i exp((f_i - C_ip - shift)/e + ln u_i) = exp(-g_p/(tau e))
// for the f of the previous pass, and the new f moves by at most tau e D+
// down and tau e D- up, so S_p lies within e^(D+) and e^(D-) of exp(P_p),
// P_p = b_p - g_p/(tau e); kq_p = -rint(P_p / ln 2) puts it in
// [2^-795, 2^867] for D+ <= 550 and D+ + D- <= 600.  Each band records its
// kind (bmode) and block 0 the frames, which the merge reads.
constexpr int UF_BANDS = 256;   // bands of rows per pass (at most)
constexpr int UF_MAX_RB = 256;  // rows per band (M <= 65535 over 256 bands)
constexpr double LAM_MAX = 1.0e6;
constexpr double FRAME_P_MAX = 1.0e8;  // |P_p| of a shifted pass (frames fit an int)

GW_DEV double col_base(double gp, double lvp, double shift, double ie) {
  const double gb = (gp - shift) * ie;
  return lvp > -INFINITY ? gb + lvp : gb;
}

template <int NTH, int EPT, int R, bool SHIFT>
__global__ __launch_bounds__(NTH) void k_uot_fused(const double* __restrict__ C, int64_t ldC,
                                                   int M, int N, int RB,
                                                   const double* __restrict__ g,
                                                   const double* __restrict__ gprev,
                                                   const double* __restrict__ lu,
                                                   const double* __restrict__ lv,
                                                   const UgwScal* __restrict__ sc,
                                                   double* __restrict__ f,
                                                   double* __restrict__ lse,
                                                   int* __restrict__ kq,
                                                   int* __restrict__ bmode,
                                                   double* __restrict__ partS,
                                                   int* __restrict__ partX) {
  constexpr int NW = NTH / 64;
  constexpr bool BL = EPT >= 16;  // b_p and the frames in LDS for the longest rows
  __shared__ double red[2][R][NW];
  __shared__ double dred[NW][3];
  __shared__ double bls[BL ? NTH * EPT : 1];
  __shared__ int kqs[BL ? NTH * EPT : 1];
  __shared__ double lse_b[UF_MAX_RB];  // the band's row bounds from the previous pass
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const double shift = sc->shift, e = sc->e, ie = 1.0 / e, tau = sc->tau;
  const int i0 = blockIdx.x * RB, i1 = min(M, i0 + RB);
  double breg[BL ? 1 : EPT], S[EPT];
  int X[EPT], kqr[BL ? 1 : EPT];
  unsigned inrow = 0;  // bit k: entry k counts in the row maxima and sums
  // the columns: b_p, and with gprev the move of g (columns in the rows) and
  // the frames; every block reduces the same D+ and D-
  double up = 0.0, dn = 0.0;
  const double itaue = 1.0 / (tau * e);
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int col = t + NTH * k;
    const int cc = min(col, N - 1);
    const double lvv = lv[cc];
    const double gv = g[cc];
    const double bv = col_base(gv, lvv, shift, ie);
    if constexpr (BL) bls[t + NTH * k] = bv;
    else breg[k] = bv;
    if (col < N && lvv > -INFINITY) inrow |= 1u << k;
    int kv = 0;
    if (gprev != nullptr && col < N) {
      if (lvv > -INFINITY) gwx::fold_move(gv, gprev[cc], up, dn);
      const double P = bv - gv * itaue;
      if (fabs(P) <= FRAME_P_MAX) kv = -(int)rint(P * gwx::INV_LN2);
      else up = INFINITY;  // also a non-finite P
    }
    if constexpr (BL) kqs[t + NTH * k] = kv;
    else kqr[k] = kv;
    if (blockIdx.x == 0 && gprev != nullptr && col < N) kq[col] = kv;
    S[k] = 0.0;
    X[k] = gwx::EXP_SENTINEL;
  }
  double dup = -1.0;  // D+ of a shifted pass, or -1: exact maxima
  if (SHIFT && gprev != nullptr) {
    double lm = 0.0;
    for (int r = t; r < i1 - i0; r += NTH) {
      const double a = lse[i0 + r];
      lse_b[r] = a;
      lm = fmax(lm, gwx::lse_mag(a));
    }
    up = gwk::wave_max(up) * ie;
    dn = gwk::wave_max(dn) * ie;
    lm = gwk::wave_max(lm);
    if (lane == 63) {
      dred[wv][0] = up;
      dred[wv][1] = dn;
      dred[wv][2] = lm;
    }
    __syncthreads();
    up = dred[0][0];
    dn = dred[0][1];
    lm = dred[0][2];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      up = fmax(up, dred[w][0]);
      dn = fmax(dn, dred[w][1]);
      lm = fmax(lm, dred[w][2]);
    }
    dup = gwx::fast_from(up, dn, lm);
  }
  const bool fast = SHIFT && dup >= 0.0;
  // each thread reads back only its own entries: no barrier needed
  auto b = [&](int k) -> double {
    if constexpr (BL) return bls[t + NTH * k];
    else return breg[k];
  };
  auto kqf = [&](int k) -> int {
    if constexpr (BL) return kqs[t + NTH * k];
    else return kqr[k];
  };
  double cur[R][EPT];
  auto load = [&](int ib) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double* row = C + (int64_t)min(ib + r, i1 - 1) * ldC;
#pragma unroll
      for (int k = 0; k < EPT; ++k) cur[r][k] = row[min(t + NTH * k, N - 1)];
    }
  };
  if (i0 < i1) load(i0);
  for (int ib = i0; ib < i1; ib += R) {
    double z[R][EPT], m[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double ml = -INFINITY;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        z[r][k] = fma(-ie, cur[r][k], b(k));
        if (!fast && (inrow >> k & 1u)) ml = fmax(ml, z[r][k]);
      }
      m[r] = ml;
    }
    load(ib + R);  // the next rows (clamped: past the band it re-reads the last row)
    double lui[R];
#pragma unroll
    for (int r = 0; r < R; ++r) lui[r] = lu[min(ib + r, i1 - 1)];
    if (fast) {
      // the shift: the row's previous bound plus D+ (no maximum)
#pragma unroll
      for (int r = 0; r < R; ++r) m[r] = lse_b[min(ib + r, i1 - 1) - i0] + dup;
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double ml = gwk::wave_max(m[r]);
        if (lane == 63) red[0][r][wv] = ml;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double mr = red[0][r][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) mr = fmax(mr, red[0][r][w]);
        m[r] = mr;
      }
    }
    // the sums go to red[1] in the exact pass (its maxima used red[0] before
    // a barrier) and alternate between the two buffers in the shifted pass,
    // which has one barrier per step
    const int sb = fast ? ((ib - i0) / R) & 1 : 1;
    int nE[R][EPT];
    double sl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double ms = m[r] > -INFINITY ? m[r] : 0.0;
      m[r] = ms;
      sl[r] = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        z[r][k] = gwx::exp_split(fmin(z[r][k] - ms, LAM_MAX), &nE[r][k]);
        if (inrow >> k & 1u) sl[r] += ldexp(z[r][k], nE[r][k]);
      }
      sl[r] = gwk::wave_sum(sl[r]);
      if (lane == 63) red[sb][r][wv] = sl[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = ib + r;
      if (i >= i1) break;
      double s = red[sb][r][0];
#pragma unroll
      for (int w = 1; w < NW; ++w) s += red[sb][r][w];
      const double fi = -tau * e * (m[r] + log(s));
      if (t == 0) {
        f[i] = fi;
        lse[i] = s > 0.0 ? gwx::row_bound(m[r], s) : -INFINITY;
      }
      if (!(s > 0.0) || !(lui[r] > -INFINITY)) continue;  // no terms, or u_i = 0
      const double lam = fmax(fmin(m[r] + ((fi - shift) * ie + lui[r]), LAM_MAX), -LAM_MAX);
      const double nd = rint(lam * gwx::INV_LN2);
      double rr = fma(-nd, gwx::LN2_HI, lam);
      rr = fma(-nd, gwx::LN2_LO, rr);
      const double mw = gwx::exp_reduced(rr);
      const int ew = (int)nd;
      if (fast) {
#pragma unroll
        for (int k = 0; k < EPT; ++k)
          S[k] = fma(ldexp(z[r][k], nE[r][k] + ew + kqf(k)), mw, S[k]);
      } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const int te = nE[r][k] + ew;
          const int ne = max(X[k], te);
          S[k] = ldexp(S[k], X[k] - ne) + ldexp(z[r][k] * mw, te - ne);
          X[k] = ne;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int col = t + NTH * k;
    if (col < N) {
      partS[(int64_t)blockIdx.x * N + col] = S[k];
      if (!fast) partX[(int64_t)blockIdx.x * N + col] = X[k];
    }
  }
  if (t == 0) bmode[blockIdx.x] = fast ? 1 : 0;
}

// Merge of the bands' column sums, in band order: 16 columns x 16 groups of
// bands per block, the groups merged in order; a band of a shifted pass left
// plain sums in the column's frame (exponent -kq_p).  g_p = -tau e (ln S_p -
// b_p); g before the merge is kept for the next pass's test.
constexpr int UM_COLS = 16, UM_GRPS = 16;
constexpr int UM_PER = 16;  // bands per group: nb <= UF_BANDS = UM_GRPS * UM_PER

__global__ __launch_bounds__(UM_COLS * UM_GRPS) void k_uot_merge(
    int N, int nb, const double* __restrict__ partS, const int* __restrict__ partX,
    const int* __restrict__ bmode, const int* __restrict__ kq, const double* __restrict__ lv,
    const UgwScal* __restrict__ sc, double* __restrict__ g, double* __restrict__ gprev,
    gwr::StatusWord* status) {
  __shared__ double ms[UM_GRPS][UM_COLS];
  __shared__ int mx[UM_GRPS][UM_COLS];
  const int c = threadIdx.x % UM_COLS, grp = threadIdx.x / UM_COLS;
  const int col = blockIdx.x * UM_COLS + c, colc = min(col, N - 1);
  const int per = (nb + UM_GRPS - 1) / UM_GRPS;
  const int b0 = grp * per, b1 = min(nb, b0 + per);
  double S = 0.0;
  int X = gwx::EXP_SENTINEL;
  {
    // the sums are requested before the pass kinds are looked at, so that
    // waiting for the kinds does not hold back the sums (indices clamped,
    // entries past the group skipped)
    double sv[UM_PER];
    int fm[UM_PER];
#pragma unroll
    for (int u = 0; u < UM_PER; ++u) sv[u] = partS[(int64_t)min(b0 + u, nb - 1) * N + colc];
#pragma unroll
    for (int u = 0; u < UM_PER; ++u) fm[u] = bmode[min(b0 + u, nb - 1)];
    const int fx = -kq[colc];  // the frame's exponent (bands of a shifted pass)
    bool frames = true;        // every band of the group left frame sums
#pragma unroll
    for (int u = 0; u < UM_PER; ++u) frames = frames && (fm[u] != 0 || b0 + u >= b1);
    if (frames) {
      // all exponents are the frame's: the pair merge below reduces to plain
      // additions in band order (every ldexp is by 0), done directly
      if (b1 > b0) X = fx;
#pragma unroll
      for (int u = 0; u < UM_PER; ++u)
        if (b0 + u < b1) S += sv[u];
    } else {
      int xv[UM_PER];  // all requested before the first is merged
#pragma unroll
      for (int u = 0; u < UM_PER; ++u)
        xv[u] = fm[u] ? fx : partX[(int64_t)min(b0 + u, nb - 1) * N + colc];
#pragma unroll
      for (int u = 0; u < UM_PER; ++u) {
        if (b0 + u < b1) {
          const int ne = max(X, xv[u]);
          S = ldexp(S, X - ne) + ldexp(sv[u], xv[u] - ne);
          X = ne;
        }
      }
    }
  }
  ms[grp][c] = S;
  mx[grp][c] = X;
  __syncthreads();
  if (grp != 0 || col >= N) return;
  for (int k = 1; k < UM_GRPS; ++k) {
    const int ne = max(X, mx[k][c]);
    S = ldexp(S, X - ne) + ldexp(ms[k][c], mx[k][c] - ne);
    X = ne;
  }
  const double shift = sc->shift, e = sc->e, ie = 1.0 / e;
  const double gold = g[col];
  const double bp = col_base(gold, lv[col], shift, ie);
  const double lnS =
      S > 0.0 ? fma((double)X, gwx::LN2_HI, fma((double)X, gwx::LN2_LO, log(S))) : -INFINITY;
  const double gn = -sc->tau * e * (lnS - bp);
  gprev[col] = gold;
  g[col] = gn;
  if (isnan(gn)) status->nonfinite = 1;
}

// Rows per band of the one-pass update: at most UF_BANDS bands, a multiple of
// the rows a step takes (2).
int uot_band_rows(int64_t M) {
  int64_t rb = (M + UF_BANDS - 1) / UF_BANDS;
  rb = (rb + 1) / 2 * 2;
  return (int)(rb < 2 ? 2 : rb);
}

gw_status launch_uot_fused(const double* C, int64_t ldC, int64_t M, int64_t N, int RB,
                           const double* g, const double* gprev, const double* lu,
                           const double* lv, const UgwScal* sc, double* f, double* lse, int* kq,
                           int* bmode, double* partS, int* partX, hipStream_t s) {
  if (RB > UF_MAX_RB) return GW_EUNSUPPORTED;
  const unsigned nb = (unsigned)((M + RB - 1) / RB);
  const int m = (int)M, n = (int)N;
#define UF_ARGS C, ldC, m, n, RB, g, gprev, lu, lv, sc, f, lse, kq, bmode, partS, partX
  // rows of 4097-8192 entries stay exact: the shifted variant's extra state
  // pushes that shape into spills (measured 9% slower per pass)
  if (N <= 256) k_uot_fused<256, 1, 2, true><<<nb, 256, 0, s>>>(UF_ARGS);
  else if (N <= 512) k_uot_fused<256, 2, 2, true><<<nb, 256, 0, s>>>(UF_ARGS);
  else if (N <= 1024) k_uot_fused<256, 4, 2, true><<<nb, 256, 0, s>>>(UF_ARGS);
  else if (N <= 2048) k_uot_fused<256, 8, 2, true><<<nb, 256, 0, s>>>(UF_ARGS);
  else if (N <= 4096) k_uot_fused<512, 8, 1, true><<<nb, 512, 0, s>>>(UF_ARGS);
  else if (N <= 8192) k_uot_fused<512, 16, 1, false><<<nb, 512, 0, s>>>(UF_ARGS);
  else return GW_EUNSUPPORTED;
#undef UF_ARGS
  return GW_OK;
}

constexpr int64_t UF_MAX_N = 8192;

// Column update, first stage: (m, s) of LSE_i((f_i - C_ip - shift)/e + ln u_i)
// over the rows of chunk blockIdx.y, for 64 columns; each wave takes a
// contiguous part of the chunk, the waves are merged in order.
__global__ __launch_bounds__(UC_COLS * UC_WAVES) void k_uot_colpart(
    const double* __restrict__ C, int64_t ldC, int M, int N, int rows_per_chunk,
    const double* __restrict__ f, const double* __restrict__ lu, const UgwScal* __restrict__ sc,
    double* __restrict__ pm, double* __restrict__ ps) {
  __shared__ double sm[UC_WAVES][UC_COLS], ss[UC_WAVES][UC_COLS];
  const int lane = threadIdx.x & (UC_COLS - 1), wv = threadIdx.x / UC_COLS;
  const int col = blockIdx.x * UC_COLS + lane, colc = min(col, N - 1);
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(M, r0 + rows_per_chunk);
  const int len = (r1 - r0 + UC_WAVES - 1) / UC_WAVES;
  const int a0 = r0 + wv * len, a1 = min(r1, a0 + len);
  const double shift = sc->shift, ie = 1.0 / sc->e;
  double m = -INFINITY, s = 0.0;
  for (int i = a0; i < a1; ++i) {
    const double z = (f[i] - C[(int64_t)i * ldC + colc] - shift) * ie + lu[i];
    if (z > m) {
      s = s * exp(m - z) + 1.0;
      m = z;
    } else if (z > -INFINITY) {
      s += exp(z - m);
    }
  }
  sm[wv][lane] = m;
  ss[wv][lane] = s;
  __syncthreads();
  if (wv != 0 || col >= N) return;
  for (int w = 1; w < UC_WAVES; ++w) lse_merge(m, s, sm[w][lane], ss[w][lane]);
  pm[(int64_t)blockIdx.y * N + col] = m;
  ps[(int64_t)blockIdx.y * N + col] = s;
}

// Column update, second stage: a wave per column, lane r holding chunk r
// (R <= 64), merged by a butterfly (a fixed order), g_p = -tau e LSE.
__global__ __launch_bounds__(256) void k_uot_colmerge(int N, int R, const double* __restrict__ pm,
                                                      const double* __restrict__ ps,
                                                      const UgwScal* __restrict__ sc,
                                                      double* __restrict__ g,
                                                      gwr::StatusWord* status) {
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6), r = threadIdx.x & 63;
  const int cc = min(col, N - 1);
  double m = -INFINITY, s = 0.0;
  if (r < R) {
    m = pm[(int64_t)r * N + cc];
    s = ps[(int64_t)r * N + cc];
  }
  for (int o = 1; o < 64; o <<= 1) {
    const double m2 = __shfl_xor(m, o, 64), s2 = __shfl_xor(s, o, 64);
    lse_merge(m, s, m2, s2);
  }
  if (r != 0 || col >= N) return;
  const double L = m == -INFINITY ? -INFINITY : m + log(s);
  const double gn = -sc->tau * sc->e * L;
  g[col] = gn;
  if (isnan(gn)) status->nonfinite = 1;
}

// T_ip = exp((f_i + g_p - C_ip - shift)/e) u_i v_p; with rowsum, each row's sum.
__global__ __launch_bounds__(256) void k_uot_plan(const double* __restrict__ C, int64_t ldC,
                                                  int N, const double* __restrict__ f,
                                                  const double* __restrict__ g,
                                                  const double* __restrict__ u,
                                                  const double* __restrict__ v,
                                                  const UgwScal* __restrict__ sc,
                                                  double* __restrict__ T, int64_t ldT,
                                                  double* __restrict__ rowsum) {
  __shared__ double red[4];
  const int64_t i = blockIdx.x;
  const double fi = f[i], ui = u[i], shift = sc->shift, ie = 1.0 / sc->e;
  double acc = 0.0;
  for (int p = threadIdx.x; p < N; p += 256) {
    const double val = exp((fi + g[p] - C[i * ldC + p] - shift) * ie) * ui * v[p];
    T[i * ldT + p] = val;
    acc += val;
  }
  acc = block_sum<256>(acc, red);
  if (rowsum != nullptr && threadIdx.x == 0) rowsum[i] = acc;
}

// rowpart[i] = sum_p T_ip log T_ip (0 log 0 = 0).
__global__ __launch_bounds__(256) void k_ugw_tlogt(const double* __restrict__ T, int64_t ldT,
                                                   int N, double* __restrict__ rowpart) {
  __shared__ double red[4];
  const int64_t i = blockIdx.x;
  double acc = 0.0;
  for (int p = threadIdx.x; p < N; p += 256) {
    const double x = T[i * ldT + p];
    if (x > 0.0) acc += x * log(x);
  }
  acc = block_sum<256>(acc, red);
  if (threadIdx.x == 0) rowpart[i] = acc;
}

// Sums of a step (one block, fixed order): m = sum a, the shift g(Th), e, tau.
struct UgwSums {
  double m, alogau, blogbv, tlogt, alogu, blogv;
};

GW_DEV UgwSums ugw_sums(const double* a, const double* b, const double* u, const double* v,
                        const double* rowpart, int M, int N, double* red) {
  double m = 0.0, au = 0.0, al = 0.0, tl = 0.0;
  double bv = 0.0, bl = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) {
    const double x = a[i];
    m += x;
    tl += rowpart[i];
    if (x > 0.0) {
      au += x * log(x / u[i]);
      al += x * log(u[i]);
    }
  }
  for (int p = threadIdx.x; p < N; p += 256) {
    const double x = b[p];
    if (x > 0.0) {
      bv += x * log(x / v[p]);
      bl += x * log(v[p]);
    }
  }
  UgwSums r;
  r.m = block_sum<256>(m, red);
  r.alogau = block_sum<256>(au, red);
  r.blogbv = block_sum<256>(bv, red);
  r.tlogt = block_sum<256>(tl, red);
  r.alogu = block_sum<256>(al, red);
  r.blogv = block_sum<256>(bl, red);
  return r;
}

__global__ __launch_bounds__(256) void k_ugw_scalars(const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ rowpart, int M,
                                                     int N, double rho, double eps,
                                                     UgwScal* __restrict__ sc) {
  __shared__ double red[4];
  const UgwSums S = ugw_sums(a, b, u, v, rowpart, M, N, red);
  if (threadIdx.x != 0) return;
  sc->m = S.m;
  sc->shift = rho * S.alogau + rho * S.blogbv + eps * ((S.tlogt - S.alogu) - S.blogv);
  sc->e = S.m * eps;
  sc->tau = rho / (rho + eps);
}

// m(u), m(v) and the initial plan's factor 1 / sqrt(m(u) m(v)).
__global__ __launch_bounds__(256) void k_ugw_masses(const double* __restrict__ u,
                                                    const double* __restrict__ v, int M, int N,
                                                    UgwScal* __restrict__ sc) {
  __shared__ double red[4];
  double su = 0.0, sv = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) su += u[i];
  for (int p = threadIdx.x; p < N; p += 256) sv += v[p];
  su = block_sum<256>(su, red);
  sv = block_sum<256>(sv, red);
  if (threadIdx.x == 0) {
    sc->mu = su;
    sc->mv = sv;
    sc->factor = 1.0 / sqrt(su * sv);
  }
}

// T_ip = factor u_i v_p.
__global__ __launch_bounds__(256) void k_ugw_outer(const double* __restrict__ u,
                                                   const double* __restrict__ v, int N,
                                                   const UgwScal* __restrict__ sc,
                                                   double* __restrict__ T, int64_t ldT) {
  const int64_t i = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < N) T[i * ldT + p] = sc->factor * u[i] * v[p];
}

// factor = sqrt(m(Th) / m(T)) from the plan's row sums; then T *= factor.
__global__ __launch_bounds__(256) void k_ugw_rescale(const double* __restrict__ rowsum, int M,
                                                     UgwScal* __restrict__ sc,
                                                     gwr::StatusWord* status) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) s += rowsum[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) {
    const double fct = sqrt(sc->m / s);
    sc->factor = fct;
    if (!isfinite(fct)) status->nonfinite = 1;  // an empty plan or a non-finite step
  }
}

__global__ __launch_bounds__(256) void k_ugw_scale(double* __restrict__ T, int64_t ldT, int N,
                                                   const UgwScal* __restrict__ sc) {
  const int64_t i = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < N) T[i * ldT + p] *= sc->factor;
}

// obj[0] = E + rho (KL(a(x)a|u(x)u) + KL(b(x)b|v(x)v)),
// obj[1] = obj[0] + eps KL(T(x)T|(u(x)v)(x)(u(x)v)),
// KL(x(x)x|y(x)y) = 2 m(x) KL(x|y) + (m(x) - m(y))^2.
__global__ __launch_bounds__(256) void k_ugw_objective(const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ rowpart, int M,
                                                       int N, double rho, double eps,
                                                       const UgwScal* __restrict__ sc,
                                                       const double* __restrict__ eobj,
                                                       double* __restrict__ obj) {
  __shared__ double red[4];
  const UgwSums S = ugw_sums(a, b, u, v, rowpart, M, N, red);
  if (threadIdx.x != 0) return;
  const double mT = S.m, mu = sc->mu, mv = sc->mv;
  const double kla = S.alogau - mT + mu, klb = S.blogbv - mT + mv;
  const double klt = ((S.tlogt - S.alogu) - S.blogv) - mT + mu * mv;
  const double qa = 2.0 * mT * kla + (mT - mu) * (mT - mu);
  const double qb = 2.0 * mT * klb + (mT - mv) * (mT - mv);
  const double qt = 2.0 * mT * klt + (mT - mu * mv) * (mT - mu * mv);
  const double U = eobj[0] + rho * (qa + qb);
  obj[0] = U;
  obj[1] = U + eps * qt;
}

int uot_chunks(int64_t M) {
  const int64_t r = (M + 255) / 256;
  return (int)(r < 1 ? 1 : (r > UC_MAX_CHUNKS ? UC_MAX_CHUNKS : r));
}

gw_status launch_uot_row(const double* C, int64_t ldC, int64_t M, int64_t N, const double* g,
                         const double* lv, const UgwScal* sc, double* f, hipStream_t s) {
  // rows up to 4096 entries: 256 threads (cheaper block reductions), longer: 1024
  const unsigned m = (unsigned)M;
  const int n = (int)N;
  if (N <= 256) k_uot_row<256, 1><<<m, 256, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else if (N <= 1024) k_uot_row<256, 4><<<m, 256, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else if (N <= 2048) k_uot_row<256, 8><<<m, 256, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else if (N <= 4096) k_uot_row<256, 16><<<m, 256, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else if (N <= 8192) k_uot_row<UR_NT, 8><<<m, UR_NT, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else if (N <= 16384) k_uot_row<UR_NT, 16><<<m, UR_NT, 0, s>>>(C, ldC, n, g, lv, sc, f);
  else return GW_EUNSUPPORTED;
  return GW_OK;
}

}  // namespace

namespace gwl {

size_t uot_scalars_bytes() { return gwr::align_up(sizeof(UgwScal), 256); }

size_t uot_ws_bytes(int64_t M, int64_t N) {
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(M);  // ln u
  a.take<double>(N);  // ln v
  if (N <= UF_MAX_N) {  // the one-pass update
    const int64_t nb = (M + uot_band_rows(M) - 1) / uot_band_rows(M);
    a.take<double>((size_t)nb * N);  // the bands' column sums
    a.take<int>((size_t)nb * N);     // and their exponents (exact pass)
    a.take<double>(M);               // row bounds
    a.take<double>(N);               // g before the last merge
    a.take<int>(N);                  // column frames of a shifted pass
    a.take<int>(nb);                 // pass kind of each band
  } else {
    const int R = uot_chunks(M);
    a.take<double>((size_t)R * N);
    a.take<double>((size_t)R * N);
  }
  a.take<double>(M);  // row sums of the plan
  return a.used;
}

gw_status uot_set_scalars(void* scal, double shift, double e, double tau, hipStream_t s) {
  k_uot_set<<<1, 64, 0, s>>>(static_cast<UgwScal*>(scal), shift, e, tau);
  return gwr::last_launch_status();
}

// Unbalanced Sinkhorn on C + shift with the step scalars in `scal`; with T the
// plan, and with rescale its mass set to m (scal) times sqrt(m / m(plan)).
gw_status uot_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, const double* u,
                       const double* v, int iters, int init_zero, double* f, double* g,
                       double* T, int64_t ldT, bool rescale, void* scal, gwr::Arena& ws,
                       hipStream_t s, gwr::StatusWord* status) {
  if (N > 16 * UR_NT) return GW_EUNSUPPORTED;
  UgwScal* sc = static_cast<UgwScal*>(scal);
  double* lu = ws.take<double>(M);
  double* lv = ws.take<double>(N);
  const bool fused = N <= UF_MAX_N;
  const int RB = uot_band_rows(M);
  const int64_t nb = (M + RB - 1) / RB;
  const int R = uot_chunks(M);
  double *pm = nullptr, *ps = nullptr, *partS = nullptr, *lse = nullptr, *gprev = nullptr;
  int *partX = nullptr, *kq = nullptr, *bmode = nullptr;
  if (fused) {
    partS = ws.take<double>((size_t)nb * N);
    partX = ws.take<int>((size_t)nb * N);
    lse = ws.take<double>(M);
    gprev = ws.take<double>(N);
    kq = ws.take<int>(N);
    bmode = ws.take<int>(nb);
  } else {
    pm = ws.take<double>((size_t)R * N);
    ps = ws.take<double>((size_t)R * N);
  }
  double* rowsum = ws.take<double>(M);
  gwr::ProfScope prof(gwr::kFamOther, s);
  const int64_t mx = M > N ? M : N;
  k_uot_logs<<<(unsigned)((mx + 255) / 256), 256, 0, s>>>(u, v, (int)M, (int)N, lu, lv, f, g,
                                                          init_zero);
  const int rpc = (int)((M + R - 1) / R);
  const dim3 cgrid((unsigned)((N + UC_COLS - 1) / UC_COLS), (unsigned)R);
  for (int it = 0; it < iters && fused; ++it) {
    // the first pass of a call is exact (no previous g to bound the moves)
    gw_status st = launch_uot_fused(C, ldC, M, N, RB, g, it > 0 ? gprev : nullptr, lu, lv, sc,
                                    f, lse, kq, bmode, partS, partX, s);
    if (st != GW_OK) return st;
    k_uot_merge<<<(unsigned)((N + UM_COLS - 1) / UM_COLS), UM_COLS * UM_GRPS, 0, s>>>(
        (int)N, (int)nb, partS, partX, bmode, kq, lv, sc, g, gprev, status);
  }
  for (int it = 0; it < iters && !fused; ++it) {
    gw_status st = launch_uot_row(C, ldC, M, N, g, lv, sc, f, s);
    if (st != GW_OK) return st;
    k_uot_colpart<<<cgrid, UC_COLS * UC_WAVES, 0, s>>>(C, ldC, (int)M, (int)N, rpc, f, lu, sc,
                                                       pm, ps);
    k_uot_colmerge<<<(unsigned)((N + 3) / 4), 256, 0, s>>>((int)N, R, pm, ps, sc, g, status);
  }
  if (T) {
    k_uot_plan<<<(unsigned)M, 256, 0, s>>>(C, ldC, (int)N, f, g, u, v, sc, T, ldT,
                                           rescale ? rowsum : nullptr);
    if (rescale) {
      k_ugw_rescale<<<1, 256, 0, s>>>(rowsum, (int)M, sc, status);
      const dim3 sg((unsigned)((N + 255) / 256), (unsigned)M);
      k_ugw_scale<<<sg, 256, 0, s>>>(T, ldT, (int)N, sc);
    }
  }
  return gwr::last_launch_status();
}

// Set-up of a UGW solve: m(u), m(v) into the step scalars and T^0.
gw_status ugw_init(const double* u, const double* v, int64_t M, int64_t N, double* T,
                   int64_t ldT, void* scal, hipStream_t s) {
  gwr::ProfScope prof(gwr::kFamOther, s);
  UgwScal* sc = static_cast<UgwScal*>(scal);
  k_ugw_masses<<<1, 256, 0, s>>>(u, v, (int)M, (int)N, sc);
  const dim3 grid((unsigned)((N + 255) / 256), (unsigned)M);
  k_ugw_outer<<<grid, 256, 0, s>>>(u, v, (int)N, sc, T, ldT);
  return gwr::last_launch_status();
}

// The step scalars from T (its marginals a, b already in place): m, g(T), e, tau.
gw_status ugw_step_scalars(const double* T, int64_t ldT, int64_t M, int64_t N, const double* a,
                           const double* b, const double* u, const double* v, double rho,
                           double eps, double* rowpart, void* scal, hipStream_t s) {
  gwr::ProfScope prof(gwr::kFamOther, s);
  k_ugw_tlogt<<<(unsigned)M, 256, 0, s>>>(T, ldT, (int)N, rowpart);
  k_ugw_scalars<<<1, 256, 0, s>>>(a, b, u, v, rowpart, (int)M, (int)N, rho, eps,
                                  static_cast<UgwScal*>(scal));
  return gwr::last_launch_status();
}

// obj from E (device, eobj[0]) and T's marginals a, b.
gw_status ugw_objective(const double* T, int64_t ldT, int64_t M, int64_t N, const double* a,
                        const double* b, const double* u, const double* v, double rho,
                        double eps, double* rowpart, const void* scal, const double* eobj,
                        double* obj, hipStream_t s) {
  gwr::ProfScope prof(gwr::kFamOther, s);
  k_ugw_tlogt<<<(unsigned)M, 256, 0, s>>>(T, ldT, (int)N, rowpart);
  k_ugw_objective<<<1, 256, 0, s>>>(a, b, u, v, rowpart, (int)M, (int)N, rho, eps,
                                    static_cast<const UgwScal*>(scal), eobj, obj);
  return gwr::last_launch_status();
}

}  // namespace gwl
