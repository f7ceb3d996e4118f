// Log-domain Sinkhorn for the entropic OT sub-problem of each mirror-descent
// step (Sec. 2.1, Eq. (GW sinkhorn); tau = eps Remark), plan materialisation,
// and the reductions behind the objective.
//
// One iteration is f_i = eps ln p_i - eps LSE_p((g_p - C_ip)/eps), then
// g_p = eps ln q_p - eps LSE_i((f_i - C_ip)/eps).  It is done in one pass over
// C plus a small merge:
//   row pass   a block owns a band of rows; for each row it computes the
//              shifted exponentials E_ip = exp(z_ip - m_i), z = (g - C)/eps,
//              m_i = max_p z_ip, and f_i from their sum s_i.  The column
//              quantity exp((f_i - C_ip)/eps) equals E_ip (p_i/s_i) e^{-g_p/eps},
//              so the same E_ip feed the column sums without a second
//              exponential.  Because E_ip (p_i/s_i) can be far below the
//              double range for a column that no row favours, each E is kept
//              as mantissa x 2^n (the exponent comes from the argument
//              reduction exp(x) = 2^n exp(x - n ln 2), Cody-Waite split of
//              ln 2) and the column sums are accumulated as (mantissa, shared
//              binary exponent) pairs, rescaled with ldexp, never with exp;
//   col merge  one thread per column merges the bands' pairs and sets
//              g_p = g_p + eps (ln q_p - ln S_p), ln S_p = ln(mant) + e ln 2,
//              which is the LSE update rewritten with the old g as the shift.
// Zero-mass rows/columns get f = -inf / g = -inf directly and contribute
// nothing.  All sums are in a fixed order.
//
// Row shift without a max pass: the shift of a row only has to bound its
// maximum from above without being far above it.  Each pass leaves
// a_i = m_i + e_i ln 2 (m_i its shift, 2^e_i > s_i), an upper bound of the
// row's log-sum-exp.  If the column merge moved g by at most D+ up and D- down
// (in units of eps), the next pass's row maximum is at most a_i + D+ and its
// shifted sum at least e^{-(ln 2N + D+ + D-)}; with D+ + D- <= 600 the pass
// shifts by a_i + D+ and skips the max reduction.  The first pass of a call,
// and any pass after a larger move, takes the exact maximum.  D+ and D- are
// maxima over columns: the column merge keeps the previous g beside the new
// one, and every row-pass block reduces the move over all columns itself (one
// block reduction per band, no atomics), so the choice, and every result, is
// deterministic.
#include <limits.h>

#include <hip/hip_ext.h>

#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "common.h"
#include "expx.h"
#include "runtime.h"

namespace {

using gwx::EXP_SENTINEL;
using gwx::INV_LN2;
using gwx::LN2_HI;
using gwx::LN2_LO;
using gwx::X_FLOOR;
using gwx::exp_reduced;
using gwx::exp_split;
using gwx::FAST_M_MAX;
using gwx::FAST_UP_MAX;
using gwx::SHIFT_SPREAD_MAX;
using gwx::fast_from;
using gwx::fold_move;
using gwx::lse_mag;
using gwx::row_bound;

// D+ for the pass (or -1: exact maxima) from g and g before the last merge
// (gprev, null in the first iteration of a call), reduced over all columns by
// the block (every block computes the same D+ and D-), and the largest |lse_i|
// of the band's rows [i0, i1).  N <= NT * NC, i1 - i0 <= NT.
template <int NT, int NC>
GW_DEV double pass_shift(const double* __restrict__ g, const double* __restrict__ gprev, int N,
                         double inv_eps, const double* __restrict__ lse, int i0, int i1,
                         double (*red3)[3]);


template <int NT, int NC>
GW_DEV double pass_shift(const double* __restrict__ g, const double* __restrict__ gprev, int N,
                         double inv_eps, const double* __restrict__ lse, int i0, int i1,
                         double (*red3)[3]) {
  if (gprev == nullptr) return -1.0;
  // every load is issued before any is used (indices clamped into range)
  double gn[NC], go[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = min((int)threadIdx.x + NT * k, N - 1);
    gn[k] = g[c];
    go[k] = gprev[c];
  }
  const double lv = lse[min(i0 + (int)threadIdx.x, i1 - 1)];
  double up = 0.0, dn = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k)
    if ((int)threadIdx.x + NT * k < N) fold_move(gn[k], go[k], up, dn);
  double lm = lse_mag(lv);
  up = gwk::wave_max(up) * inv_eps;
  dn = gwk::wave_max(dn) * inv_eps;
  lm = gwk::wave_max(lm);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) {
    red3[w][0] = up;
    red3[w][1] = dn;
    red3[w][2] = lm;
  }
  __syncthreads();
  up = red3[0][0];
  dn = red3[0][1];
  lm = red3[0][2];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) {
    up = fmax(up, red3[k][0]);
    dn = fmax(dn, red3[k][1]);
    lm = fmax(lm, red3[k][2]);
  }
  return fast_from(up, dn, lm);
}

template <int NTH>
GW_DEV double block_max(double v, double* red) {
  v = gwk::wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < NTH / 64; ++i) r = fmax(r, red[i]);
  return r;
}

template <int NTH>
GW_DEV double block_sum(double v, double* red) {
  v = gwk::wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < NTH / 64; ++i) r += red[i];
  return r;
}

// threadIdx.x behind an empty asm statement: values derived from it cannot be
// hoisted out of the persistent item loops of the batched kernels, where they
// would stay live across the loop and push the band bodies into spills.
GW_DEV int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ---- fast pass: rows shifted by a multiple of ln 2, columns in fixed frames
//
// A fast pass shifts row i by M_i = nm_i ln 2, nm_i = ceil((lse_i + D+) / ln 2),
// so exp(z - M_i) = 2^(rint(z / ln 2) - nm_i) e^r with r = z - rint(z / ln 2) ln 2:
// the reduction works on z itself and the shift only enters the exponent.
// Adding z / ln 2 to SHIFTER - nm_i (SHIFTER = 1.5 2^52) rounds it to an
// integer and leaves rint(z / ln 2) - nm_i in the low 32 bits of the sum, so
// one FMA gives both the reduction integer and the final exponent.  The
// two-constant split stays exact while |rint(z / ln 2)| < 2^21, which holds
// for |M_i| < FAST_M_MAX and z >= M_i - FAST_ZSPAN (z is clamped there; terms
// below the clamp are 0 in every frame used).
//
// Column sums of a fast pass are plain doubles in a frame 2^kq_p per column
// (kq_p = max(0, -e_p - FRAME_OFFSET), q_p = m 2^e_p, m in [0.5, 1)), so
// q_p 2^kq_p lies in [2^-101, 1].  After the previous merge,
// sum_i exp((f_i - C_ip + g_p)/eps) = q_p for the f of the previous pass; the
// new f differs from it by at most D+ eps below and D- eps above (the row
// log-sum-exp moves by at most the largest move of g), so the frame sum lies
// in q_p 2^kq_p [e^-D+, e^D-], inside [2^-895, 2^866] for D+ <= FAST_UP_MAX
// and D+ + D- <= SHIFT_SPREAD_MAX: no (mantissa, exponent) pairs are needed.
constexpr double SHIFTER = 0x1.8p52;
constexpr double FAST_ZSPAN = 2560.0;
constexpr int FRAME_OFFSET = 100;

struct FastShift {
  double sh;    // SHIFTER - nm
  double zlo;   // clamp of z
  double mrow;  // nm ln 2, the shift applied
};

GW_DEV FastShift fast_shift(double m) {
  const double nm = ceil(m * INV_LN2);
  FastShift fs;
  fs.sh = SHIFTER - nm;
  fs.mrow = fma(nm, LN2_HI, nm * LN2_LO);
  fs.zlo = fs.mrow - FAST_ZSPAN;
  return fs;
}

// exp(z - M) = e^r 2^n for the shift of fs.
GW_DEV double exp_fast(double z, const FastShift& fs, int& n) {
  z = fmax(z, fs.zlo);
  const double u = fma(z, INV_LN2, fs.sh);
  const double nd = u - fs.sh;
  double r = fma(-nd, LN2_HI, z);
  r = fma(-nd, LN2_LO, r);
  n = __double2loint(u);
  return exp_reduced(r);
}


// Log-marginals, the column frames of the fast pass and (cold start) zero
// potentials.
__global__ __launch_bounds__(256) void k_sk_prep(const double* __restrict__ p,
                                                  const double* __restrict__ q, int M, int N,
                                                  int init_zero, double* __restrict__ logp,
                                                  double* __restrict__ logq,
                                                  int* __restrict__ kq,
                                                  double* __restrict__ f,
                                                  double* __restrict__ g) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < M) logp[idx] = p[idx] > 0.0 ? log(p[idx]) : -INFINITY;
  if (idx < N) {
    const double qv = q[idx];
    logq[idx] = qv > 0.0 ? log(qv) : -INFINITY;
    int eq = 0;
    (void)frexp(qv, &eq);
    kq[idx] = qv > 0.0 ? max(0, -eq - FRAME_OFFSET) : 0;
    if (init_zero) g[idx] = 0.0;
  }
  if (init_zero && idx < M) f[idx] = 0.0;
}

// Row pass.  A block of NTH threads owns rows [blockIdx.x * RB, +RB); thread t
// owns columns t + NTH * e.  Rows are taken R at a time (their reductions share
// barriers) and the next R rows are loaded before the current ones are
// reduced, so loads stay in flight across the barriers.
// The body works on band `band` so that the batched kernels of the request
// loop run exactly the same arithmetic on a band as the single-problem kernel.
// LDS of a row-pass shape, shared by its two variants (one static allocation
// per shape, not per variant).
// Rows per band are at most 256 (M <= 65535 over 256 bands).  The band's
// per-row scalars (p_i, the row bound lse_i, and the row's shift and sum) live
// in LDS while the band runs: read at the band's start, written back at its
// end, so the row steps issue no loads or stores of them.
constexpr int kMaxBandRows = 256;
struct BandRows {
  double p[kMaxBandRows];
  double lse[kMaxBandRows];
  double m[kMaxBandRows];
  double s[kMaxBandRows];
};

template <int NTH, int EPT, int R, bool GL>
struct RowLds {
  double red[2][R][NTH / 64];
  double dred[NTH / 64][3];
  double gls[GL ? EPT * NTH : 1];
  BandRows br;
};
template <int NTH, int EPT, int R, bool GL>
GW_DEV RowLds<NTH, EPT, R, GL>& row_lds() {
  __shared__ RowLds<NTH, EPT, R, GL> l;
  return l;
}

template <int EPT, int NG>
struct RowgLds {
  union {
    double gie[EPT * (1024 / NG)];                    // g/eps while the rows run
    double mS[NG > 1 ? NG - 1 : 1][EPT][1024 / NG];  // then the groups' mantissas
  } u;
  int mX[NG > 1 ? NG - 1 : 1][EPT][1024 / NG];
  int kqs[EPT * (1024 / NG)];  // column frames of the fast pass
  double dred[16][3];
  double red[2][NG][1024 / NG / 64];
  BandRows br;
};

// The band's p_i and (fast pass) lse_i into LDS; thread t < rows loads row
// i0 + t.  Visible after the caller's next barrier.
GW_DEV void band_rows_load(BandRows& br, const double* __restrict__ p,
                           const double* __restrict__ lse, int i0, int rows, int t,
                           bool need_lse) {
  if (t < rows) {
    br.p[t] = p[i0 + t];
    if (need_lse) br.lse[t] = lse[i0 + t];
  }
}

// Row bounds, and with write_f the rows' (shift, sum), back to global memory;
// zero-mass rows get f = -inf.  After a barrier that follows the last row.
GW_DEV void band_rows_store(const BandRows& br, double* __restrict__ lse, double* __restrict__ ms,
                            double* __restrict__ f, int write_f, int i0, int rows, int t) {
  if (t < rows) {
    const int i = i0 + t;
    lse[i] = br.lse[t];
    if (!(br.p[t] > 0.0)) {
      f[i] = -INFINITY;
    } else if (write_f) {
      ms[2 * i] = br.m[t];
      ms[2 * i + 1] = br.s[t];
    }
  }
}
template <int EPT, int NG>
GW_DEV RowgLds<EPT, NG>& rowg_lds() {
  __shared__ RowgLds<EPT, NG> l;
  return l;
}

// GL: g_p / eps is kept in LDS instead of registers.  PF: the next rows are
// loaded while the current ones are reduced (two row buffers); without it the
// next rows are loaded after the column update into the same registers, which
// leaves room for up to 32 entries per thread at 512 threads.
// FAST (dup = D+ >= 0): rows shifted by their bound lse_i + D+ rounded up to a
// multiple of ln 2, column sums in the per-column frames 2^kq_p; otherwise the
// exact row maxima and (mantissa, exponent) column pairs.  bmode[band] records
// which of the two the band's partials are.
template <int NTH, int EPT, int R, bool GL, bool PF, bool FAST>
GW_DEV void sk_row_band(const double* __restrict__ C, int64_t ldC, int M, int N, int RB,
                        double cs, double inv_eps, const double* __restrict__ p,
                        const double* __restrict__ logp, const double* __restrict__ g,
                        const int* __restrict__ kq, double* __restrict__ f,
                        double* __restrict__ ms, double* __restrict__ partS,
                        int* __restrict__ partX, int* __restrict__ bmode,
                        double* __restrict__ lse, double dup, int write_f, int band) {
  constexpr int NW = NTH / 64;
  auto& lds = row_lds<NTH, EPT, R, GL>();
  auto& red = lds.red;
  double* gls = lds.gls;
  const int t = opaque_tid(), wv = t >> 6, lane = t & 63;
  const double csie = cs * inv_eps;
  double S[EPT];
  int Xe[FAST ? 1 : EPT];
  int kqc[FAST ? EPT : 1];   // column frames (fast pass)
  double gir[GL ? 1 : EPT];  // g_p / eps
  if constexpr (FAST) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) kqc[e] = kq[min(t + NTH * e, N - 1)];
  }
  if constexpr (GL && EPT > 24) {
    // g/eps to LDS one entry at a time (the longest rows have no registers to
    // spare for a batch of loads)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int col = t + NTH * e;
      S[e] = 0.0;
      if constexpr (!FAST) Xe[e] = EXP_SENTINEL;
      gls[t + NTH * e] = col < N ? g[col] * inv_eps : -INFINITY;
    }
  } else if constexpr (GL) {
    // g/eps to LDS, loads issued 8 at a time before they are used
#pragma unroll
    for (int e0 = 0; e0 < EPT; e0 += 8) {
      double graw[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) graw[u] = g[min(t + NTH * min(e0 + u, EPT - 1), N - 1)];
#pragma unroll
      for (int u = 0; u < 8 && e0 + u < EPT; ++u) {
        const int e = e0 + u, col = t + NTH * e;
        S[e] = 0.0;
        if constexpr (!FAST) Xe[e] = EXP_SENTINEL;
        gls[col] = col < N ? graw[u] * inv_eps : -INFINITY;
      }
    }
  } else {
    double graw[EPT];  // all loads issued before any is used (indices clamped)
#pragma unroll
    for (int e = 0; e < EPT; ++e) graw[e] = g[min(t + NTH * e, N - 1)];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      S[e] = 0.0;
      if constexpr (!FAST) Xe[e] = EXP_SENTINEL;
      gir[e] = t + NTH * e < N ? graw[e] * inv_eps : -INFINITY;
    }
  }
  if constexpr (GL) __syncthreads();
  auto gie = [&](int e) -> double {
    if constexpr (GL) return gls[t + NTH * e];
    else return gir[e];
  };
  const int i0 = band * RB, i1 = min(M, i0 + RB);
  double cur[R][EPT];
  // Loads are unconditional (row and column indices clamped into range) so the
  // compiler can keep the next rows in flight across the reductions.
  int colc[EPT];  // column of each entry, clamped into range
#pragma unroll
  for (int e = 0; e < EPT; ++e) colc[e] = min(t + NTH * e, N - 1);
  auto load = [&](double (&dst)[R][EPT], int ib) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = min(ib + r, i1 - 1);
      const double* row = C + (int64_t)i * ldC;
#pragma unroll
      for (int e = 0; e < EPT; ++e) dst[r][e] = row[colc[e]];
    }
  };
  if (i0 < i1) load(cur, i0);
  // The next R rows are loaded into `cur` as soon as the current rows have
  // been turned into exponents, so the loads overlap the reductions, the
  // exponentials and the column updates.
  auto& br = lds.br;  // the band's p_i and row bounds, staged by the caller
  for (int ib = i0; ib < i1; ib += R) {
    double pv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pv[r] = br.p[min(ib + r, i1 - 1) - i0];
    double z[R][EPT];
    double m[R];  // the shift of each row
    FastShift fs[FAST ? R : 1];
    if constexpr (FAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        fs[r] = fast_shift(br.lse[min(ib + r, i1 - 1) - i0] + dup);
        m[r] = fs[r].mrow;
#pragma unroll
        for (int e = 0; e < EPT; ++e) z[r][e] = fma(-csie, cur[r][e], gie(e));
      }
      if constexpr (PF) load(cur, ib + R);  // clamped: past the band it re-reads the last row
    } else {
      double mloc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mloc[r] = -INFINITY;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          z[r][e] = fma(-csie, cur[r][e], gie(e));
          mloc[r] = fmax(mloc[r], z[r][e]);
        }
      }
      if constexpr (PF) load(cur, ib + R);  // clamped: past the band it re-reads the last row
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mloc[r] = gwk::wave_max(mloc[r]);
        if (lane == 63) red[0][r][wv] = mloc[r];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        m[r] = red[0][r][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m[r] = fmax(m[r], red[0][r][w]);
      }
    }
    int nE[R][EPT];
    double sl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      sl[r] = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if constexpr (FAST) z[r][e] = exp_fast(z[r][e], fs[r], nE[r][e]);
        else z[r][e] = exp_split(z[r][e] - m[r], &nE[r][e]);
        sl[r] += ldexp(z[r][e], nE[r][e]);
      }
    }
    // Without the max pass there is one barrier per row step, so the sums of
    // consecutive steps alternate between the two buffers: a wave that writes
    // step k + 2 has passed step k + 1's barrier, after every read of step k.
    const int sb = FAST ? (((ib - i0) / R) & 1) : 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
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
      // the row's bound for the next pass and, for f (an output only, formed
      // after the last iteration by k_sk_f), its shift and sum
      if (t == 0) {
        br.lse[i - i0] = row_bound(m[r], s);
        br.m[i - i0] = m[r];
        br.s[i - i0] = s;
      }
      const double pi = pv[r];
      if (!(pi > 0.0)) continue;
      int ew;
      const double mw = frexp(pi / s, &ew);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if constexpr (FAST) {
          S[e] = fma(ldexp(z[r][e], nE[r][e] + ew + kqc[e]), mw, S[e]);
        } else {
          const double tv = z[r][e] * mw;
          const int te = nE[r][e] + ew;
          const int ne = max(Xe[e], te);
          S[e] = ldexp(S[e], Xe[e] - ne) + ldexp(tv, te - ne);
          Xe[e] = ne;
        }
      }
    }
    if constexpr (!PF) load(cur, ib + R);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int col = t + NTH * e;
    if (col < N) {
      partS[(int64_t)band * N + col] = S[e];
      if constexpr (!FAST) partX[(int64_t)band * N + col] = Xe[e];
    }
  }
  if (t == 0) bmode[band] = FAST ? 1 : 0;
  __syncthreads();
  band_rows_store(br, lse, ms, f, write_f, i0, i1 - i0, t);
}

template <int NTH, int EPT, int R, bool GL, bool PF>
__global__ __launch_bounds__(NTH) void k_sk_row(const double* __restrict__ C, int64_t ldC, int M,
                                                 int N, int RB, double cs, double inv_eps,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ logp,
                                                 const double* __restrict__ g,
                                                 const int* __restrict__ kq,
                                                 double* __restrict__ f,
                                                 double* __restrict__ ms,
                                                 double* __restrict__ partS,
                                                 int* __restrict__ partX,
                                                 int* __restrict__ bmode,
                                                 double* __restrict__ lse,
                                                 const double* __restrict__ gprev,
                                                 int write_f, const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;  // a tolerance stop has ended the call
  {
    const int i0 = blockIdx.x * RB;
    band_rows_load(row_lds<NTH, EPT, R, GL>().br, p, lse, i0, min(M, i0 + RB) - i0,
                   (int)threadIdx.x, PF && gprev != nullptr);
    __syncthreads();
  }
  // the longest rows (no register prefetch) always take the exact maxima:
  // their fast variant spills more registers than it saves
  double dup = -1.0;
  if constexpr (PF)
    dup = pass_shift<NTH, EPT>(g, gprev, N, inv_eps, lse, blockIdx.x * RB,
                               min(M, (int)blockIdx.x * RB + RB), row_lds<NTH, EPT, R, GL>().dred);
  if (PF && dup >= 0.0)
    sk_row_band<NTH, EPT, R, GL, PF, PF>(C, ldC, M, N, RB, cs, inv_eps, p, logp, g, kq, f, ms,
                                         partS, partX, bmode, lse, dup, write_f, blockIdx.x);
  else
    sk_row_band<NTH, EPT, R, GL, PF, false>(C, ldC, M, N, RB, cs, inv_eps, p, logp, g, kq, f,
                                            ms, partS, partX, bmode, lse, 0.0, write_f,
                                            blockIdx.x);
}

// Grouped row pass for rows of up to 8 x 512 entries: a block of 1024 threads
// is split into NG groups of GT = 1024/NG threads and each group reduces its
// own rows, so a lane owns EPT = N/GT entries of a row and the per-row work
// (two reductions, the weight p_i/s_i) is spread over more entries.  g/eps
// lives in LDS.  The NG groups' column sums are merged through LDS in group
// order and written as the block's partial.
//
// The rows of a band, given its first row in x (loaded by sk_rowg_band) and
// g/eps in LDS; FAST as in sk_row_band.
template <int EPT, int NG, bool PF, bool FAST>
GW_DEV void sk_rowg_rows(const double* __restrict__ C, int64_t ldC, int M, int N, int RB,
                         double csie, const double* __restrict__ p, const int* __restrict__ kq,
                         double* __restrict__ f, double* __restrict__ ms,
                         double* __restrict__ partS, int* __restrict__ partX,
                         int* __restrict__ bmode, double* __restrict__ lse, double dup,
                         int write_f, int band, int t, double (&x)[EPT]) {
  constexpr int GT = 1024 / NG, GW = GT / 64;
  auto& lds = rowg_lds<EPT, NG>();
  const double* gie = lds.u.gie;
  auto& red = lds.red;
  // group and wave indices are the same in every lane of a wave: kept in
  // scalar registers, so row addresses are scalar bases
  const int gi = __builtin_amdgcn_readfirstlane(t / GT), tl = t - gi * GT;
  const int wv = __builtin_amdgcn_readfirstlane(tl >> 6), lane = t & 63;
  double S[EPT];
  int Xe[FAST ? 1 : EPT];
  int kqc[FAST ? EPT : 1];  // column frames (fast pass), staged with g/eps
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    S[e] = 0.0;
    if constexpr (FAST) kqc[e] = lds.kqs[tl + GT * e];
    else Xe[e] = EXP_SENTINEL;
  }
  const int i0 = band * RB, i1 = min(M, i0 + RB);
  const int nr = (RB + NG - 1) / NG;  // row steps, the same for every group
  // row j of the group through a buffer resource over the row: entry e at byte
  // offset 8 tl + 8 GT e (a lane offset plus a scalar one), columns past N read 0
  auto load = [&](double (&dst)[EPT], int j) {
    const int i = min(i0 + j * NG + gi, i1 - 1);
    const auto rs = gwk::buffer_rsrc_n(C + (int64_t)i * ldC, N * 8);
#pragma unroll
    for (int e = 0; e < EPT; ++e) dst[e] = gwk::buffer_load_f64(rs, 8 * tl, 8 * GT * e);
  };
  // one row step on the row in xc; with PF the next row is loaded into xn
  // first (the two buffers swap roles from one step to the next; a second
  // row of prefetch measured slower)
  auto& br = lds.br;
  auto step = [&](int j, double (&xc)[EPT], double (&xn)[EPT]) {
    if (PF) load(xn, j + 1);
    const int i = i0 + j * NG + gi;
    const bool valid = i < i1;
    const int li = min(i, i1 - 1) - i0;  // the row within the band
    const double pi = br.p[li];
    double m;
    int nE[EPT];
    double sl = 0.0;
    if constexpr (FAST) {
      const FastShift fs = fast_shift(br.lse[li] + dup);
      m = fs.mrow;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        xc[e] = exp_fast(fma(-csie, xc[e], gie[tl + GT * e]), fs, nE[e]);
        sl += ldexp(xc[e], nE[e]);
      }
    } else {
      double mloc = -INFINITY;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        xc[e] = fma(-csie, xc[e], gie[tl + GT * e]);
        mloc = fmax(mloc, xc[e]);
      }
      mloc = gwk::wave_max(mloc);
      if (lane == 63) red[0][gi][wv] = mloc;
      __syncthreads();
      m = red[0][gi][0];
#pragma unroll
      for (int w = 1; w < GW; ++w) m = fmax(m, red[0][gi][w]);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        xc[e] = exp_split(xc[e] - m, &nE[e]);
        sl += ldexp(xc[e], nE[e]);
      }
    }
    // one barrier per row step in the fast pass: alternate the buffers of
    // consecutive steps (see the single-group pass)
    const int sb = FAST ? (j & 1) : 1;
    sl = gwk::wave_sum(sl);
    if (lane == 63) red[sb][gi][wv] = sl;
    __syncthreads();
    double s = red[sb][gi][0];
#pragma unroll
    for (int w = 1; w < GW; ++w) s += red[sb][gi][w];
    // the row's bound for the next pass and, for f (an output only, formed
    // after the last iteration by k_sk_f), its shift and sum
    if (valid && tl == 0) {
      br.lse[li] = row_bound(m, s);
      br.m[li] = m;
      br.s[li] = s;
    }
    if (valid && pi > 0.0) {
      int ew;
      const double mw = frexp(pi / s, &ew);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if constexpr (FAST) {
          S[e] = fma(ldexp(xc[e], nE[e] + ew + kqc[e]), mw, S[e]);
        } else {
          const double tv = xc[e] * mw;
          const int te = nE[e] + ew;
          const int ne = max(Xe[e], te);
          S[e] = ldexp(S[e], Xe[e] - ne) + ldexp(tv, te - ne);
          Xe[e] = ne;
        }
      }
    }
    if (!PF) load(xc, j + 1);
  };
  if constexpr (PF) {
    double y[EPT];
    int j = 0;
    for (; j + 1 < nr; j += 2) {
      step(j, x, y);
      step(j + 1, y, x);
    }
    if (j < nr) step(j, x, y);
  } else {
    for (int j = 0; j < nr; ++j) step(j, x, x);
  }
  // the band's row scalars back to global memory; then merge the groups'
  // column sums into group 0 in group order: one exchange through LDS (the
  // sums take the place of g/eps, which no row reads any more)
  __syncthreads();
  band_rows_store(br, lse, ms, f, write_f, i0, i1 - i0, t);
  if constexpr (NG > 1) {
    auto& mS = lds.u.mS;
    auto& mX = lds.mX;
    if (gi > 0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        mS[gi - 1][e][tl] = S[e];
        if constexpr (!FAST) mX[gi - 1][e][tl] = Xe[e];
      }
    }
    __syncthreads();
    if (gi > 0) return;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
#pragma unroll
      for (int k = 0; k < NG - 1; ++k) {
        if constexpr (FAST) {
          S[e] += mS[k][e][tl];
        } else {
          const int xb = mX[k][e][tl];
          const int ne = max(Xe[e], xb);
          S[e] = ldexp(S[e], Xe[e] - ne) + ldexp(mS[k][e][tl], xb - ne);
          Xe[e] = ne;
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int col = tl + GT * e;
    if (col < N) {
      partS[(int64_t)band * N + col] = S[e];
      if constexpr (!FAST) partX[(int64_t)band * N + col] = Xe[e];
    }
  }
  if (tl == 0) bmode[band] = FAST ? 1 : 0;
}

// One band of the grouped pass: the band's first row is loaded before the
// move of g is reduced (D+, D-) and g/eps is staged in LDS, so its latency
// overlaps both; then the rows run in the fast or the exact variant.
template <int EPT, int NG, bool PF>
GW_DEV void sk_rowg_band(const double* __restrict__ C, int64_t ldC, int M, int N, int RB,
                         double cs, double inv_eps, const double* __restrict__ p,
                         const double* __restrict__ g, const double* __restrict__ gprev,
                         const int* __restrict__ kq, double* __restrict__ f,
                         double* __restrict__ ms, double* __restrict__ partS,
                         int* __restrict__ partX, int* __restrict__ bmode,
                         double* __restrict__ lse, int write_f, int band) {
  constexpr int GT = 1024 / NG;
  auto& lds = rowg_lds<EPT, NG>();
  const int t = opaque_tid(), gi = __builtin_amdgcn_readfirstlane(t / GT), tl = t - gi * GT;
  const int i0 = band * RB, i1 = min(M, i0 + RB);
  // g (and g before the last merge) are loaded once: g/eps goes to LDS and
  // the move of g and the band's row bounds are reduced over the block, one
  // barrier for all.  These loads are issued before the band's first row, so
  // waiting for them does not wait for the row (loads return in issue order);
  // the row's latency overlaps the reductions.
  double dup = -1.0;
  double x[EPT];
  {
    constexpr int NF = EPT * GT / 1024;
    double* gie = lds.u.gie;
    double gv[NF], go[NF];  // all loads issued before any is used (indices clamped)
    int kv[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) gv[k] = g[min(t + 1024 * k, N - 1)];
    double lv = 0.0;
    if (gprev != nullptr) {
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        go[k] = gprev[min(t + 1024 * k, N - 1)];
        kv[k] = kq[min(t + 1024 * k, N - 1)];
      }
      lv = lse[min(i0 + t, i1 - 1)];
    }
    band_rows_load(lds.br, p, lse, i0, i1 - i0, t, gprev != nullptr);
    {
      const auto rs = gwk::buffer_rsrc_n(C + (int64_t)min(i0 + gi, i1 - 1) * ldC, N * 8);
#pragma unroll
      for (int e = 0; e < EPT; ++e) x[e] = gwk::buffer_load_f64(rs, 8 * tl, 8 * GT * e);
    }
    double up = 0.0, dn = 0.0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int c = t + 1024 * k;
      gie[c] = c < N ? gv[k] * inv_eps : -INFINITY;
      if (gprev != nullptr) lds.kqs[c] = kv[k];
      if (gprev != nullptr && c < N) fold_move(gv[k], go[k], up, dn);
    }
    if (gprev != nullptr) {
      double lm = lse_mag(lv);
      up = gwk::wave_max(up) * inv_eps;
      dn = gwk::wave_max(dn) * inv_eps;
      lm = gwk::wave_max(lm);
      if ((t & 63) == 63) {
        lds.dred[t >> 6][0] = up;
        lds.dred[t >> 6][1] = dn;
        lds.dred[t >> 6][2] = lm;
      }
    }
    __syncthreads();
    if (gprev != nullptr) {
      up = lds.dred[0][0];
      dn = lds.dred[0][1];
      double lm = lds.dred[0][2];
#pragma unroll
      for (int w = 1; w < 16; ++w) {
        up = fmax(up, lds.dred[w][0]);
        dn = fmax(dn, lds.dred[w][1]);
        lm = fmax(lm, lds.dred[w][2]);
      }
      dup = fast_from(up, dn, lm);
    }
  }
  const double csie = cs * inv_eps;
  if (dup >= 0.0)
    sk_rowg_rows<EPT, NG, PF, true>(C, ldC, M, N, RB, csie, p, kq, f, ms, partS, partX, bmode,
                                    lse, dup, write_f, band, t, x);
  else
    sk_rowg_rows<EPT, NG, PF, false>(C, ldC, M, N, RB, csie, p, kq, f, ms, partS, partX, bmode,
                                     lse, 0.0, write_f, band, t, x);
}

template <int EPT, int NG, bool PF>
__global__ __launch_bounds__(1024) void k_sk_rowg(const double* __restrict__ C, int64_t ldC,
                                                   int M, int N, int RB, double cs,
                                                   double inv_eps,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ g,
                                                   const int* __restrict__ kq,
                                                   double* __restrict__ f,
                                                   double* __restrict__ ms,
                                                   double* __restrict__ partS,
                                                   int* __restrict__ partX,
                                                   int* __restrict__ bmode,
                                                   double* __restrict__ lse,
                                                   const double* __restrict__ gprev,
                                                   int write_f, const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;  // a tolerance stop has ended the call
  sk_rowg_band<EPT, NG, PF>(C, ldC, M, N, RB, cs, inv_eps, p, g, gprev, kq, f, ms, partS, partX,
                            bmode, lse, write_f, blockIdx.x);
}

// ---------------------------------------------------------------- wide rows
// Rows of more than 16384 entries do not fit on chip; they run in slabs of
// WIDE_SLAB columns and two passes over C per iteration:
//   k_skw_rowpart  block (band, slab): each row's maximum over the slab and
//                  its sum of exp(z - max) there, z = (g - C_eff)/eps;
//   k_skw_colpart  block (band, slab): each row's maximum and shifted sum over
//                  all slabs (the same arithmetic in every block of the row),
//                  then the exponentials again, weighted by p_i / s_i, into
//                  (mantissa, exponent) column pairs for the band, as the exact
//                  single-pass variant writes them; k_sk_col merges the bands.
constexpr int WIDE_NT = 512, WIDE_EPT = 16, WIDE_SLAB = WIDE_NT * WIDE_EPT;

// g/eps of the slab's columns and the slab's first column
GW_DEV void wide_gie(const double* __restrict__ g, int N, double inv_eps, int c0, int t,
                     double (&gie)[WIDE_EPT]) {
  double graw[WIDE_EPT];
#pragma unroll
  for (int e = 0; e < WIDE_EPT; ++e) graw[e] = g[min(c0 + t + WIDE_NT * e, N - 1)];
#pragma unroll
  for (int e = 0; e < WIDE_EPT; ++e)
    gie[e] = c0 + t + WIDE_NT * e < N ? graw[e] * inv_eps : -INFINITY;
}

__global__ __launch_bounds__(WIDE_NT) void k_skw_rowpart(const double* __restrict__ C,
                                                         int64_t ldC, int M, int N, int RB,
                                                         double cs, double inv_eps,
                                                         const double* __restrict__ g,
                                                         double* __restrict__ part_m,
                                                         double* __restrict__ part_s,
                                                         const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;  // a tolerance stop has ended the call
  __shared__ double red[2][WIDE_NT / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int band = blockIdx.x, slab = blockIdx.y, c0 = slab * WIDE_SLAB;
  const int i0 = band * RB, i1 = min(M, i0 + RB);
  const double csie = cs * inv_eps;
  double gie[WIDE_EPT];
  wide_gie(g, N, inv_eps, c0, t, gie);
  for (int i = i0; i < i1; ++i) {
    const double* row = C + (int64_t)i * ldC;
    double z[WIDE_EPT];
    double mloc = -INFINITY;
#pragma unroll
    for (int e = 0; e < WIDE_EPT; ++e) {
      z[e] = fma(-csie, row[min(c0 + t + WIDE_NT * e, N - 1)], gie[e]);
      mloc = fmax(mloc, z[e]);
    }
    mloc = gwk::wave_max(mloc);
    if (lane == 63) red[0][wv] = mloc;
    __syncthreads();
    double m = red[0][0];
#pragma unroll
    for (int w = 1; w < WIDE_NT / 64; ++w) m = fmax(m, red[0][w]);
    double sl = 0.0;
    if (m > -INFINITY) {
#pragma unroll
      for (int e = 0; e < WIDE_EPT; ++e) {
        int n;
        const double x = exp_split(z[e] - m, &n);
        sl += ldexp(x, n);
      }
    }
    sl = gwk::wave_sum(sl);
    if (lane == 63) red[1][wv] = sl;
    __syncthreads();
    if (t == 0) {
      double s = red[1][0];
#pragma unroll
      for (int w = 1; w < WIDE_NT / 64; ++w) s += red[1][w];
      part_m[(int64_t)slab * M + i] = m;
      part_s[(int64_t)slab * M + i] = s;
    }
  }
}

__global__ __launch_bounds__(WIDE_NT) void k_skw_colpart(
    const double* __restrict__ C, int64_t ldC, int M, int N, int RB, int ns, double cs,
    double inv_eps, const double* __restrict__ p, const double* __restrict__ g,
    const double* __restrict__ part_m, const double* __restrict__ part_s, double* __restrict__ f,
    double* __restrict__ ms, double* __restrict__ partS, int* __restrict__ partX,
    int* __restrict__ bmode, int write_f, const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;  // a tolerance stop has ended the call
  const int t = threadIdx.x;
  const int band = blockIdx.x, slab = blockIdx.y, c0 = slab * WIDE_SLAB;
  const int i0 = band * RB, i1 = min(M, i0 + RB);
  const double csie = cs * inv_eps;
  double gie[WIDE_EPT];
  wide_gie(g, N, inv_eps, c0, t, gie);
  double S[WIDE_EPT];
  int Xe[WIDE_EPT];
#pragma unroll
  for (int e = 0; e < WIDE_EPT; ++e) {
    S[e] = 0.0;
    Xe[e] = EXP_SENTINEL;
  }
  for (int i = i0; i < i1; ++i) {
    const double pi = p[i];
    // the row's maximum and shifted sum over all slabs, in slab order
    double m = -INFINITY;
    for (int j = 0; j < ns; ++j) m = fmax(m, part_m[(int64_t)j * M + i]);
    double s = 0.0;
    for (int j = 0; j < ns; ++j) {
      const double mj = part_m[(int64_t)j * M + i];
      if (mj > -INFINITY) s += part_s[(int64_t)j * M + i] * exp(mj - m);
    }
    if (!(pi > 0.0)) {
      if (slab == 0 && t == 0) f[i] = -INFINITY;
      continue;
    }
    // f_i is an output only: the last iteration leaves (m_i, s_i) for k_sk_f
    if (write_f && slab == 0 && t == 0) {
      ms[2 * i] = m;
      ms[2 * i + 1] = s;
    }
    int ew;
    const double mw = frexp(pi / s, &ew);
    const double* row = C + (int64_t)i * ldC;
#pragma unroll
    for (int e = 0; e < WIDE_EPT; ++e) {
      int n;
      const double x = exp_split(fma(-csie, row[min(c0 + t + WIDE_NT * e, N - 1)], gie[e]) - m, &n);
      const double tv = x * mw;
      const int te = n + ew;
      const int ne = max(Xe[e], te);
      S[e] = ldexp(S[e], Xe[e] - ne) + ldexp(tv, te - ne);
      Xe[e] = ne;
    }
  }
#pragma unroll
  for (int e = 0; e < WIDE_EPT; ++e) {
    const int col = c0 + t + WIDE_NT * e;
    if (col < N) {
      partS[(int64_t)band * N + col] = S[e];
      partX[(int64_t)band * N + col] = Xe[e];
    }
  }
  if (slab == 0 && t == 0) bmode[band] = 0;
}

// Column merge: a block covers 16 columns x 16 groups of bands; each thread
// merges its groups' (mantissa, exponent) pairs in band order, then the 16
// group results of a column are merged in group order.  A band written by a
// fast pass (bmode) left only the mantissa: its exponent is -kq_p, the
// column's frame.
constexpr int MERGE_COLS = gwb::kMergeCols, MERGE_GRPS = 16;
constexpr int MERGE_PER = 16;  // bands per group: nb <= 256 = MERGE_GRPS * MERGE_PER

// With errpart (uniform), the block also writes sum |S_p - q_p| over its
// columns to errpart[cblock]: S_p is the column sum of the plan (f, g before
// this merge), so the blocks' sums make the half-step's column violation.
GW_DEV void sk_col_block(int N, int nb, const double* __restrict__ partS,
                         const int* __restrict__ partX, const int* __restrict__ bmode,
                         const int* __restrict__ kq, const double* __restrict__ q,
                         const double* __restrict__ logq, double eps, double* __restrict__ g,
                         gwr::StatusWord* status, double* __restrict__ gprev, int cblock,
                         double* __restrict__ errpart) {
  __shared__ double ms[MERGE_GRPS][MERGE_COLS];
  __shared__ int mx[MERGE_GRPS][MERGE_COLS];
  const int c = threadIdx.x & (MERGE_COLS - 1), grp = threadIdx.x / MERGE_COLS;
  const int col = cblock * MERGE_COLS + c;
  double S = 0.0;
  int X = EXP_SENTINEL;
  {
    // a group's bands (at most MERGE_PER) are all requested before the first
    // is merged: indices clamped into range, entries past the group skipped
    const int per = (nb + MERGE_GRPS - 1) / MERGE_GRPS;
    const int b0 = grp * per, b1 = min(nb, b0 + per);
    const int colc = min(col, N - 1);
    const int fx = -kq[colc];
    double sv[MERGE_PER];
    int xv[MERGE_PER];
    int fm[MERGE_PER];
#pragma unroll
    for (int u = 0; u < MERGE_PER; ++u) fm[u] = bmode[min(b0 + u, nb - 1)];
#pragma unroll
    for (int u = 0; u < MERGE_PER; ++u) {
      const int64_t b = min(b0 + u, nb - 1);
      sv[u] = partS[b * N + colc];
      xv[u] = fm[u] ? fx : partX[b * N + colc];
    }
    if (col < N) {
#pragma unroll
      for (int u = 0; u < MERGE_PER; ++u) {
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
  if (errpart == nullptr && (grp != 0 || col >= N)) return;
  double e = 0.0;
  if (grp == 0 && col < N) {
    for (int k = 1; k < MERGE_GRPS; ++k) {
      const int ne = max(X, mx[k][c]);
      S = ldexp(S, X - ne) + ldexp(ms[k][c], mx[k][c] - ne);
      X = ne;
    }
    const double qc = q[col];
    if (errpart != nullptr) e = fabs(ldexp(S, X) - qc);
    const double gold = g[col];
    gprev[col] = gold;
    if (!(qc > 0.0)) {
      g[col] = -INFINITY;
    } else {
      // ln(S 2^X) with X ln 2 split so that X * LN2_HI is exact
      const double lnS = fma((double)X, LN2_HI, fma((double)X, LN2_LO, log(S)));
      const double gn = gold + eps * (logq[col] - lnS);
      g[col] = gn;
      if (!isfinite(gn)) status->nonfinite = 1;
    }
  }
  if (errpart == nullptr) return;
  // the block's columns summed in column order (the group-0 threads are lanes
  // 0..MERGE_COLS-1 of the first wave)
  __shared__ double es[MERGE_COLS];
  if (grp == 0) es[c] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < MERGE_COLS; ++k) t += es[k];
    errpart[cblock] = t;
  }
}

__global__ __launch_bounds__(256) void k_sk_col(int N, int nb, const double* __restrict__ partS,
                                                 const int* __restrict__ partX,
                                                 const int* __restrict__ bmode,
                                                 const int* __restrict__ kq,
                                                 const double* __restrict__ q,
                                                 const double* __restrict__ logq, double eps,
                                                 double* __restrict__ g,
                                                 gwr::StatusWord* status, double* gprev,
                                                 const int* __restrict__ stop,
                                                 double* __restrict__ errpart) {
  if (stop != nullptr && *stop) return;  // a tolerance stop has ended the call
  sk_col_block(N, nb, partS, partX, bmode, kq, q, logq, eps, g, status, gprev, blockIdx.x,
               errpart);
}

// Tolerance stop, state of one call: stop flag, iterations done, last err.
struct SkCtl {
  int stop;
  int done;
  double err;
};

__global__ void k_sk_ctl_init(SkCtl* ctl, int iters, int* iters_out, double* err_out) {
  if (threadIdx.x != 0) return;
  ctl->stop = 0;
  ctl->done = iters;
  ctl->err = NAN;
  if (iters_out) *iters_out = iters;
  if (err_out) *err_out = NAN;
}

// After the merge of iteration `it` (0-based) on a check iteration: err = the
// column blocks' sums added in block order by one wave; stop if err <= tol.
__global__ __launch_bounds__(64) void k_sk_check(const double* __restrict__ errpart, int ncb,
                                                  double tol, int it, SkCtl* ctl,
                                                  int* iters_out, double* err_out) {
  if (ctl->stop) return;
  const int l = threadIdx.x;
  double t = 0.0;
  for (int b = l; b < ncb; b += 64) t += errpart[b];
  // fixed-order tree over the 64 lanes
  for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
  if (l != 0) return;
  ctl->err = t;
  if (err_out) *err_out = t;
  if (t <= tol) {
    ctl->stop = 1;
    ctl->done = it + 1;
    if (iters_out) *iters_out = it + 1;
  }
}

// f_i = eps (ln p_i - m_i - ln s_i) from the last row pass's row maximum and
// shifted sum; zero-mass rows were already set to -inf by the row pass.
__global__ __launch_bounds__(256) void k_sk_f(int M, const double* __restrict__ p,
                                               const double* __restrict__ logp,
                                               const double* __restrict__ ms, double eps,
                                               double* __restrict__ f,
                                               gwr::StatusWord* status) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M || !(p[i] > 0.0)) return;
  const double fi = eps * ((logp[i] - ms[2 * i]) - log(ms[2 * i + 1]));
  f[i] = fi;
  if (!isfinite(fi)) status->nonfinite = 1;
}

__global__ __launch_bounds__(256) void k_plan(const double* __restrict__ C, int64_t ldC, int M,
                                               int N, double cs, const double* __restrict__ f,
                                               const double* __restrict__ g, double inv_eps,
                                               double* __restrict__ T, int64_t ldT) {
  const int64_t i = blockIdx.y;
  const double fi = f[i];
  for (int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x; col < N;
       col += (int64_t)gridDim.x * 256)
    T[i * ldT + col] = exp(((fi + g[col]) - cs * C[i * ldC + col]) * inv_eps);
}

__global__ __launch_bounds__(256) void k_outer(const double* __restrict__ p,
                                                const double* __restrict__ q, int M, int N,
                                                double* __restrict__ T, int64_t ldT) {
  const int64_t i = blockIdx.y;
  const double pi = p[i];
  for (int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x; col < N;
       col += (int64_t)gridDim.x * 256)
    T[i * ldT + col] = pi * q[col];
}

// row sums: one block per row
__global__ __launch_bounds__(256) void k_rowsum(const double* __restrict__ T, int64_t ldT, int N,
                                                 double* __restrict__ r) {
  __shared__ double red[4];
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int col = threadIdx.x; col < N; col += 256) s += T[i * ldT + col];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) r[i] = s;
}

// column sums: a block of 1024 threads covers 16 columns x 64 row groups
// (contiguous row ranges), the groups' sums added in group order
constexpr int CS_COLS = 16, CS_GRPS = 64;
__global__ __launch_bounds__(CS_COLS * CS_GRPS) void k_colsum(const double* __restrict__ T,
                                                              int64_t ldT, int M, int N,
                                                              double* __restrict__ c) {
  __shared__ double part[CS_GRPS][CS_COLS];
  const int lane = threadIdx.x & (CS_COLS - 1), grp = threadIdx.x / CS_COLS;
  const int col = blockIdx.x * CS_COLS + lane;
  double s = 0.0;
  if (col < N) {
    const int chunk = (M + CS_GRPS - 1) / CS_GRPS;
    const int r0 = grp * chunk, r1 = min(M, r0 + chunk);
#pragma unroll 8
    for (int i = r0; i < r1; ++i) s += T[(int64_t)i * ldT + col];
  }
  part[grp][lane] = s;
  __syncthreads();
  if (grp == 0 && col < N) {
    double r = part[0][lane];
    for (int g = 1; g < CS_GRPS; ++g) r += part[g][lane];
    c[col] = r;
  }
}

// partial sums of G*T and T (ln T - 1) per block (rows band), fixed order
__global__ __launch_bounds__(256) void k_obj_partial(const double* __restrict__ G, int64_t ldG,
                                                      const double* __restrict__ T, int64_t ldT,
                                                      int M, int N, int RB,
                                                      double* __restrict__ part,
                                                      gwr::StatusWord* status) {
  __shared__ double red[4];
  const int i0 = blockIdx.x * RB, i1 = min(M, i0 + RB);
  double a = 0.0, h = 0.0;
  bool bad = false;
  for (int i = i0; i < i1; ++i)
    for (int col = threadIdx.x; col < N; col += 256) {
      const double tv = T[(int64_t)i * ldT + col];
      const double gv = G[(int64_t)i * ldG + col];
      a = fma(gv, tv, a);
      if (tv > 0.0) h = fma(tv, log(tv) - 1.0, h);
      bad |= !isfinite(tv) || !isfinite(gv);
    }
  a = block_sum<256>(a, red);
  h = block_sum<256>(h, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = h;
  }
  if (bad) status->nonfinite = 1;
}

__global__ __launch_bounds__(256) void k_obj_final(const double* __restrict__ part, int nb,
                                                    double eps, double* __restrict__ obj) {
  __shared__ double red[4];
  double a = 0.0, h = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    a += part[2 * b];
    h += part[2 * b + 1];
  }
  a = block_sum<256>(a, red);
  h = block_sum<256>(h, red);
  if (threadIdx.x == 0) {
    obj[0] = a;
    obj[1] = a + eps * h;
  }
}

int sk_rows_per_block(int64_t M) {
  int rb = (int)((M + 255) / 256);
  return rb < 1 ? 1 : rb;
}

// Rows reduced together by the row pass: 4 for short rows, 2 at 1024
// threads (register pressure), 1 for rows of 16 entries per thread.
template <int NTH, int EPT>
constexpr int row_group() {
  return EPT > 4 ? 1 : (NTH >= 1024 ? 2 : 4);
}

// Rows of more than 16 entries per thread keep g / eps in LDS, and above 18
// they give up the register prefetch.
template <int NTH, int EPT>
constexpr bool row_gl() {
  return EPT > 16;
}
template <int NTH, int EPT>
constexpr bool row_pf() {
  return EPT <= 18;
}

template <int NTH, int EPT>
void launch_row(int nb, hipStream_t s, hipEvent_t eb, hipEvent_t ee, const double* C,
                int64_t ldC, int M, int N, int RB, double cs, double inv_eps, const double* p,
                const double* logp, const double* g, const int* kq, double* f, double* ms,
                double* pS, int* pX, int* bmode, double* lse, const double* gprev, int last,
                const int* stop) {
  constexpr int R = row_group<NTH, EPT>();
  hipExtLaunchKernelGGL(k_sk_row<NTH, EPT, R, row_gl<NTH, EPT>(), row_pf<NTH, EPT>()>, dim3(nb),
                        dim3(NTH), 0, s, eb, ee, 0, C, ldC, M, N, RB, cs, inv_eps, p, logp, g, kq,
                        f, ms, pS, pX, bmode, lse, gprev, last, stop);
}

// ---------------------------------------------------------------------------
// Batched kernels of the request loop.  Each block walks the item list of its
// class with a fixed stride (the grid is fixed when the step is captured);
// an item names a request slot and a band (row pass) or a column block
// (merge).  A request takes part in iteration j of a step only if j < its.
// The per-band arithmetic is the single-problem kernel's, so a request's
// result does not depend on what else is in the batch.
template <int NTH, int EPT>
__global__ __launch_bounds__(NTH) void k_skb_row(const gwb::SkSlot* __restrict__ slots,
                                                  const gwb::SkTableHead* __restrict__ head,
                                                  const uint32_t* __restrict__ items, int cls,
                                                  int j) {
  const int n = head->count[cls];
  const uint32_t* list = items + head->offset[cls];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const uint32_t code = list[w];
    const gwb::SkSlot& a = slots[code >> gwb::kBandBits];
    if (j >= a.its) continue;
    __syncthreads();
    const int tt = a.it0 + j;  // iteration within the request's Sinkhorn call
    const int band = (int)(code & ((1u << gwb::kBandBits) - 1));
    constexpr int R = row_group<NTH, EPT>();
    constexpr bool GL = row_gl<NTH, EPT>();
    constexpr bool PF = row_pf<NTH, EPT>();
    {
      const int i0 = band * a.RB;
      band_rows_load(row_lds<NTH, EPT, R, GL>().br, a.p, a.lse, i0, min(a.M, i0 + a.RB) - i0,
                     (int)threadIdx.x, PF && tt > 0);
      __syncthreads();
    }
    double dup = -1.0;  // exact maxima without the register prefetch, as in k_sk_row
    if constexpr (PF)
      dup = pass_shift<NTH, EPT>(a.g, tt > 0 ? a.gprev : nullptr, a.N, a.inv_eps, a.lse,
                                 band * a.RB, min(a.M, band * a.RB + a.RB),
                                 row_lds<NTH, EPT, R, GL>().dred);
    const int wf = a.last && j == a.its - 1;
    if (PF && dup >= 0.0)
      sk_row_band<NTH, EPT, R, GL, PF, PF>(a.C, a.ldC, a.M, a.N, a.RB, a.cs, a.inv_eps, a.p,
                                             a.logp, a.g, a.kq, a.f, a.ms, a.pS, a.pX, a.bmode,
                                             a.lse, dup, wf, band);
    else
      sk_row_band<NTH, EPT, R, GL, PF, false>(a.C, a.ldC, a.M, a.N, a.RB, a.cs, a.inv_eps, a.p,
                                              a.logp, a.g, a.kq, a.f, a.ms, a.pS, a.pX, a.bmode,
                                              a.lse, 0.0, wf, band);
  }
}

__global__ __launch_bounds__(1024) void k_skb_rowg(const gwb::SkSlot* __restrict__ slots,
                                                    const gwb::SkTableHead* __restrict__ head,
                                                    const uint32_t* __restrict__ items, int cls,
                                                    int j) {
  const int n = head->count[cls];
  const uint32_t* list = items + head->offset[cls];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const uint32_t code = list[w];
    const gwb::SkSlot& a = slots[code >> gwb::kBandBits];
    if (j >= a.its) continue;
    __syncthreads();
    const int tt = a.it0 + j;
    const int band = (int)(code & ((1u << gwb::kBandBits) - 1));
    sk_rowg_band<8, 2, true>(a.C, a.ldC, a.M, a.N, a.RB, a.cs, a.inv_eps, a.p, a.g,
                             tt > 0 ? a.gprev : nullptr, a.kq, a.f, a.ms, a.pS, a.pX, a.bmode,
                             a.lse, a.last && j == a.its - 1, band);
  }
}

__global__ __launch_bounds__(256) void k_skb_col(const gwb::SkSlot* __restrict__ slots,
                                                  const gwb::SkTableHead* __restrict__ head,
                                                  const uint32_t* __restrict__ items, int j) {
  const int n = head->count[gwb::kClsCol];
  const uint32_t* list = items + head->offset[gwb::kClsCol];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const uint32_t code = list[w];
    const gwb::SkSlot& a = slots[code >> gwb::kCBlockBits];
    if (j >= a.its) continue;
    __syncthreads();
    sk_col_block(a.N, a.nb, a.pS, a.pX, a.bmode, a.kq, a.q, a.logq, a.eps, a.g, a.status, a.gprev,
                 (int)(code & ((1u << gwb::kCBlockBits) - 1)), nullptr);
  }
}

// Persistent grids: enough blocks to fill the chip at the class's occupancy.
constexpr unsigned kBatchBlocks256 = 2048, kBatchBlocks512 = 1024, kBatchBlocks1024 = 512;

// Host view of a tolerance stop: after each check the device's stop flag is
// copied to pinned host memory, so the host can stop enqueueing iterations
// once a check has stopped the call (the launches it no longer enqueues
// would return at once: results are unchanged).  Probes are pooled per
// device and reused; a probe is taken only after its previous user's copies
// have landed.
constexpr int kProbeSlots = 2;

struct StopProbe {
  int dev = -1;
  int* flag = nullptr;  // pinned, kProbeSlots flags
  hipEvent_t ev[kProbeSlots] = {};
};

std::mutex g_probe_mu;
std::vector<StopProbe*> g_probe_free;

void probe_destroy(StopProbe* pr) {
  for (hipEvent_t e : pr->ev)
    if (e) (void)hipEventDestroy(e);
  if (pr->flag) (void)hipHostFree(pr->flag);
  delete pr;
}

// nullptr if no probe can be had (the call then enqueues every iteration).
StopProbe* probe_take() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  StopProbe* pr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_probe_mu);
    for (size_t i = 0; i < g_probe_free.size(); ++i)
      if (g_probe_free[i]->dev == dev) {
        pr = g_probe_free[i];
        g_probe_free.erase(g_probe_free.begin() + (ptrdiff_t)i);
        break;
      }
  }
  if (!pr) {
    pr = new (std::nothrow) StopProbe();
    if (!pr) return nullptr;
    pr->dev = dev;
    bool ok = hipHostMalloc(reinterpret_cast<void**>(&pr->flag), kProbeSlots * sizeof(int),
                            hipHostMallocDefault) == hipSuccess;
    for (int i = 0; i < kProbeSlots && ok; ++i)
      ok = hipEventCreateWithFlags(&pr->ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      probe_destroy(pr);
      return nullptr;
    }
    return pr;
  }
  for (hipEvent_t e : pr->ev)
    if (hipEventSynchronize(e) != hipSuccess) {
      probe_destroy(pr);
      return nullptr;
    }
  return pr;
}

void probe_give(StopProbe* pr) {
  if (!pr) return;
  std::lock_guard<std::mutex> lock(g_probe_mu);
  g_probe_free.push_back(pr);
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

}  // namespace

namespace gwl {

size_t sinkhorn_ws_bytes(int64_t M, int64_t N) {
  const int rb = sk_rows_per_block(M);
  const int64_t nb = (M + rb - 1) / rb;
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(M);
  a.take<double>(N);
  a.take<double>((size_t)nb * N);
  a.take<int>((size_t)nb * N);
  a.take<double>(2 * (size_t)M);
  a.take<double>(M);  // row bounds
  a.take<double>(N);  // g before the last merge
  a.take<int>(N);     // column frames
  a.take<int>(nb);    // pass kind of each band's partials
  if (N > 16384) {    // wide rows: per-slab row maxima and sums
    const int64_t ns = (N + WIDE_SLAB - 1) / WIDE_SLAB;
    a.take<double>((size_t)ns * M);
    a.take<double>((size_t)ns * M);
  }
  a.take<double>(4);  // tolerance-stop state
  a.take<double>((N + MERGE_COLS - 1) / MERGE_COLS);  // column violation per merge block
  return a.used;
}

gw_status sinkhorn_prep(const double* p, const double* q, int64_t M, int64_t N, int init_zero,
                        double* logp, double* logq, int* kq, double* f, double* g,
                        hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  const int64_t mx = M > N ? M : N;
  k_sk_prep<<<(unsigned)((mx + 255) / 256), 256, 0, s>>>(p, q, (int)M, (int)N, init_zero, logp,
                                                         logq, kq, f, g);
  return gwr::last_launch_status();
}

gw_status sinkhorn_finish(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                          const double* p, const double* logp, const double* ms, double eps,
                          int iters, double* f, const double* g, double* T, int64_t ldT,
                          hipStream_t s, gwr::StatusWord* status) {
  if (iters > 0) {
    gwr::ProfScope ps(gwr::kFamOther, s);
    k_sk_f<<<(unsigned)((M + 255) / 256), 256, 0, s>>>((int)M, p, logp, ms, eps, f, status);
  }
  if (T) return plan(C, ldC, M, N, c_scale, f, g, eps, T, ldT, s);
  return gwr::last_launch_status();
}

int sk_rows_per_band(int64_t M) { return sk_rows_per_block(M); }

gw_status sk_batch_launch(int cls, int j, const gwb::SkSlot* slots, const gwb::SkTableHead* head,
                          const uint32_t* items, hipStream_t s) {
  switch (cls) {
    case gwb::kClsN256: k_skb_row<256, 1><<<kBatchBlocks256, 256, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN512: k_skb_row<512, 1><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN1024: k_skb_row<1024, 1><<<kBatchBlocks1024, 1024, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN2048: k_skb_row<1024, 2><<<kBatchBlocks1024, 1024, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN3072: k_skb_row<256, 12><<<kBatchBlocks256, 256, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN4096: k_skb_rowg<<<kBatchBlocks1024, 1024, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN6144: k_skb_row<512, 12><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN8192: k_skb_row<512, 16><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN9216: k_skb_row<512, 18><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN12288: k_skb_row<512, 24><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsN16384: k_skb_row<512, 32><<<kBatchBlocks512, 512, 0, s>>>(slots, head, items, cls, j); break;
    case gwb::kClsCol: k_skb_col<<<kBatchBlocks256, 256, 0, s>>>(slots, head, items, j); break;
    default: return GW_EINVAL;
  }
  return gwr::last_launch_status();
}

gw_status sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                   const double* p, const double* q, double eps, int iters, int init_zero,
                   double* f, double* g, double* T, int64_t ldT, gwr::Arena& ws, hipStream_t s,
                   gwr::StatusWord* status, const gwr::SkStop* stop_opts) {
  const int rb = sk_rows_per_block(M);
  const int nb = (int)((M + rb - 1) / rb);
  double* logp = ws.take<double>(M);
  double* logq = ws.take<double>(N);
  double* pS = ws.take<double>((size_t)nb * N);
  int* pX = ws.take<int>((size_t)nb * N);
  double* ms = ws.take<double>(2 * (size_t)M);
  double* lse = ws.take<double>(M);
  double* gprev = ws.take<double>(N);
  int* kq = ws.take<int>(N);
  int* bmode = ws.take<int>(nb);
  const bool wide = N > 16384;
  const int ns = wide ? (int)((N + WIDE_SLAB - 1) / WIDE_SLAB) : 0;
  double* part_m = wide ? ws.take<double>((size_t)ns * M) : nullptr;
  double* part_s = wide ? ws.take<double>((size_t)ns * M) : nullptr;
  SkCtl* ctl = reinterpret_cast<SkCtl*>(ws.take<double>(4));
  const int ncb = (int)((N + MERGE_COLS - 1) / MERGE_COLS);
  double* errpart = ws.take<double>(ncb);
  const double inv_eps = 1.0 / eps;
  gw_status st = sinkhorn_prep(p, q, M, N, init_zero, logp, logq, kq, f, g, s);
  if (st != GW_OK) return st;
  // tolerance stop: every `every` iterations the merge measures the column
  // violation and k_sk_check may raise the flag that the later launches of
  // this call test first
  const int every = stop_opts ? stop_opts->check_every : 0;
  const int* stop = stop_opts ? &ctl->stop : nullptr;
  if (stop_opts) {
    gwr::ProfScope ps(gwr::kFamOther, s);
    k_sk_ctl_init<<<1, 64, 0, s>>>(ctl, iters, stop_opts->iters_out, stop_opts->err_out);
  }
  // the host follows the checks one period behind (not while the stream is
  // captured into a graph, which cannot wait on the host)
  StopProbe* probe = every > 0 && !stream_capturing(s) ? probe_take() : nullptr;
  int nchecks = 0;
  const int Mi = (int)M, Ni = (int)N;
  for (int it = 0; it < iters; ++it) {
    const bool check = every > 0 && (it + 1) % every == 0;
    {
      gwr::ProfDispatch pd(gwr::kFamSinkRow);
      hipEvent_t eb = pd.b, ee = pd.e;
      // a pass that may be the last one leaves (m_i, s_i) for k_sk_f
      const int lst = it == iters - 1 || check;
      const double* gp = it > 0 ? gprev : nullptr;
      if (wide) {
        hipExtLaunchKernelGGL(k_skw_rowpart, dim3(nb, ns), dim3(WIDE_NT), 0, s, eb, nullptr, 0, C,
                              ldC, Mi, Ni, rb, c_scale, inv_eps, g, part_m, part_s, stop);
        hipExtLaunchKernelGGL(k_skw_colpart, dim3(nb, ns), dim3(WIDE_NT), 0, s, nullptr, ee, 0,
                              C, ldC, Mi, Ni, rb, ns, c_scale, inv_eps, p, g, part_m, part_s, f,
                              ms, pS, pX, bmode, lst, stop);
      } else switch (gwb::row_class(N)) {
        case gwb::kClsN256: launch_row<256, 1>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN512: launch_row<512, 1>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN1024: launch_row<1024, 1>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN2048: launch_row<1024, 2>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN3072: launch_row<256, 12>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN4096: hipExtLaunchKernelGGL(k_sk_rowg<8, 2, true>, dim3(nb), dim3(1024), 0, s, eb, ee, 0, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN6144: launch_row<512, 12>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN8192: launch_row<512, 16>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN9216: launch_row<512, 18>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        case gwb::kClsN12288: launch_row<512, 24>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
        default: launch_row<512, 32>(nb, s, eb, ee, C, ldC, Mi, Ni, rb, c_scale, inv_eps, p, logp, g, kq, f, ms, pS, pX, bmode, lse, gp, lst, stop); break;
      }
    }
    {
      gwr::ProfDispatch pd(gwr::kFamSinkCol);
      hipExtLaunchKernelGGL(k_sk_col, dim3((unsigned)ncb), dim3(256), 0, s, pd.b, pd.e, 0, Ni,
                            nb, pS, pX, bmode, kq, q, logq, eps, g, status, gprev, stop,
                            check ? errpart : nullptr);
    }
    if (check) {
      {
        gwr::ProfScope ps(gwr::kFamOther, s);
        k_sk_check<<<1, 64, 0, s>>>(errpart, ncb, stop_opts->tol, it, ctl, stop_opts->iters_out,
                                     stop_opts->err_out);
      }
      if (probe) {
        // this check's flag to the host; then wait for the previous check's
        // (the device still has this period queued) and stop enqueueing if
        // it stopped the call.  The slot written now held the flag of two
        // checks ago, whose copy was waited for one check ago.
        const int slot = nchecks % kProbeSlots;
        if (hipMemcpyAsync(&probe->flag[slot], &ctl->stop, sizeof(int), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipEventRecord(probe->ev[slot], s) != hipSuccess) {
          probe_give(probe);
          return GW_EDEVICE;
        }
        ++nchecks;
        if (nchecks >= 2) {
          const int prev = (nchecks - 2) % kProbeSlots;
          if (hipEventSynchronize(probe->ev[prev]) != hipSuccess) {
            probe_give(probe);
            return GW_EDEVICE;
          }
          if (probe->flag[prev]) break;
        }
      }
    }
  }
  probe_give(probe);
  return sinkhorn_finish(C, ldC, M, N, c_scale, p, logp, ms, eps, iters, f, g, T, ldT, s, status);
}

gw_status plan(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
               const double* f, const double* g, double eps, double* T, int64_t ldT,
               hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamPlan, s);
  const unsigned gx = (unsigned)((N + 255) / 256 < 16 ? (N + 255) / 256 : 16);
  k_plan<<<dim3(gx, (unsigned)M), 256, 0, s>>>(C, ldC, (int)M, (int)N, c_scale, f, g, 1.0 / eps, T, ldT);
  return gwr::last_launch_status();
}

gw_status outer_product(const double* p, const double* q, int64_t M, int64_t N, double* T,
                        int64_t ldT, hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  const unsigned gx = (unsigned)((N + 255) / 256 < 16 ? (N + 255) / 256 : 16);
  k_outer<<<dim3(gx, (unsigned)M), 256, 0, s>>>(p, q, (int)M, (int)N, T, ldT);
  return gwr::last_launch_status();
}

gw_status marginals(const double* T, int64_t ldT, int64_t M, int64_t N, double* r, double* c,
                    gwr::Arena&, hipStream_t s) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  k_rowsum<<<(unsigned)M, 256, 0, s>>>(T, ldT, (int)N, r);
  k_colsum<<<(unsigned)((N + CS_COLS - 1) / CS_COLS), CS_COLS * CS_GRPS, 0, s>>>(T, ldT, (int)M,
                                                                                (int)N, c);
  return gwr::last_launch_status();
}

size_t objective_reduce_ws_bytes(int64_t M, int64_t) {
  const int64_t nb = (M + 15) / 16;
  gwr::Arena a{nullptr, 0, 0};
  a.take<double>(2 * nb);
  return a.used;
}

gw_status objective_reduce(const double* G, int64_t ldG, const double* T, int64_t ldT,
                           int64_t M, int64_t N, double eps, double* obj, gwr::Arena& ws,
                           hipStream_t s, gwr::StatusWord* status) {
  gwr::ProfScope ps(gwr::kFamOther, s);
  const int RB = 16;
  const int nb = (int)((M + RB - 1) / RB);
  double* part = ws.take<double>(2 * (size_t)nb);
  k_obj_partial<<<(unsigned)nb, 256, 0, s>>>(G, ldG, T, ldT, (int)M, (int)N, RB, part, status);
  k_obj_final<<<1, 256, 0, s>>>(part, nb, eps, obj);
  return gwr::last_launch_status();
}

}  // namespace gwl
