// Exponentials with an unbounded binary exponent for the log-domain
// Sinkhorn passes (balanced and unbalanced), and the test that lets a pass
// skip its row maxima.
#pragma once
#include "common.h"

namespace gwx {

// ln 2 = LN2_HI + LN2_LO with LN2_HI carrying 32 significant bits, so n*LN2_HI
// is exact for |n| < 2^21 (Cody and Waite's two-constant argument reduction).
constexpr double LN2_HI = 0x1.62e42fee00000p-1;
constexpr double LN2_LO = 0x1.a39ef35793c76p-33;
constexpr double INV_LN2 = 0x1.71547652b82fep+0;
constexpr int EXP_SENTINEL = -(1 << 30);
constexpr double X_FLOOR = -1.0e6;  // exp(-1e6) is 0 in any precision used here

// e^r for |r| <= ln(2)/2: the degree-11 polynomial of best relative
// approximation on that interval (Remez exchange; 3.1e-18 relative before its
// coefficients are rounded to double, about one ulp when evaluated by Horner
// in double).
GW_DEV double exp_reduced(double r) {
  double y = 0x1.ad66238d9d610p-26;
  y = fma(y, r, 0x1.28b311bbb39f6p-22);
  y = fma(y, r, 0x1.71df451c45e1ap-19);
  y = fma(y, r, 0x1.a01992d10c9e6p-16);
  y = fma(y, r, 0x1.a01a011059272p-13);
  y = fma(y, r, 0x1.6c16c187810c2p-10);
  y = fma(y, r, 0x1.1111111130dd0p-7);
  y = fma(y, r, 0x1.555555554f370p-5);
  y = fma(y, r, 0x1.55555555554a2p-3);
  y = fma(y, r, 0x1.0000000000010p-1);
  y = fma(y, r, 1.0);
  return fma(y, r, 1.0);
}

// exp(x) for -1e6 <= x <= 1e6 (x below is taken as -1e6) as E * 2^n, E in [0.70, 1.42]: n = rint(x / ln 2), the
// remainder x - n ln 2 is formed with the two-constant split of ln 2.
GW_DEV double exp_split(double x, int* n) {
  x = fmax(x, X_FLOOR);
  const double nd = rint(x * INV_LN2);
  double r = fma(-nd, LN2_HI, x);
  r = fma(-nd, LN2_LO, r);
  *n = (int)nd;
  return exp_reduced(r);
}

// ---- the shifted pass
// A row pass may shift each row by an upper bound of its log-sum-exp instead
// of reducing the row maximum: the previous pass's bound a_i (below) plus D+,
// the largest move of the row's exponents since that pass (a log-sum-exp
// moves by at most the largest move of its arguments).  D- is the largest
// move down.  Then the shifted row sum lies in [e^-(D+ + D- + ln 2), 1], and
// column sums can be kept as plain doubles in per-column frames.
constexpr double SHIFT_SPREAD_MAX = 600.0;  // D+ + D- up to which the max pass is skipped
constexpr double FAST_UP_MAX = 550.0;       // largest D+ of a shifted pass
constexpr double FAST_M_MAX = 1.0e6;        // bound on |a_i| + D+

// Folds one column's move into (up, dn): its value now (gn) and before the
// last update (go).  A column that became or stopped being finite rules the
// shifted pass out.
GW_DEV void fold_move(double gn, double go, double& up, double& dn) {
  if (isfinite(gn) && isfinite(go)) {
    up = fmax(up, gn - go);
    dn = fmax(dn, go - gn);
  } else if (isfinite(gn) != isfinite(go)) {
    up = dn = INFINITY;
  }
}

// |a_i| of a row for the test (a non-finite bound rules it out).
GW_DEV double lse_mag(double v) { return isfinite(v) ? fabs(v) : INFINITY; }

// Upper bound of ln(sum) for a row shifted by m with shifted sum s > 0:
// m + e ln 2 for s = f 2^e, f in [0.5, 1).
GW_DEV double row_bound(double m, double s) {
  int es;
  (void)frexp(s, &es);
  return m + (double)es * 0.6931471805599453;
}

// The decision from the moves (up = D+, dn = D-, in units of the exponents)
// and the largest |a_i| of the band: D+ if the pass may be shifted, else -1
// (exact row maxima).
GW_DEV double fast_from(double up, double dn, double lmax) {
  return (up + dn <= SHIFT_SPREAD_MAX && up <= FAST_UP_MAX && lmax + up < FAST_M_MAX) ? up : -1.0;
}

}  // namespace gwx
