// Exponentials with an unbounded binary exponent for the log-domain
// Sinkhorn passes (balanced and unbalanced).
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

}  // namespace gwx
