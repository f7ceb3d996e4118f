// Shared device helpers for the GW kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gw.h"

#define GW_DEV __device__ __forceinline__

namespace gwk {

constexpr int kWave = 64;

// Binomial coefficients C(r, s) for r, s <= 8.
GW_DEV constexpr double binom(int r, int s) {
  double v = 1.0;
  for (int t = 1; t <= s; ++t) v = v * (double)(r - s + t) / (double)t;
  return v;
}

// One step of the Pascal recursion (Sec. 3, Eq. (1d recursive relation)):
// a_r <- x + sum_{s<=r} C(r,s) a_s, evaluated from r = K down to 0 so the
// right-hand side sees the old state.
template <int K>
GW_DEV void pascal_step(double (&a)[K + 1], double x) {
#pragma unroll
  for (int r = K; r >= 0; --r) {
    double acc = a[r];
#pragma unroll
    for (int s = r - 1; s >= 0; --s) acc = fma(binom(r, s), a[s], acc);
    a[r] = acc + x;
  }
}

// Advance a state over w positions with zero input:
// a_r <- sum_{s<=r} C(r,s) w^{r-s} a_s (all coefficients >= 0).
template <int K>
GW_DEV void pascal_shift(double (&a)[K + 1], double w) {
  double wp[K + 1];
  wp[0] = 1.0;
#pragma unroll
  for (int r = 1; r <= K; ++r) wp[r] = wp[r - 1] * w;
#pragma unroll
  for (int r = K; r >= 1; --r) {
    double acc = a[r];
#pragma unroll
    for (int s = r - 1; s >= 0; --s) acc = fma(binom(r, s) * wp[r - s], a[s], acc);
    a[r] = acc;
  }
}

GW_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

GW_DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

GW_DEV int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

// |d|^k for an integer distance d >= 0, as an exact double while < 2^53.
GW_DEV double ipow(double d, int k) {
  double v = 1.0;
  for (int i = 0; i < k; ++i) v *= d;
  return v;
}

}  // namespace gwk
