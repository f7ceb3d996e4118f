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

// Move a double across lanes with one DPP pattern (both 32-bit halves);
// lanes the pattern does not write receive `old`.
template <int CTRL, int ROW_MASK = 0xF>
GW_DEV double dpp_f64(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL,
                                             ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL,
                                             ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// The same move where the lanes the pattern does not write may hold any value
// (no register has to be initialised with an `old` value first).
template <int CTRL, int ROW_MASK = 0xF>
GW_DEV double dpp_any_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

GW_DEV double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Wave64 reductions with DPP: swaps within quads, half-row and row mirrors,
// then the two row broadcasts leave the total in lane 63 (GCN/CDNA pattern).
// The result is returned in every lane.  Only lane 63's value is read: the
// first four patterns write every lane, and the two broadcasts write the row
// of lane 63 and the row it reads next (from lanes the earlier patterns
// wrote), so the lanes a pattern leaves alone may hold any value.
GW_DEV double wave_sum(double v) {
  v += dpp_any_f64<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_any_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_any_f64<0x141>(v);       // row_half_mirror
  v += dpp_any_f64<0x140>(v);       // row_mirror
  v += dpp_any_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_any_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return readlane_f64(v, 63);
}

GW_DEV double wave_max(double v) {
  v = fmax(v, dpp_any_f64<0xB1>(v));
  v = fmax(v, dpp_any_f64<0x4E>(v));
  v = fmax(v, dpp_any_f64<0x141>(v));
  v = fmax(v, dpp_any_f64<0x140>(v));
  v = fmax(v, dpp_any_f64<0x142, 0xA>(v));
  v = fmax(v, dpp_any_f64<0x143, 0xC>(v));
  return readlane_f64(v, 63);
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

// Masked stores without a branch: a raw buffer resource over `base` (a
// wave-uniform address) covering kRsrcBytes, and a store that every lane
// issues; lanes whose byte offset is kOffDrop or above fall outside the
// resource's range and are dropped by the hardware.  With no branch around
// stores, the number of memory operations in flight is the same on every
// path, so later waits for loads are not widened to cover the stores.
// In-range offsets must stay below kRsrcBytes.
constexpr int kRsrcBytes = 1 << 16;
constexpr int kOffDrop = 1 << 30;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

GW_DEV __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base) {
  // 0x00020000: the raw-buffer data format word of the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, kRsrcBytes,
                                           0x00020000);
}

// A raw buffer resource over `bytes` bytes from `base` (a wave-uniform
// address): loads at byte offsets at or beyond `bytes` return 0.
GW_DEV __amdgpu_buffer_rsrc_t buffer_rsrc_n(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// A double at byte offset voff + soff of the resource (soff wave-uniform).
GW_DEV double buffer_load_f64(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// AUX: cache policy bits of the store (0 default; 2 non-temporal, for output
// that is streamed out and not read back soon).
template <int AUX = 0>
GW_DEV void buffer_store_f64(double v, __amdgpu_buffer_rsrc_t r, int byte_off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, byte_off, 0, AUX);
}

}  // namespace gwk
