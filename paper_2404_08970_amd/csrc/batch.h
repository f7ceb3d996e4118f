// Device work table of the request loop: one descriptor per active request
// (slot) and, per kernel class, a list of work items.  The host rewrites the
// table between steps; the captured step graph reads it.
#pragma once
#include <stdint.h>

#include "runtime.h"

namespace gwb {

// Row-pass classes by row length N, each with the same block shape as the
// single-problem Sinkhorn kernel for that length, plus the column merge.
enum {
  kClsN256 = 0,    // N <= 256:   256 threads, 1 entry per thread
  kClsN512 = 1,    // N <= 512:   512 threads, 1 entry
  kClsN1024 = 2,   // N <= 1024: 1024 threads, 1 entry
  kClsN2048 = 3,   // N <= 2048: 1024 threads, 2 entries
  kClsN3072 = 4,   // N <= 3072:  256 threads, 12 entries
  kClsN4096 = 5,   // N <= 4096: two 512-thread row groups, 8 entries
  kClsN6144 = 6,   // N <= 6144:  512 threads, 12 entries
  kClsN8192 = 7,   // N <= 8192:  512 threads, 16 entries
  kClsN9216 = 8,   // N <= 9216:  512 threads, 18 entries, g / eps in LDS
  kClsN12288 = 9,  // N <= 12288: 512 threads, 24 entries, g / eps in LDS
  kClsN16384 = 10, // N <= 16384: 512 threads, 32 entries, g / eps in LDS
  kNumRowCls = 11,
  kClsCol = 11,    // column merge items
  kNumLists = 12
};

inline int row_class(int64_t N) {
  if (N <= 256) return kClsN256;
  if (N <= 512) return kClsN512;
  if (N <= 1024) return kClsN1024;
  if (N <= 2048) return kClsN2048;
  if (N <= 3072) return kClsN3072;
  if (N <= 4096) return kClsN4096;
  if (N <= 6144) return kClsN6144;
  if (N <= 8192) return kClsN8192;
  if (N <= 9216) return kClsN9216;
  if (N <= 12288) return kClsN12288;
  return kClsN16384;
}

// Columns merged by one column-pass item (a block of 256 threads).
constexpr int kMergeCols = 16;

// Item encodings: row items (slot << 9) | band (band < 512), column items
// (slot << 11) | column block (block < 2048).
constexpr int kBandBits = 9, kCBlockBits = 11;

// One Sinkhorn problem as the batched kernels see it (all device pointers).
struct SkSlot {
  const double* C;  // cost matrix, C_eff = cs * C
  int64_t ldC;
  const double* p;
  const double* logp;
  const double* q;
  const double* logq;
  double* f;
  double* g;
  double* ms;  // (m_i, s_i) of the last row pass
  double* pS;  // [nb x N] partial column mantissas
  int* pX;     // [nb x N] partial column exponents
  gwr::StatusWord* status;
  double* lse;    // [M] upper bounds of the rows' log-sum-exp (row shifts)
  double* gprev;  // [N] g before the last column merge
  const int* kq;  // [N] column frames of the fast pass
  int* bmode;     // [nb] pass kind of each band's partials
  double cs, inv_eps, eps;
  int32_t M, N, RB, nb;
  int32_t its;   // Sinkhorn iterations this request takes in the current step
  int32_t last;  // 1 if the step's last iteration is the request's last one
  int32_t it0;   // index, within the request's Sinkhorn call, of the step's first iteration
  int32_t pad;
};

struct SkTableHead {
  int32_t count[kNumLists];
  int32_t offset[kNumLists];  // in items, from the start of the item array
};

}  // namespace gwb

namespace gwl {
// Launch the batched row pass of class `cls` (or the column merge for
// gwb::kClsCol) for iteration `j` of a step, with a fixed persistent grid.
gw_status sk_batch_launch(int cls, int j, const gwb::SkSlot* slots, const gwb::SkTableHead* head,
                          const uint32_t* items, hipStream_t s);
// Per-request pieces of a Sinkhorn call around the batched iterations:
// log-marginals (and zero potentials if init_zero), and after the last
// iteration f from (m, s) and the plan.
gw_status sinkhorn_prep(const double* p, const double* q, int64_t M, int64_t N, int init_zero,
                        double* logp, double* logq, int* kq, double* f, double* g,
                        hipStream_t s);
gw_status sinkhorn_finish(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                          const double* p, const double* logp, const double* ms, double eps,
                          int iters, double* f, const double* g, double* T, int64_t ldT,
                          hipStream_t s, gwr::StatusWord* status);
int sk_rows_per_band(int64_t M);
}  // namespace gwl
