// Host-side helpers shared by the launchers: grid descriptors, workspace
// layout, kernel timing and error mapping.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gw.h"

namespace gwr {

// A validated grid in the form the kernels use.
struct Grid {
  int ndim;
  int k;
  int metric;
  int64_t Z, H, W;  // 1D: Z = H = 1, W = n; 2D: Z = 1
  double h;
  int64_t n() const { return Z * H * W; }
  // h^k as k left-to-right products (h^2 for SQEUCLID).
  double hk() const {
    int kk = metric == GW_METRIC_SQEUCLID ? 2 : k;
    double v = 1.0;
    for (int i = 0; i < kk; ++i) v = v * h;
    return v;
  }
  // Exponent used by the 1D recursion (1D grids only).
  int k1d() const { return metric == GW_METRIC_SQEUCLID ? 2 : k; }
};

// Host-side validation of a public grid; returns GW_OK or GW_EINVAL.
gw_status to_grid(const gw_grid* g, Grid* out);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace.
struct Arena {
  char* base;
  size_t used;
  size_t cap;
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used, 256);
    used = off + align_up(count * sizeof(T), 256);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Workspace bytes for each building block (all multiples of 256).
size_t ws_status_bytes();
size_t ws_grad_bytes(const Grid& X, const Grid& Y, int path);
size_t ws_sinkhorn_bytes(int64_t M, int64_t N);
size_t ws_objective_bytes(const Grid& X, const Grid& Y);
size_t ws_objective_tail_bytes(const Grid& X, const Grid& Y);

// Kernel timing families (see gw.h).
enum Family {
  kFamFastMain = 0,
  kFamFastCarry = 1,
  kFamDense = 2,
  kFamSinkRow = 3,
  kFamSinkCol = 4,
  kFamPlan = 5,
  kFamOther = 6,
  kFam2D = 7,
  kFamServeStep = 8,
  kNumFamilies = 9
};
void prof_begin(int family, hipStream_t s);
void prof_end(int family, hipStream_t s);

// Times everything enqueued on `s` during the scope (events recorded before
// and after: includes the dispatch latency of each launch).
struct ProfScope {
  int fam;
  hipStream_t s;
  ProfScope(int f, hipStream_t st) : fam(f), s(st) { prof_begin(fam, s); }
  ~ProfScope() { prof_end(fam, s); }
};

// Times one kernel dispatch by its own begin and end timestamps: pass b and e
// as the start / stop events of hipExtLaunchKernelGGL.  Both are null (a plain
// launch) when the family is not being timed.
void prof_dispatch_events(int family, hipEvent_t* b, hipEvent_t* e);
void prof_dispatch_done(int family, hipEvent_t b, hipEvent_t e);
struct ProfDispatch {
  int fam;
  hipEvent_t b = nullptr, e = nullptr;
  explicit ProfDispatch(int f) : fam(f) { prof_dispatch_events(fam, &b, &e); }
  ~ProfDispatch() { prof_dispatch_done(fam, b, e); }
};

// A side stream for work that may run beside the caller's stream, pooled per
// device.  side_take(s) hands one out that waits for what `s` has enqueued so
// far; side_join makes `s` wait for what was enqueued on it and returns it to
// the pool.  Both are event waits, so they also hold while `s` is being
// captured into a graph (where no new side stream is created: nullptr then,
// and the caller uses `s`).
struct SideStream {
  int dev = -1;
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};
SideStream* side_take(hipStream_t s);
gw_status side_join(SideStream* ss, hipStream_t s);

// Joins a side stream (if any) when the work that needs it is about to be
// enqueued, or on leaving the scope.
struct SideJoin {
  SideStream* ss;
  hipStream_t s;
  gw_status join() {
    SideStream* x = ss;
    ss = nullptr;
    return x ? side_join(x, s) : GW_OK;
  }
  ~SideJoin() { (void)join(); }
};

// Raise a kernel's dynamic LDS limit on the current device to at least
// `bytes` (hipFuncSetAttribute once per kernel, device and larger size;
// thread-safe).  GW_EDEVICE if the runtime refuses.
gw_status allow_dyn_lds(const void* kernel, size_t bytes);

inline gw_status last_launch_status() {
  return hipGetLastError() == hipSuccess ? GW_OK : GW_EDEVICE;
}

// Status word kept at the start of every workspace (first 256 bytes).
struct StatusWord {
  int32_t nonfinite;
};

gw_status clear_status(StatusWord* st, hipStream_t s);

// Fused GW terms: feature vectors fa [M], fb [N] (c_ip = fa_i - fb_p) and the
// weight theta of the GW part.
struct Fgw {
  const double* fa;
  const double* fb;
  double theta;
};

// Elementwise step applied to a gradient as it is written:
// G <- a G + b (fa_i - fb_p)^2 (the fused GW feature term).  Passed by value
// to kernels.
struct Epilogue {
  const double* fa;
  const double* fb;
  double a;
  double b;
};

// Tolerance stop of a Sinkhorn call: every check_every iterations the column
// violation of the half-step plan is measured; the call stops after the first
// check with violation <= tol.  iters_out / err_out (device, may be null)
// receive the iterations done and the last measured violation.
struct SkStop {
  int check_every;
  double tol;
  int* iters_out;
  double* err_out;
};

// Gradient on `path` with optional precomputed constant terms and optional
// epilogue, and the objective of a plan (its own marginals, Gbuf [M x N] as
// scratch; the fused objective when fgw is given); both take their scratch
// from `a`.
gw_status run_grad(const Grid& X, const Grid& Y, const double* p, const double* q,
                   const double* T, int64_t ldT, double* G, int64_t ldG, int path, Arena& a,
                   hipStream_t s, const double* c1, const double* c2,
                   const Epilogue* epi = nullptr);
gw_status run_objective(const Grid& X, const Grid& Y, const double* T, int64_t ldT, double eps,
                        double* obj, double* Gbuf, Arena& a, hipStream_t s, StatusWord* status,
                        const Fgw* fgw);

}  // namespace gwr

// Launchers implemented in the kernel translation units.
namespace gwl {
// c[i] = hk^2 * sum_j d(i,j)^2 w[j] for grid g (recursion in 1D, separable form
// in 2D).
gw_status const_term(const gwr::Grid& g, const double* w, double* c, hipStream_t s);
// c1 for (X, p) and c2 for (Y, q), in one launch when both are 1D with the same
// exponent.
gw_status const_terms(const gwr::Grid& X, const double* p, double* c1, const gwr::Grid& Y,
                      const double* q, double* c2, hipStream_t s);
// Use the precomputed constant terms where given (c1_pre, c2_pre may be null),
// else compute them into *c1, *c2 (workspace).
gw_status resolve_const_terms(const gwr::Grid& X, const double* p, const double* c1_pre,
                              double** c1, const gwr::Grid& Y, const double* q,
                              const double* c2_pre, double** c2, hipStream_t s);
// FAST 1D x 1D gradient (tiled recursion).  ws: arena for its scratch; epi
// (may be null) is applied by the kernel that writes G.
gw_status fast1d(const gwr::Grid& X, const gwr::Grid& Y, const double* p, const double* q,
                 const double* T, int64_t ldT, double* G, int64_t ldG, gwr::Arena& ws,
                 hipStream_t s, const double* c1_pre, const double* c2_pre,
                 const gwr::Epilogue* epi);
size_t fast1d_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y);
// The unscaled 2D grid operator on every row of `in` (rows x H W), for images of
// at most 64 x 64 points; GW_EUNSUPPORTED otherwise.
gw_status img_rowop(const double* in, int64_t ldi, int64_t rows, const gwr::Grid& g,
                    double* out, int64_t ldo, hipStream_t s);
// The same for 3D grids with every axis of at most 16 points.
gw_status img3_rowop(const double* in, int64_t ldi, int64_t rows, const gwr::Grid& g,
                     double* out, int64_t ldo, hipStream_t s);
// Generic FAST gradient for 2D (and mixed 1D/2D) grids; epi as for fast1d.
gw_status fast_generic(const gwr::Grid& X, const gwr::Grid& Y, const double* p,
                       const double* q, const double* T, int64_t ldT, double* G, int64_t ldG,
                       gwr::Arena& ws, hipStream_t s, const double* c1_pre,
                       const double* c2_pre, const gwr::Epilogue* epi);
size_t fast_generic_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y);
// Dense gradient on matrix cores.
gw_status dense(const gwr::Grid& X, const gwr::Grid& Y, const double* p, const double* q,
                const double* T, int64_t ldT, double* G, int64_t ldG, int path, gwr::Arena& ws,
                hipStream_t s, const double* c1_pre, const double* c2_pre);
size_t dense_ws_bytes(const gwr::Grid& X, const gwr::Grid& Y, int path);
// Sinkhorn.
gw_status sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                   const double* p, const double* q, double eps, int iters, int init_zero,
                   double* f, double* g, double* T, int64_t ldT, gwr::Arena& ws, hipStream_t s,
                   gwr::StatusWord* status, const gwr::SkStop* stop = nullptr);
size_t sinkhorn_ws_bytes(int64_t M, int64_t N);
gw_status plan(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
               const double* f, const double* g, double eps, double* T, int64_t ldT,
               hipStream_t s);
gw_status outer_product(const double* p, const double* q, int64_t M, int64_t N, double* T,
                        int64_t ldT, hipStream_t s);
// Row sums, column sums, and the reductions sum G*T, sum T(ln T - 1).
gw_status marginals(const double* T, int64_t ldT, int64_t M, int64_t N, double* r, double* c,
                    gwr::Arena& ws, hipStream_t s);
gw_status objective_reduce(const double* G, int64_t ldG, const double* T, int64_t ldT,
                           int64_t M, int64_t N, double eps, double* obj, gwr::Arena& ws,
                           hipStream_t s, gwr::StatusWord* status);
size_t objective_reduce_ws_bytes(int64_t M, int64_t N);
// Unbalanced GW: step scalars (device block of uot_scalars_bytes()), the
// unbalanced Sinkhorn and the solve's set-up / step / objective pieces.
size_t uot_scalars_bytes();
size_t uot_ws_bytes(int64_t M, int64_t N);
gw_status uot_set_scalars(void* scal, double shift, double e, double tau, hipStream_t s);
gw_status uot_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, const double* u,
                       const double* v, int iters, int init_zero, double* f, double* g,
                       double* T, int64_t ldT, bool rescale, void* scal, gwr::Arena& ws,
                       hipStream_t s, gwr::StatusWord* status);
gw_status ugw_init(const double* u, const double* v, int64_t M, int64_t N, double* T,
                   int64_t ldT, void* scal, hipStream_t s);
gw_status ugw_step_scalars(const double* T, int64_t ldT, int64_t M, int64_t N, const double* a,
                           const double* b, const double* u, const double* v, double rho,
                           double eps, double* rowpart, void* scal, hipStream_t s);
gw_status ugw_objective(const double* T, int64_t ldT, int64_t M, int64_t N, const double* a,
                        const double* b, const double* u, const double* v, double rho,
                        double eps, double* rowpart, const void* scal, const double* eobj,
                        double* obj, hipStream_t s);
// G <- a G + b (fa_i - fb_p)^2 (fused GW terms).
gw_status fgw_blend(double* G, int64_t ldG, int64_t M, int64_t N, const double* fa,
                    const double* fb, double a, double b, hipStream_t s);
}  // namespace gwl
