// C ABI entry points of libgw.so: argument validation, workspace layout,
// dispatch to the kernel launchers, status reporting and kernel timing.
#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "runtime.h"

namespace gwr {

static const int64_t kMaxExtent = 65535;

namespace {
std::mutex g_side_mu;
std::vector<SideStream*> g_side_free;

void side_destroy(SideStream* ss) {
  if (ss->fork_ev) (void)hipEventDestroy(ss->fork_ev);
  if (ss->join_ev) (void)hipEventDestroy(ss->join_ev);
  if (ss->side) (void)hipStreamDestroy(ss->side);
  delete ss;
}

void side_give(SideStream* ss) {
  std::lock_guard<std::mutex> lock(g_side_mu);
  g_side_free.push_back(ss);
}

// A pooled side stream that was forked from a stream under capture stays in
// that capture until the capture ends, even after it was joined back and
// returned.  It may only be handed out again to work on a stream of the same
// capture; eager work, or another capture, must not enqueue on it.
bool side_usable(SideStream* ss, hipStream_t s) {
  hipStreamCaptureStatus cs_side = hipStreamCaptureStatusNone;
  unsigned long long id_side = 0;
  if (hipStreamGetCaptureInfo(ss->side, &cs_side, &id_side) != hipSuccess) return false;
  if (cs_side == hipStreamCaptureStatusNone) return true;
  hipStreamCaptureStatus cs_s = hipStreamCaptureStatusNone;
  unsigned long long id_s = 0;
  if (hipStreamGetCaptureInfo(s, &cs_s, &id_s) != hipSuccess) return false;
  return cs_side == hipStreamCaptureStatusActive && cs_s == hipStreamCaptureStatusActive &&
         id_s == id_side;
}
}  // namespace

SideStream* side_take(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  SideStream* ss = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_side_mu);
    for (size_t i = 0; i < g_side_free.size(); ++i)
      if (g_side_free[i]->dev == dev && side_usable(g_side_free[i], s)) {
        ss = g_side_free[i];
        g_side_free.erase(g_side_free.begin() + (ptrdiff_t)i);
        break;
      }
  }
  if (!ss) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return nullptr;
    ss = new (std::nothrow) SideStream();
    if (!ss) return nullptr;
    ss->dev = dev;
    // default priority, like every stream of this library
    if (hipStreamCreateWithFlags(&ss->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ss->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ss->join_ev, hipEventDisableTiming) != hipSuccess) {
      side_destroy(ss);
      return nullptr;
    }
  }
  if (hipEventRecord(ss->fork_ev, s) != hipSuccess ||
      hipStreamWaitEvent(ss->side, ss->fork_ev, 0) != hipSuccess) {
    side_give(ss);
    return nullptr;
  }
  return ss;
}

gw_status side_join(SideStream* ss, hipStream_t s) {
  const bool ok = hipEventRecord(ss->join_ev, ss->side) == hipSuccess &&
                  hipStreamWaitEvent(s, ss->join_ev, 0) == hipSuccess;
  side_give(ss);
  return ok ? GW_OK : GW_EDEVICE;
}

gw_status allow_dyn_lds(const void* kernel, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GW_EDEVICE;
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> set;  // largest size set so far
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = set[{dev, kernel}];
  if (bytes <= cur) return GW_OK;
  if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
      hipSuccess)
    return GW_EDEVICE;
  cur = bytes;
  return GW_OK;
}

gw_status to_grid(const gw_grid* g, Grid* out) {
  if (!g) return GW_EINVAL;
  if (g->reserved != 0) return GW_EINVAL;
  if (g->ndim < 1 || g->ndim > 3) return GW_EINVAL;
  if (g->metric != GW_METRIC_L1POW && g->metric != GW_METRIC_SQEUCLID) return GW_EINVAL;
  if (g->k < 1 || g->k > GW_KMAX) return GW_EINVAL;
  if (g->metric == GW_METRIC_SQEUCLID && g->k != 2) return GW_EINVAL;
  if (!(g->h > 0.0) || !isfinite(g->h)) return GW_EINVAL;
  if (g->shape[0] < 1 || g->shape[1] < 1 || g->shape[2] < 1) return GW_EINVAL;
  if (g->ndim == 1 && g->shape[1] != 1) return GW_EINVAL;
  if (g->ndim <= 2 && g->shape[2] != 1) return GW_EINVAL;
  Grid r;
  r.ndim = g->ndim;
  r.k = g->k;
  r.metric = g->metric;
  r.h = g->h;
  r.Z = 1;
  if (g->ndim == 1) {
    r.H = 1;
    r.W = g->shape[0];
  } else if (g->ndim == 2) {
    r.H = g->shape[0];
    r.W = g->shape[1];
  } else {
    r.Z = g->shape[0];
    r.H = g->shape[1];
    r.W = g->shape[2];
  }
  if (r.Z > kMaxExtent || r.H > kMaxExtent || r.W > kMaxExtent) return GW_EUNSUPPORTED;
  if (r.Z * r.H > kMaxExtent || r.n() > kMaxExtent) return GW_EUNSUPPORTED;
  *out = r;
  return GW_OK;
}

size_t ws_status_bytes() { return 256; }

size_t ws_grad_bytes(const Grid& X, const Grid& Y, int path) {
  if (path == GW_PATH_FAST_F64) {
    if (X.ndim == 1 && Y.ndim == 1) return gwl::fast1d_ws_bytes(X, Y);
    return gwl::fast_generic_ws_bytes(X, Y);
  }
  return gwl::dense_ws_bytes(X, Y, path);
}

size_t ws_sinkhorn_bytes(int64_t M, int64_t N) { return gwl::sinkhorn_ws_bytes(M, N); }

// Objective scratch after the M x N gradient buffer: marginals, the FAST
// gradient's own workspace and the reduction partials.
size_t ws_objective_tail_bytes(const Grid& X, const Grid& Y) {
  Arena a{nullptr, 0, 0};
  a.take<double>(X.n());  // row sums
  a.take<double>(Y.n());  // column sums
  return a.used + ws_grad_bytes(X, Y, GW_PATH_FAST_F64) +
         gwl::objective_reduce_ws_bytes(X.n(), Y.n());
}

size_t ws_objective_bytes(const Grid& X, const Grid& Y) {
  Arena a{nullptr, 0, 0};
  a.take<double>((size_t)X.n() * Y.n());  // gradient at T's own marginals
  return a.used + ws_objective_tail_bytes(X, Y);
}

// ------------------------------------------------------------------ timing
namespace {
struct ProfState {
  std::mutex mu;
  int32_t mask = 0;
  std::vector<hipEvent_t> pool[kNumFamilies];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kNumFamilies];
  size_t used[kNumFamilies] = {};
  double total_ms[kNumFamilies] = {};
  int64_t launches[kNumFamilies] = {};
  hipEvent_t open[kNumFamilies] = {};
  int32_t every = 1;                    // time one launch in `every`
  int64_t seq[kNumFamilies] = {};       // launches seen since the last enable
};
ProfState& prof() {
  static ProfState* p = new ProfState();
  return *p;
}
hipEvent_t pool_event(ProfState& P, int fam) {
  if (P.used[fam] < P.pool[fam].size()) return P.pool[fam][P.used[fam]++];
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  P.pool[fam].push_back(e);
  P.used[fam]++;
  return e;
}
void drain(ProfState& P, int fam) {
  for (auto& pr : P.pending[fam]) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess &&
        hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      P.total_ms[fam] += ms;
      P.launches[fam] += 1;
    }
  }
  P.pending[fam].clear();
  P.used[fam] = 0;
}
}  // namespace

// The launches of a family are counted and every P.every-th one is timed.
bool sampled(ProfState& P, int fam) { return P.seq[fam]++ % P.every == 0; }

void prof_begin(int fam, hipStream_t s) {
  ProfState& P = prof();
  if (!(P.mask & (1 << fam))) return;
  std::lock_guard<std::mutex> g(P.mu);
  P.open[fam] = nullptr;
  if (!sampled(P, fam)) return;
  if (P.used[fam] + 2 > (size_t(1) << 20)) drain(P, fam);
  hipEvent_t e = pool_event(P, fam);
  if (e) (void)hipEventRecord(e, s);
  P.open[fam] = e;
}

void prof_dispatch_events(int fam, hipEvent_t* b, hipEvent_t* e) {
  *b = *e = nullptr;
  ProfState& P = prof();
  if (!(P.mask & (1 << fam))) return;
  std::lock_guard<std::mutex> g(P.mu);
  if (!sampled(P, fam)) return;
  if (P.used[fam] + 2 > (size_t(1) << 20)) drain(P, fam);
  *b = pool_event(P, fam);
  *e = pool_event(P, fam);
  if (!*b || !*e) *b = *e = nullptr;
}

void prof_dispatch_done(int fam, hipEvent_t b, hipEvent_t e) {
  if (!b || !e) return;
  ProfState& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.pending[fam].push_back({b, e});
}

void prof_end(int fam, hipStream_t s) {
  ProfState& P = prof();
  if (!(P.mask & (1 << fam))) return;
  std::lock_guard<std::mutex> g(P.mu);
  hipEvent_t b = P.open[fam];
  hipEvent_t e = pool_event(P, fam);
  if (b && e) {
    (void)hipEventRecord(e, s);
    P.pending[fam].push_back({b, e});
  }
  P.open[fam] = nullptr;
}

}  // namespace gwr

using gwr::Arena;
using gwr::Grid;

namespace {

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }
bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* ca = (const char*)a;
  const char* cb = (const char*)b;
  return ca < cb + bn && cb < ca + an;
}

gw_status check_matrix(const double* ptr, int64_t rows, int64_t cols, int64_t ld) {
  if (!ptr || !aligned8(ptr)) return GW_EINVAL;
  if (ld < cols) return GW_EINVAL;
  if (rows > 0 && ld > (int64_t(1) << 40) / rows) return GW_EINVAL;
  return GW_OK;
}

gw_status check_vec(const double* ptr) { return (ptr && aligned8(ptr)) ? GW_OK : GW_EINVAL; }

gw_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need > ws_bytes) return GW_ENOMEM;
  if (need > 0 && (!ws || !aligned256(ws))) return GW_EINVAL;
  return GW_OK;
}

gwr::StatusWord* status_of(void* ws) { return reinterpret_cast<gwr::StatusWord*>(ws); }

size_t grad_need(const Grid& X, const Grid& Y, int path) {
  return gwr::ws_status_bytes() + gwr::ws_grad_bytes(X, Y, path);
}

bool path_valid(int path) { return path >= GW_PATH_FAST_F64 && path <= GW_PATH_DENSE_F32_SPLIT; }

// UGW solve: scalars, a, b, row partials, G, E, then the larger of the UOT
// scratch, the gradient's and the objective's.
size_t ugw_need(const Grid& X, const Grid& Y, int path) {
  const int64_t M = X.n(), N = Y.n();
  Arena a{nullptr, 0, 0};
  a.take<char>(gwr::ws_status_bytes());
  a.take<char>(gwl::uot_scalars_bytes());
  a.take<double>(M);              // a = T 1
  a.take<double>(N);              // b = T^T 1
  a.take<double>(M);              // row partials
  a.take<double>((size_t)M * N);  // G
  a.take<double>(2);              // E
  size_t tail = gwr::ws_grad_bytes(X, Y, path);
  const size_t uo = gwl::uot_ws_bytes(M, N);
  if (uo > tail) tail = uo;
  const size_t ob = gwr::ws_objective_tail_bytes(X, Y);
  if (ob > tail) tail = ob;
  return a.used + tail;
}

size_t uot_need(int64_t M, int64_t N) {
  Arena a{nullptr, 0, 0};
  a.take<char>(gwr::ws_status_bytes());
  a.take<char>(gwl::uot_scalars_bytes());
  return a.used + gwl::uot_ws_bytes(M, N);
}

size_t solve_need(const Grid& X, const Grid& Y, int path) {
  const int64_t M = X.n(), N = Y.n();
  Arena a{nullptr, 0, 0};
  a.take<char>(gwr::ws_status_bytes());
  a.take<double>((size_t)M * N);  // G
  a.take<double>(M);              // c1
  a.take<double>(N);              // c2
  size_t tail = gwr::ws_grad_bytes(X, Y, path);
  const size_t sk = gwr::ws_sinkhorn_bytes(M, N);
  if (sk > tail) tail = sk;
  const size_t ob = gwr::ws_objective_tail_bytes(X, Y);  // the objective reuses G
  if (ob > tail) tail = ob;
  return a.used + tail;
}

}  // namespace

namespace gwr {

gw_status run_grad(const Grid& X, const Grid& Y, const double* p, const double* q,
                   const double* T, int64_t ldT, double* G, int64_t ldG, int path, Arena& a,
                   hipStream_t s, const double* c1, const double* c2, const Epilogue* epi) {
  if (path == GW_PATH_FAST_F64) {
    if (X.ndim == 1 && Y.ndim == 1)
      return gwl::fast1d(X, Y, p, q, T, ldT, G, ldG, a, s, c1, c2, epi);
    return gwl::fast_generic(X, Y, p, q, T, ldT, G, ldG, a, s, c1, c2, epi);
  }
  gw_status st = gwl::dense(X, Y, p, q, T, ldT, G, ldG, path, a, s, c1, c2);
  if (st != GW_OK || !epi) return st;
  return gwl::fgw_blend(G, ldG, X.n(), Y.n(), epi->fa, epi->fb, epi->a, epi->b, s);
}

gw_status run_objective(const Grid& X, const Grid& Y, const double* T, int64_t ldT, double eps,
                        double* obj, double* Gbuf, Arena& a, hipStream_t s,
                        gwr::StatusWord* status, const Fgw* fgw) {
  const int64_t M = X.n(), N = Y.n();
  double* r = a.take<double>(M);
  double* c = a.take<double>(N);
  gw_status st = gwl::marginals(T, ldT, M, N, r, c, a, s);
  if (st != GW_OK) return st;
  // fused objective: sum T (theta G' + (1 - theta) c^2)
  const bool fused = fgw && fgw->theta != 1.0;
  const Epilogue epi{fused ? fgw->fa : nullptr, fused ? fgw->fb : nullptr,
                     fused ? fgw->theta : 1.0, fused ? 1.0 - fgw->theta : 0.0};
  st = run_grad(X, Y, r, c, T, ldT, Gbuf, N, GW_PATH_FAST_F64, a, s, nullptr, nullptr,
                fused ? &epi : nullptr);
  if (st != GW_OK) return st;
  return gwl::objective_reduce(Gbuf, N, T, ldT, M, N, eps, obj, a, s, status);
}

__global__ void k_clear_status(StatusWord* st) { st->nonfinite = 0; }

gw_status clear_status(StatusWord* st, hipStream_t s) {
  ProfScope ps(kFamOther, s);
  k_clear_status<<<1, 1, 0, s>>>(st);
  return last_launch_status();
}

}  // namespace gwr

namespace {
using gwr::run_grad;
using gwr::run_objective;

gw_status check_fgw(const gwr::Fgw& fw) {
  if (!isfinite(fw.theta) || fw.theta < 0.0 || fw.theta > 1.0) return GW_EINVAL;
  if (check_vec(fw.fa) != GW_OK || check_vec(fw.fb) != GW_OK) return GW_EINVAL;
  return GW_OK;
}

// Gradient (Sec. 2, decomposition of the gradient), GW or fused GW (fgw non-null).
gw_status grad_impl(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                    const gwr::Fgw* fgw, const double* T, int64_t ldT, double* G, int64_t ldG,
                    int32_t path, void* ws, size_t ws_bytes, void* stream) {
  Grid X, Y;
  gw_status st;
  if ((st = gwr::to_grid(Xp, &X)) != GW_OK) return st;
  if ((st = gwr::to_grid(Yp, &Y)) != GW_OK) return st;
  if (!path_valid(path)) return GW_EINVAL;
  if (fgw && (st = check_fgw(*fgw)) != GW_OK) return st;
  const int64_t M = X.n(), N = Y.n();
  if ((st = check_vec(p)) != GW_OK || (st = check_vec(q)) != GW_OK) return st;
  if ((st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  if ((st = check_matrix(G, M, N, ldG)) != GW_OK) return st;
  if (overlaps(T, sizeof(double) * ((M - 1) * ldT + N), G, sizeof(double) * ((M - 1) * ldG + N)))
    return GW_EINVAL;
  if ((st = check_ws(ws, ws_bytes, grad_need(X, Y, path))) != GW_OK) return st;
  if (path != GW_PATH_FAST_F64 && (X.ndim != 1 || Y.ndim != 1)) return GW_EUNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Arena a{static_cast<char*>(ws), 0, ws_bytes};
  a.take<char>(gwr::ws_status_bytes());
  // fused GW: half gradient theta G + (1 - theta)/2 c^2 (skipped at theta = 1)
  const bool fused = fgw && fgw->theta != 1.0;
  const gwr::Epilogue epi{fused ? fgw->fa : nullptr, fused ? fgw->fb : nullptr,
                          fused ? fgw->theta : 1.0, fused ? 0.5 * (1.0 - fgw->theta) : 0.0};
  return run_grad(X, Y, p, q, T, ldT, G, ldG, path, a, s, nullptr, nullptr,
                  fused ? &epi : nullptr);
}

gw_status check_stop(const gwr::SkStop& so) {
  if (so.check_every < 1 || isnan(so.tol)) return GW_EINVAL;
  if (so.iters_out && reinterpret_cast<uintptr_t>(so.iters_out) % alignof(int32_t)) return GW_EINVAL;
  if (so.err_out && !aligned8(so.err_out)) return GW_EINVAL;
  return GW_OK;
}

// Log-domain Sinkhorn (Sec. 2.1), fixed iteration count or tolerance stop (so non-null).
gw_status sinkhorn_impl(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                        const double* p, const double* q, double eps, int32_t iters,
                        int32_t init_zero, const gwr::SkStop* so, double* f, double* g,
                        double* T, int64_t ldT, void* ws, size_t ws_bytes, void* stream,
                        bool clear = false) {
  gw_status st;
  if (M < 1 || N < 1) return GW_EINVAL;
  if (M > gwr::kMaxExtent || N > gwr::kMaxExtent) return GW_EUNSUPPORTED;
  if (!(eps > 0.0) || !isfinite(eps) || !isfinite(c_scale) || iters < 0) return GW_EINVAL;
  if (so && (st = check_stop(*so)) != GW_OK) return st;
  if ((st = check_matrix(C, M, N, ldC)) != GW_OK) return st;
  if ((st = check_vec(p)) != GW_OK || (st = check_vec(q)) != GW_OK) return st;
  if ((st = check_vec(f)) != GW_OK || (st = check_vec(g)) != GW_OK) return st;
  if (T && (st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  const size_t need = gwr::ws_status_bytes() + gwr::ws_sinkhorn_bytes(M, N);
  if ((st = check_ws(ws, ws_bytes, need)) != GW_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (clear && (st = gwr::clear_status(status_of(ws), s)) != GW_OK) return st;
  Arena a{static_cast<char*>(ws), 0, ws_bytes};
  a.take<char>(gwr::ws_status_bytes());
  return gwl::sinkhorn(C, ldC, M, N, c_scale, p, q, eps, iters, init_zero, f, g, T, ldT, a, s,
                       status_of(ws), so);
}

// Scratch of the no-allocation Sinkhorn: a static device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is kept per device.
constexpr size_t kStaticScratchBytes = GW_NOALLOC_SCRATCH_BYTES;
}  // namespace
namespace gwnoalloc {
__device__ __align__(256) char scratch[kStaticScratchBytes];
}  // namespace gwnoalloc
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gw_status static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GW_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(gwnoalloc::scratch)) != hipSuccess || ptr == nullptr)
      return GW_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GW_OK;
}

// Mirror descent (Sec. 2.1), GW or fused GW (fgw non-null).
// With so (non-null), each Sinkhorn call stops by tolerance; its iterations
// done go to so->iters_out[l] for outer step l (if given).
gw_status solve_impl(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                     const gwr::Fgw* fgw, double eps, int32_t outer, int32_t inner,
                     int32_t path, int32_t flags, double* T, int64_t ldT, double* f, double* g,
                     double* obj, void* ws, size_t ws_bytes, void* stream,
                     const gwr::SkStop* so = nullptr) {
  Grid X, Y;
  gw_status st;
  if ((st = gwr::to_grid(Xp, &X)) != GW_OK) return st;
  if ((st = gwr::to_grid(Yp, &Y)) != GW_OK) return st;
  if (!path_valid(path)) return GW_EINVAL;
  if (!(eps > 0.0) || !isfinite(eps) || outer < 0 || inner < 0) return GW_EINVAL;
  if (flags & ~GW_FLAG_WARM_START) return GW_EINVAL;
  if (fgw && (st = check_fgw(*fgw)) != GW_OK) return st;
  if (so && (st = check_stop(*so)) != GW_OK) return st;
  const int64_t M = X.n(), N = Y.n();
  if ((st = check_vec(p)) != GW_OK || (st = check_vec(q)) != GW_OK) return st;
  if ((st = check_vec(f)) != GW_OK || (st = check_vec(g)) != GW_OK) return st;
  if ((st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  if (obj && !aligned8(obj)) return GW_EINVAL;
  if ((st = check_ws(ws, ws_bytes, solve_need(X, Y, path))) != GW_OK) return st;
  if (path != GW_PATH_FAST_F64 && (X.ndim != 1 || Y.ndim != 1)) return GW_EUNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Arena a{static_cast<char*>(ws), 0, ws_bytes};
  a.take<char>(gwr::ws_status_bytes());
  double* G = a.take<double>((size_t)M * N);
  double* c1 = a.take<double>(M);
  double* c2 = a.take<double>(N);
  const size_t mark = a.used;
  // fused GW: the Sinkhorn cost 2 G becomes (1 - theta) c^2 + theta grad E
  const bool fused = fgw && fgw->theta != 1.0;
  const gwr::Epilogue epi{fused ? fgw->fa : nullptr, fused ? fgw->fb : nullptr,
                          fused ? fgw->theta : 1.0, fused ? 0.5 * (1.0 - fgw->theta) : 0.0};
  if ((st = gwl::const_terms(X, p, c1, Y, q, c2, s)) != GW_OK) return st;
  if ((st = gwl::outer_product(p, q, M, N, T, ldT, s)) != GW_OK) return st;
  if ((st = gwr::clear_status(status_of(ws), s)) != GW_OK) return st;
  for (int l = 0; l < outer; ++l) {
    a.used = mark;
    st = run_grad(X, Y, p, q, T, ldT, G, N, path, a, s, c1, c2, fused ? &epi : nullptr);
    if (st != GW_OK) return st;
    a.used = mark;
    const int cold = (flags & GW_FLAG_WARM_START) && l > 0 ? 0 : 1;
    gwr::SkStop sl{};
    if (so) sl = gwr::SkStop{so->check_every, so->tol, so->iters_out ? so->iters_out + l : nullptr,
                             nullptr};
    st = gwl::sinkhorn(G, N, M, N, 2.0, p, q, eps, inner, cold, f, g, T, ldT, a, s, status_of(ws),
                       so ? &sl : nullptr);
    if (st != GW_OK) return st;
  }
  if (obj) {
    a.used = mark;
    return run_objective(X, Y, T, ldT, eps, obj, G, a, s, status_of(ws), fgw);
  }
  return gwr::last_launch_status();
}

gw_status objective_impl(const gw_grid* Xp, const gw_grid* Yp, const double* T, int64_t ldT,
                         const gwr::Fgw* fgw, double eps, double* obj, void* ws,
                         size_t ws_bytes, void* stream) {
  Grid X, Y;
  gw_status st;
  if ((st = gwr::to_grid(Xp, &X)) != GW_OK) return st;
  if ((st = gwr::to_grid(Yp, &Y)) != GW_OK) return st;
  if (!isfinite(eps) || eps < 0.0) return GW_EINVAL;
  if (fgw && (st = check_fgw(*fgw)) != GW_OK) return st;
  const int64_t M = X.n(), N = Y.n();
  if ((st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  if (!obj || !aligned8(obj)) return GW_EINVAL;
  if ((st = check_ws(ws, ws_bytes, gwr::ws_status_bytes() + gwr::ws_objective_bytes(X, Y))) != GW_OK)
    return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Arena a{static_cast<char*>(ws), 0, ws_bytes};
  a.take<char>(gwr::ws_status_bytes());
  double* Gbuf = a.take<double>((size_t)M * N);
  return run_objective(X, Y, T, ldT, eps, obj, Gbuf, a, s, status_of(ws), fgw);
}

}  // namespace

extern "C" {

size_t gw_workspace_bytes(const gw_grid* Xp, const gw_grid* Yp, int32_t path, int32_t op) {
  Grid X, Y;
  if (gwr::to_grid(Xp, &X) != GW_OK || gwr::to_grid(Yp, &Y) != GW_OK) return 0;
  switch (op) {
    case GW_OP_GRAD:
      if (!path_valid(path)) return 0;
      return grad_need(X, Y, path);
    case GW_OP_SINKHORN:
      return gwr::ws_status_bytes() + gwr::ws_sinkhorn_bytes(X.n(), Y.n());
    case GW_OP_SOLVE:
      if (!path_valid(path)) return 0;
      return solve_need(X, Y, path);
    case GW_OP_OBJECTIVE:
      return gwr::ws_status_bytes() + gwr::ws_objective_bytes(X, Y);
    case GW_OP_UOT_SINKHORN:
      return uot_need(X.n(), Y.n());
    case GW_OP_SOLVE_UGW:
      if (!path_valid(path)) return 0;
      return ugw_need(X, Y, path);
  }
  return 0;
}

gw_status gw_grad(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                  const double* T, int64_t ldT, double* G, int64_t ldG, int32_t path, void* ws,
                  size_t ws_bytes, void* stream) {
  return grad_impl(Xp, Yp, p, q, nullptr, T, ldT, G, ldG, path, ws, ws_bytes, stream);
}

gw_status gw_grad_fgw(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                      const double* fa, const double* fb, double theta, const double* T,
                      int64_t ldT, double* G, int64_t ldG, int32_t path, void* ws,
                      size_t ws_bytes, void* stream) {
  const gwr::Fgw fw{fa, fb, theta};
  return grad_impl(Xp, Yp, p, q, &fw, T, ldT, G, ldG, path, ws, ws_bytes, stream);
}

gw_status gw_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                      const double* p, const double* q, double eps, int32_t iters,
                      int32_t init_zero, double* f, double* g, double* T, int64_t ldT, void* ws,
                      size_t ws_bytes, void* stream) {
  return sinkhorn_impl(C, ldC, M, N, c_scale, p, q, eps, iters, init_zero, nullptr, f, g, T, ldT,
                       ws, ws_bytes, stream);
}

gw_status gw_sinkhorn_noalloc(const double* C, int64_t ldC, int64_t M, int64_t N,
                              double c_scale, const double* p, const double* q, double eps,
                              int32_t iters, int32_t init_zero, double* f, double* g, double* T,
                              int64_t ldT, void* stream) {
  // sizes the Sinkhorn kernels take but the static scratch does not hold
  if (M >= 1 && N >= 1 && M <= gwr::kMaxExtent && N <= gwr::kMaxExtent &&
      gwr::ws_status_bytes() + gwr::ws_sinkhorn_bytes(M, N) > kStaticScratchBytes)
    return GW_ENOMEM;
  void* ws = nullptr;
  gw_status st = static_scratch(&ws);
  if (st != GW_OK) return st;
  return sinkhorn_impl(C, ldC, M, N, c_scale, p, q, eps, iters, init_zero, nullptr, f, g, T, ldT,
                       ws, kStaticScratchBytes, stream, /*clear=*/true);
}

gw_status gw_sinkhorn_tol(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                          const double* p, const double* q, double eps, int32_t max_iters,
                          int32_t check_every, double tol, int32_t init_zero, double* f,
                          double* g, double* T, int64_t ldT, int32_t* iters_done, double* err,
                          void* ws, size_t ws_bytes, void* stream) {
  const gwr::SkStop so{check_every, tol, iters_done, err};
  return sinkhorn_impl(C, ldC, M, N, c_scale, p, q, eps, max_iters, init_zero, &so, f, g, T, ldT,
                       ws, ws_bytes, stream);
}

gw_status gw_solve(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                   double eps, int32_t outer, int32_t inner, int32_t path, int32_t flags,
                   double* T, int64_t ldT, double* f, double* g, double* obj, void* ws,
                   size_t ws_bytes, void* stream) {
  return solve_impl(Xp, Yp, p, q, nullptr, eps, outer, inner, path, flags, T, ldT, f, g, obj, ws,
                    ws_bytes, stream);
}

gw_status gw_solve_tol(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                       double eps, int32_t outer, int32_t max_inner, int32_t check_every,
                       double tol, int32_t path, int32_t flags, double* T, int64_t ldT, double* f,
                       double* g, double* obj, int32_t* inner_done, void* ws, size_t ws_bytes,
                       void* stream) {
  const gwr::SkStop so{check_every, tol, inner_done, nullptr};
  return solve_impl(Xp, Yp, p, q, nullptr, eps, outer, max_inner, path, flags, T, ldT, f, g, obj,
                    ws, ws_bytes, stream, &so);
}

gw_status gw_uot_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_shift,
                          const double* u, const double* v, double rho, double eps,
                          int32_t iters, int32_t init_zero, double* f, double* g, double* T,
                          int64_t ldT, void* ws, size_t ws_bytes, void* stream) {
  gw_status st;
  if (M < 1 || N < 1) return GW_EINVAL;
  if (M > gwr::kMaxExtent || N > gwr::kMaxExtent) return GW_EUNSUPPORTED;
  if (N > 16384) return GW_EUNSUPPORTED;
  if (!(eps > 0.0) || !isfinite(eps) || !(rho > 0.0) || !isfinite(rho) || !isfinite(c_shift) ||
      iters < 0)
    return GW_EINVAL;
  if ((st = check_matrix(C, M, N, ldC)) != GW_OK) return st;
  if ((st = check_vec(u)) != GW_OK || (st = check_vec(v)) != GW_OK) return st;
  if ((st = check_vec(f)) != GW_OK || (st = check_vec(g)) != GW_OK) return st;
  if (T && (st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  if ((st = check_ws(ws, ws_bytes, uot_need(M, N))) != GW_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Arena a{static_cast<char*>(ws), 0, ws_bytes};
  a.take<char>(gwr::ws_status_bytes());
  void* scal = a.take<char>(gwl::uot_scalars_bytes());
  if ((st = gwl::uot_set_scalars(scal, c_shift, eps, rho / (rho + eps), s)) != GW_OK) return st;
  return gwl::uot_sinkhorn(C, ldC, M, N, u, v, iters, init_zero, f, g, T, ldT, false, scal, a, s,
                           status_of(ws));
}

gw_status gw_solve_ugw(const gw_grid* Xp, const gw_grid* Yp, const double* u, const double* v,
                       double rho, double eps, int32_t outer, int32_t inner, int32_t path,
                       double* T, int64_t ldT, double* f, double* g, double* obj, void* ws,
                       size_t ws_bytes, void* stream) {
  Grid X, Y;
  gw_status st;
  if ((st = gwr::to_grid(Xp, &X)) != GW_OK) return st;
  if ((st = gwr::to_grid(Yp, &Y)) != GW_OK) return st;
  if (!path_valid(path)) return GW_EINVAL;
  if (!(eps > 0.0) || !isfinite(eps) || !(rho > 0.0) || !isfinite(rho) || outer < 0 || inner < 0)
    return GW_EINVAL;
  const int64_t M = X.n(), N = Y.n();
  if (N > 16384) return GW_EUNSUPPORTED;
  if ((st = check_vec(u)) != GW_OK || (st = check_vec(v)) != GW_OK) return st;
  if ((st = check_vec(f)) != GW_OK || (st = check_vec(g)) != GW_OK) return st;
  if ((st = check_matrix(T, M, N, ldT)) != GW_OK) return st;
  if (obj && !aligned8(obj)) return GW_EINVAL;
  if ((st = check_ws(ws, ws_bytes, ugw_need(X, Y, path))) != GW_OK) return st;
  if (path != GW_PATH_FAST_F64 && (X.ndim != 1 || Y.ndim != 1)) return GW_EUNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Arena ar{static_cast<char*>(ws), 0, ws_bytes};
  ar.take<char>(gwr::ws_status_bytes());
  void* scal = ar.take<char>(gwl::uot_scalars_bytes());
  double* a = ar.take<double>(M);
  double* b = ar.take<double>(N);
  double* rowpart = ar.take<double>(M);
  double* G = ar.take<double>((size_t)M * N);
  double* eobj = ar.take<double>(2);
  const size_t mark = ar.used;
  if ((st = gwr::clear_status(status_of(ws), s)) != GW_OK) return st;
  if ((st = gwl::ugw_init(u, v, M, N, T, ldT, scal, s)) != GW_OK) return st;
  for (int l = 0; l < outer; ++l) {
    ar.used = mark;
    // the step at Th = T: marginals, scalars, the half gradient at T's own marginals
    if ((st = gwl::marginals(T, ldT, M, N, a, b, ar, s)) != GW_OK) return st;
    if ((st = gwl::ugw_step_scalars(T, ldT, M, N, a, b, u, v, rho, eps, rowpart, scal, s)) !=
        GW_OK)
      return st;
    if ((st = run_grad(X, Y, a, b, T, ldT, G, N, path, ar, s, nullptr, nullptr)) != GW_OK)
      return st;
    ar.used = mark;
    st = gwl::uot_sinkhorn(G, N, M, N, u, v, inner, 1, f, g, T, ldT, true, scal, ar, s,
                           status_of(ws));
    if (st != GW_OK) return st;
  }
  if (outer == 0) {  // potentials of no step: zero
    ar.used = mark;
    if ((st = gwl::uot_sinkhorn(G, N, M, N, u, v, 0, 1, f, g, nullptr, ldT, false, scal, ar, s,
                                status_of(ws))) != GW_OK)
      return st;
  }
  if (obj) {
    ar.used = mark;
    if ((st = run_objective(X, Y, T, ldT, 0.0, eobj, G, ar, s, status_of(ws), nullptr)) != GW_OK)
      return st;
    if ((st = gwl::marginals(T, ldT, M, N, a, b, ar, s)) != GW_OK) return st;
    return gwl::ugw_objective(T, ldT, M, N, a, b, u, v, rho, eps, rowpart, scal, eobj, obj, s);
  }
  return gwr::last_launch_status();
}

gw_status gw_solve_fgw(const gw_grid* Xp, const gw_grid* Yp, const double* p, const double* q,
                       const double* fa, const double* fb, double theta, double eps,
                       int32_t outer, int32_t inner, int32_t path, int32_t flags, double* T,
                       int64_t ldT, double* f, double* g, double* obj, void* ws,
                       size_t ws_bytes, void* stream) {
  const gwr::Fgw fw{fa, fb, theta};
  return solve_impl(Xp, Yp, p, q, &fw, eps, outer, inner, path, flags, T, ldT, f, g, obj, ws,
                    ws_bytes, stream);
}

gw_status gw_objective(const gw_grid* Xp, const gw_grid* Yp, const double* T, int64_t ldT,
                       double eps, double* obj, void* ws, size_t ws_bytes, void* stream) {
  return objective_impl(Xp, Yp, T, ldT, nullptr, eps, obj, ws, ws_bytes, stream);
}

gw_status gw_objective_fgw(const gw_grid* Xp, const gw_grid* Yp, const double* T, int64_t ldT,
                           const double* fa, const double* fb, double theta, double eps,
                           double* obj, void* ws, size_t ws_bytes, void* stream) {
  const gwr::Fgw fw{fa, fb, theta};
  return objective_impl(Xp, Yp, T, ldT, &fw, eps, obj, ws, ws_bytes, stream);
}

const char* gw_status_string(gw_status s) {
  switch (s) {
    case GW_OK: return "GW_OK";
    case GW_EINVAL: return "GW_EINVAL: invalid argument";
    case GW_ENOMEM: return "GW_ENOMEM: workspace too small";
    case GW_EDEVICE: return "GW_EDEVICE: HIP runtime error";
    case GW_ENUMERIC: return "GW_ENUMERIC: non-finite value detected on the device";
    case GW_EUNSUPPORTED: return "GW_EUNSUPPORTED: request outside what this library implements";
  }
  return "unknown gw_status";
}

gw_status gw_check_status(void* ws, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return GW_EDEVICE;
  if (hipGetLastError() != hipSuccess) return GW_EDEVICE;
  if (!ws) return GW_OK;
  gwr::StatusWord w{0};
  if (hipMemcpy(&w, ws, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) return GW_EDEVICE;
  if (w.nonfinite) {
    if (gwr::clear_status(status_of(ws), s) != GW_OK) return GW_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return GW_EDEVICE;
    return GW_ENUMERIC;
  }
  return GW_OK;
}

void gw_profile_enable(int32_t mask) {
  gwr::ProfState& P = gwr::prof();
  std::lock_guard<std::mutex> g(P.mu);
  for (int f = 0; f < gwr::kNumFamilies; ++f) {
    P.pending[f].clear();
    P.used[f] = 0;
    P.total_ms[f] = 0.0;
    P.launches[f] = 0;
    P.open[f] = nullptr;
    P.seq[f] = 0;
  }
  P.mask = mask;
}

gw_status gw_profile_sample(int32_t every) {
  if (every < 1) return GW_EINVAL;
  gwr::ProfState& P = gwr::prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.every = every;
  for (int f = 0; f < gwr::kNumFamilies; ++f) P.seq[f] = 0;
  return GW_OK;
}

gw_status gw_profile_read(int32_t family, double* total_ms, int64_t* launches) {
  if (family < 0 || family >= gwr::kNumFamilies || !total_ms || !launches) return GW_EINVAL;
  gwr::ProfState& P = gwr::prof();
  std::lock_guard<std::mutex> g(P.mu);
  gwr::drain(P, family);
  *total_ms = P.total_ms[family];
  *launches = P.launches[family];
  return GW_OK;
}

const char* gw_version(void) { return "libgw 0.1 (gfx950)"; }

}  // extern "C"
