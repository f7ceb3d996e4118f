// Request loop: continuous batching of mirror-descent GW solves (Sec. 2.1)
// of uneven sizes on one stream.
//
// Per request the loop runs exactly the calls of gw_solve on the FAST path:
// constant terms, T = p q^T, then per outer iteration the gradient, the
// Sinkhorn set-up, `inner` Sinkhorn iterations, f and the plan.  Everything
// except the Sinkhorn iterations is launched per request; the iterations of
// all requests in their Sinkhorn phase run together as one replay of a
// captured graph of persistent batched kernels (row pass per length class,
// column merge) that take their work from a device table rewritten between
// replays.  Admission is first-come first-served, bounded by slots and by a
// first-fit range of the arena of the request's footprint.
#include <math.h>

#include <deque>
#include <map>
#include <new>
#include <vector>

#include "arena_alloc.h"
#include "batch.h"
#include "runtime.h"

using gwr::Arena;
using gwr::Grid;
using gwr::RangeAllocator;

namespace {

enum Phase { kQueued, kGrad, kSink, kDone };

constexpr int kMaxSlots = 4096;
constexpr int kMaxItersPerStep = 1000;
constexpr int kMaxBoost = 8;
constexpr size_t kMaxGraphs = 256;  // step graphs kept; least recently used ones go first
constexpr int kLevels = 4;  // iteration ranges of a step: [0, S), [S, 2S), [2S, 4S), [4S, 8S)
static_assert(kLevels * gwb::kNumRowCls <= 64, "graph key holds a class mask per range");
static_assert(kMaxBoost == 1 << (kLevels - 1), "one iteration range per doubling");
constexpr int64_t kMaxRows = 65535;
constexpr int64_t kMaxCols = 16384;

// Small pinned record a finished request's objective and status land in.
struct HostRecord {
  double obj[2];
  int32_t nonfinite;
  int32_t pad;
};

struct Req {
  int64_t id = 0;
  gw_request r{};
  Grid X{}, Y{};
  int64_t M = 0, N = 0;
  size_t bytes = 0;
  size_t off = RangeAllocator::kFail;
  int slot = -1;
  Phase phase = kQueued;
  int outer_done = 0;
  int inner_left = 0;
  int its = 0;  // Sinkhorn iterations taken in the current step
  int rb = 0, nb = 0;
  gwr::StatusWord* st = nullptr;
  double *T = nullptr, *G = nullptr, *c1 = nullptr, *c2 = nullptr, *f = nullptr, *g = nullptr;
  double *obj = nullptr, *logp = nullptr, *logq = nullptr, *ms = nullptr, *pS = nullptr;
  double *lse = nullptr, *gprev = nullptr;
  int* pX = nullptr;
  int *kq = nullptr, *bmode = nullptr;
  char* tail = nullptr;
  size_t tail_bytes = 0;
  hipEvent_t done = nullptr;
  HostRecord* rec = nullptr;
};

size_t tail_bytes_of(const Grid& X, const Grid& Y) {
  const size_t a = gwr::ws_grad_bytes(X, Y, GW_PATH_FAST_F64);
  const size_t b = gwr::ws_objective_tail_bytes(X, Y);
  return a > b ? a : b;
}

// Carve a request's buffers from `base` (nullptr: sizes only); returns bytes.
size_t carve(Req& q, char* base) {
  const int64_t M = q.M, N = q.N;
  Arena a{base, 0, 0};
  q.st = a.take<gwr::StatusWord>(1);
  q.T = a.take<double>((size_t)M * N);
  q.G = a.take<double>((size_t)M * N);
  q.c1 = a.take<double>(M);
  q.c2 = a.take<double>(N);
  q.f = a.take<double>(M);
  q.g = a.take<double>(N);
  q.obj = a.take<double>(2);
  q.logp = a.take<double>(M);
  q.logq = a.take<double>(N);
  q.ms = a.take<double>(2 * (size_t)M);
  q.lse = a.take<double>(M);
  q.gprev = a.take<double>(N);
  q.pS = a.take<double>((size_t)q.nb * N);
  q.pX = a.take<int>((size_t)q.nb * N);
  q.kq = a.take<int>(N);
  q.bmode = a.take<int>(q.nb);
  q.tail_bytes = tail_bytes_of(q.X, q.Y);
  q.tail = a.take<char>(q.tail_bytes);
  return a.used;
}

// Validates a request and fills the size fields of q.
gw_status describe(const gw_request* r, Req* q) {
  if (!r) return GW_EINVAL;
  gw_status st;
  if ((st = gwr::to_grid(&r->X, &q->X)) != GW_OK) return st;
  if ((st = gwr::to_grid(&r->Y, &q->Y)) != GW_OK) return st;
  if (!(r->eps > 0.0) || !isfinite(r->eps) || r->outer < 0 || r->inner < 0) return GW_EINVAL;
  if (r->flags & ~(GW_FLAG_WARM_START | GW_REQ_OBJECTIVE)) return GW_EINVAL;
  if (r->reserved != 0) return GW_EINVAL;
  if (!r->p || !r->q || ((uintptr_t)r->p & 7u) || ((uintptr_t)r->q & 7u)) return GW_EINVAL;
  q->M = q->X.n();
  q->N = q->Y.n();
  if (q->N > kMaxCols || q->M > kMaxRows) return GW_EUNSUPPORTED;
  q->rb = gwl::sk_rows_per_band(q->M);
  q->nb = (int)((q->M + q->rb - 1) / q->rb);
  q->r = *r;
  q->bytes = carve(*q, nullptr);
  return GW_OK;
}

struct TableLayout {
  size_t head, slots, items, total;
  size_t item_cap;
};

TableLayout table_layout(int max_slots) {
  TableLayout L;
  L.head = 0;
  L.slots = gwr::align_up(sizeof(gwb::SkTableHead), 256);
  L.items = L.slots + gwr::align_up((size_t)max_slots * sizeof(gwb::SkSlot), 256);
  // per request at most 256 bands and ceil(16384 / 16) column blocks
  L.item_cap = (size_t)max_slots * (256 + kMaxCols / gwb::kMergeCols);
  L.total = L.items + gwr::align_up(L.item_cap * sizeof(uint32_t), 256);
  return L;
}

}  // namespace

struct gw_server {
  hipStream_t s = nullptr;
  hipStream_t cap = nullptr;  // capture only; nothing runs on it
  char* arena = nullptr;
  TableLayout L{};
  RangeAllocator alloc;
  int max_slots = 0, S = 0;
  int boost = 1;  // largest iteration share of a small request (power of two, <= kMaxBoost)
  std::vector<int> free_slots;
  std::deque<int64_t> queue;
  std::map<int64_t, Req> reqs;
  std::vector<int64_t> running;  // admitted, not finished, in admission order
  char* h_stage[2] = {nullptr, nullptr};
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  struct CachedGraph {
    hipGraphExec_t exec;
    int64_t last_step;  // step whose replay used it last
  };
  std::map<uint64_t, CachedGraph> graphs;  // by the class masks of the step's iteration ranges
  std::vector<uint32_t> lists[gwb::kNumLists];
  std::vector<HostRecord*> rec_free;
  std::vector<void*> rec_chunks;
  hipEvent_t ev0 = nullptr;
  bool ready = false;  // creation finished
  int64_t next_id = 1;
  int64_t steps = 0;
};

namespace {

gw_status hip_ok(hipError_t e) { return e == hipSuccess ? GW_OK : GW_EDEVICE; }

gw_status take_record(gw_server* sv, HostRecord** out) {
  if (sv->rec_free.empty()) {
    constexpr int kChunk = 256;
    void* p = nullptr;
    if (hipHostMalloc(&p, kChunk * sizeof(HostRecord), hipHostMallocDefault) != hipSuccess)
      return GW_EDEVICE;
    sv->rec_chunks.push_back(p);
    HostRecord* r = static_cast<HostRecord*>(p);
    for (int i = kChunk - 1; i >= 0; --i) sv->rec_free.push_back(r + i);
  }
  *out = sv->rec_free.back();
  sv->rec_free.pop_back();
  (*out)->obj[0] = (*out)->obj[1] = NAN;
  (*out)->nonfinite = 0;
  return GW_OK;
}

// Last work of a request: objective, host copies of obj and status, and the
// completion event.  The slot is returned; the arena range stays.
gw_status complete(gw_server* sv, Req& q) {
  hipStream_t s = sv->s;
  gw_status st;
  if (q.r.flags & GW_REQ_OBJECTIVE) {
    Arena a{q.tail, 0, q.tail_bytes};
    if ((st = gwr::run_objective(q.X, q.Y, q.T, q.N, q.r.eps, q.obj, q.G, a, s, q.st, nullptr)) != GW_OK)
      return st;
    if ((st = hip_ok(hipMemcpyAsync(q.rec->obj, q.obj, 2 * sizeof(double),
                                    hipMemcpyDeviceToHost, s))) != GW_OK)
      return st;
  }
  if ((st = hip_ok(hipMemcpyAsync(&q.rec->nonfinite, &q.st->nonfinite, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s))) != GW_OK)
    return st;
  if ((st = hip_ok(hipEventRecord(q.done, s))) != GW_OK) return st;
  q.phase = kDone;
  sv->free_slots.push_back(q.slot);
  q.slot = -1;
  return GW_OK;
}

gw_status finish_outer(gw_server* sv, Req& q) {
  gw_status st = gwl::sinkhorn_finish(q.G, q.N, q.M, q.N, 2.0, q.r.p, q.logp, q.ms, q.r.eps,
                                      q.r.inner, q.f, q.g, q.T, q.N, sv->s, q.st);
  if (st != GW_OK) return st;
  q.outer_done += 1;
  if (q.outer_done == q.r.outer) return complete(sv, q);
  q.phase = kGrad;
  return GW_OK;
}

// Gradient and Sinkhorn set-up of the next outer iteration(s); with
// inner = 0 the outer iterations need no batched work and all run here.
gw_status start_outer(gw_server* sv, Req& q) {
  while (q.phase == kGrad) {
    Arena a{q.tail, 0, q.tail_bytes};
    gw_status st = gwr::run_grad(q.X, q.Y, q.r.p, q.r.q, q.T, q.N, q.G, q.N, GW_PATH_FAST_F64, a,
                                 sv->s, q.c1, q.c2);
    if (st != GW_OK) return st;
    const int cold = (q.r.flags & GW_FLAG_WARM_START) && q.outer_done > 0 ? 0 : 1;
    st = gwl::sinkhorn_prep(q.r.p, q.r.q, q.M, q.N, cold, q.logp, q.logq, q.kq, q.f, q.g,
                            sv->s);
    if (st != GW_OK) return st;
    q.phase = kSink;
    q.inner_left = q.r.inner;
    if (q.r.inner == 0 && (st = finish_outer(sv, q)) != GW_OK) return st;
  }
  return GW_OK;
}

gw_status admit(gw_server* sv, Req& q) {
  hipStream_t s = sv->s;
  carve(q, sv->arena + sv->L.total + q.off);
  gw_status st;
  if ((st = hip_ok(hipEventCreate(&q.done))) != GW_OK) return st;
  if ((st = take_record(sv, &q.rec)) != GW_OK) return st;
  if ((st = gwr::clear_status(q.st, s)) != GW_OK) return st;
  if ((st = gwl::const_terms(q.X, q.r.p, q.c1, q.Y, q.r.q, q.c2, s)) != GW_OK) return st;
  if ((st = gwl::outer_product(q.r.p, q.r.q, q.M, q.N, q.T, q.N, s)) != GW_OK) return st;
  if (q.r.outer == 0) return complete(sv, q);
  q.phase = kGrad;
  return GW_OK;
}

// Row classes launched in iteration range l of a step (see kLevels), packed
// 11 bits per range: the ranges are nested (a request that takes iterations
// of range l takes every earlier one), so the first empty range ends the step.
uint32_t level_mask(uint64_t key, int l) {
  return (uint32_t)(key >> (l * gwb::kNumRowCls)) & ((1u << gwb::kNumRowCls) - 1u);
}

int level_start(int S, int l) { return l == 0 ? 0 : S << (l - 1); }

// Destroy the least recently used graph if it last ran two or more steps ago
// (the step's wait on its staging event has then seen that replay finish).
void evict_graph(gw_server* sv) {
  auto victim = sv->graphs.end();
  for (auto it = sv->graphs.begin(); it != sv->graphs.end(); ++it)
    if (it->second.last_step <= sv->steps - 2 &&
        (victim == sv->graphs.end() || it->second.last_step < victim->second.last_step))
      victim = it;
  if (victim == sv->graphs.end()) return;
  (void)hipGraphExecDestroy(victim->second.exec);
  sv->graphs.erase(victim);
}

gw_status graph_for(gw_server* sv, uint64_t key, hipGraphExec_t* out) {
  auto it = sv->graphs.find(key);
  if (it != sv->graphs.end()) {
    it->second.last_step = sv->steps;
    *out = it->second.exec;
    return GW_OK;
  }
  if (sv->graphs.size() >= kMaxGraphs) evict_graph(sv);
  const gwb::SkTableHead* head = reinterpret_cast<const gwb::SkTableHead*>(sv->arena + sv->L.head);
  const gwb::SkSlot* slots = reinterpret_cast<const gwb::SkSlot*>(sv->arena + sv->L.slots);
  const uint32_t* items = reinterpret_cast<const uint32_t*>(sv->arena + sv->L.items);
  if (hipStreamBeginCapture(sv->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return GW_EDEVICE;
  gw_status st = GW_OK;
  for (int l = 0; l < kLevels && st == GW_OK; ++l) {
    const uint32_t mask = level_mask(key, l);
    if (!mask) break;
    for (int j = level_start(sv->S, l); j < level_start(sv->S, l + 1) && st == GW_OK; ++j) {
      for (int c = 0; c < gwb::kNumRowCls && st == GW_OK; ++c)
        if (mask & (1u << c)) st = gwl::sk_batch_launch(c, j, slots, head, items, sv->cap);
      if (st == GW_OK) st = gwl::sk_batch_launch(gwb::kClsCol, j, slots, head, items, sv->cap);
    }
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(sv->cap, &g);
  if (st != GW_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return st != GW_OK ? st : GW_EDEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return GW_EDEVICE;
  sv->graphs[key] = {exec, sv->steps};
  *out = exec;
  return GW_OK;
}

// Iterations a request in its Sinkhorn phase takes in a step: S, or with size
// quotas b S for the largest power of two b <= boost with b M N at most the
// largest M N in the Sinkhorn phase (never more than the call has left).
int step_quota(const gw_server* sv, const Req& q, int64_t wmax) {
  int b = 1;
  while (b < sv->boost && 2 * b * (q.M * q.N) <= wmax) b *= 2;
  const int quota = b * sv->S;
  return q.inner_left < quota ? q.inner_left : quota;
}

// Write the work table for the requests in their Sinkhorn phase into the
// staging buffer; returns the graph key (the class masks of the iteration
// ranges, 0: nothing to run) and the bytes to upload.
uint64_t build_table(gw_server* sv, char* stage, size_t* upload) {
  for (auto& l : sv->lists) l.clear();
  auto* slots = reinterpret_cast<gwb::SkSlot*>(stage + sv->L.slots);
  int64_t wmax = 0;
  for (int64_t id : sv->running) {
    const Req& q = sv->reqs[id];
    if (q.phase == kSink && q.M * q.N > wmax) wmax = q.M * q.N;
  }
  uint64_t key = 0;
  for (int64_t id : sv->running) {
    Req& q = sv->reqs[id];
    if (q.phase != kSink) continue;
    q.its = step_quota(sv, q, wmax);
    gwb::SkSlot& d = slots[q.slot];
    d.C = q.G;
    d.ldC = q.N;
    d.p = q.r.p;
    d.logp = q.logp;
    d.q = q.r.q;
    d.logq = q.logq;
    d.f = q.f;
    d.g = q.g;
    d.ms = q.ms;
    d.pS = q.pS;
    d.pX = q.pX;
    d.status = q.st;
    d.lse = q.lse;
    d.gprev = q.gprev;
    d.kq = q.kq;
    d.bmode = q.bmode;
    d.cs = 2.0;
    d.inv_eps = 1.0 / q.r.eps;
    d.eps = q.r.eps;
    d.M = (int32_t)q.M;
    d.N = (int32_t)q.N;
    d.RB = q.rb;
    d.nb = q.nb;
    d.its = q.its;
    d.last = q.inner_left == q.its ? 1 : 0;
    d.it0 = q.r.inner - q.inner_left;
    d.pad = 0;
    const int cls = gwb::row_class(q.N);
    for (int l = 0; l < kLevels; ++l)
      if (q.its > level_start(sv->S, l)) key |= (uint64_t)(1u << cls) << (l * gwb::kNumRowCls);
    for (int b = 0; b < q.nb; ++b)
      sv->lists[cls].push_back(((uint32_t)q.slot << gwb::kBandBits) | (uint32_t)b);
    const int ncb = (int)((q.N + gwb::kMergeCols - 1) / gwb::kMergeCols);
    for (int b = 0; b < ncb; ++b)
      sv->lists[gwb::kClsCol].push_back(((uint32_t)q.slot << gwb::kCBlockBits) | (uint32_t)b);
  }
  auto* head = reinterpret_cast<gwb::SkTableHead*>(stage + sv->L.head);
  auto* items = reinterpret_cast<uint32_t*>(stage + sv->L.items);
  size_t n = 0;
  for (int c = 0; c < gwb::kNumLists; ++c) {
    head->count[c] = (int32_t)sv->lists[c].size();
    head->offset[c] = (int32_t)n;
    for (uint32_t v : sv->lists[c]) items[n++] = v;
  }
  *upload = sv->L.items + n * sizeof(uint32_t);
  return key;
}

gw_status step(gw_server* sv, int32_t* active, int32_t* queued) {
  const int b = (int)(sv->steps & 1);
  gw_status st;
  if (sv->stage_used[b] && (st = hip_ok(hipEventSynchronize(sv->stage_ev[b]))) != GW_OK)
    return st;
  // 1. admission, first come first served
  while (!sv->queue.empty() && !sv->free_slots.empty()) {
    Req& q = sv->reqs[sv->queue.front()];
    const size_t off = sv->alloc.alloc(q.bytes);
    if (off == RangeAllocator::kFail) break;
    sv->queue.pop_front();
    q.off = off;
    q.slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    sv->running.push_back(q.id);
    if ((st = admit(sv, q)) != GW_OK) return st;
  }
  // 2. gradients of requests at the start of an outer iteration
  for (int64_t id : sv->running) {
    Req& q = sv->reqs[id];
    if (q.phase == kGrad && (st = start_outer(sv, q)) != GW_OK) return st;
  }
  // 3. the batched Sinkhorn iterations
  size_t upload = 0;
  const uint64_t key = build_table(sv, sv->h_stage[b], &upload);
  if (key) {
    hipGraphExec_t exec = nullptr;
    if ((st = graph_for(sv, key, &exec)) != GW_OK) return st;
    if ((st = hip_ok(hipMemcpyAsync(sv->arena, sv->h_stage[b], upload, hipMemcpyHostToDevice,
                                    sv->s))) != GW_OK)
      return st;
    gwr::ProfScope ps(gwr::kFamServeStep, sv->s);
    if ((st = hip_ok(hipGraphLaunch(exec, sv->s))) != GW_OK) return st;
  }
  if ((st = hip_ok(hipEventRecord(sv->stage_ev[b], sv->s))) != GW_OK) return st;
  sv->stage_used[b] = true;
  // 4. requests whose Sinkhorn call ended this step
  for (int64_t id : sv->running) {
    Req& q = sv->reqs[id];
    if (q.phase != kSink) continue;
    q.inner_left -= q.its;
    if (q.inner_left == 0 && (st = finish_outer(sv, q)) != GW_OK) return st;
  }
  std::vector<int64_t> still;
  still.reserve(sv->running.size());
  for (int64_t id : sv->running)
    if (sv->reqs[id].phase != kDone) still.push_back(id);
  sv->running.swap(still);
  sv->steps += 1;
  if (active) *active = (int32_t)sv->running.size();
  if (queued) *queued = (int32_t)sv->queue.size();
  return GW_OK;
}

void destroy_request(gw_server* sv, Req& q) {
  if (q.done) (void)hipEventDestroy(q.done);
  if (q.rec) sv->rec_free.push_back(q.rec);
  if (q.off != RangeAllocator::kFail) sv->alloc.release(q.off);
}

}  // namespace

extern "C" {

size_t gw_server_request_bytes(const gw_request* r) {
  Req q;
  return describe(r, &q) == GW_OK ? q.bytes : 0;
}

size_t gw_server_table_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > kMaxSlots) return 0;
  return table_layout(max_slots).total;
}

gw_status gw_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                           int32_t iters_per_step, void* stream, gw_server** out) {
  if (!out) return GW_EINVAL;
  *out = nullptr;
  if (!arena || ((uintptr_t)arena & 255u)) return GW_EINVAL;
  if (max_slots < 1 || max_slots > kMaxSlots) return GW_EINVAL;
  if (iters_per_step < 1 || iters_per_step > kMaxItersPerStep) return GW_EINVAL;
  const TableLayout L = table_layout(max_slots);
  if (arena_bytes < L.total + RangeAllocator::kAlign) return GW_ENOMEM;
  gw_server* sv = new (std::nothrow) gw_server();
  if (!sv) return GW_ENOMEM;
  sv->s = reinterpret_cast<hipStream_t>(stream);
  sv->arena = static_cast<char*>(arena);
  sv->L = L;
  sv->alloc.reset(arena_bytes - L.total);
  sv->max_slots = max_slots;
  sv->S = iters_per_step;
  for (int i = max_slots - 1; i >= 0; --i) sv->free_slots.push_back(i);
  bool ok = hipStreamCreateWithFlags(&sv->cap, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipHostMalloc(reinterpret_cast<void**>(&sv->h_stage[i]), L.total,
                       hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&sv->stage_ev[i], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreate(&sv->ev0) == hipSuccess &&
       hipEventRecord(sv->ev0, sv->s) == hipSuccess && hipEventSynchronize(sv->ev0) == hipSuccess;
  if (!ok) {
    gw_server_destroy(sv);
    return GW_EDEVICE;
  }
  sv->ready = true;
  *out = sv;
  return GW_OK;
}

gw_status gw_server_set_boost(gw_server* sv, int32_t max_boost) {
  if (!sv) return GW_EINVAL;
  if (max_boost < 1 || max_boost > kMaxBoost || (max_boost & (max_boost - 1))) return GW_EINVAL;
  if ((int64_t)sv->S * max_boost > kMaxItersPerStep) return GW_EINVAL;
  sv->boost = max_boost;
  return GW_OK;
}

gw_status gw_server_submit(gw_server* sv, const gw_request* r, int64_t* id) {
  if (!sv || !id) return GW_EINVAL;
  Req q;
  gw_status st = describe(r, &q);
  if (st != GW_OK) return st;
  if (RangeAllocator::round(q.bytes) > sv->alloc.capacity()) return GW_ENOMEM;
  q.id = sv->next_id++;
  *id = q.id;
  sv->reqs.emplace(q.id, q);
  sv->queue.push_back(q.id);
  return GW_OK;
}

gw_status gw_server_step(gw_server* sv, int32_t* active, int32_t* queued) {
  if (!sv) return GW_EINVAL;
  return step(sv, active, queued);
}

gw_status gw_server_poll(gw_server* sv, int64_t id, int32_t* state) {
  if (!sv || !state) return GW_EINVAL;
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return GW_EINVAL;
  const Req& q = it->second;
  if (q.phase == kQueued) {
    *state = GW_REQ_QUEUED;
  } else if (q.phase != kDone) {
    *state = GW_REQ_RUNNING;
  } else {
    const hipError_t e = hipEventQuery(q.done);
    if (e == hipSuccess) *state = GW_REQ_DONE;
    else if (e == hipErrorNotReady) *state = GW_REQ_RUNNING;
    else return GW_EDEVICE;
  }
  return GW_OK;
}

gw_status gw_server_result(gw_server* sv, int64_t id, gw_result* out) {
  if (!sv || !out) return GW_EINVAL;
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return GW_EINVAL;
  Req& q = it->second;
  if (q.phase != kDone) return GW_EAGAIN;
  if (hipEventSynchronize(q.done) != hipSuccess) return GW_EDEVICE;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, sv->ev0, q.done) != hipSuccess) return GW_EDEVICE;
  out->T = q.T;
  out->f = q.f;
  out->g = q.g;
  out->M = q.M;
  out->N = q.N;
  out->obj[0] = q.rec->obj[0];
  out->obj[1] = q.rec->obj[1];
  out->done_ms = (double)ms;
  out->status = q.rec->nonfinite ? GW_ENUMERIC : GW_OK;
  out->reserved = 0;
  return GW_OK;
}

gw_status gw_server_release(gw_server* sv, int64_t id) {
  if (!sv) return GW_EINVAL;
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return GW_EINVAL;
  Req& q = it->second;
  if (q.phase == kQueued) {
    for (auto qi = sv->queue.begin(); qi != sv->queue.end(); ++qi)
      if (*qi == id) {
        sv->queue.erase(qi);
        break;
      }
  } else if (q.phase != kDone) {
    return GW_EAGAIN;
  } else if (hipEventSynchronize(q.done) != hipSuccess) {
    return GW_EDEVICE;
  }
  destroy_request(sv, q);
  sv->reqs.erase(it);
  return GW_OK;
}

gw_status gw_server_destroy(gw_server* sv) {
  if (!sv) return GW_EINVAL;
  gw_status st = GW_OK;
  if (sv->ready) st = hip_ok(hipStreamSynchronize(sv->s));
  for (auto& kv : sv->reqs)
    if (kv.second.done) (void)hipEventDestroy(kv.second.done);
  for (auto& kv : sv->graphs) (void)hipGraphExecDestroy(kv.second.exec);
  for (int i = 0; i < 2; ++i) {
    if (sv->h_stage[i]) (void)hipHostFree(sv->h_stage[i]);
    if (sv->stage_ev[i]) (void)hipEventDestroy(sv->stage_ev[i]);
  }
  for (void* p : sv->rec_chunks) (void)hipHostFree(p);
  if (sv->ev0) (void)hipEventDestroy(sv->ev0);
  if (sv->cap) (void)hipStreamDestroy(sv->cap);
  delete sv;
  return st;
}

}  // extern "C"
