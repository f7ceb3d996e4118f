/*
 * gw.h - C ABI of libgw.so: entropic Gromov-Wasserstein on uniform grids for
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow arXiv 2404.08970 ("Fast Gradient Computation for
 * Gromov-Wasserstein Distance"):
 *   - grids and distance matrices: Sec. 2, Eq. (1d distance matrices);
 *     2D grids Sec. 3.1, Eq. (2d Dx);
 *   - gradient: Sec. 2, the decomposition C_1 - 4 D_X Gamma D_Y that follows
 *     Eq. (gradient entry); the fast evaluation of D_X Gamma D_Y is Sec. 3,
 *     Eq. (Dx), Eq. (1d recursive relation) and Eq. (2D kronecker);
 *   - Sinkhorn sub-problem: Sec. 2.1, Eq. (GW sinkhorn) with tau = eps (Remark);
 *   - solve: mirror descent, Sec. 2.1, Eq. (GW proximal gradient).
 *
 * Conventions shared by every call:
 *   - Matrices are row-major FP64 (unless a path says otherwise) with a leading
 *     dimension in elements.  Pointers marked "device" are device pointers that
 *     must be 8-byte aligned; the workspace must be 256-byte aligned.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream), except the tolerance-stopped calls (see there).  A return of
 *     GW_OK means the arguments were valid and the work was enqueued.  On any
 *     other return nothing was enqueued.  Work that does not depend on the
 *     stream's earlier results beyond the inputs (the constant terms of a FAST
 *     gradient) may run on a side stream forked from `stream` and joined back
 *     with events before the results are used, so ordering on `stream` and
 *     graph capture of `stream` hold as if everything ran on it.
 *   - The caller owns every buffer, including the workspace sized by
 *     gw_workspace_bytes().  The library never frees caller memory and does not
 *     allocate device memory on these calls.  Per device it creates, on first
 *     use and never while `stream` is being captured, a small pool of side
 *     streams (default priority) and events, and pinned host flags for the
 *     tolerance stop; they live until the process ends.
 *   - Marginals are expected to be non-negative, finite and to sum to 1; zero
 *     entries are allowed (their potential is -inf and their plan row/column
 *     is zero).  These preconditions are documented, not checked per call.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gw_status;
#define GW_OK 0
#define GW_EINVAL (-1)        /* invalid argument (null/misaligned pointer, bad size, bad scalar) */
#define GW_ENOMEM (-2)        /* workspace too small */
#define GW_EDEVICE (-3)       /* a HIP runtime call failed */
#define GW_ENUMERIC (-4)      /* device detected a non-finite value (gw_check_status) */
#define GW_EUNSUPPORTED (-5)  /* valid request outside what this library implements */
#define GW_EAGAIN (-6)        /* request loop: the result is not ready yet */

/* Distance on a grid (Sec. 2 and Sec. 3.1).
 *   GW_METRIC_L1POW:    h^k * (|dr| + |dc|)^k; in 1D h^k * |i - j|^k.
 *   GW_METRIC_SQEUCLID: h^2 * (dr^2 + dc^2) (requires k = 2; in 1D equal to
 *                       L1POW with k = 2). */
#define GW_METRIC_L1POW 0
#define GW_METRIC_SQEUCLID 1

#define GW_KMAX 4

/* Gradient evaluation paths.
 *   FAST_F64:   the paper's exact O(MN) recursion (Sec. 3), FP64.
 *   DENSE_F64:  the plain product D_X T D_Y on FP64 matrix cores (the O(N^3)
 *               "original" computation), distance tiles generated from indices.
 *   DENSE_F32:  as DENSE_F64 with FP32 inputs and FP32 accumulation.
 *   DENSE_BF16: BF16 inputs, FP32 accumulation.
 *   DENSE_BF16_SPLIT / DENSE_F32_SPLIT: split-precision refinement (the
 *               inputs are split into a high and a low part and the leading
 *               cross products are accumulated in FP64 over K-chunks). */
#define GW_PATH_FAST_F64 0
#define GW_PATH_DENSE_F64 1
#define GW_PATH_DENSE_F32 2
#define GW_PATH_DENSE_BF16 3
#define GW_PATH_DENSE_BF16_SPLIT 4
#define GW_PATH_DENSE_F32_SPLIT 5

#define GW_OP_GRAD 0
#define GW_OP_SINKHORN 1
#define GW_OP_SOLVE 2
#define GW_OP_OBJECTIVE 3
#define GW_OP_UOT_SINKHORN 4
#define GW_OP_SOLVE_UGW 5

/* gw_solve flags */
#define GW_FLAG_WARM_START 1  /* Sinkhorn starts from the previous outer step's potentials */

/* A uniform grid (Sec. 2; Sec. 3.1, which states that more axes work alike).
 * ndim = 1: shape = {n, 1, 1}; ndim = 2: shape = {H, W, 1}, points flattened
 * row-major (flat = r * W + c); ndim = 3: shape = {D, H, W},
 * flat = (d * H + r) * W + c, distance (|dd| + |dr| + |dc|)^k (L1POW) or
 * dd^2 + dr^2 + dc^2 (SQEUCLID), times h^k.  3D grids run on GW_PATH_FAST_F64
 * only (the dense paths are 1D).  h > 0 is the
 * spacing, k in [1, GW_KMAX] the exponent, metric one of GW_METRIC_*. */
typedef struct gw_grid {
  int32_t ndim;
  int32_t k;
  int32_t metric;
  int32_t reserved; /* must be 0 */
  int64_t shape[3];
  double h;
} gw_grid;

/* Bytes of device workspace needed by `op` (GW_OP_*) for grids X (rows, M
 * points) and Y (columns, N points) on `path` (GW_PATH_*; ignored for
 * GW_OP_SINKHORN).  Returns 0 for invalid arguments.  Host-only arithmetic. */
size_t gw_workspace_bytes(const gw_grid* X, const gw_grid* Y, int32_t path, int32_t op);

/* G = c1 1^T + 1 c2^T - 2 D_X T D_Y with c1 = (D_X o D_X) p, c2 = (D_Y o D_Y) q
 * (Sec. 2, decomposition after Eq. (gradient entry); G is half of the paper's
 * gradient).  X has M points, Y has N points.
 *   p [M], q [N], T [M x N, ldT >= N], G [M x N, ldG >= N]: device FP64.
 *   G must not overlap T.  ws: device workspace of ws_bytes bytes. */
gw_status gw_grad(const gw_grid* X, const gw_grid* Y, const double* p, const double* q,
                  const double* T, int64_t ldT, double* G, int64_t ldG, int32_t path, void* ws,
                  size_t ws_bytes, void* stream);

/* Log-domain Sinkhorn for min <C_eff, P> + eps H(P) over couplings of (p, q),
 * C_eff = c_scale * C (Sec. 2.1, Eq. (GW sinkhorn) is this problem with
 * C_eff = the gradient).  One iteration sets
 *   f_i = eps ln p_i - eps LSE_p((g_p - C_eff_ip)/eps), then
 *   g_p = eps ln q_p - eps LSE_i((f_i - C_eff_ip)/eps).
 * If init_zero != 0 the potentials start at 0, else at the values in f, g.
 *   C [M x N, ldC >= N], p [M], q [N]: device FP64 inputs.
 *   f [M], g [N]: device FP64 in/out.
 *   T: optional (may be NULL) device FP64 [M x N, ldT >= N]; receives the plan
 *      P_ip = exp((f_i + g_p - C_eff_ip)/eps) after the last iteration.
 * eps > 0; M, N <= 65535.  Rows of up to 16384 entries are held on chip (one
 * pass over C per iteration); longer rows run in slabs of 8192 columns with
 * two passes per iteration. */
gw_status gw_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                      const double* p, const double* q, double eps, int32_t iters,
                      int32_t init_zero, double* f, double* g, double* T, int64_t ldT, void* ws,
                      size_t ws_bytes, void* stream);

/* gw_sinkhorn without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and validation as
 * gw_sinkhorn; its scratch (band partials, log-marginals, row bounds, status
 * word) is a static device array of GW_NOALLOC_SCRATCH_BYTES per GPU, held
 * from the first call on that GPU until the process ends.  Sizes whose
 * gw_sinkhorn workspace (gw_workspace_bytes with GW_OP_SINKHORN) exceeds it
 * return GW_ENOMEM before anything is enqueued (about M, N <= 10000 at
 * M = N).  Calls no allocating routine.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.  The status word in the array is cleared
 * at the start of each call and is not reported by gw_check_status; a
 * non-finite result shows in f and g. */
#define GW_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
gw_status gw_sinkhorn_noalloc(const double* C, int64_t ldC, int64_t M, int64_t N,
                              double c_scale, const double* p, const double* q, double eps,
                              int32_t iters, int32_t init_zero, double* f, double* g, double* T,
                              int64_t ldT, void* stream);

/* Entropic GW by mirror descent with tau = eps (Sec. 2.1): T^0 = p q^T, then
 * `outer` times { G = gw_grad(T); Sinkhorn on the cost 2G with `inner`
 * iterations; T = its plan }.  Afterwards obj[0] = E(T) (the QAP objective of
 * Sec. 2 with T's own marginals) and obj[1] = E(T) + eps H(T).
 *   p [M], q [N]: device FP64.  T [M x N, ldT >= N], f [M], g [N]: device FP64
 *   outputs.  obj: device double[2] (may be NULL to skip the objective).
 *   flags: GW_FLAG_*. */
gw_status gw_solve(const gw_grid* X, const gw_grid* Y, const double* p, const double* q,
                   double eps, int32_t outer, int32_t inner, int32_t path, int32_t flags,
                   double* T, int64_t ldT, double* f, double* g, double* obj, void* ws,
                   size_t ws_bytes, void* stream);

/* obj[0] = E(T), obj[1] = E(T) + eps H(T) for an arbitrary non-negative T
 * (Sec. 2, discrete objective and Eq. (entropic GW)).  T [M x N]: device FP64;
 * obj: device double[2]. */
gw_status gw_objective(const gw_grid* X, const gw_grid* Y, const double* T, int64_t ldT,
                       double eps, double* obj, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Tolerance-stopped Sinkhorn.  The paper runs fixed iteration counts and
 * states no stopping rule (Sec. 2.1 and the experiments of Sec. 5); this is
 * an optional one.  Iteration t (1-based) is gw_sinkhorn's update.  When t is
 * a multiple of check_every, the column merge of iteration t also measures
 *   err_t = sum_p | sum_i exp((f_i + g_p - C_eff_ip)/eps) - q_p |
 * with f after and g before the update of iteration t (the plan whose row
 * sums are p), the g update is applied, and if err_t <= tol the call stops
 * there: f, g (and T) are those after iteration t.  The decision is taken on
 * the device: later launches of the call see a flag and return at once.  The
 * host follows it one check behind: after enqueueing check c it waits for
 * check c - 1 to finish on the device (a 4-byte copy of the flag to pinned
 * host memory) and enqueues nothing more once a check has stopped the call,
 * so these calls return only when the device has reached the stopping check
 * (or the last one), and a stopped call enqueues at most two check periods
 * past its stop.  On a stream being captured into a graph the host does not
 * wait: all max_iters launches are enqueued (stopped ones return at once).
 * Results are the same either way.  The pinned flags and events are pooled
 * per device (host memory, allocated on first use).
 * check_every >= 1; tol must not be NaN (tol < 0 never stops).
 * ------------------------------------------------------------------------ */

/* gw_sinkhorn with a tolerance stop.  iters_done: device int32 (may be NULL),
 * receives the iterations done (max_iters if no check met tol).  err: device
 * double (may be NULL), receives the last measured err_t (NaN if none). */
gw_status gw_sinkhorn_tol(const double* C, int64_t ldC, int64_t M, int64_t N, double c_scale,
                          const double* p, const double* q, double eps, int32_t max_iters,
                          int32_t check_every, double tol, int32_t init_zero, double* f,
                          double* g, double* T, int64_t ldT, int32_t* iters_done, double* err,
                          void* ws, size_t ws_bytes, void* stream);

/* gw_solve whose Sinkhorn calls stop by tolerance (at most max_inner
 * iterations each).  inner_done: device int32 [outer] (may be NULL), the
 * iterations done by each outer step's Sinkhorn call. */
gw_status gw_solve_tol(const gw_grid* X, const gw_grid* Y, const double* p, const double* q,
                       double eps, int32_t outer, int32_t max_inner, int32_t check_every,
                       double tol, int32_t path, int32_t flags, double* T, int64_t ldT, double* f,
                       double* g, double* obj, int32_t* inner_done, void* ws, size_t ws_bytes,
                       void* stream);

/* ------------------------------------------------------------------------
 * Unbalanced GW (Remark on UGW, Sec. 3): for positive measures u [M], v [N]
 * (device FP64, not necessarily of mass 1) and rho > 0 the divergence
 *   E(T) + rho KL(T1 (x) T1 | u (x) u) + rho KL(T^T 1 (x) T^T 1 | v (x) v),
 * KL(a|b) = sum a log(a/b) - m(a) + m(b), minimised with the entropic term
 * eps KL(T (x) T | (u (x) v) (x) (u (x) v)).  The Remark gives the step
 *   T = argmin <G(Th) + g(Th), T> + m(Th) (rho KL(T1|u) + rho KL(T^T 1|v)
 *                                          + eps KL(T|u (x) v)),
 * G(Th) the half gradient at Th's own marginals; the scalar g(Th), the solver
 * of the step and the mass rescaling are those of the UGW work it cites:
 *   g(Th) = rho <log(a/u), a> + rho <log(b/v), b> + eps <log(Th/(u (x) v)), Th>,
 *   unbalanced Sinkhorn with tau = rho / (rho + eps) and e = m(Th) eps,
 *   T <- sqrt(m(Th) / m(T)) T after each step, T^0 = u (x) v / sqrt(m(u) m(v)).
 * Workspace: gw_workspace_bytes with GW_OP_UOT_SINKHORN / GW_OP_SOLVE_UGW.
 * u and v must have positive mass; a non-finite potential or rescale factor
 * (e.g. from an empty measure) sets the workspace status (gw_check_status ->
 * GW_ENUMERIC).  gw_solve_ugw clears the status first; gw_uot_sinkhorn, like
 * gw_sinkhorn, leaves an earlier flag in place.
 * ------------------------------------------------------------------------ */

/* Unbalanced entropic OT on C_eff = C + c_shift:
 *   min <C_eff, T> + rho KL(T1|u) + rho KL(T^T 1|v) + eps KL(T|u (x) v).
 * One iteration: f_i = -tau eps LSE_p((g_p - C_eff_ip)/eps + ln v_p), then
 * g_p = -tau eps LSE_i((f_i - C_eff_ip)/eps + ln u_i), tau = rho/(rho+eps).
 * init_zero: start from f = g = 0 (else from the given f, g).  T (may be
 * NULL) receives exp((f_i + g_p - C_eff_ip)/eps) u_i v_p.  N <= 16384. */
gw_status gw_uot_sinkhorn(const double* C, int64_t ldC, int64_t M, int64_t N, double c_shift,
                          const double* u, const double* v, double rho, double eps,
                          int32_t iters, int32_t init_zero, double* f, double* g, double* T,
                          int64_t ldT, void* ws, size_t ws_bytes, void* stream);

/* Entropic UGW: `outer` steps, each `inner` unbalanced Sinkhorn iterations
 * from zero potentials.  T [M x N]: the plan; f, g: the last step's
 * potentials (0 if outer = 0); obj (may be NULL): obj[0] = the divergence at
 * T, obj[1] = obj[0] + its entropic term.  The gradient runs on `path`. */
gw_status gw_solve_ugw(const gw_grid* X, const gw_grid* Y, const double* u, const double* v,
                       double rho, double eps, int32_t outer, int32_t inner, int32_t path,
                       double* T, int64_t ldT, double* f, double* g, double* obj, void* ws,
                       size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Fused GW (Remark on FGW, Sec. 3): the objective
 *   E_fgw(T) = (1 - theta) sum_ip c_ip^2 T_ip + theta E(T),  theta in [0, 1],
 * with the feature cost c_ip = fa_i - fb_p between scalar features fa [M] of
 * X's points and fb [N] of Y's points (device FP64).  Its gradient is
 * (1 - theta) C o C + theta grad E, so only the GW part goes through the
 * gradient paths; the feature term is one extra elementwise pass over G.
 * Workspace: what gw_workspace_bytes reports for the matching GW operation
 * (GW_OP_GRAD, GW_OP_SOLVE, GW_OP_OBJECTIVE).  theta outside [0, 1] or not
 * finite, or a NULL / misaligned fa or fb, is GW_EINVAL.  At theta = 1 the
 * results are bitwise those of the GW entry points (the feature pass is
 * skipped).
 * ------------------------------------------------------------------------ */

/* G = (1 - theta)/2 c o c + theta (c1 1^T + 1 c2^T - 2 D_X T D_Y), half the
 * FGW gradient, arguments as gw_grad. */
gw_status gw_grad_fgw(const gw_grid* X, const gw_grid* Y, const double* p, const double* q,
                      const double* fa, const double* fb, double theta, const double* T,
                      int64_t ldT, double* G, int64_t ldG, int32_t path, void* ws,
                      size_t ws_bytes, void* stream);

/* Entropic FGW by mirror descent (Sec. 2.1 with the FGW gradient): as gw_solve
 * with the Sinkhorn cost 2 G from gw_grad_fgw.  obj[0] = E_fgw(T) (T's own
 * marginals in E), obj[1] = obj[0] + eps H(T). */
gw_status gw_solve_fgw(const gw_grid* X, const gw_grid* Y, const double* p, const double* q,
                       const double* fa, const double* fb, double theta, double eps,
                       int32_t outer, int32_t inner, int32_t path, int32_t flags, double* T,
                       int64_t ldT, double* f, double* g, double* obj, void* ws,
                       size_t ws_bytes, void* stream);

/* obj[0] = E_fgw(T), obj[1] = E_fgw(T) + eps H(T) for a non-negative T. */
gw_status gw_objective_fgw(const gw_grid* X, const gw_grid* Y, const double* T, int64_t ldT,
                           const double* fa, const double* fb, double theta, double eps,
                           double* obj, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Request loop: continuous batching of gw_solve problems of uneven sizes.
 *
 * Not an operation of the paper; a serving layer that runs the mirror-descent
 * solve of Sec. 2.1 (exactly the arithmetic of gw_solve on GW_PATH_FAST_F64)
 * for many requests at once.  Each request keeps its plan T, potentials f, g,
 * gradient and Sinkhorn state resident in the server's arena from admission
 * until it is released.  One host thread drives a server (not thread-safe).
 *
 * A step (gw_server_step) does, on the server's stream:
 *   1. admission: queued requests, in submission order, while a slot is free
 *      and the arena has a free range of the request's footprint
 *      (gw_server_request_bytes); the first that does not fit stops admission;
 *   2. for each request at the start of an outer iteration: its gradient and
 *      Sinkhorn set-up (per-request launches);
 *   3. one replay of a captured HIP graph that runs `iters_per_step` Sinkhorn
 *      iterations of every request in its Sinkhorn phase (a multiple of it for
 *      small requests under size quotas, gw_server_set_boost): persistent batched
 *      kernels read a device work table (per request: sizes, pointers and
 *      how many of the step's iterations it takes) that the host rewrites
 *      between replays, so request shapes are data, not launch shapes;
 *   4. for each request whose Sinkhorn call ended: its potentials and plan;
 *      after the last outer iteration the objective (if asked) and a
 *      completion event.
 * The host never runs more than two steps ahead of the device.  A request's
 * results do not depend on the other requests in the batch: each band of
 * each iteration runs the single-problem kernel's arithmetic, and no
 * reduction crosses requests.
 * ------------------------------------------------------------------------ */
typedef struct gw_server gw_server; /* opaque */

#define GW_REQ_OBJECTIVE 2 /* request flag: compute obj after the last outer iteration */

/* Request states reported by gw_server_poll. */
#define GW_REQ_QUEUED 0  /* submitted, not admitted */
#define GW_REQ_RUNNING 1 /* admitted; device work not finished */
#define GW_REQ_DONE 2    /* device work finished; gw_server_result is ready */

/* One solve: the arguments of gw_solve on GW_PATH_FAST_F64.
 *   p [M], q [N]: device FP64, owned by the caller, read until the request is
 *   released.  flags: GW_FLAG_WARM_START | GW_REQ_OBJECTIVE.  Requires
 *   N <= 16384, eps > 0, outer >= 0, inner >= 0; reserved must be 0. */
typedef struct gw_request {
  gw_grid X;
  gw_grid Y;
  const double* p;
  const double* q;
  double eps;
  int32_t outer;
  int32_t inner;
  int32_t flags;
  int32_t reserved;
} gw_request;

/* Result of a finished request.  T [M x N] (leading dimension N), f [M], g [N]
 * are device pointers into the server's arena, valid until the request is
 * released.  f and g are the last Sinkhorn call's potentials (unset if
 * outer = 0).  obj: host copy of gw_solve's obj (NaN without
 * GW_REQ_OBJECTIVE).  done_ms: device time of completion in ms after
 * gw_server_create returned (HIP event clock).  status: GW_OK, or
 * GW_ENUMERIC if a kernel of this request saw a non-finite value. */
typedef struct gw_result {
  const double* T;
  const double* f;
  const double* g;
  int64_t M;
  int64_t N;
  double obj[2];
  double done_ms;
  gw_status status;
  int32_t reserved;
} gw_result;

/* Arena bytes one request holds while admitted (T, gradient, potentials,
 * Sinkhorn partials, gradient scratch); 0 for an invalid request. Host-only. */
size_t gw_server_request_bytes(const gw_request* r);

/* Arena bytes the server keeps for its device work table. Host-only. */
size_t gw_server_table_bytes(int32_t max_slots);

/* Create a server over `arena` (device memory of arena_bytes bytes, 256-byte
 * aligned, owned by the caller and not touched by it until
 * gw_server_destroy).  max_slots (1..4096) bounds the requests admitted at
 * once; iters_per_step (1..1000) is the Sinkhorn iterations per step.  The
 * server allocates pinned host staging buffers, HIP events and graphs, never
 * device memory.  stream: the hipStream_t all work goes to. */
gw_status gw_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                           int32_t iters_per_step, void* stream, gw_server** out);

/* Size-aware iteration quotas (a scheduling policy of the request loop, not
 * an operation of the paper).  With max_boost b > 1 (1, 2, 4 or 8), a request
 * in its Sinkhorn phase whose problem has at most M N / 2^m entries, where
 * M N is the largest among the requests in their Sinkhorn phase in that
 * step, takes 2^m iters_per_step iterations in the step (2^m <= b); the
 * largest take iters_per_step.  Small requests finish in fewer steps while
 * the step time grows only by their extra (small) work.  Results do not
 * change: every request still runs its iterations in order with the same
 * arithmetic.  Default 1 (every request takes iters_per_step).  GW_EINVAL if
 * b is not one of 1, 2, 4, 8 or iters_per_step * b > 1000.  Host-only; may be
 * called between steps. */
gw_status gw_server_set_boost(gw_server* sv, int32_t max_boost);

/* Queue a request; *id receives its handle.  GW_ENOMEM if its footprint can
 * never fit the arena.  Nothing is launched. */
gw_status gw_server_submit(gw_server* sv, const gw_request* r, int64_t* id);

/* One step (see above).  *active: requests admitted and not finished after
 * the step; *queued: requests waiting for admission (either may be NULL). */
gw_status gw_server_step(gw_server* sv, int32_t* active, int32_t* queued);

/* *state = GW_REQ_*; GW_EINVAL for an unknown or released id. */
gw_status gw_server_poll(gw_server* sv, int64_t id, int32_t* state);

/* Fill *out for a finished request (waits for its completion event if its
 * work is all enqueued); GW_EAGAIN if the request is queued or still has
 * steps to go. */
gw_status gw_server_result(gw_server* sv, int64_t id, gw_result* out);

/* Give back a finished or queued request's arena range and handle.
 * GW_EAGAIN if it is admitted and not finished. */
gw_status gw_server_release(gw_server* sv, int64_t id);

/* Wait for the stream and free the server's host resources (the arena stays
 * the caller's). */
gw_status gw_server_destroy(gw_server* sv);

/* Human-readable name of a status code (static storage). */
const char* gw_status_string(gw_status s);

/* Waits for `stream`, then reports GW_EDEVICE if a HIP error is pending and
 * GW_ENUMERIC if a kernel that used workspace `ws` (may be NULL) flagged a
 * non-finite value since the workspace was last cleared; the flag is cleared. */
gw_status gw_check_status(void* ws, void* stream);

/* Kernel timing with HIP events on the launching stream.  Families:
 *   0 fast-gradient main tile kernel, 1 fast-gradient carry/moment kernels,
 *   2 dense gradient GEMMs, 3 Sinkhorn row pass, 4 Sinkhorn column merge,
 *   5 plan materialisation, 6 other (init, objective, constant terms),
 *   7 2D gradient kernels, 8 request-loop step graphs (batched Sinkhorn).
 * gw_profile_enable(mask) records the families whose bit (1 << family) is set
 * in `mask` (0 stops recording; every call clears the counts); gw_profile_read
 * waits for the recorded events and returns total milliseconds and launch
 * count of a family (the launches timed).  Timing adds an event pair around
 * each timed launch; gw_profile_sample(every) times only the first of every
 * `every` launches of each family (default 1: all), which keeps that cost off
 * the untimed ones.  every < 1 returns GW_EINVAL. */
void gw_profile_enable(int32_t mask);
gw_status gw_profile_read(int32_t family, double* total_ms, int64_t* launches);
gw_status gw_profile_sample(int32_t every);

/* Library version string. */
const char* gw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GW_H */
