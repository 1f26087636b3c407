/*
 * qqa.h -- C ABI of libqqa, an MI355X (gfx950) solver for Parallel Quasi-Quantum
 * Annealing (PQQA, arXiv 2409.02135).
 *
 * The solver runs S coupled replicas of relaxed binary variables P in [0,1]^{N x S}
 * through K updates of
 *     g  = grad l^(P) + gamma_t grad s(P) + grad(-S alpha_c sum_i STD_s P_i)
 *     P <- Clamp(step(P, g) + sqrt(2 eta T) xi)
 * and finally rounds x = [P > 1/2] and evaluates each replica exactly in integers:
 *   * relaxed objectives l^: the MIS and max-cut energies of the appendix section
 *     "Energy Function of Benchmark Problems";
 *   * alpha-entropy s(p) = sum_i 1 - (2 p_i - 1)^alpha: Eq. 7, annealed with gamma_t
 *     rising linearly from gamma_min to gamma_max (Sec. 5 "Implementation", appendix
 *     "Annealing Schedule");
 *   * replica communication: the STD term of Eq. 10;
 *   * update: the sensitive-transition step on p of Eq. 11 with AdamW in place of
 *     the plain step (Sec. 3.4), or the plain step itself; Clamp to [0,1] (Sec. 5 "Implementation");
 *   * rounding x_i = Theta(p_i - 1/2) (Sec. 5 "Implementation"), with Theta(0) = 0.
 *
 * Conventions for every function:
 *   * Return value: QQA_OK (0), QQA_PENDING (1) or a negative QQA_E_* code.  Nothing
 *     aborts or throws across this ABI; qqa_last_error() describes the last failure
 *     of a context (the qqa_dev_* functions report through qqa_dev_last_error()).
 *   * Layout of replica state: row-major N x stride float32, replica index contiguous,
 *     stride = qqa_replica_stride(S) = S rounded up to a multiple of 4.  Columns
 *     S..stride-1 are padding: written as 0, never read as replicas.
 *   * "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory
 *     (for example from torch.empty(..., device="cuda")).
 *   * `stream` arguments are hipStream_t passed as void*; NULL is the null stream.
 *     qqa_dev_* calls are asynchronous on that stream.
 */
#ifndef QQA_H
#define QQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QQA_OK 0
#define QQA_PENDING 1
#define QQA_E_ARG (-1)         /* bad argument: NULL, S <= 0, steps <= 0, odd alpha, gamma_min > gamma_max, ... */
#define QQA_E_GRAPH (-2)       /* invalid graph: asymmetric, self-loop, duplicate, index out of range, weight off grid */
#define QQA_E_NOMEM (-3)       /* device memory exhausted */
#define QQA_E_ADMISSION (-4)   /* request footprint exceeds the context's HBM budget even when idle */
#define QQA_E_DEVICE (-5)      /* HIP runtime error */
#define QQA_E_UNKNOWN_REQ (-6) /* unknown or already collected request handle */
#define QQA_E_CANCELLED (-7)   /* request was cancelled */

/* Problems (appendix "Energy Function of Benchmark Problems"), relaxed objective l^(p) of
 * one replica, lambda = penalty_lambda:
 *   QQA_MIS        -sum_i p_i + lambda p^T A p / 2
 *   QQA_MAXCUT     -sum_{i<j} A_ij (1 - (2p_i - 1)(2p_j - 1)) / 2
 *   QQA_MAXCLIQUE  -sum_i p_i + lambda/2 (1^T p (1^T p - 1) - p^T A p); its gradient
 *                  needs the per-replica sum 1^T p over all variables in every update.
 *                  Max clique runs on the streaming and sliced engines of plain solves
 *                  only (not in batches or the server).
 *   QQA_COLORING   categorical K-state variant (appendix "Generalization to discrete
 *                  optimization problems"): per replica V in [0,1]^(N x K), sigma_ik =
 *                  V_ik / sum_k' V_ik' (uniform for an all-zero row), objective
 *                  sum_{(i,j) in E} sum_k sigma_ik sigma_jk (expected conflicts), the
 *                  categorical alpha-entropy s_K, the replica STD per (variable, colour).
 *                  Solved with qqa_solve_coloring (it needs K); streaming engine only. */
typedef enum { QQA_MIS = 0, QQA_MAXCUT = 1, QQA_MAXCLIQUE = 2, QQA_COLORING = 3 } qqa_problem;
typedef enum { QQA_STEP_ADAMW = 0, QQA_STEP_LANGEVIN = 1 } qqa_step_rule;

/* Hyper-parameters of one solve.  qqa_schedule_default() fills the paper's values:
 * gamma -2 -> 0.1 (max-cut: gamma_min -20 for N >= 1000, else -5; appendix "Annealing
 * Schedule"), alpha = 4 (Sec. 5 "Implementation"), weight decay 0.01 and T = 0.001 (appendix
 * "Configuration of Optimizer"), MIS lambda = 2 (appendix MIS energy), and the choices
 * the paper leaves open: lr 0.1 (from its set {1, 0.1, 0.01}), comm_alpha 0.1,
 * Adam betas 0.9 / 0.999, eps 1e-8. */
typedef struct {
    float gamma_min, gamma_max;  /* entropy coefficient schedule, linear in the update index */
    float lr;                    /* eta */
    float weight_decay;          /* AdamW decoupled weight decay */
    float temperature;           /* T of the sqrt(2 eta T) xi noise */
    float comm_alpha;            /* alpha of the STD communication term, in [0, 1] */
    int32_t entropy_alpha;       /* alpha-entropy exponent: even, >= 2 */
    float beta1, beta2, adam_eps;
    int32_t penalty_lambda;      /* MIS constraint penalty (integer, so objectives stay exact) */
    int32_t rule;                /* qqa_step_rule */
} qqa_schedule;

void qqa_schedule_default(qqa_schedule *s, qqa_problem problem, int32_t n);

/* Replica-row stride (floats) used for an S-replica state: S rounded up to 4. */
int32_t qqa_replica_stride(int32_t S);

/* ---------------------------------------------------------------------------------
 * Request-level API.  One context per device and host thread; it owns every device
 * buffer it allocates.
 * --------------------------------------------------------------------------------- */
typedef struct qqa_ctx qqa_ctx;
typedef int64_t qqa_req;
typedef int64_t qqa_graph_id;

/* Undirected graph in host memory.  Sparse: symmetric CSR (row_ptr[n+1], col_idx[nnz]),
 * no self-loops, no duplicate entries; weight[nnz] or NULL (all ones).  Dense: `dense`
 * is an n x n row-major symmetric matrix with zero diagonal and row_ptr/col_idx are
 * ignored.  Max-cut weights must be integer multiples of 2^-16 with |w| < 128 (so
 * cut values are exact integers in units of 2^-16); MIS ignores weights (A is the
 * 0/1 adjacency).  The library copies the graph; the caller may free it on return. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const float *weight;
    const float *dense;
} qqa_graph;

/* Check a host graph against the rules above for `problem` without a context and without
 * touching the device.  Returns QQA_OK or QQA_E_GRAPH; a message for the failure is
 * written to `why` (may be NULL, else at least `why_len` bytes). */
int qqa_graph_validate(const qqa_graph *g, qqa_problem problem, char *why, size_t why_len);

/* Result of a finished request.  The caller owns the optional arrays (NULL = not
 * wanted) and qqa_poll fills them when it returns QQA_OK.
 * Objectives are exact integers: MIS l = -size + lambda * violations (selected adjacent
 * pairs); max-cut l = -cut with cut counted in units of 2^-16; max clique
 * l = -size + lambda * violations (selected pairs that are not adjacent); coloring
 * l = size_or_cut = violations = edges whose ends share a colour (x_i = argmax_k V_ik, first
 * maximum), best_x = the colours (< K).  best_replica minimises (violations > 0, l,
 * replica index) lexicographically. */
typedef struct {
    int32_t best_replica;
    int32_t feasible;            /* best replica has no violated constraint */
    int64_t best_objective;
    int64_t best_size_or_cut;    /* MIS / clique set size, or cut in units of 2^-16 */
    int64_t best_violations;     /* MIS edges with both ends selected; 0 for max-cut */
    int64_t *replica_objective;  /* [S] or NULL */
    int64_t *replica_size_or_cut;/* [S] or NULL */
    int64_t *replica_violations; /* [S] or NULL */
    uint8_t *best_x;             /* [n] or NULL: rounded solution of best_replica */
    double queue_ms;             /* submit -> start on device (host clock) */
    double device_ms;            /* device time from first to last kernel of the request */
    double step_loop_ms;         /* device time of the K-update loop */
    double latency_ms;           /* submit -> result ready (host clock) */
    int32_t engine;              /* qqa_engine that ran the update loop */
    double kernel_us;            /* streaming engines: mean device duration of the dominant
                                  * launch of an update (the coupling product for dense
                                  * graphs, the update kernel otherwise), timed with events on
                                  * up to 32 updates spread over the schedule; -1 otherwise */
    double first_update_ms;      /* submit -> first update launched (host clock); for
                                  * requests outside the server, equal to queue_ms */
} qqa_result;

/* How the update loop runs.  STREAM: one launch per update, state streamed through
 * memory.  PERSISTENT: one cooperative launch for all updates; every lane group keeps
 * its rows' p, m, v in registers and only the new p goes to memory, updates separated by
 * a grid barrier.  LDS_BLOCK: one workgroup with P (and the CSR when it fits) in LDS
 * (small instances); its normals are formed by the whole GPU before each chunk of updates,
 * into a device table of at most 64 MiB that the request's footprint includes.  BATCH: a
 * ragged multi-instance launch (qqa_solve_batch, the server).  SLICED: streaming, with
 * the replica axis cut into 8 slices, slice s of every row updated on XCD s so that the
 * neighbour gathers of an XCD stay within 1/8 of P (its L2); one launch per update, which
 * also leaves each slice's partial statistics {mean, M2} of the new values for the next
 * update.  Sparse graphs with S >= 61 (at least 2 replica quads per slice).  STREAM,
 * PERSISTENT, LDS_BLOCK and BATCH perform the same arithmetic per row and give identical
 * results (STREAM layouts that split a row's edges over lane slices add the coupling sum in
 * another order).  SLICED performs the same arithmetic except for the replica statistics,
 * which it combines from the slices' partials: its results agree with the others to
 * rounding after one update, and its trajectories then diverge from theirs as any two
 * roundings of the method do.  It is deterministic and resumable like the others.
 * COMPACT: one replica per variable (S = 1, sparse MIS or max-cut): P, m, v held as one
 * float per variable instead of a padded quad, one lane per variable, one launch per
 * update; bitwise STREAM's results at one lane per row (the default layout for S = 1).
 * BATCH_RESIDENT: a ragged batch (qqa_solve_batch) in one cooperative launch for all of its
 * updates: each instance is run by a team of workgroups on one XCD whose lane groups keep
 * their rows' p, m, v in registers, the new P of every update is shared through that XCD's
 * L2, and the team meets at a barrier between updates.  Used by qqa_solve_batch under the
 * automatic policy when all instances share one replica layout with one quad per lane
 * (S = 4 x lanes per row), none has rows split into chunks, and each instance's rows fit
 * the registers of one XCD's workgroups; otherwise, and under QQA_ENGINE_STREAM, a batch
 * runs as BATCH.  Same arithmetic per row as STREAM: identical results. */
typedef enum {
    QQA_ENGINE_AUTO = -1,
    QQA_ENGINE_STREAM = 0,
    QQA_ENGINE_PERSISTENT = 1,
    QQA_ENGINE_LDS_BLOCK = 2,
    QQA_ENGINE_BATCH = 3,
    QQA_ENGINE_SLICED = 4,
    QQA_ENGINE_COMPACT = 5,
    QQA_ENGINE_BATCH_RESIDENT = 6
} qqa_engine;

/* device: HIP ordinal.  hbm_budget_bytes: cap on the device memory the context may
 * hold for requests (0 = 90% of free memory at creation).  hip_stream: stream to run
 * on (NULL = the context creates its own). */
int qqa_create(qqa_ctx **out, int device, size_t hbm_budget_bytes, void *hip_stream);
void qqa_destroy(qqa_ctx *c);
const char *qqa_last_error(const qqa_ctx *c);

/* Validate a host graph and copy it into device memory once; solves that name the id
 * read it in place.  Release with qqa_graph_release once no request uses it. */
int qqa_graph_upload(qqa_ctx *c, const qqa_graph *g, qqa_problem problem, qqa_graph_id *out);
int qqa_graph_release(qqa_ctx *c, qqa_graph_id id);

/* Submit one solve (asynchronous): init P ~ U(0,1) from `seed`, `steps` updates,
 * rounding and exact evaluation.  qqa_solve copies the host graph; qqa_solve_resident
 * uses an uploaded one.  `sched` NULL = qqa_schedule_default. */
int qqa_solve(qqa_ctx *c, const qqa_graph *g, qqa_problem problem, const qqa_schedule *sched,
              int32_t S, int32_t steps, uint64_t seed, qqa_req *out_id);
int qqa_solve_resident(qqa_ctx *c, qqa_graph_id g, qqa_problem problem, const qqa_schedule *sched,
                       int32_t S, int32_t steps, uint64_t seed, qqa_req *out_id);

/* Graph coloring with `colors` colours (2..255) on a CSR graph: the categorical update
 * (QQA_COLORING) for `steps` updates, then the colouring of every replica and its conflict
 * count; qqa_poll returns it as for the other problems.  Device state is colors x the
 * binary problems'.  qqa_solve_coloring_resident takes a graph uploaded with QQA_COLORING.
 * QQA_E_ARG for colors outside [2, 255]; qqa_solve / qqa_solve_resident refuse
 * QQA_COLORING.  An update is a gradient launch and an update launch; under the automatic
 * engine policy, shapes where one variable's colours x replica quads fit a wavefront (at most
 * 8 colours, a power-of-two number of quads served one per lane) run both in one launch with
 * bitwise the same results (QQA_ENGINE_STREAM keeps two launches).  kernel_us times the
 * gradient launch, or the single launch. */
int qqa_solve_coloring(qqa_ctx *c, const qqa_graph *g, int32_t colors, const qqa_schedule *sched,
                       int32_t S, int32_t steps, uint64_t seed, qqa_req *out_id);
int qqa_solve_coloring_resident(qqa_ctx *c, qqa_graph_id g, int32_t colors, const qqa_schedule *sched,
                                int32_t S, int32_t steps, uint64_t seed, qqa_req *out_id);

/* Submit `count` independent solves packed into one ragged batch: every update of the
 * batch is a single launch covering all instances (each at its own update index), the
 * update loop is replayed from a captured HIP graph.  Instances never interact: each
 * result equals that of the same solve run alone on the whole-row engines (under the
 * automatic policy a solve alone with S >= 128 may run on SLICED, which agrees to
 * rounding after one update; see qqa_engine).  Graph ids come from
 * qqa_graph_upload.  Arrays have `count` entries; sched may be NULL (defaults).  Dense
 * graphs and max clique are solved one at a time (QQA_E_ARG here). */
int qqa_solve_batch(qqa_ctx *c, int32_t count, const qqa_graph_id *graphs, const qqa_problem *problems,
                    const qqa_schedule *sched, const int32_t *S, const int32_t *steps,
                    const uint64_t *seeds, qqa_req *out_ids);

/* Batch autotuner: runs shortened copies of the batch described (arguments as for
 * qqa_solve_batch; the longest instance runs 64 updates, the others their share of that,
 * seeds 1..count, each candidate twice, results discarded) and keeps what is fastest:
 * for every S in the batch, the replica layout (as qqa_autotune) on the slot launches,
 * timed over that S's instances; and, when all instances share one S under the automatic
 * policy, whether the resident engine (at the default layout) or the slot launches (at the
 * layout found) run the batch in less device time per update.  Later batches and plain
 * solves of this context use those layouts, and later batches of one layout class with
 * that S use that engine.  lanes_out (count entries, may be NULL): the lanes per row each
 * instance's S now runs with.  *resident_out (may be NULL): 1 if the resident engine was kept.
 * The layout decides the summation order of the replica statistics, so results after
 * tuning equal those of the same solves under the same layouts.  QQA_E_ARG under a policy
 * other than AUTO or STREAM; errors of the timed batches are returned, with the context's
 * layouts and engine choices left as they were. */
int qqa_autotune_batch(qqa_ctx *c, int32_t count, const qqa_graph_id *graphs, const qqa_problem *problems,
                       const qqa_schedule *sched, const int32_t *S, const int32_t *steps,
                       int32_t *lanes_out, int32_t *resident_out);

/* Replica layout: how many adjacent lanes of a 64-lane wavefront serve the S replicas of
 * one variable (a power of two <= 64; each lane then owns ceil(S / (4 * lanes)) float4
 * quads, and a wavefront serves 64 / lanes variables).  The layout changes only the
 * summation order of the cross-replica mean and STD (a fixed tree per layout).  A context
 * applies one layout per S to all of its solves -- plain, batched and served -- so a
 * result never depends on which form ran it.  lanes_per_row = 0 restores the default
 * (the fewest quads per lane).  Set it before submitting solves with that S. */
int qqa_set_replica_layout(qqa_ctx *c, int32_t S, int32_t lanes_per_row);

/* Autotuner: time every supported layout for S on an uploaded graph (a few updates each,
 * on scratch state, with the streaming update kernel, or the compact one for S = 1 under
 * the automatic or COMPACT policy), keep the fastest for S in this context and return it
 * in *lanes_per_row (may be NULL). */
int qqa_autotune(qqa_ctx *c, qqa_graph_id g, qqa_problem problem, int32_t S, int32_t *lanes_per_row);

/* Engine policy of a context for single solves: QQA_ENGINE_AUTO (default) runs an instance
 * on LDS_BLOCK when it qualifies (one quad per lane in a full-width layout, no rows split
 * into chunks, P fits in one workgroup's LDS), else COMPACT for S = 1 (sparse MIS or
 * max-cut), else SLICED when the graph is sparse, S >= 256 and P (n x stride floats) is at
 * most 24 MiB, or when the solve can keep its state slice-major (S a multiple of the slice
 * count times the slice's lanes, not max clique), S >= 128 and P at most 64 MiB; else
 * STREAM.  (The per-stage qqa_dev_run keeps the row-major rule alone);
 * QQA_ENGINE_PERSISTENT runs the register-resident engine when the instance fits on chip
 * (else STREAM); QQA_ENGINE_LDS_BLOCK / QQA_ENGINE_SLICED / QQA_ENGINE_COMPACT /
 * QQA_ENGINE_STREAM force those engines where possible.  QQA_E_ARG for BATCH or an unknown
 * value. */
int qqa_set_engine(qqa_ctx *c, qqa_engine policy);

/* Wait up to timeout_us (0 = do not wait, < 0 = forever) for a request.  Returns QQA_OK
 * and fills *out when done (the handle is then released), QQA_PENDING if still
 * running, or an error. */
int qqa_poll(qqa_ctx *c, qqa_req id, qqa_result *out, int32_t timeout_us);
int qqa_cancel(qqa_ctx *c, qqa_req id);

/* ---------------------------------------------------------------------------------
 * Continuous-batching server.  A server thread advances admitted requests together:
 * every update is one launch per replica-layout class covering every running request,
 * each at its own update index, so requests that arrive while others run overlap on
 * the device.  It works in rounds of 16 updates; at each round boundary it retires
 * finished requests (rounded, evaluated and copied back during the previous round) and
 * admits queued requests first-come-first-served while a slot is free and the request's
 * HBM footprint (state, graph, schedule table, result) fits the server budget (the
 * context budget not in use when the server started).  Each round advances the admitted
 * requests with the least remaining work (updates left x rows x replica stride) until an
 * update covers about 8M replica-variables; the others keep their place for the round.
 * So small requests finish at close to their time alone.  A served result is identical to
 * the same solve run alone on the whole-row engines (STREAM, and BATCH); under the
 * automatic policy a solve alone with S >= 128 may run on SLICED, whose results agree with
 * the served one to rounding after one update (see qqa_engine).  Replica layouts set on the
 * context before qqa_serve_start apply.  Collect results with qqa_poll (queue_ms = submit ->
 * admission, first_update_ms = submit -> first update launched, latency_ms = submit ->
 * result).  Dense graphs, max clique and coloring are not served (QQA_E_ARG).
 *   qqa_serve_start: max_slots concurrent requests on the device.
 *   qqa_serve_submit: validates and copies the host graph (the caller may free it on
 *     return) and queues the request; QQA_E_ADMISSION if it can never fit, or if it is
 *     shed (below).
 *   qqa_serve_set_deadline: load shedding.  With deadline_ms > 0, qqa_serve_submit refuses
 *     (QQA_E_ADMISSION, "shed: ...") a request unless it and every admitted request can
 *     still finish within deadline_ms of their submission.  The projection: under
 *     least-remaining-work-first a request of work w waits for the pending work with no more
 *     remaining work than its own, W_<=, and for smaller work arriving meanwhile at the rate
 *     a_w measured over the admitted submissions of the last 5 s; at the device rate R
 *     (replica-variable updates per second, measured over rounds that leave work waiting) it
 *     finishes after (W_<= + w) / (R - a_w), and no sooner than its updates times the
 *     shortest update time seen.  Admitting it
 *     delays each pending request with more remaining work by w / R; it is refused if one
 *     of them would then be projected past its deadline (also one that is late already, so
 *     that it is not overtaken by ever more smaller work).  With a deadline, each round
 *     first runs the requests older than half of it, oldest first, then the others by least
 *     remaining work.  0 (the default) sheds nothing.
 *   qqa_serve_get_stats: counts of submitted, admitted, shed and completed requests since
 *     qqa_serve_start, the measured device rate and the server's device memory.
 *   qqa_serve_stop: returns after every queued and admitted request has finished;
 *     results stay available to qqa_poll.  A context runs at most one server at a time.
 * --------------------------------------------------------------------------------- */
typedef struct {
    int64_t submitted;           /* qqa_serve_submit calls that passed validation */
    int64_t admitted;            /* of which queued for the device */
    int64_t shed;                /* of which refused by the deadline */
    int64_t completed;           /* admitted requests whose result is ready */
    double rate_updates_per_s;   /* measured device rate R */
    double deadline_ms;
    size_t device_bytes_held;    /* request buffers the server's pool holds (in use or idle) */
    size_t device_bytes_cached;  /* of which idle, kept for reuse (capped at 4 GiB) */
} qqa_serve_stats;

int qqa_serve_start(qqa_ctx *c, int32_t max_slots);
int qqa_serve_submit(qqa_ctx *c, const qqa_graph *g, qqa_problem problem, const qqa_schedule *sched,
                     int32_t S, int32_t steps, uint64_t seed, qqa_req *out_id);
int qqa_serve_set_deadline(qqa_ctx *c, double deadline_ms);
int qqa_serve_get_stats(qqa_ctx *c, qqa_serve_stats *out);
int qqa_serve_stop(qqa_ctx *c);

/* ---------------------------------------------------------------------------------
 * Device-level entry points: one stage of the path on caller-owned device buffers,
 * asynchronous on `stream`.  They exist so that each stage can be checked on its own.
 * --------------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;  /* device, n+1 (sparse) */
    const int32_t *col_idx;  /* device, nnz (sparse) */
    const float *weight;     /* device, nnz or NULL */
    const float *dense;      /* device, n x n row-major, or NULL for sparse */
} qqa_dev_graph;

const char *qqa_dev_last_error(void);

/* Raw Philox4x32-10 integers (SC'11 generator) for rows [0,n) and quads [0,nquads):
 * out[(i*nquads + q)*4 + j] = word j of Philox(key = seed, counter = (i, q, k, stream_id)). */
int qqa_dev_philox(uint64_t seed, int32_t n, int32_t nquads, uint32_t k, uint32_t stream_id,
                   uint32_t *out, void *stream);

/* Gaussian noise of update k (Box-Muller on 24-bit uniforms): xi[i*stride + s]. */
int qqa_dev_noise(uint64_t seed, int32_t n, int32_t S, uint32_t k, float *xi, void *stream);

/* Initial state: P[i*stride + s] ~ U(0,1) from `seed`; m = v = 0 (m, v may be NULL). */
int qqa_dev_init(uint64_t seed, int32_t n, int32_t S, float *P, float *m, float *v, void *stream);

/* Dense coupling product on the matrix cores (FP32 MFMA, FP32 accumulation):
 * C[i*stride + s] = sum_k W[i*n + k] f(P[k*stride + s]), f(p) = 2p - 1 (QQA_MAXCUT) or p
 * (QQA_MIS), for a symmetric n x n W (device).  P, C: device n x stride.  The k range may
 * be split over workgroups, with the parts' partial products (stream-ordered scratch)
 * added in a fixed order: the result is deterministic. */
int qqa_dev_dense_coupling(const float *W, const float *P, float *C, int32_t n, int32_t S, qqa_problem problem,
                           void *stream);

/* Per-replica sums of P for max clique, exact in 2^-32 fixed point:
 * T[s] = sum_i round(P[i*stride + s] * 2^32) for s < stride (padding replicas included),
 * for P with entries in [0, 1].  T: device, stride uint64, overwritten.  The integer sum
 * does not depend on the order of additions, so T is bit-reproducible. */
int qqa_dev_replica_sums(const float *P, int32_t n, int32_t S, uint64_t *T, void *stream);

/* One update t (0-based, AdamW step count t+1) of a K-update schedule:
 * reads P_in, writes P_out (must not alias P_in: neighbours read P_in), updates m, v in
 * place.  lanes_per_row selects the replica layout (0 = default; see
 * qqa_set_replica_layout).  Rows of more than 64 neighbours are split into 16-edge chunks
 * whose partial sums are added in chunk order, as in every solve.  A dense graph takes the
 * coupling product from qqa_dev_dense_coupling's kernel.  Max clique computes the
 * per-replica sums of P_in (qqa_dev_replica_sums) before the update. */
int qqa_dev_step(const qqa_dev_graph *g, qqa_problem problem, const qqa_schedule *sched, int32_t S,
                 int32_t t, int32_t K, uint64_t seed, const float *P_in, float *P_out, float *m,
                 float *v, int32_t lanes_per_row, void *stream);

/* Updates t0 .. t1-1 of a K-update schedule with the given engine (QQA_ENGINE_AUTO picks
 * as a context would) on caller buffers: P0 and P1 ping-pong (P[t0 & 1] holds the state
 * before update t0, P[t1 & 1] the state after), m and v updated in place.  Returns
 * QQA_E_ARG if the engine cannot run this instance, QQA_E_DEVICE if a persistent
 * launch's barrier timed out.  Synchronous for the persistent engines' abort check.  The
 * LDS_BLOCK engine allocates (stream-ordered) a table of the normals of at most 64 MiB for
 * the call and frees it before returning. */
int qqa_dev_run(const qqa_dev_graph *g, qqa_problem problem, const qqa_schedule *sched, int32_t S,
                int32_t t0, int32_t t1, int32_t K, uint64_t seed, float *P0, float *P1, float *m, float *v,
                int32_t engine, int32_t lanes_per_row, void *stream);

/* One graph-coloring update t of a K-update schedule on caller buffers: V_in, V_out, m, v
 * are device arrays of n * colors rows x stride floats (row i*colors + k holds colour k of
 * variable i for every replica); V_out must not alias V_in; m, v updated in place.  The
 * Clamp-normalised sigma of V_in is formed internally (stream-ordered scratch).  Shapes that
 * the single-launch form serves (see qqa_solve_coloring) use it. */
int qqa_dev_color_step(const qqa_dev_graph *g, int32_t colors, const qqa_schedule *sched, int32_t S,
                       int32_t t, int32_t K, uint64_t seed, const float *V_in, float *V_out, float *m,
                       float *v, int32_t lanes_per_row, void *stream);

/* Colouring of every replica and its exact cost: X (device, n x stride bytes) receives
 * x_i = argmax_k V_ik (first maximum) for replica s at X[i*stride + s]; conflicts[S]
 * (device int64) the edges whose ends share a colour; best[1] (device int32) the replica
 * with the fewest (lowest index among ties). */
int qqa_dev_color_eval(const qqa_dev_graph *g, int32_t colors, int32_t S, const float *V, uint8_t *X,
                       int64_t *conflicts, int32_t *best, void *stream);

/* Round x = [P > 1/2] and evaluate every replica exactly.  Outputs are device arrays:
 * size_or_cut[S], viol[S], obj[S] (int64) and best[1] (int32). */
int qqa_dev_eval(const qqa_dev_graph *g, qqa_problem problem, int32_t penalty_lambda, int32_t S,
                 const float *P, int64_t *size_or_cut, int64_t *viol, int64_t *obj, int32_t *best,
                 void *stream);

/* qqa_dev_eval for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as qqa_dev_eval, but its per-replica accumulators live in a fixed 64 KiB
 * device array of the library (2 x 4096 uint64, enough for every S <= 4096) instead of
 * stream-ordered scratch, so it calls no allocator; it is launched as three kernels (a fill
 * that clears the accumulators, the counts, the objectives) and no memset, copy or
 * synchronisation.  Each GPU holds its own copy of the array from the first call on that
 * device until the process ends.  Every call on one GPU shares that array: calls that may
 * overlap on one GPU (different streams without ordering between them) race and must be
 * serialised by the caller.  QQA_E_ARG for S outside [1, 4096]. */
int qqa_dev_eval_noalloc(const qqa_dev_graph *g, qqa_problem problem, int32_t penalty_lambda, int32_t S,
                         const float *P, int64_t *size_or_cut, int64_t *viol, int64_t *obj, int32_t *best,
                         void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QQA_H */
