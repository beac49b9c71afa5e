/*
 * prop.h -- C ABI of the MI355X (gfx950) domain-propagation library.
 *
 * The library propagates variable bounds through linear constraints
 *
 *     lhs_i <= sum_j A_ij x_j <= rhs_i      (i = 0..m-1)
 *     lb_j  <= x_j <= ub_j                  (j = 0..n-1, some x_j integer)
 *
 * in synchronous rounds, as in Sofranac, Gleixner and Pokutta,
 * "Accelerating Domain Propagation: an Efficient GPU-Parallel Algorithm
 * over Sparse Matrices" (arXiv 2009.07785):
 *
 *   - every row's minimum and maximum activity (Sec. 1.1, Definition 1),
 *     split into a finite part and a count of infinite contributions
 *     (Sec. 3.4), from the bounds as they stood at the start of the round;
 *   - one lower and one upper bound candidate per nonzero (Sec. 1.1, Step 3,
 *     eqs. bound_candidates_pos / bound_candidates_neg), rounded inward for
 *     integer variables;
 *   - candidates that improve on the start-of-round bound are applied with
 *     atomic max (lower) / min (upper) (Sec. 3.5, Algorithm 3);
 *   - rounds repeat until no bound changes, a domain becomes empty or the
 *     round limit is reached (Algorithm 2).
 *
 * Numerical contract (the same as the test oracle's, stated in full in the
 * repository's design notes):
 *   - activities are the exact sum of the products, rounded once to the
 *     nearest double; every other operation is one IEEE double operation in
 *     the order of the paper's formulas: (beta - activity) / a + bound;
 *   - integer candidates: lower = ceil(c - eps_int), upper =
 *     floor(c + eps_int);
 *   - a candidate is applied when it beats the start-of-round bound b:
 *     b infinite: any finite candidate; integer: strictly; continuous: by
 *     more than cont_rel_tol * max(1, |b|); candidates beyond 2^200 in
 *     magnitude are dropped;
 *   - a domain is empty when l > u (integer) or
 *     l - u > feas_tol * max(1, |l|, |u|) (continuous).
 *
 * Input domain (checked; violations return PROP_EINVAL): coefficients are
 * finite and either 0 (skipped) or of magnitude in [2^-64, 2^64]; column
 * indices are in [0, n) and distinct within a row; row_ptr starts at 0 and
 * never decreases; lhs is finite or -inf, rhs finite or +inf; lb finite or
 * -inf, ub finite or +inf; finite values have magnitude <= 2^200; no NaN;
 * vartype is 0 (continuous) or 1 (integer; a binary is an integer in [0,1]).
 *
 * Threading: a prop_problem may be used by one thread at a time.  Calls on
 * different problems may run concurrently.
 */
#ifndef PROP_H
#define PROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Outcome of a run (prop_result.status). */
#define PROP_CONVERGED 0  /* a round changed nothing */
#define PROP_INFEASIBLE 1 /* some domain became empty (bounds then unspecified) */
#define PROP_MAX_ROUNDS 2 /* the round limit was reached with changes pending */

/* Return codes: 0 on success, negative on error; the library never aborts. */
#define PROP_OK 0
#define PROP_EINVAL (-1)  /* invalid argument or input outside the domain above */
#define PROP_ENOMEM (-2)  /* device or host allocation failed */
#define PROP_EDEVICE (-3) /* HIP runtime error, no usable GPU, or device timeout */
#define PROP_EBUSY (-4)   /* serving: the request queue is full */

/* vartype values */
#define PROP_CONTINUOUS 0
#define PROP_INTEGER 1

/* Bound stores (prop_set_store). */
#define PROP_STORE_F64 64 /* default: bounds kept as doubles */
#define PROP_STORE_F32 32 /* bounds kept in single precision, rounded outward */

/* Round-loop drivers (prop_set_loop).  All give identical results. */
#define PROP_LOOP_PERSISTENT 0 /* one cooperative launch, grid barriers between phases */
#define PROP_LOOP_STREAM 1     /* default: per-round kernels queued in batches; the host
                                  reads the device's done flag one batch behind */
#define PROP_LOOP_HOST 2       /* per-round kernels, host reads the flag every round */
#define PROP_LOOP_GRAPH 3      /* as STREAM, each batch of rounds one replay of a HIP graph
                                  captured on the first run (kernels exit early once done) */
#define PROP_LOOP_GRAPH_ALL 4  /* the replays of GRAPH for all max_rounds rounds queued at
                                  once: the host reads nothing until the end, and rounds
                                  after the last one exit at once */

typedef struct prop_problem prop_problem; /* opaque */

/* Constraint matrix in CSR form, host memory.  row_ptr has m+1 entries. */
typedef struct {
  int32_t m;
  int32_t n;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* vals;
} prop_csr;

/* Tolerances and layout; a NULL pointer means 1e-6 for each tolerance and
 * steps = 0. */
typedef struct {
  double eps_int;      /* integer rounding slack, >= 0 and < 0.5 */
  double cont_rel_tol; /* relative gain a continuous bound needs, >= 0 */
  double feas_tol;     /* relative crossing a continuous domain may show, >= 0 */
  int32_t steps;       /* layout: entries per lane of a short row, 4, 8 or 16 (rows longer
                          than 64 * steps go to 1024-entry segments); 0 = the value
                          prop_autotune recorded for a matrix of this shape, else by
                          size: 4 up to 100,000 stored entries, 8 up to 5,000,000,
                          16 above */
  int32_t layout;      /* 0: rows in length classes, K lanes per row, in wave-sized
                          chunks (default); 1: nnz split (merge-path style): rows in
                          input order packed into waves of 512 entries, 8 consecutive
                          entries per lane, rows spanning lanes joined by a segmented
                          scan, rows longer than 512 entries in segments (steps is
                          then ignored).  Layout 1 serves single runs only (batches
                          and serving return PROP_EINVAL) and processes every row in
                          marked rounds (same results). */
} prop_params;

typedef struct {
  int32_t status; /* PROP_CONVERGED / PROP_INFEASIBLE / PROP_MAX_ROUNDS */
  int32_t rounds; /* rounds executed, counting the last change-free one */
} prop_result;

/* Size and layout figures of a created problem. */
typedef struct {
  int32_t m, n;
  int64_t nnz;             /* nonzero coefficients (explicit zeros dropped) */
  int64_t nnz_stored;      /* stored entries including layout padding */
  int32_t n_chunks;        /* wave-sized tiles of rows with <= 64 * steps entries */
  int32_t n_long_rows;     /* rows with more than 64 * steps entries */
  int32_t n_segments;      /* 1024-entry segments of those rows */
  int32_t grid_blocks;     /* blocks of the persistent launch */
  int64_t device_bytes;    /* device memory held by the problem */
  int64_t alg_bytes_round; /* algorithmic bytes per round: 12 nnz + 20 m + 33 n + 4 */
  int32_t steps;           /* entries per lane of a short row in the layout (4, 8, 16) */
  int32_t layout;          /* prop_params.layout of the problem */
} prop_info;

/* Builds a problem on the current HIP device.  The inputs are copied; the
 * caller keeps ownership of every array.  Rows are reordered and variables
 * relabelled internally; results come back in the caller's order.
 * Rows with lhs > rhs, and empty rows whose sides exclude 0, make every
 * later run report PROP_INFEASIBLE after 0 rounds.  `params` may be NULL.
 * Returns PROP_OK and stores the handle in *out, or an error code. */
int prop_create(const prop_csr* A, const double* lhs, const double* rhs, const uint8_t* vartype,
                const prop_params* params, prop_problem** out);

/* Autotuner: builds the problem with each layout (steps = 16, 8, 4), times
 * full propagations from lb[n], ub[n] (host, not modified; max_rounds as
 * for prop_run) with the stream driver, and stores the fastest steps in
 * *steps_out and in the tuning cache under the matrix's shape signature
 * (m, n, nnz and the histogram of row lengths by powers of two), where
 * prop_create with steps = 0 looks it up.  The cache lives in the process
 * and, when the environment variable PROP_TUNE_CACHE names a file, in that
 * file (one "signature steps" line per entry, appended).  Needs the device
 * memory of two layouts at a time.  Returns like prop_create / prop_run. */
int prop_autotune(const prop_csr* A, const double* lhs, const double* rhs, const uint8_t* vartype,
                  const prop_params* params, const double* lb, const double* ub,
                  int32_t max_rounds, int32_t* steps_out);

/* Propagates host arrays lb[n], ub[n] in place (caller-owned, overwritten
 * with the result; unspecified when the status is PROP_INFEASIBLE).
 * Copies in, runs, copies out and synchronises.  max_rounds >= 0. */
int prop_run(prop_problem* p, double* lb, double* ub, int32_t max_rounds, prop_result* out);

/* Same on device arrays d_lb[n], d_ub[n] (HIP device memory, caller-owned,
 * updated in place), queued on `stream` (a hipStream_t; NULL = the null
 * stream).  Allocates no device memory (the graph driver captures its
 * rounds on its first run, and kernel timing creates its events on first
 * use).  Host waits: the stream and graph drivers queue rounds in batches
 * of 4 and, after queueing a batch, wait on the event of the batch before
 * it to read the device's done flag; the host driver synchronises the
 * stream after every round; the persistent driver runs every round in one
 * launch, and the graph-all driver queues ceil(max_rounds / 4) graph
 * replays before waiting on anything (each round after the run has ended
 * costs three kernel launches that exit at once).  All of them synchronise
 * the stream at the end to fill *out (host memory).  Bound validation happens on the device; an invalid bound makes
 * the call return PROP_EINVAL. */
int prop_run_device(prop_problem* p, double* d_lb, double* d_ub, int32_t max_rounds,
                    void* stream, prop_result* out);

/* Propagates `nodes` bound vectors of the same problem together (for
 * example branch-and-bound nodes: the paper propagates at every node of a
 * search, Sec. 1, and names propagation after branching as the case that
 * needs GPU-suited methods, Sec. 5).  d_lb, d_ub: device arrays of nodes * n
 * doubles, node k's bounds at [k * n, (k + 1) * n), caller-owned, updated in
 * place.  out: host array of `nodes` results.  Each node's status, rounds
 * and bounds are bitwise those a separate prop_run_device call on that node
 * returns; nodes that finish early stop consuming work.  Rounds are queued
 * on `stream` in batches as by PROP_LOOP_STREAM (or replayed as by
 * PROP_LOOP_GRAPH; PROP_LOOP_GRAPH_ALL: see prop_set_loop).  When the nodes
 * still running would fit in fewer groups of 8, the call synchronises `stream`,
 * writes the finished nodes' rows of d_lb / d_ub, and packs the running
 * nodes into fewer groups; the rest of the rows are written at the end.  The first call with more nodes than any
 * earlier call allocates the batch workspace (32 * n * ceil(nodes / 8) * 8
 * bytes of bounds, about n / 8 bytes of touch flags per group of 8 nodes,
 * plus per-node counters and lists, and 80 + 48 bytes of long-row partial
 * and row state per long-row segment and node),
 * kept until prop_destroy; later calls allocate nothing.  An invalid bound
 * in any node returns PROP_EINVAL. */
int prop_run_batch_device(prop_problem* p, int32_t nodes, double* d_lb, double* d_ub,
                          int32_t max_rounds, void* stream, prop_result* out);

/* prop_run_batch_device on host arrays lb[nodes * n], ub[nodes * n]
 * (caller-owned, node k at [k * n, (k + 1) * n), overwritten with the
 * result; a node's bounds are unspecified when its status is
 * PROP_INFEASIBLE).  Copies in, runs on the null stream, copies out and
 * synchronises.  Besides the batch workspace, the first call with more
 * nodes than any earlier one allocates device staging of 16 * n * nodes
 * bytes, kept until prop_destroy. */
int prop_run_batch(prop_problem* p, int32_t nodes, double* lb, double* ub, int32_t max_rounds,
                   prop_result* out);

/* prop_run_batch_device for callers that cannot allocate device memory:
 * code being captured into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors, but the batch
 * workspace lives in a fixed 64 MiB device array of the library instead of
 * memory the call allocates, and the call allocates nothing.  The
 * workspace takes 32 * n * 8 * ceil(nodes / 8) bytes of bound pairs plus
 * n / 8 bytes of touch flags per group (rounded up to 256 bytes), 80
 * bytes per long-row segment and node, and 40 bytes per node, each region
 * rounded up to 256 bytes; a call that needs more than 64 MiB returns
 * PROP_EINVAL before touching the device.  Every group of 8 nodes runs
 * until all nodes have finished (no compaction), with rounds queued on
 * `stream` in batches as by PROP_LOOP_STREAM, whatever prop_set_loop
 * selected; the done flag is read through pinned memory once per batch.
 * Each device the library runs on holds its own copy of the array until
 * the process ends, and every call on that device reuses it (the call
 * clears what must start at zero): calls that overlap on one device, from
 * several threads or on several streams, race and must be serialised by
 * the caller. */
int prop_run_batch_device_static(prop_problem* p, int32_t nodes, double* d_lb, double* d_ub,
                                 int32_t max_rounds, void* stream, prop_result* out);

/* Selects the round-loop driver (PROP_LOOP_*) for later runs.  Batches with
 * PROP_LOOP_GRAPH_ALL queue every replay up front as well and read nothing
 * until the end, so they are never compacted: finished nodes leave their
 * groups, which keep running with the nodes left. */
int prop_set_loop(prop_problem* p, int32_t mode);

/* Marked rounds (enable != 0; off by default), for prop_run and
 * prop_run_device with the stream, graph, graph-all or host driver, and for
 * prop_run_batch / prop_run_batch_device (the persistent driver and
 * prop_run_batch_device_static ignore it).  A row is then processed in
 * round r >= 2 only when one of its variables changed in round r - 1 (in a
 * batch: in any node of the row's group of 8 nodes): a row whose variables
 * did not change would compute the activities and candidates of the
 * previous round, against the same bounds, and those changed nothing (a
 * candidate that counted would have changed its variable).  Results,
 * status and round counts are bitwise those of unmarked rounds; when more
 * than n / 32 variables changed, the next round processes every row (in a
 * batch: every row of that group; also after a compaction).  This is the
 * constraint marking of the paper's sequential Algorithm 1 (Sec. 2.1)
 * applied to the synchronous rounds of Algorithm 2.  The first enable
 * uploads the rows of every variable (4 bytes per nonzero, 8 per variable,
 * 12 per piece of 64 rows of a variable), a row stamp per row and a
 * changed-variable bitmap; a marked batch also allocates 4 bytes per row
 * and n / 8 bytes per group of 8 nodes.  These stay until prop_destroy. */
int prop_set_marking(prop_problem* p, int32_t enable);

/* Parent fixed point for marked runs (branch-and-bound children; the
 * paper's outlook, Sec. 5, and the marking of Algorithm 1, Sec. 2.1).
 * d_lb, d_ub: device arrays of n doubles holding bounds that are a fixed
 * point of this problem's propagation, such as the bounds a CONVERGED run
 * returned; the library keeps a copy (integer bounds rounded as at the
 * start of a run, and rounded outward under the single-precision store of
 * prop_set_store, which must be the store the parent was computed with),
 * so the caller's arrays may be reused at once.  While a parent is set and marked rounds are enabled, round 1 of prop_run,
 * prop_run_device, prop_run_batch and prop_run_batch_device processes only
 * the rows holding a variable whose start bounds differ from the parent's
 * (in a batch: in any node of the row's group): every other row would
 * compute the candidates of the parent's last round from the same bounds,
 * and none of those counted.  Results are then bitwise those of an unmarked
 * run, provided the parent really is a fixed point (the library does not
 * check it: if it is not, rows that would have tightened a bound in round 1
 * are skipped).  NULL, NULL clears the parent.  Runs on `stream` and
 * synchronises it.  A bound that prop_run would reject returns PROP_EINVAL
 * and clears the parent.  The first call allocates 16 * n bytes (and the
 * marking data, as prop_set_marking does). */
int prop_set_parent(prop_problem* p, const double* d_lb, const double* d_ub, void* stream);

/* Bound store for later runs of prop_run and prop_run_device (every
 * driver): PROP_STORE_F64 (default) or PROP_STORE_F32, the mixed-precision
 * variant of the paper's single-precision runs (Sec. 4.5, where the method
 * run wholly in single precision gives wrong results).  With PROP_STORE_F32
 * the arithmetic is unchanged (the numerical contract above), but every
 * bound is kept on the grid G of 0, -inf, +inf and the normal single-precision
 * numbers, rounded outward: a lower bound becomes the largest member of G
 * not above it, an upper bound the smallest member not below it.  This
 * applies to the input bounds after their integer rounding and to every
 * bound a round commits, before the round decides whether anything
 * changed; a gain smaller than one step of G therefore changes nothing.
 * Outward rounding only loosens bounds, so no point that the FP64 store
 * keeps is cut off and no problem is reported infeasible that the FP64
 * store finds feasible; bounds beyond the single-precision range become
 * infinite, and integer bounds stay integers (every integer up to 2^24 is
 * in G).  The activity pass then gathers 8 bytes per continuous variable
 * instead of 16.  Returned bounds are doubles holding members of G.
 * Results are bitwise those of the test oracle's single-precision store.
 * The first PROP_STORE_F32 allocates 8 * n bytes, kept until prop_destroy.
 * Changing the store clears the parent (prop_set_parent) and any captured
 * rounds.  The nnz-split layout (prop_params.layout 1) returns
 * PROP_EINVAL, and while PROP_STORE_F32 is set, prop_run_batch,
 * prop_run_batch_device, prop_run_batch_device_static and
 * prop_srv_add_instance return PROP_EINVAL. */
int prop_set_store(prop_problem* p, int32_t bits);

/* Fills *out with the problem's sizes. */
int prop_get_info(const prop_problem* p, prop_info* out);

/* Device time of the last run's round loop in milliseconds (HIP events on
 * the launch stream around the loop kernels, pack/unpack excluded), and the
 * same with the bound pack and unpack kernels included. */
int prop_last_timing(const prop_problem* p, double* loop_ms, double* total_ms);

/* With enable != 0, later runs of the stream and host drivers record HIP
 * events around every launch of the per-round matrix kernel (the dominant
 * kernel) on the launch stream; prop_last_kernel_timing then returns the
 * summed duration in milliseconds and the number of launches of the last
 * run.  Off by default; the events cost a few microseconds per round. */
int prop_set_kernel_timing(prop_problem* p, int32_t enable);
int prop_last_kernel_timing(const prop_problem* p, double* ms, int32_t* launches);

/* Releases the problem (NULL is allowed). */
void prop_destroy(prop_problem* p);

/* ------------------------------------------------------------------------
 * Serving: many propagation requests over resident problems.
 *
 * A request is one bound vector (a node of a search, a what-if query) to be
 * propagated on a problem added to the server.  Requests on the same problem
 * share its node slots, laid out as by prop_run_batch_device, and run with
 * continuous batching: a request enters a free slot at the next round
 * boundary of its problem, advances one round per round of that problem,
 * and leaves when it converges, becomes infeasible or reaches its own round
 * limit, while the other requests keep running.  Each request's status,
 * rounds and bounds are bitwise those prop_run returns for the same problem
 * and input.
 *
 * Admission by device-memory footprint: slots come in groups of 8, each
 * group holding 384 * n bytes (start-of-round and candidate bound pairs,
 * and the request's input/output staging) plus about n / 8 bytes of touch
 * flags; groups are allocated when a
 * request finds no free slot and the budget has room, and idle groups are
 * released when another problem needs the room.  Each added problem also
 * holds 32 * max_slots bytes of per-slot state plus 64 * max_slots bytes
 * per long-row segment, and the server about 100 KB of its own; this fixed
 * state is never released.  A request waits in its problem's queue (first
 * in, first out) while neither a slot nor room is available.
 *
 * One host thread per server schedules.  The kernels go to one HIP stream
 * of the server, the copies of request bounds and results to a second one
 * (both default priority, ordered with events) so that the copies overlap
 * the rounds: each round of every problem with running requests is one
 * launch per phase, so the host's launch count does not grow with the
 * number of problems.  At most 256 problems per server,
 * all on one device.  The server reads only a problem's matrix and keeps its own
 * control state: prop_run calls on an added problem stay allowed, from one
 * thread at a time as always.  Destroy the server before its problems.
 * Server calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct prop_server prop_server; /* opaque */

typedef struct {
  int64_t budget_bytes;    /* device bytes for slot groups and per-problem state, > 0 */
  int32_t max_slots;       /* slots per problem, a multiple of 8 (0: 256) */
  int32_t rounds_per_step; /* rounds queued between status reads (0: 1) */
  int32_t max_pending;     /* requests held (queued, running or unread) before
                              prop_srv_submit returns PROP_EBUSY (0: 1 << 20) */
  int32_t marking;         /* != 0: marked rounds per group of 8 slots, as by
                              prop_set_marking for batches (a row is processed only
                              when one of its variables changed in the previous round
                              in a slot of the group; a request joining a group makes
                              the group's next round process every row); results are
                              bitwise those without.  prop_srv_add_instance then
                              uploads the problem's variable rows (as the first
                              prop_set_marking does, charged to the problem) and adds
                              4 bytes per row and n / 8 + 8 bytes per group of slots
                              to the instance's state (charged to the budget). */
} prop_srv_config;

typedef struct {
  int64_t submitted;          /* accepted by prop_srv_submit */
  int64_t completed;          /* results ready */
  int64_t queued;             /* waiting for a slot */
  int64_t running;            /* in a slot */
  int64_t device_bytes;       /* device memory the server holds now */
  int64_t peak_device_bytes;  /* most it has held */
  int64_t steps;              /* round steps queued over all problems */
  double p50_ms, p99_ms;      /* latency, submission to result ready */
  double mean_ms, max_ms;
  double wall_s;              /* first submission to last completion */
  double req_per_s;           /* completed / wall_s */
} prop_srv_stats;

/* Starts a server (and its scheduler thread; no device work yet). */
int prop_srv_create(const prop_srv_config* cfg, prop_server** out);

/* Makes problem p servable under the id stored in *id (0, 1, ...).  The
 * problem must outlive the server.  Returns PROP_ENOMEM when its per-problem
 * state does not fit the remaining budget, PROP_EINVAL beyond 256 problems
 * or for a problem on another device than the first one. */
int prop_srv_add_instance(prop_server* s, prop_problem* p, int32_t* id);

/* Queues a request: lb[n], ub[n] (host, copied before the call returns;
 * the caller keeps them) under the input domain of prop_run, and a round
 * limit >= 0.  Stores a ticket in *ticket.  PROP_EINVAL for an unknown id
 * or an invalid bound, PROP_ENOMEM when one slot group of the problem
 * cannot fit the budget beside the fixed state of the server and its
 * problems, PROP_EBUSY when max_pending requests are held. */
int prop_srv_submit(prop_server* s, int32_t id, const double* lb, const double* ub,
                    int32_t max_rounds, int64_t* ticket);

/* Returns 1 and fills *out, lb[n], ub[n] (host, caller-owned; either may be
 * NULL to skip it) when the request has finished, releasing the ticket; 0
 * while it is pending; a negative code for an unknown ticket or when the
 * server failed (the request is then lost). */
int prop_srv_poll(prop_server* s, int64_t ticket, prop_result* out, double* lb, double* ub);

/* As prop_srv_poll, waiting up to timeout_ms milliseconds (< 0: no limit). */
int prop_srv_wait(prop_server* s, int64_t ticket, int32_t timeout_ms, prop_result* out, double* lb,
                  double* ub);

/* Counters and latency percentiles since the server started or the last
 * prop_srv_reset_stats. */
int prop_srv_get_stats(prop_server* s, prop_srv_stats* out);
int prop_srv_reset_stats(prop_server* s);

/* Stops the scheduler, waits for queued device work and releases the
 * server's memory (NULL is allowed).  Unread results are discarded. */
void prop_srv_destroy(prop_server* s);

/* Message describing the last error on the calling thread ("" if none). */
const char* prop_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PROP_H */
