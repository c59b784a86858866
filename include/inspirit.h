/*
 * inspirit.h -- C ABI of the MI355X (gfx950) INSPIRIT scheduling library.
 *
 * INSPIRIT (Y. Wang et al., "INSPIRIT: Inspiring Ability and Efficiency for
 * Task Scheduling", arXiv 2404.03226) orders ready tasks of a task DAG on
 * heterogeneous workers by two per-task attributes, inspiring ability (IA)
 * and inspiring efficiency (IE), and switches between them by watching the
 * number of ready tasks (Nready).  This library computes the attributes on
 * the GPU and runs an integer-time, event-driven list-scheduling simulation
 * of CPU and GPU workers with those priorities, for one DAG or for many DAGs
 * in one persistent launch.
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (for example torch tensors on the
 *     ROCm device) unless marked "host".
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued on it asynchronously; calls that must validate device
 *     data (insp_build_dag) synchronise the stream before returning.
 *   - Every call returns an insp_status.  On a non-OK status no output array
 *     has been written (outputs of a call that fails during the simulation,
 *     INSP_E_HANG, are unspecified) and insp_last_error() describes why.
 *     Nothing is thrown or aborted across the ABI.
 *   - Durations and estimates are integer ticks in [1, 2^20].  A DAG has at
 *     most 2^21 tasks; a machine has 1..1024 workers.
 *   - Worker w < n_cpu is a CPU worker (kind 0), the rest are GPU workers
 *     (kind 1).  Per-task tick tables are int32 [n][2]: column 0 = CPU,
 *     column 1 = GPU; they are read a row (8 bytes) at a time and must be
 *     8-byte aligned (INSP_E_INVAL otherwise).
 */
#ifndef INSPIRIT_H
#define INSPIRIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    INSP_OK = 0,
    INSP_E_INVAL = 1,  /* malformed argument: bad CSR, self loop, null pointer, bad enum */
    INSP_E_CYCLE = 2,  /* the dependency graph has a cycle */
    INSP_E_RANGE = 3,  /* a size or tick value outside the documented limits */
    INSP_E_NOMEM = 4,  /* device or host allocation failed */
    INSP_E_DEVICE = 5, /* a HIP runtime call failed */
    INSP_E_HANG = 6    /* the simulation needed more events than allowed */
} insp_status;

typedef enum {
    INSP_POLICY_INSPIRIT = 0,     /* adaptive: Nready regulator picks the pop rule */
    INSP_POLICY_FIFO = 1,         /* plain DMDA: each worker pops in push order */
    INSP_POLICY_ABILITY_ONLY = 2, /* always the high-ability rule */
    INSP_POLICY_EFI_ONLY = 3,     /* always the high-efficiency rule */
    INSP_POLICY_HEFT = 4,         /* HEFT list baseline (Section 6): highest upward rank
                                     R(v) = n_cpu est_cpu(v) + n_gpu est_gpu(v) + max over
                                     successors R(s), then earliest push; R < 2^42 or the
                                     DAG fails with INSP_E_RANGE at insp_sync_status */
    INSP_POLICY_LOCALITY = 5      /* always the efficiency-with-locality rule */
} insp_policy;

/* Pop rule in force at a pop (mode_at_pop) and in trace records. */
typedef enum {
    INSP_MODE_ABILITY = 0, /* highest IA, then highest IE, then earliest push */
    INSP_MODE_EFI = 1,     /* highest IE, then highest IA, then earliest push */
    INSP_MODE_EFI_LOC = 2, /* efficiency with locality: with the data model the tasks whose inputs
                              have arrived first, then as EFI; without it, as EFI */
    INSP_MODE_FIFO = 3,    /* earliest push */
    INSP_MODE_RANK = 4     /* highest HEFT upward rank, then earliest push */
} insp_mode;

#define INSP_ALL_DAGS (-1)
#define INSP_MAX_TASKS (1 << 21)
#define INSP_MAX_TICK (1 << 20)
#define INSP_MAX_WORKERS 1024
#define INSP_MAX_TRANSITIVE_TASKS (1 << 15)

/* Which reading of the attributes orders the queues (insp_params.attr_mode). */
typedef enum {
    INSP_ATTR_DIRECT = 0,    /* IA = out-degree, IE over successors at the current in-degrees */
    INSP_ATTR_TRANSITIVE = 1 /* fixed IA_T, IE_T of insp_transitive_attributes */
} insp_attr_mode;

/* Opaque, library-owned device copy of B >= 1 canonical DAGs. */
typedef struct insp_dag insp_dag;

typedef struct {
    int32_t n_cpu, n_gpu;
} insp_workers;

/*
 * Scheduling parameters.  The regulator parameters are the ones named in the
 * Section 4.4 pseudocode; the paper prints no values, so a field <= 0 (c < 0;
 * k_num or k_den <= 0 for the pair) selects the default, with W workers and
 * tau_bar = max(1, floor(mean GPU estimate)) (CPU estimate without GPUs):
 *   s_inc    task window / ascending step          default ceil(W/4)
 *   s_dec    descending step of the peak threshold default ceil(W/2)
 *   dec_step INC/DEC margin below the peak         default s_dec
 *   c        slack of the descending test          default floor(s_dec/2)
 *   k_num/k_den  expected ascending slope k_inc    default W / tau_bar
 * unit_time is IE's unit time U in ticks (0 = automatic ladder, Section 4.3).
 * max_events bounds the simulation's event count (0 = n + 1, the most a
 * correct run can need); exceeding it returns INSP_E_HANG.
 * k_num and k_den must not exceed 2^20.
 * attr_mode picks the attribute reading the queues are ordered by: with
 * INSP_ATTR_TRANSITIVE the keys are IA_T and IE_T (insp_transitive_attributes,
 * unit_time being their window U), fixed for the run.
 * data_bw > 0 turns on the data model (Section 2: DMDA weighs data transfers
 * and the push starts them; Section 4.4: the efficiency-with-locality rule).
 * The handle needs per-task output sizes (insp_set_task_data).  Memory node
 * of a worker: the host for CPU workers, its own memory for each GPU worker.
 * Task u leaves one output item of data_kib[u] KiB on its worker's node (not
 * replicated); a consumer on another node moves it in
 * ceil(1024 data_kib[u] / data_bw) ticks.  The push cost adds X(v, w), the
 * ticks of v's inputs not on w's node; the queue length still grows by the
 * estimate alone (the transfers start at the push and overlap other work);
 * v's inputs arrive at t + X(v, chosen worker), and a popped task starts when
 * they have arrived (its worker waits).  X above 2^20 ticks fails the DAG
 * with INSP_E_RANGE at insp_sync_status.
 */
typedef struct {
    int32_t policy;
    int32_t unit_time;
    int32_t s_inc, s_dec, dec_step, c, k_num, k_den;
    int32_t max_events;
    int32_t attr_mode; /* insp_attr_mode; TRANSITIVE needs DAGs of <= INSP_MAX_TRANSITIVE_TASKS */
    int32_t data_bw;   /* data model: bytes moved per tick between memory nodes; 0 = no data model */
} insp_params;

/* One record per simulation event: the Nready the regulator observed (after
 * the pushes of the event, before its pops), the rule then in force, the
 * regulator's decrement count and peak, and the tasks pushed and popped. */
typedef struct {
    int64_t t;
    int32_t nready, mode, cnt, peak, pushed, popped;
} insp_trace_rec;

/*
 * insp_build_dag -- copy B DAGs to library-owned device memory in canonical
 * form (Section 2: tasks are vertices, dependencies are edges; Section 4.3:
 * traversal from the tasks with zero in-degree).
 *   n_dags    B >= 1
 *   task_off  host int64 [B+1], prefix sums of task counts (task_off[0] = 0)
 *   edge_off  host int64 [B+1], prefix sums of edge counts
 *   row_ptr   device int32, DAG b's local CSR row pointer of n_b + 1 entries
 *             starts at element task_off[b] + b; row_ptr values are local
 *             (0 .. m_b)
 *   col       device int32 [edge_off[B]], successor ids local to their DAG
 *   type      device int32 [task_off[B]] task kind (stored, may be NULL)
 *   out       receives the handle; free it with insp_free_dag
 * Rows are sorted and repeated edges merged on the device.  Errors:
 * INSP_E_INVAL for a non-monotone row pointer, an id out of range or a self
 * loop; INSP_E_CYCLE for a cycle; INSP_E_RANGE for n_b > 2^21.  The call
 * synchronises `stream` to report these.  The caller keeps its buffers.
 * The handle lives on the device current at this call; the calls that take
 * it make that device current before they launch.
 */
int insp_build_dag(int32_t n_dags, const int64_t *task_off, const int64_t *edge_off, const int32_t *row_ptr,
                   const int32_t *col, const int32_t *type, void *stream, insp_dag **out);

/*
 * insp_set_task_data -- attach per-task output sizes to a handle for the data
 * model (see insp_params.data_bw).
 *   data_kib  device int32 [task_off[B]], KiB of each task's output item, in
 *             [0, 2^20]; copied (the caller keeps its buffer); NULL detaches
 * INSP_E_RANGE for a size out of range.  The call synchronises `stream`.
 */
int insp_set_task_data(insp_dag *dag, const int32_t *data_kib, void *stream);

/* Release a handle from insp_build_dag (NULL is ignored).  The caller must
 * make sure no work using it is still running. */
void insp_free_dag(insp_dag *dag);

/* Task and edge counts of DAG `dag` after canonicalisation (host outputs). */
int insp_dag_info(const insp_dag *dag, int32_t index, int64_t *n_tasks, int64_t *n_edges, int32_t *n_dags);

/*
 * insp_attributes -- inspiring ability and efficiency of every task
 * (Section 4.2 definitions, Section 4.3 computation).
 *   IA(v) = out-degree of v: the dependencies v's completion resolves.
 *   IE(v) = #{successors s : rem[s] == 1 and tau(v) + tau(s) <= U}: the
 *           successors v's completion makes ready that can also finish
 *           within U of v's start, tau being the GPU estimate (the CPU
 *           estimate if the machine has no GPU worker).
 *   U     = unit_time if > 0, else the automatic choice: among U = 2^j,
 *           j = 0..J with 2^J the first power of two >= 2 max tau, the U that
 *           maximises #{v : 0 < IE(v) < IA(v)} (larger U on a tie).
 *   dag         index of one DAG, or INSP_ALL_DAGS for every DAG
 *   est         device int32 [n][2] estimates of the selected task range
 *   workers     host, one entry (or B entries for INSP_ALL_DAGS)
 *   rem         device int32 [n] remaining in-degrees, or NULL for the
 *               initial in-degrees; the ladder is scored at this rem
 *   ia, ie      device int32 [n] outputs
 *   unit_time_used host int32 [1] (or [B]) output; the call synchronises
 *               `stream` to fill it
 * Task ranges are DAG-local: index 0 is the first task of the selected DAG
 * (of DAG 0 for INSP_ALL_DAGS, the DAGs then following back to back).
 */
int insp_attributes(const insp_dag *dag, int32_t index, const int32_t *est, const insp_workers *workers,
                    int32_t unit_time, const int32_t *rem, int32_t *ia, int32_t *ie, int32_t *unit_time_used,
                    void *stream);

/*
 * insp_transitive_attributes -- the transitive reading of the attributes
 * (Section 4.3: the source of a fully connected DAG scores the number of its
 * tasks; Section 4.2: with a large unit time IE converges to IA; Section 7:
 * IE looks at a time window after the task), on the whole graph:
 *   D(v)       = v and every task reachable from v;
 *   IA_T(v)    = |D(v)|;
 *   EF_v(d)    = the longest tau-weighted path from v to d, both ends
 *                included (d's earliest finish when v starts at 0 on
 *                unlimited workers), tau as for insp_attributes;
 *   IE_T(v; U) = #{d in D(v) : EF_v(d) <= U}.
 *   U = unit_time if > 0, else the ladder U = 2^j, j = 0..J, 2^J the first
 *       power of two at least the DAG's longest path, maximising
 *       #{v : 0 < IE_T(v) < IA_T(v)} (the larger U on a tie).
 *   index, est, workers, ia, ie   as for insp_attributes (no rem: the
 *                                 attributes are fixed for a run)
 *   unit_time_used host int32 [1] (or [B]) output
 *   longest_path   host int64 [1] (or [B]) output, nullable
 * The call synchronises `stream`.  INSP_E_RANGE for a DAG of more than
 * INSP_MAX_TRANSITIVE_TASKS tasks, a longest path of 2^30 ticks or more, or
 * an estimate out of range.  Cost: one pass over D(v) per task, O(n (n + m))
 * per DAG at worst.  The first call on a handle builds the DAGs' level order.
 */
int insp_transitive_attributes(const insp_dag *dag, int32_t index, const int32_t *est, const insp_workers *workers,
                               int32_t unit_time, int32_t *ia, int32_t *ie, int32_t *unit_time_used,
                               int64_t *longest_path, void *stream);

/*
 * insp_schedule -- simulate one DAG on the given workers (Section 2 DMDA
 * push, Section 4.1 per-worker queues, Section 4.4 adaptive pop rule).
 * Integer time; at each event time, in this order: newly ready tasks are
 * pushed in ascending id to the worker minimising expected free time +
 * queued estimates + own estimate (ties to the lowest worker id); the
 * regulator observes Nready (queued tasks, running ones excluded); every
 * idle worker pops the top task of its own queue under the current rule,
 * with IE taken at the current remaining in-degrees; time advances to the
 * next completion, whose successors' dependencies are released.  Decisions
 * use `est`, time advances with `dur`.
 *   dur, est     device int32 [n][2] of this DAG
 *   worker       device int32 [n] output: worker that ran each task
 *   start,finish device int64 [n] outputs
 *   makespan     device int64 [1] output
 *   ie_at_pop    device int32 [n] output, IE when popped (nullable)
 *   mode_at_pop  device int8 [n] output, rule of that pop (nullable)
 *   trace        device insp_trace_rec [max_events or n+1] (nullable)
 *   n_events     device int32 [1] output: events simulated (nullable)
 * INSP_E_HANG is detected on the device and reported by the next
 * insp_sync_status(); the call itself returns once the work is enqueued.
 */
int insp_schedule(const insp_dag *dag, int32_t index, const insp_workers *workers, const int32_t *dur,
                  const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start, int64_t *finish,
                  int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop, insp_trace_rec *trace,
                  int32_t *n_events, void *stream);

/*
 * insp_schedule_batch -- insp_schedule for all B DAGs of the handle in one
 * persistent launch (workgroups take DAGs, largest first, from an atomic
 * counter).  Arrays are indexed by the global task id (task_off of the
 * handle); makespan is [B].  workers is host [B].  tune_key selects a
 * launch configuration: NULL = the library's default for this device, or a
 * comma-separated string of "grid=<g>" (persistent work-groups, each one
 * wave simulating one DAG at a time), "lds_blocks=<b>" (queue blocks per DAG
 * whose maxima live in LDS, <= 8192), "lds_slots=<s>" (queue blocks per DAG
 * whose entries live in LDS), "lds_keys=<k>" (queue blocks per DAG whose
 * keys live in LDS, at least lds_slots: a pop's scan reads only keys; the
 * default is 128 maxima, 24 full blocks and keys of 40, with three
 * work-groups per CU), "prio=<k>" (the k largest DAGs run at raised
 * wave priority), "scan=<k>" (<= 16: a pop reads every queue entry of a
 * worker with at most k queue blocks, and picks a block by its maximum
 * first above that) and "waves=1" (the only accepted value; any other is
 * INSP_E_INVAL).  Each work-group of the launch is one wave that simulates
 * and, for machines of at most 64 workers, one that reads ahead for it.
 * Results never depend on the key.  The first call with a new machine shape
 * allocates workspace; later calls reuse it.
 */
int insp_schedule_batch(const insp_dag *dag, const insp_workers *workers, const int32_t *dur, const int32_t *est,
                        const insp_params *params, int32_t *worker, int64_t *start, int64_t *finish,
                        int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop, const char *tune_key,
                        void *stream);

/*
 * insp_schedule_batch_trace -- insp_schedule_batch that also records every
 * DAG's per-event trace (the Nready analysis of the paper's Section 5, per
 * DAG of the batch).  trace is device insp_trace_rec [N + B] (N = tasks of
 * the handle): DAG b's records start at index task_off[b] + b and number
 * min(n_events[b], max_events or n_b + 1) -- a run takes at most n_b + 1
 * events, so n_b + 1 slots always suffice.  n_events is device [B]: the
 * events of each DAG's run (max_events + 1 when the run stopped at the
 * max_events limit, which insp_sync_status reports as INSP_E_HANG; 0 for an
 * empty DAG).  Both arrays are caller-owned and required (NULL is
 * INSP_E_INVAL); every other argument, result and error is as for
 * insp_schedule_batch.
 */
int insp_schedule_batch_trace(const insp_dag *dag, const insp_workers *workers, const int32_t *dur,
                              const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start,
                              int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                              insp_trace_rec *trace, int32_t *n_events, const char *tune_key, void *stream);

/*
 * insp_schedule_batch_noalloc -- insp_schedule_batch for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, results and status
 * reporting (insp_sync_status) as insp_schedule_batch; the caller passes the
 * inputs and outputs as before.  The call allocates nothing: the per-call
 * state -- task records (32 B per task), dependency words (8 B per task),
 * frontier buffers (12 B per task),
 * per-DAG attribute records and launch tables, and the queue pools (about
 * 2,076 B per 64-task block, ceil(n/64) + W blocks and 4 W (ceil(n/64) + 1) B
 * of block lists per DAG of n tasks on W workers) -- is carved out of one
 * static device array of INSP_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds from the first call on that GPU until the process ends.  A
 * batch needing more fails with INSP_E_RANGE before any device work.  Only
 * the direct attributes without the data model are served (policies
 * INSPIRIT, FIFO, ABILITY_ONLY and EFI_ONLY, attr_mode DIRECT, data_bw 0);
 * the HEFT and locality policies, transitive attributes and the data model
 * build handle state on first use and are INSP_E_INVAL here.  The launch
 * tables are uploaded (and the stream synchronised) only when the handle or
 * the machine shape differs from the previous call's on the same GPU.  All
 * calls on one GPU share the array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.
 */
#define INSP_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int insp_schedule_batch_noalloc(const insp_dag *dag, const insp_workers *workers, const int32_t *dur,
                                const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start,
                                int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                                const char *tune_key, void *stream);

/*
 * The batch step as a HIP graph the library owns (batching in one launch
 * replayed without per-call host work).  insp_batch_graph_create takes the
 * arguments of insp_schedule_batch: it runs one eager step on `stream`
 * (which builds every buffer made on first use and synchronises the stream),
 * then captures the same step -- the attribute pass, the persistent
 * simulation and the unpacking of the schedules, kernel launches only -- on a
 * stream of its own.  Each insp_batch_graph_launch enqueues one replay on
 * `stream`, reading the input arrays given at creation and writing the same
 * output arrays (update their contents in place between replays, never
 * their addresses); failures are reported by insp_sync_status as for an
 * eager call.  The handle and every array must outlive the graph, and the
 * handle must not be used by other calls while a replay runs.
 * insp_batch_graph_free releases the graph (NULL is ignored).
 */
typedef struct insp_graph insp_graph;
int insp_batch_graph_create(const insp_dag *dag, const insp_workers *workers, const int32_t *dur,
                            const int32_t *est, const insp_params *params, int32_t *worker, int64_t *start,
                            int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                            const char *tune_key, void *stream, insp_graph **out);
int insp_batch_graph_launch(insp_graph *graph, void *stream);
void insp_batch_graph_free(insp_graph *graph);

/* Synchronise `stream` and report a device-side failure of the schedule
 * calls (insp_schedule, insp_schedule_batch) enqueued on the handle since the
 * last check: INSP_E_HANG, or INSP_E_RANGE for a tick value out of range, a
 * HEFT rank >= 2^42, a longest path >= 2^30 under transitive attributes or
 * input transfers above 2^20 ticks.  Failures are kept across later schedule
 * calls until this call reports them (the first one found is returned, and
 * all are cleared).  A DAG that failed before its simulation started (an
 * estimate, HEFT rank or longest path out of range) has makespan -1 and its
 * other outputs untouched; one that hung has makespan -1 and its other
 * outputs unspecified, as are the outputs of a DAG with a duration or a
 * transfer out of range.  The standalone attribute calls report their own
 * failures and do not affect this one. */
int insp_sync_status(const insp_dag *dag, void *stream);

/*
 * Kernel timing (for benchmarks and tuning).  While enabled, every kernel the
 * library launches is bracketed by HIP events recorded on the caller's
 * stream; insp_profile_read waits for the recorded events and returns the
 * summed elapsed time and launch count of the kernels whose name starts with
 * `kernel` ("sim", "attr_a", "attr_b", "attr_select", "" for all).
 * insp_profile_enable(0) stops recording and drops pending records;
 * insp_profile_enable(2) records only the outermost scope of each call (the
 * whole attribute pass, the simulation, the unpacking), so that no event
 * record sits between the kernels it brackets.  The recorder is process-wide
 * and not meant for concurrent streams.
 */
int insp_profile_enable(int on);
int insp_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/*
 * Learned cost model (an extension of the paper's per-type average
 * execution times, Section 4.3): a 32 -> 256 -> 256 -> 2 ReLU network that
 * predicts ln(duration) on the CPU and GPU worker kinds from 32 task
 * features.  Weights, activations and activation gradients are bfloat16,
 * accumulation, biases, outputs, gradients and the Adam state are fp32.
 * Parameters are packed as W1 [32][256], b1 [256], W2 [256][256], b2 [256],
 * W3 [256][2], b3 [2] (row-major, INSP_MLP_PARAMS floats).
 *   insp_mlp_create     copy host fp32 initial parameters to a new model
 *   insp_mlp_grads      loss (mean squared error over batch x 2 outputs) and
 *                       its gradients for one batch, without updating; x is
 *                       device fp32 [batch][32], t device fp32 [batch][2]
 *                       (targets in ln ticks); grads device fp32 [PARAMS],
 *                       y device fp32 [batch][2], loss device fp32 [1]
 *                       (each nullable)
 *   insp_mlp_train_step the same gradients followed by one Adam step
 *                       (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr)
 *   insp_mlp_train      `epochs` passes over rows [0, n) of device x [n][32]
 *                       and t [n][2] in minibatches of `batch` rows (the
 *                       last n mod batch rows are not used): the same result,
 *                       bit for bit, as one insp_mlp_train_step per
 *                       minibatch in order, with the steps replayed from a
 *                       captured HIP graph of up to 32 steps.  loss (device,
 *                       nullable) receives the last step's loss.  At most
 *                       2^28 steps per call (INSP_E_RANGE); n < batch or
 *                       epochs == 0 does nothing.  The graph is kept with
 *                       the model and captured again when x, t, the step
 *                       count, batch or lr change.  Host-synchronizes with
 *                       `stream` once, at the start, while it uploads the
 *                       step table.
 *   insp_mlp_predict    y = network(x) for n rows and/or integer estimates
 *                       est = clamp(rint(exp(y)), 1, 2^20), int32 [n][2];
 *                       x must be 16-byte aligned (INSP_E_INVAL otherwise)
 *   insp_mlp_state      copy parameters, Adam moments and step count to the
 *                       host (to_host = 1) or from it (to_host = 0), for
 *                       checkpoint and resume; any pointer may be NULL
 * batch must be a positive multiple of 32.  Work runs on `stream`.  The
 * model lives on the device current at insp_mlp_create, and grads,
 * train_step, train and predict fail with INSP_E_INVAL when another device
 * is current.  Calls on one model share its buffers and must not overlap;
 * insp_mlp_free waits for the device before it releases them.
 */
#define INSP_MLP_PARAMS 74754
typedef struct insp_mlp insp_mlp;
int insp_mlp_create(const float *params, insp_mlp **out);
void insp_mlp_free(insp_mlp *m);
int insp_mlp_grads(insp_mlp *m, const float *x, const float *t, int32_t batch, float *grads, float *y, float *loss,
                   void *stream);
int insp_mlp_train_step(insp_mlp *m, const float *x, const float *t, int32_t batch, float lr, float *loss,
                        void *stream);
int insp_mlp_train(insp_mlp *m, const float *x, const float *t, int64_t n, int32_t batch, int32_t epochs, float lr,
                   float *loss, void *stream);
int insp_mlp_predict(insp_mlp *m, const float *x, int64_t n, float *y, int32_t *est, void *stream);
int insp_mlp_state(insp_mlp *m, float *params, float *adam_m, float *adam_v, int64_t *step, int to_host);

/* Thread-local description of the last non-OK status. */
const char *insp_last_error(void);

/*
 * Testing hook for the allocation-failure paths: after `after` more device
 * allocations made by the library succeed, the next one fails as if the
 * device were out of memory (the call making it returns INSP_E_NOMEM), and
 * injection then stops.  -1 turns injection off.  Process-wide; INSP_E_INVAL
 * for after < -1.
 */
int insp_test_fail_alloc(int64_t after);

#ifdef __cplusplus
}
#endif

#endif /* INSPIRIT_H */
