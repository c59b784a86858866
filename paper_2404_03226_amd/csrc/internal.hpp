// Host-side internals of libinspirit: the DAG handle, per-shape launch
// workspaces and error reporting.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "inspirit.h"

namespace insp {

int set_error(int code, const char *fmt, ...);

#define INSP_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::insp::set_error(e_ == hipErrorOutOfMemory ? INSP_E_NOMEM : INSP_E_DEVICE, \
                                     "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

// Device memory owned by a handle or workspace, or borrowed from memory the
// library does not free (the static scratch array).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool own = true;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    int alloc(size_t nbytes);
    void release();
    // Point at `nbytes` of memory owned elsewhere; release() then forgets it.
    void borrow(void *q, size_t nbytes) {
        release();
        p = q;
        bytes = nbytes;
        own = false;
    }
    void swap(DevBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(own, o.own);
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Per-task simulation record (32 bytes, 32-byte aligned).  Bytes 16..31 are
// one aligned vector (IE, IA, tau, first edge) read together; bytes 8..15
// (queue slot, push order) likewise.  The dependency word lives apart, in a
// dense 8-byte array (the structure every release touches, kept small for
// the caches).  Once the task is popped, bytes 0..15 hold its schedule:
//   word = start | duration << 42,  qpos = -2 - worker,
//   seq  = IE at pop | mode << 22.
// While the task is queued under the data model, `word` holds the arrival
// time of its inputs.
struct TaskRec {
    unsigned long long word;  // schedule once popped (see above)
    int32_t qpos;             // queue slot; -1 before the push; <= -2 once popped
    int32_t seq;              // push sequence number once queued
    int32_t iev;              // current inspiring efficiency
    int32_t ia, tau, rs;      // out-degree, tau, first edge (fixed during a run)
};
static_assert(sizeof(TaskRec) == 32, "TaskRec layout");

// Queue slot: key word, payload word and the task's first edge (32 bytes of
// pool per slot, the size the allocators reserve).
struct Slot {
    unsigned long long k, x;
    int32_t rs, pad0;
    int32_t pad1, pad2;
};

// The global queue pool as three arrays -- keys, payloads, first edges --
// so that a pop's scan of a block's keys reads 512 contiguous bytes.
struct SlotPool {
    unsigned long long *k, *x;
    int32_t *rs;
    // the pool in `bytes` of memory sized as Slot [slots]
    __host__ __device__ static SlotPool over(void *p, size_t bytes) {
        const size_t n = bytes / sizeof(Slot);
        SlotPool s;
        s.k = static_cast<unsigned long long *>(p);
        s.x = s.k + n;
        s.rs = reinterpret_cast<int32_t *>(s.x + n);
        return s;
    }
    __host__ __device__ SlotPool at(int64_t off) const {
        SlotPool s;
        s.k = k + off;
        s.x = x + off;
        s.rs = rs + off;
        return s;
    }
};

// One DAG of a launch, as the kernels see it.
struct DagDesc {
    int64_t toff, eoff;   // first global task / edge
    int64_t blk_off;      // first queue block of the DAG's pool
    int64_t wl_off;       // first slot of the DAG's worker block lists
    int32_t id;           // DAG index in the handle
    int32_t n, m;
    int32_t n_cpu, n_gpu;
    int32_t nblk, maxb;   // blocks in the pool; block-list slots per worker
    int32_t path;         // attribute pass: 0 = one work-group per DAG, 1 = the whole grid (large DAG)
    int32_t hub0, nhub;   // large DAG: its hub rows (first index in the handle's list, count)
    int32_t long0, nlong; // ... and those cut into pieces
};

// Launch state for one machine shape (DAG range and worker counts): the
// kernels' DAG descriptors, the attribute and simulation orders and the
// queue pools.  Built once, reused by every call with the same shape.
struct Workspace {
    int32_t count = 0;            // DAGs described
    int32_t first = 0;            // first DAG of the range
    int32_t max_w = 0;
    int64_t max_nblk = 0;
    int64_t base = 0;             // first global task of the range
    int64_t total_wl = 0;         // block-list slots before the free-block stacks in paux
    int64_t tasks = 0;
    int32_t n_small = 0;          // non-empty DAGs of the per-DAG attribute pass
    int32_t max_small = 0;        // tasks of the largest of them
    DevBuf desc;                  // DagDesc [count]
    DevBuf order;                 // int32 [count]: desc indices, largest first
    DevBuf sorder;                // int32 [n_small]: desc indices of the per-DAG pass, largest first
    DevBuf slots;                 // Slot [64 per block]: queue entries
    DevBuf sums;                  // uint64 x2 per block: max key under each rule
    DevBuf paux;                  // int32: per-worker block lists, then free-block stacks
    DevBuf barr;                  // int64 per block: latest input arrival (data model)
    DevBuf counter;               // int32 [4]: DAG dispenser
    DevBuf tlong, tu;             // transitive attributes: longest path per DAG (+ a counter), chosen U
    std::vector<int32_t> h_order, h_sorder;
    std::vector<int32_t> h_large;      // desc indices of the DAGs of the grid-wide attribute pass
    std::vector<DagDesc> h_desc;
    // Per-call state the attribute pass and the simulation write, indexed by
    // global task or DAG id: the handle's buffers, or regions of the static
    // scratch array for the allocation-free batch call.
    TaskRec *tr = nullptr;             // [N]
    unsigned long long *dep = nullptr; // [N]: dependency words (remaining in-degree << 43 | sum of unfinished predecessors)
    int32_t *fbuf = nullptr;           // [3 N]
    int32_t *dag_u = nullptr, *dag_taubar = nullptr, *dag_maxtau = nullptr;  // [B]
    int32_t *dag_score = nullptr;      // [B * kRungs]
    unsigned long long *dag_tausum = nullptr;  // [B]
    int32_t *dag_done = nullptr;       // [B]: finished blocks of the grid-wide attribute pass
    int32_t *apart = nullptr;          // [kBigGrid * 32]: its per-block partial results
    uint32_t *apkg = nullptr;          // [rows of the largest large DAG]: its task words
    unsigned long long *asumm = nullptr;  // [same]: its rows' pass-A summaries
};

}  // namespace insp

struct insp_dag {
    int32_t B = 0;
    int device = 0;
    uint64_t serial = 0;               // unique per handle in the process
    int64_t N = 0, M = 0;
    std::vector<int64_t> toff, eoff;   // canonical prefix sums (host)
    std::vector<int32_t> order;        // DAG ids by n + m descending
    insp::DevBuf d_toff, d_eoff;       // int64 [B+1]
    insp::DevBuf rp;                   // int32 [N + B] local canonical row pointers
    insp::DevBuf col;                  // int32 [M] canonical successor lists
    insp::DevBuf type;                 // int32 [N] (may be empty)
    insp::DevBuf word0;                // uint64 [N] in-degree << 43 | sum of predecessor ids
    // per-task simulation state, shared by every shape (allocated on first use)
    insp::DevBuf tr;                   // TaskRec [N]
    insp::DevBuf dep;                  // uint64 [N]: dependency words of the simulation
    insp::DevBuf fbuf;                 // int32 [3 N]: frontier runs, merged frontier, candidates
    // per-DAG attribute and status records
    insp::DevBuf dag_u, dag_taubar;    // int32 [B]
    insp::DevBuf dag_maxtau;           // int32 [B]
    insp::DevBuf dag_tausum;           // int64 [B]
    insp::DevBuf dag_score;            // int32 [B * 24] ladder score, difference form
    insp::DevBuf dag_done;             // int32 [B]: finished blocks of the grid-wide attribute pass
    insp::DevBuf apart;                // int32 [kBigGrid * 32]: its per-block partial results
    insp::DevBuf apkg;                 // uint32 [rows of the largest large DAG]: task words of the grid pass
    insp::DevBuf asumm;                // uint64 [same]: pass-A row summaries of the grid pass
    // large DAGs (at least kGridMin tasks): rows with more than kHubDeg
    // successors, longest first (built with the handle)
    std::vector<int32_t> hub0, nhub;   // per DAG: first entry, entries
    insp::DevBuf hub;                  // int4 [entries]: DAG-local row, piece, pieces, first piece slot
    insp::DevBuf pslot;                // int32 [4 * entries]: partial results of the pieces of long rows
    std::vector<int32_t> long0, nlong; // per DAG: first long row, long rows
    insp::DevBuf lrow;                 // int4 [long rows]: row, 0, pieces, first piece slot
    // status words (allocated with the handle)
    insp::DevBuf dag_stat;             // int32 [B * 2]: status of the current schedule call, events
    insp::DevBuf dag_astat;            // int32 [B * 2]: status of the current attribute-only call
    insp::DevBuf dag_sticky;           // int32 [B]: schedule failures not yet reported by insp_sync_status
    // HEFT: topological levels (built on first use) and upward ranks
    insp::DevBuf topo;                 // int32 [N]: each DAG's tasks in level order
    insp::DevBuf lvl;                  // int32 [N + B]: start of each level in topo, then the end
    insp::DevBuf nlev;                 // int32 [B]: levels per DAG
    insp::DevBuf rank;                 // int64 [N]: upward rank of the last HEFT call
    // transitive attributes: positions in level order (built on first use),
    // per-call tau by position and ladder counts, attributes for the simulation
    insp::DevBuf prow;                 // int2 [N]: row of the task at each position
    insp::DevBuf plev;                 // int32 [N]: level of each position
    insp::DevBuf pcol;                 // int32 [M]: position of each edge's target
    insp::DevBuf ptau;                 // int32 [N]: tau by position
    insp::DevBuf pedge;                // int2 [M]: each edge's target position and its tau
    insp::DevBuf tcum;                 // int32 [N * kTRungs]: members within 2^j
    insp::DevBuf tia, tie;             // int32 [N]: transitive IA, IE of the last schedule call
    // data model: output KiB per task (insp_set_task_data), predecessor lists
    insp::DevBuf dkib;                 // int32 [N]
    insp::DevBuf pprp;                 // int32 [N + B]: local predecessor row pointers (as rp)
    insp::DevBuf ppred;                // int32 [M]: predecessor ids (local)
    insp::DevBuf dxc;                  // int32 [N]: transfer ticks of each output (per run)
    std::map<std::string, std::unique_ptr<insp::Workspace>> ws;
};

namespace insp {

constexpr int kRungs = 24;       // ladder rungs 2^0 .. 2^22 plus a sentinel

// Per-DAG status bits (dag_stat[2 b]): estimate or duration out of range, the
// event budget exhausted, a HEFT rank too wide for the queue key.
enum { ST_EST = 1, ST_DUR = 2, ST_HANG = 4, ST_RANK = 8, ST_PATH = 16, ST_XFER = 32 };
constexpr int kRankBits = 42;
constexpr int kTRungs = 32;  // transitive ladder rungs 2^0 .. 2^31
constexpr int kAttrThreads = 256;
constexpr int32_t kGridMin = 32768;  // DAGs this large take the grid-wide attribute pass
constexpr int32_t kHubDeg = 64;      // ... where rows with more successors get a wave each
constexpr int32_t kPieceMin = 1024;  // ... or, this long, one wave per piece
constexpr int32_t kPiece = 512;      // successors per piece
constexpr int kBigGrid = 2048;       // work-groups of the grid-wide pass

// Hub rows of the handle's large DAGs (insp_build_dag).
int build_hubs(insp_dag *dag, hipStream_t st);

int ensure_state(insp_dag *dag, hipStream_t st);

// Tasks of the handle's largest DAG of the grid-wide attribute pass (0: none).
int32_t large_rows(const insp_dag *dag);

// The handle's status words, zeroed (called once, by insp_build_dag).
int alloc_status(insp_dag *dag);

// Raise a kernel's dynamic LDS limit to at least `bytes` on the current
// device, once: later launches of the same size make no attribute call (so a
// warmed-up call can be captured in a graph).
int set_lds_limit(const void *kernel, size_t bytes);

// Kernel timing hook: brackets a launch with events when profiling is on.
void prof_mark(hipStream_t st, const char *kernel, bool begin);
// Stop (true) or resume (false) the calling thread's marks (graph capture).
void prof_suspend(bool on);
struct ProfScope {
    hipStream_t st;
    const char *name;
    ProfScope(hipStream_t s, const char *n) : st(s), name(n) { prof_mark(st, name, true); }
    ~ProfScope() { prof_mark(st, name, false); }
};

// Workspace for DAGs [first, first + count) with per-DAG workers (host).
int get_workspace(insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers, bool per_dag,
                  Workspace **out);

// The host side of a workspace: sizes, simulation order, the DAG descriptors
// (no device memory touched).  total_wl and the
// returned block count size the queue pools.
int64_t workspace_shape(const insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers,
                        bool per_dag, Workspace *w, std::vector<DagDesc> *desc);

// Attribute pipeline over a workspace's DAGs: per-DAG max and sum of tau,
// ladder scores (unit_time == 0), the chosen U, then IA and IE.  User arrays
// are indexed relative to the workspace's first task.  With `sim_init` the
// per-task simulation records are reset as well.
int run_attributes(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, const int32_t *rem,
                   int32_t *ia_out, int32_t *ie_out, bool sim_init, hipStream_t st);

// HEFT upward ranks of a workspace's DAGs into dag->rank (levels are built
// on the first call).  Runs after run_attributes, which clears the status.
int run_rank(insp_dag *dag, Workspace *ws, const int32_t *est, hipStream_t st);

// Exclusive prefix sum of n values into out[0 .. n] (out[n] = the total),
// enqueued on `st` (the call may synchronise `st` before it returns).
int exclusive_scan(const int32_t *in, int64_t n, int64_t *out, hipStream_t st);
int exclusive_scan(const int64_t *in, int64_t n, int64_t *out, hipStream_t st);

// Predecessor lists of every DAG of the handle (built once).
int ensure_preds(insp_dag *dag, hipStream_t st);

// Kahn levels of every DAG of the handle (built once).
int ensure_levels(insp_dag *dag, hipStream_t st);

// Transitive IA and IE of a workspace's DAGs into ia / ie (task-indexed
// relative to the workspace's first task); the chosen U per DAG lands in
// ws->tu, the longest path in ws->tlong.  With clear_status the DAGs' status
// words are reset first (a standalone call); a schedule keeps the bits the
// attribute pass set.
int run_transitive(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, int32_t *ia, int32_t *ie,
                   bool clear_status, hipStream_t st);

// Launch shape of a batch call.
struct BatchLaunch {
    int grid = 1, sum_cap = 0, slot_cap = 0, key_cap = 0, prio = 0, scan = 16;
};

// Argument checks and the launch shape of a batch schedule call (host only;
// makes the handle's device current).
int batch_prologue(insp_dag *dag, const insp_workers *workers, const int32_t *dur, const int32_t *est,
                   const insp_params *params, const int32_t *worker, const int64_t *start, const int64_t *finish,
                   const int64_t *makespan, const char *tune_key, BatchLaunch *launch);

int launch_sim(insp_dag *dag, Workspace *ws, const insp_params &p, const int32_t *dur, const int32_t *est,
               int32_t *worker, int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
               int8_t *mode_at_pop, insp_trace_rec *trace, int32_t *n_events, int waves, int grid,
               int sum_cap, int slot_cap, int key_cap, hipStream_t st, int prio_top, int scan_max);

}  // namespace insp
