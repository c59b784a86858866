// Allocation-free batch schedule call (insp_schedule_batch_noalloc).
//
// The batch call's per-call state -- task records, frontier buffers, per-DAG
// attribute records, the launch tables and the queue pools -- is carved out
// of one static device array instead of memory the library allocates.  The
// array exists once per GPU (each device holds its own copy at its own
// address); host code never passes the array's name to a kernel, only the
// device address hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace insp {
namespace {

constexpr size_t kScratchBytes = (size_t)INSP_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// What one GPU's copy of the array holds.
struct DeviceScratch {
    unsigned char *ptr = nullptr;      // device address of `scratch` on this GPU
    uint64_t serial = 0;               // handle whose launch tables are resident (0: none)
    std::vector<int32_t> shape;        // machine shape of the resident tables (n_cpu, n_gpu per DAG)
    Workspace ws;                      // views into the array
};

std::mutex g_mu;
std::map<int, std::unique_ptr<DeviceScratch>> g_dev;

// The array's address on `device` (current), looked up once per device.
int device_scratch(int device, DeviceScratch **out) {
    auto it = g_dev.find(device);
    if (it == g_dev.end()) {
        std::unique_ptr<DeviceScratch> ds(new DeviceScratch());
        void *p = nullptr;
        INSP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(INSP_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        ds->ptr = static_cast<unsigned char *>(p);
        it = g_dev.emplace(device, std::move(ds)).first;
    }
    *out = it->second.get();
    return INSP_OK;
}

// Lay the batch's per-call state out in the array and upload the launch
// tables, unless the array already holds this handle's tables for this
// machine shape.
int prepare(insp_dag *dag, const insp_workers *workers, DeviceScratch *ds, hipStream_t st) {
    std::vector<int32_t> shape(2 * (size_t)dag->B);
    for (int32_t b = 0; b < dag->B; b++) {
        shape[2 * b] = workers[b].n_cpu;
        shape[2 * b + 1] = workers[b].n_gpu;
    }
    if (ds->serial == dag->serial && ds->shape == shape) return INSP_OK;
    ds->serial = 0;
    Workspace &w = ds->ws;
    w.max_w = 0;
    w.max_nblk = 0;
    w.max_small = 0;
    std::vector<DagDesc> desc;
    const int64_t boff = workspace_shape(dag, 0, dag->B, workers, true, &w, &desc);
    const size_t N = (size_t)std::max<int64_t>(dag->N, 1), B = (size_t)dag->B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_tr = take(sizeof(TaskRec) * N), o_dep = take(8 * N), o_fbuf = take(12 * N);
    const size_t o_u = take(4 * B), o_taubar = take(4 * B), o_maxtau = take(4 * B), o_tausum = take(8 * B);
    const size_t o_score = take(4 * kRungs * B), o_done = take(4 * B);
    const size_t o_desc = take(sizeof(DagDesc) * B), o_order = take(4 * B), o_sorder = take(4 * B);
    const size_t o_apart = take(4 * 32 * kBigGrid);
    const size_t big = (size_t)large_rows(dag), o_apkg = take(4 * big), o_asumm = take(8 * big);
    const size_t o_slots = take(sizeof(Slot) * 64 * (size_t)boff), o_sums = take(16 * (size_t)boff);
    const size_t o_paux = take(4 * (size_t)(w.total_wl + boff)), o_barr = take(8 * (size_t)boff);
    const size_t o_counter = take(16);
    if (off > kScratchBytes)
        return set_error(INSP_E_RANGE,
                         "insp_schedule_batch_noalloc: the batch needs %zu bytes of scratch, the static array "
                         "holds %zu (INSP_NOALLOC_SCRATCH_BYTES)",
                         off, kScratchBytes);
    unsigned char *p = ds->ptr;
    w.tr = reinterpret_cast<TaskRec *>(p + o_tr);
    w.dep = reinterpret_cast<unsigned long long *>(p + o_dep);
    w.fbuf = reinterpret_cast<int32_t *>(p + o_fbuf);
    w.dag_u = reinterpret_cast<int32_t *>(p + o_u);
    w.dag_taubar = reinterpret_cast<int32_t *>(p + o_taubar);
    w.dag_maxtau = reinterpret_cast<int32_t *>(p + o_maxtau);
    w.dag_tausum = reinterpret_cast<unsigned long long *>(p + o_tausum);
    w.dag_score = reinterpret_cast<int32_t *>(p + o_score);
    w.dag_done = reinterpret_cast<int32_t *>(p + o_done);
    w.apart = reinterpret_cast<int32_t *>(p + o_apart);
    w.apkg = reinterpret_cast<uint32_t *>(p + o_apkg);
    w.asumm = reinterpret_cast<unsigned long long *>(p + o_asumm);
    w.desc.borrow(p + o_desc, sizeof(DagDesc) * B);
    w.order.borrow(p + o_order, 4 * B);
    w.sorder.borrow(p + o_sorder, 4 * B);
    w.slots.borrow(p + o_slots, sizeof(Slot) * 64 * (size_t)boff);
    w.sums.borrow(p + o_sums, 16 * (size_t)boff);
    w.paux.borrow(p + o_paux, 4 * (size_t)(w.total_wl + boff));
    w.barr.borrow(p + o_barr, 8 * (size_t)boff);
    w.counter.borrow(p + o_counter, 16);
    // the tables are read by kernels of earlier calls still queued on `st`:
    // the copies are ordered after them on the same stream, and the stream is
    // synchronised before the host vectors go away
    INSP_HIP(hipMemcpyAsync(w.desc.p, desc.data(), sizeof(DagDesc) * B, hipMemcpyHostToDevice, st));
    INSP_HIP(hipMemcpyAsync(w.order.p, w.h_order.data(), 4 * B, hipMemcpyHostToDevice, st));
    if (w.n_small > 0)
        INSP_HIP(hipMemcpyAsync(w.sorder.p, w.h_sorder.data(), 4 * (size_t)w.n_small, hipMemcpyHostToDevice, st));
    INSP_HIP(hipStreamSynchronize(st));
    ds->shape.swap(shape);
    ds->serial = dag->serial;
    return INSP_OK;
}

}  // namespace
}  // namespace insp

using namespace insp;

extern "C" int insp_schedule_batch_noalloc(const insp_dag *cdag, const insp_workers *workers, const int32_t *dur,
                                           const int32_t *est, const insp_params *params, int32_t *worker,
                                           int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
                                           int8_t *mode_at_pop, const char *tune_key, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    BatchLaunch bl;
    int rc;
    if ((rc = batch_prologue(dag, workers, dur, est, params, worker, start, finish, makespan, tune_key, &bl)))
        return rc;
    if (params->policy == INSP_POLICY_HEFT || params->policy == INSP_POLICY_LOCALITY ||
        params->attr_mode != INSP_ATTR_DIRECT || params->data_bw != 0)
        return set_error(INSP_E_INVAL,
                         "insp_schedule_batch_noalloc serves the direct attributes without the data model only "
                         "(policy %d, attr_mode %d, data_bw %d)",
                         params->policy, params->attr_mode, params->data_bw);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch *ds;
    if ((rc = device_scratch(dag->device, &ds))) return rc;
    if ((rc = prepare(dag, workers, ds, st))) return rc;
    if ((rc = run_attributes(dag, &ds->ws, est, params->unit_time, nullptr, nullptr, nullptr, true, st))) return rc;
    return launch_sim(dag, &ds->ws, *params, dur, est, worker, start, finish, makespan, ie_at_pop, mode_at_pop,
                      nullptr, nullptr, 1, bl.grid, bl.sum_cap, bl.slot_cap, bl.key_cap, st, bl.prio, bl.scan);
}
