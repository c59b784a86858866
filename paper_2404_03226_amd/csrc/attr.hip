// Inspiring ability and efficiency (Sections 4.2 and 4.3 of the paper).
//
//   IA(v) = out-degree of v.
//   IE(v) = #{ s in succ(v) : rem[s] == 1 and tau(v) + tau(s) <= U }, tau the
//           GPU estimate (CPU estimate on machines without GPU workers).
//   U     = given, or the ladder choice: U = 2^j for j = 0..J, 2^J the first
//           power of two >= 2 max tau, maximising #{v : 0 < IE(v) < IA(v)},
//           the larger U on a tie.
//
// Layout: one 256-thread block per 256-task chunk of one DAG (a host-built
// block map), so a block's ladder histogram belongs to a single DAG.  A task
// contributes to the score of rung j exactly when IE(v; 2^j) is positive but
// below IA(v): with x_s = tau(v) + tau(s) over successors with rem == 1,
// IE > 0 iff 2^j >= min x_s, and IE == IA iff every successor has rem == 1
// and 2^j >= max x_s.  So each task adds +1 at rung ceil(log2 min x) and -1 at
// rung ceil(log2 max x) (or never), a difference histogram that the select
// kernel integrates.  Pass A therefore reads every successor list once for
// all rungs; pass B reads it again to count IE at the chosen U.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "internal.hpp"

namespace insp {

__device__ __forceinline__ int ceil_log2(int32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// Work-groups are dealt to the 8 XCDs round-robin (block i runs on XCD i % 8),
// and each XCD has its own L2.  Give XCD x a contiguous run of the chunk list
// so the chunks of one DAG -- whose successor gathers hit the same few hundred
// KB -- share one L2.  Bijective for any grid size.
__device__ __forceinline__ int32_t xcd_chunk(int32_t i, int32_t nb) {
    const int32_t x = i & 7, k = i >> 3, q = nb >> 3, rmd = nb & 7;
    return x * q + min(x, rmd) + k;
}

struct AttrArgs {
    const DagDesc *desc;
    const int2 *blkmap;
    const int32_t *rp, *col;
    const unsigned long long *word0;
    const int32_t *est, *rem;   // user arrays, indexed relative to `base`
    int64_t base;
    int32_t unit_time;
    int32_t *maxtau, *score, *u, *taubar;
    int32_t *stat;    // this call's status words (stride 2)
    int32_t *sticky;  // schedule calls: failures of earlier calls kept for insp_sync_status (nullable)
    int32_t *anybad;  // [1]: some DAG of the call has an estimate out of range
    unsigned long long *tausum;
};

__global__ void k_attr_clear(AttrArgs a, int32_t count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *a.anybad = 0;
    if (i >= count * kRungs) return;
    int32_t id = a.desc[i / kRungs].id;
    int j = i % kRungs;
    a.score[id * kRungs + j] = 0;
    if (j == 0) {
        a.maxtau[id] = 0;
        a.tausum[id] = 0;
        // a schedule call keeps the previous call's failures until they are
        // reported: they move to the sticky word before the status restarts
        if (a.sticky) a.sticky[id] |= a.stat[2 * id];
        a.stat[2 * id] = 0;
    }
}

__global__ __launch_bounds__(kAttrThreads) void k_attr_a(AttrArgs a) {
    __shared__ int32_t hist[kRungs];
    __shared__ uint32_t wmax[kAttrThreads / kWave];
    __shared__ unsigned long long wsum[kAttrThreads / kWave];
    __shared__ int32_t bad;
    const int tid = threadIdx.x;
    if (tid < kRungs) hist[tid] = 0;
    if (tid == 0) bad = 0;
    __syncthreads();
    const int2 bm = a.blkmap[xcd_chunk(blockIdx.x, gridDim.x)];
    const DagDesc d = a.desc[bm.x];
    const int32_t lv = bm.y * kAttrThreads + tid;
    const int g = d.n_gpu > 0 ? 1 : 0;
    const int32_t *r = a.rp + d.toff + d.id;
    const int32_t *c = a.col + d.eoff;
    const int64_t ub = d.toff - a.base;  // user index of the DAG's task 0
    uint32_t tv = 0;
    if (lv < d.n) {
        int32_t e0 = a.est[2 * (ub + lv)], e1 = a.est[2 * (ub + lv) + 1];
        if (e0 < 1 || e0 > INSP_MAX_TICK || e1 < 1 || e1 > INSP_MAX_TICK) bad = 1;
        tv = (uint32_t)(g ? e1 : e0);
        if (a.unit_time == 0) {
            int32_t e = r[lv], z = r[lv + 1];
            int32_t cnt1 = 0, lo = 0x7fffffff, hi = 0;
            for (; e < z; e++) {
                int32_t s = c[e];
                int32_t rs = a.rem ? a.rem[ub + s] : (int32_t)(a.word0[d.toff + s] >> 43);
                if (rs == 1) {
                    int32_t x = (int32_t)tv + a.est[2 * (ub + s) + g];
                    cnt1++;
                    lo = min(lo, x);
                    hi = max(hi, x);
                }
            }
            if (cnt1 > 0) {
                int jlo = ceil_log2(lo);
                int jhi = cnt1 == r[lv + 1] - r[lv] ? ceil_log2(hi) : kRungs - 1;
                if (jlo < jhi) {
                    atomicAdd(&hist[jlo], 1);
                    atomicAdd(&hist[jhi], -1);
                }
            }
        }
    }
    uint32_t m = wave_max_u32(tv);
    unsigned long long sm = wave_sum_u64(tv);
    if ((tid & (kWave - 1)) == 0) {
        wmax[tid / kWave] = m;
        wsum[tid / kWave] = sm;
    }
    __syncthreads();
    if (tid < kRungs && hist[tid] != 0) atomicAdd(&a.score[d.id * kRungs + tid], hist[tid]);
    if (tid == 0) {
        uint32_t bm2 = 0;
        unsigned long long bs = 0;
        for (int w = 0; w < kAttrThreads / kWave; w++) {
            bm2 = max(bm2, wmax[w]);
            bs += wsum[w];
        }
        atomicMax(&a.maxtau[d.id], (int32_t)bm2);
        atomicAdd(&a.tausum[d.id], bs);
        if (bad) {
            atomicOr(&a.stat[2 * d.id], ST_EST);
            *a.anybad = 1;
        }
    }
}

// One thread per DAG: integrate the score histogram over the ladder and pick
// U (largest rung among the best scores); mean tau for the regulator.
__global__ void k_attr_select(AttrArgs a, int32_t count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const DagDesc d = a.desc[i];
    int32_t mt = a.maxtau[d.id];
    int J = 0;
    while (((int64_t)1 << J) < 2 * (int64_t)mt) J++;
    int32_t run = 0, best = -1, bj = 0;
    for (int j = 0; j <= J; j++) {
        run += a.score[d.id * kRungs + j];
        if (run >= best) {
            best = run;
            bj = j;
        }
    }
    a.u[d.id] = a.unit_time > 0 ? a.unit_time : (1 << bj);
    long long tb = d.n > 0 ? (long long)(a.tausum[d.id] / (unsigned long long)d.n) : 1;
    a.taubar[d.id] = (int32_t)(tb < 1 ? 1 : tb);
}

struct AttrOut {
    int32_t *ia_out, *ie_out;   // user arrays (nullable), relative to base
    int sim_init;
    TaskRec *tr;
};

__global__ __launch_bounds__(kAttrThreads) void k_attr_b(AttrArgs a, AttrOut o) {
    const int2 bm = a.blkmap[xcd_chunk(blockIdx.x, gridDim.x)];
    const DagDesc d = a.desc[bm.x];
    const int32_t lv = bm.y * kAttrThreads + threadIdx.x;
    if (lv >= d.n) return;
    // an estimate out of range fails the call: an attribute-only call then
    // writes no output at all; a schedule does not simulate that DAG, whose
    // records are marked unscheduled so that no stale schedule reaches the
    // caller's arrays
    if (o.sim_init ? (a.stat[2 * d.id] & ST_EST) != 0 : *a.anybad != 0) {
        if (o.sim_init) {
            TaskRec rec;
            memset(&rec, 0, sizeof rec);
            rec.qpos = -1;
            o.tr[d.toff + lv] = rec;
        }
        return;
    }
    const int g = d.n_gpu > 0 ? 1 : 0;
    const int32_t *r = a.rp + d.toff + d.id;
    const int32_t *c = a.col + d.eoff;
    const int64_t ub = d.toff - a.base;
    const int64_t U = a.u[d.id];
    const int32_t tv = a.est[2 * (ub + lv) + g];
    const int32_t e0 = r[lv], z = r[lv + 1];
    int32_t ie = 0;
    for (int32_t e = e0; e < z; e++) {
        int32_t s = c[e];
        int32_t rs = a.rem ? a.rem[ub + s] : (int32_t)(a.word0[d.toff + s] >> 43);
        if (rs == 1 && (int64_t)tv + a.est[2 * (ub + s) + g] <= U) ie++;
    }
    if (o.ia_out) o.ia_out[ub + lv] = z - e0;
    if (o.ie_out) o.ie_out[ub + lv] = ie;
    if (o.sim_init) {
        const int64_t v = d.toff + lv;
        TaskRec rec;
        rec.word = a.word0[v];
        rec.iev = ie;
        rec.qpos = -1;
        rec.ia = z - e0;
        rec.tau = tv;
        rec.rs = e0;
        rec.seq = 0;
        o.tr[v] = rec;
    }
}

static AttrArgs make_args(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, const int32_t *rem) {
    AttrArgs a;
    a.desc = ws->desc.as<DagDesc>();
    a.blkmap = ws->blkmap.as<int2>();
    a.rp = dag->rp.as<int32_t>();
    a.col = dag->col.as<int32_t>();
    a.word0 = dag->word0.as<unsigned long long>();
    a.est = est;
    a.rem = rem;
    a.base = ws->base;
    a.unit_time = unit_time;
    a.maxtau = ws->dag_maxtau;
    a.score = ws->dag_score;
    a.u = ws->dag_u;
    a.taubar = ws->dag_taubar;
    a.stat = dag->dag_stat.as<int32_t>();
    a.sticky = dag->dag_sticky.as<int32_t>();
    a.anybad = ws->counter.as<int32_t>() + 3;
    a.tausum = ws->dag_tausum;
    return a;
}

int run_attributes(insp_dag *dag, Workspace *ws, const int32_t *est, int32_t unit_time, const int32_t *rem,
                   int32_t *ia_out, int32_t *ie_out, bool sim_init, hipStream_t st) {
    AttrArgs a = make_args(dag, ws, est, unit_time, rem);
    if (!sim_init) {
        // an attribute-only call has status words of its own: it neither
        // clears nor reports a schedule's pending failures
        a.stat = dag->dag_astat.as<int32_t>();
        a.sticky = nullptr;
    }
    hipLaunchKernelGGL(k_attr_clear, dim3((ws->count * kRungs + 255) / 256), dim3(256), 0, st, a, ws->count);
    if (ws->attr_blocks > 0) {
        ProfScope ps(st, "attr_a");
        hipLaunchKernelGGL(k_attr_a, dim3(ws->attr_blocks), dim3(kAttrThreads), 0, st, a);
    }
    {
        ProfScope ps(st, "attr_select");
        hipLaunchKernelGGL(k_attr_select, dim3((ws->count + 63) / 64), dim3(64), 0, st, a, ws->count);
    }
    AttrOut o;
    o.ia_out = ia_out;
    o.ie_out = ie_out;
    o.sim_init = sim_init ? 1 : 0;
    o.tr = ws->tr;
    if (ws->attr_blocks > 0) {
        ProfScope ps(st, "attr_b");
        hipLaunchKernelGGL(k_attr_b, dim3(ws->attr_blocks), dim3(kAttrThreads), 0, st, a, o);
    }
    INSP_HIP(hipGetLastError());
    return INSP_OK;
}

int alloc_status(insp_dag *dag) {
    int rc;
    if ((rc = dag->dag_stat.alloc(8 * dag->B)) || (rc = dag->dag_astat.alloc(8 * dag->B)) ||
        (rc = dag->dag_sticky.alloc(4 * dag->B)))
        return rc;
    INSP_HIP(hipMemset(dag->dag_stat.p, 0, 8 * dag->B));
    INSP_HIP(hipMemset(dag->dag_astat.p, 0, 8 * dag->B));
    INSP_HIP(hipMemset(dag->dag_sticky.p, 0, 4 * dag->B));
    return INSP_OK;
}

int ensure_state(insp_dag *dag, hipStream_t st) {
    (void)st;
    if (dag->tr.p) return INSP_OK;
    const int64_t N = std::max<int64_t>(dag->N, 1);
    int rc;
    if ((rc = dag->tr.alloc(sizeof(TaskRec) * N)) || (rc = dag->fbuf.alloc(12 * N)) ||
        (rc = dag->dag_u.alloc(4 * dag->B)) ||
        (rc = dag->dag_taubar.alloc(4 * dag->B)) || (rc = dag->dag_maxtau.alloc(4 * dag->B)) ||
        (rc = dag->dag_tausum.alloc(8 * dag->B)) || (rc = dag->dag_score.alloc(4 * kRungs * dag->B))) {
        dag->tr.release();
        return rc;
    }
    return INSP_OK;
}

// Queue pool of one DAG: every worker's queue is a list of 64-slot blocks;
// at any time sum over workers of ceil(len/64) <= n/64 + W blocks are in use.
static void pool_shape(int32_t n, int32_t W, int32_t *nblk, int32_t *maxb) {
    *nblk = (n + 63) / 64 + W;
    *maxb = (n + 63) / 64 + 1;
}

int64_t workspace_shape(const insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers,
                        bool per_dag, Workspace *w, std::vector<DagDesc> *desc, std::vector<int2> *blk) {
    w->count = count;
    w->first = first;
    w->base = dag->toff[first];
    w->tasks = dag->toff[first + count] - dag->toff[first];
    desc->assign(count, DagDesc());
    blk->clear();
    w->h_order.clear();
    int64_t boff = 0, wloff = 0;
    for (int32_t i = 0; i < count; i++) {
        const insp_workers &wk = workers[per_dag ? i : 0];
        int32_t b = first + i;
        DagDesc &d = (*desc)[i];
        memset(&d, 0, sizeof d);
        d.id = b;
        d.toff = dag->toff[b];
        d.eoff = dag->eoff[b];
        d.n = (int32_t)(dag->toff[b + 1] - dag->toff[b]);
        d.m = (int32_t)(dag->eoff[b + 1] - dag->eoff[b]);
        d.n_cpu = wk.n_cpu;
        d.n_gpu = wk.n_gpu;
        pool_shape(d.n, wk.n_cpu + wk.n_gpu, &d.nblk, &d.maxb);
        d.blk_off = boff;
        d.wl_off = wloff;
        boff += d.nblk;
        wloff += (int64_t)(wk.n_cpu + wk.n_gpu) * d.maxb;
        w->max_w = std::max(w->max_w, wk.n_cpu + wk.n_gpu);
        w->max_nblk = std::max<int64_t>(w->max_nblk, d.nblk);
        for (int32_t c = 0; c * kAttrThreads < d.n; c++) blk->push_back(make_int2(i, c));
    }
    w->attr_blocks = (int32_t)blk->size();
    // simulation order: largest DAGs first
    for (int32_t b : dag->order)
        if (b >= first && b < first + count) w->h_order.push_back(b - first);
    w->total_wl = wloff;
    return boff;
}

int get_workspace(insp_dag *dag, int32_t first, int32_t count, const insp_workers *workers, bool per_dag,
                  Workspace **out) {
    std::string key = std::to_string(first) + ":" + std::to_string(count);
    for (int32_t i = 0; i < (per_dag ? count : 1); i++)
        key += ":" + std::to_string(workers[i].n_cpu) + "," + std::to_string(workers[i].n_gpu);
    auto it = dag->ws.find(key);
    Workspace *w = nullptr;
    if (it != dag->ws.end()) {
        w = it->second.get();
    } else {
        std::unique_ptr<Workspace> nw(new Workspace());
        std::vector<DagDesc> desc;
        std::vector<int2> blk;
        const int64_t boff = workspace_shape(dag, first, count, workers, per_dag, nw.get(), &desc, &blk);
        int rc;
        if ((rc = nw->desc.alloc(sizeof(DagDesc) * count)) || (rc = nw->blkmap.alloc(sizeof(int2) * blk.size())) ||
            (rc = nw->order.alloc(sizeof(int32_t) * count)) || (rc = nw->slots.alloc(sizeof(Slot) * 64 * (size_t)boff)) ||
            (rc = nw->sums.alloc(16 * (size_t)boff)) || (rc = nw->paux.alloc(4 * (size_t)(nw->total_wl + boff))) ||
            (rc = nw->barr.alloc(8 * (size_t)boff)) ||
            (rc = nw->counter.alloc(16)))
            return rc;
        INSP_HIP(hipMemcpy(nw->desc.p, desc.data(), sizeof(DagDesc) * count, hipMemcpyHostToDevice));
        if (!blk.empty())
            INSP_HIP(hipMemcpy(nw->blkmap.p, blk.data(), sizeof(int2) * blk.size(), hipMemcpyHostToDevice));
        INSP_HIP(hipMemcpy(nw->order.p, nw->h_order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice));
        w = nw.get();
        dag->ws[key] = std::move(nw);
    }
    // the handle's per-call state (ensure_state has run)
    w->tr = dag->tr.as<TaskRec>();
    w->fbuf = dag->fbuf.as<int32_t>();
    w->dag_u = dag->dag_u.as<int32_t>();
    w->dag_taubar = dag->dag_taubar.as<int32_t>();
    w->dag_maxtau = dag->dag_maxtau.as<int32_t>();
    w->dag_score = dag->dag_score.as<int32_t>();
    w->dag_tausum = dag->dag_tausum.as<unsigned long long>();
    *out = w;
    return INSP_OK;
}

}  // namespace insp

using namespace insp;

static int check_workers(const insp_workers *w, int32_t count) {
    for (int32_t i = 0; i < count; i++) {
        if (w[i].n_cpu < 0 || w[i].n_gpu < 0) return set_error(INSP_E_INVAL, "negative worker count");
        int32_t W = w[i].n_cpu + w[i].n_gpu;
        if (W < 1 || W > INSP_MAX_WORKERS) return set_error(INSP_E_RANGE, "worker count %d outside [1, 1024]", W);
    }
    return INSP_OK;
}

extern "C" int insp_attributes(const insp_dag *cdag, int32_t index, const int32_t *est, const insp_workers *workers,
                               int32_t unit_time, const int32_t *rem, int32_t *ia, int32_t *ie,
                               int32_t *unit_time_used, void *stream) {
    insp_dag *dag = const_cast<insp_dag *>(cdag);
    if (!dag || !workers || !unit_time_used) return set_error(INSP_E_INVAL, "null argument");
    if (index != INSP_ALL_DAGS && (index < 0 || index >= dag->B))
        return set_error(INSP_E_INVAL, "dag index %d out of range", index);
    if (unit_time < 0) return set_error(INSP_E_INVAL, "negative unit_time");
    const int32_t first = index == INSP_ALL_DAGS ? 0 : index;
    const int32_t count = index == INSP_ALL_DAGS ? dag->B : 1;
    int rc = check_workers(workers, count);
    if (rc) return rc;
    const int64_t n = dag->toff[first + count] - dag->toff[first];
    if (n > 0 && (!est || !ia || !ie)) return set_error(INSP_E_INVAL, "null est/ia/ie");
    hipStream_t st = (hipStream_t)stream;
    INSP_HIP(hipSetDevice(dag->device));
    if ((rc = ensure_state(dag, st))) return rc;
    Workspace *ws;
    if ((rc = get_workspace(dag, first, count, workers, true, &ws))) return rc;
    if ((rc = run_attributes(dag, ws, est, unit_time, rem, ia, ie, false, st))) return rc;
    std::vector<int32_t> stat(2 * dag->B), uu(count);
    INSP_HIP(hipMemcpyAsync(uu.data(), ws->dag_u + first, sizeof(int32_t) * count,
                            hipMemcpyDeviceToHost, st));
    INSP_HIP(hipMemcpyAsync(stat.data(), dag->dag_astat.p, sizeof(int32_t) * 2 * dag->B, hipMemcpyDeviceToHost, st));
    INSP_HIP(hipStreamSynchronize(st));
    for (int32_t i = first; i < first + count; i++)
        if (stat[2 * i] & ST_EST) return set_error(INSP_E_RANGE, "estimate outside [1, 2^20] in DAG %d", i);
    for (int32_t i = 0; i < count; i++) unit_time_used[i] = uu[i];
    return INSP_OK;
}
