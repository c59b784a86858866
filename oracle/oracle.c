/*
 * CPU oracle for the INSPIRIT adaptive-priority scheduling hot path
 * (Y. Wang et al., arXiv 2404.03226).
 *
 * TEST INFRASTRUCTURE.  This is a plain, slow, single-threaded-per-DAG
 * reference that only the tests, the smoke check and the benchmark's CPU
 * baseline leg load.  The HIP library never links, includes or calls it, and
 * the two share no code, header, table or helper.
 *
 * What it computes, in the paper's terms:
 *   - inspiring ability IA(v): the dependencies that v's completion resolves
 *     (Section 4.2), read as the out-degree of v;
 *   - inspiring efficiency IE(v; U, rem): successors s of v that v's
 *     completion makes ready (rem[s] == 1) and that can complete within the
 *     unit time U measured from v's start, using GPU execution times
 *     (Sections 4.2 and 4.3): tau(v) + tau(s) <= U;
 *   - the unit-time search of Section 4.3 (IE must separate tasks: neither
 *     all zero nor converged to IA) as a power-of-two ladder;
 *   - a DMDA-style list-scheduling simulation (Section 2: push to the worker
 *     with the least expected termination time; Section 4.1: per-worker
 *     queues, FIFO head by default, attribute-driven precedence), with the
 *     Nready regulator of Section 4.4 choosing between the high-ability and
 *     the high-efficiency pop rule;
 *   - the transitive reading of the attributes (all descendants, and the
 *     descendants finishing within a unit-time window, Sections 4.3 and 7),
 *     used as fixed keys when a schedule asks for them;
 *   - the HEFT upward-rank list baseline the paper compares against;
 *   - a data model: per-task output items on memory nodes, DMDA's transfer
 *     term at push and the efficiency-with-locality pop rule.
 * Readings taken where the paper is silent or garbled are listed at the
 * function that applies them.
 *
 * Two pop implementations exist: ORC_PLAIN scans a worker's queue linearly and
 * recomputes IE from its definition for every queued task at every pop;
 * ORC_HEAP keeps IE incrementally (by scanning a successor's predecessors for
 * the one still unfinished) and uses lazy-deletion binary heaps.  The tests
 * require both to give identical schedules; ORC_HEAP exists only so that the
 * oracle finishes the million-task workloads in reasonable time.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_CYCLE = 2, ORC_E_RANGE = 3, ORC_E_NOMEM = 4, ORC_E_HANG = 6 };
enum { POL_INSPIRIT = 0, POL_FIFO = 1, POL_ABILITY = 2, POL_EFI = 3, POL_RANK = 4, POL_LOCALITY = 5 };
enum { M_ABILITY = 0, M_EFI = 1, M_EFI_LOC = 2, M_FIFO = 3, M_RANK = 4 };
enum { ORC_PLAIN = 0, ORC_HEAP = 1 };

#define ORC_MAX_N (1 << 21)
#define ORC_MAX_TICK (1 << 20)
#define ORC_MAX_W 1024
#define ORC_MAX_PATH (1 << 30) /* transitive attributes: longest path in ticks, exclusive */

typedef struct {
    int32_t policy, unit_time;
    int32_t s_inc, s_dec, dec_step, c, k_num, k_den;
    int32_t max_events;
    int32_t attr_mode;  /* 0: direct attributes; 1: transitive (static) attributes */
    int32_t data_bw;    /* data model: bytes moved per tick between memory nodes (0 = no data model) */
    const int32_t *data_kib; /* data model: KiB of each task's output item */
} orc_params;

typedef struct {
    int64_t t;
    int32_t nready, mode, cnt, peak, pushed, popped;
} orc_trace;

/* ------------------------------------------------------------------ DAG */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Validate a user CSR and write its canonical form: each successor row
 * sorted ascending with repeated edges dropped.  Self loops and ids out of
 * range are structural errors; a cycle (checked by Kahn's traversal from the
 * tasks with no predecessors, Section 4.3) is reported as ORC_E_CYCLE.
 * rp_out has n+1 entries and col_out room for rp[n] entries. */
int orc_canon(int32_t n, const int32_t *rp, const int32_t *col, int32_t *rp_out, int32_t *col_out) {
    if (n < 0) return ORC_E_INVAL;
    if (n > ORC_MAX_N) return ORC_E_RANGE;
    if (rp[0] != 0) return ORC_E_INVAL;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] < rp[v]) return ORC_E_INVAL;
    for (int64_t e = 0; e < rp[n]; e++)
        if (col[e] < 0 || col[e] >= n) return ORC_E_INVAL;
    for (int32_t v = 0; v < n; v++)
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (col[e] == v) return ORC_E_INVAL;
    int32_t m = 0;
    rp_out[0] = 0;
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
    if (!row) return ORC_E_NOMEM;
    for (int32_t v = 0; v < n; v++) {
        int32_t d = rp[v + 1] - rp[v];
        memcpy(row, col + rp[v], sizeof(int32_t) * (size_t)d);
        qsort(row, (size_t)d, sizeof(int32_t), cmp_i32);
        for (int32_t i = 0; i < d; i++)
            if (i == 0 || row[i] != row[i - 1]) col_out[m++] = row[i];
        rp_out[v + 1] = m;
    }
    free(row);
    /* Kahn: repeatedly remove tasks whose predecessors are all removed. */
    int32_t *indeg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!indeg || !stack) { free(indeg); free(stack); return ORC_E_NOMEM; }
    for (int32_t e = 0; e < m; e++) indeg[col_out[e]]++;
    int32_t top = 0, seen = 0;
    for (int32_t v = 0; v < n; v++)
        if (indeg[v] == 0) stack[top++] = v;
    while (top > 0) {
        int32_t v = stack[--top];
        seen++;
        for (int32_t e = rp_out[v]; e < rp_out[v + 1]; e++)
            if (--indeg[col_out[e]] == 0) stack[top++] = col_out[e];
    }
    free(indeg);
    free(stack);
    return seen == n ? ORC_OK : ORC_E_CYCLE;
}

/* ----------------------------------------------------------- attributes */

/* tau(v): the GPU estimate when the machine has GPU workers, else the CPU
 * estimate (Section 4.3 computes IE with GPU execution times). */
static int32_t tau_of(const int32_t *est, int32_t n_gpu, int32_t v) {
    return est[2 * (int64_t)v + (n_gpu > 0 ? 1 : 0)];
}

/* IE(v; U, rem) straight from its definition. */
static int32_t ie_def(const int32_t *rp, const int32_t *col, const int32_t *est, int32_t n_gpu,
                      const int32_t *rem, int64_t U, int32_t v) {
    int32_t c = 0;
    int64_t tv = tau_of(est, n_gpu, v);
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
        int32_t s = col[e];
        if (rem[s] == 1 && tv + tau_of(est, n_gpu, s) <= U) c++;
    }
    return c;
}

/* Unit-time search (Section 4.3): try U = 1, 2, 4, ... up to the first power
 * of two that is at least twice the largest tau (beyond that every IE has
 * converged to its limit), score each U by the number of tasks whose IE is
 * neither zero nor equal to IA (the two degenerate ends named in Section 4.2),
 * and keep the best score, the larger U on a tie. */
static int64_t auto_unit_time(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *est,
                              int32_t n_gpu, const int32_t *rem) {
    int64_t maxtau = 0;
    for (int32_t v = 0; v < n; v++)
        if (tau_of(est, n_gpu, v) > maxtau) maxtau = tau_of(est, n_gpu, v);
    int J = 0;
    while (((int64_t)1 << J) < 2 * maxtau) J++;
    int64_t bestU = 1, bestScore = -1;
    for (int j = 0; j <= J; j++) {
        int64_t U = (int64_t)1 << j, score = 0;
        for (int32_t v = 0; v < n; v++) {
            int32_t ia = rp[v + 1] - rp[v];
            int32_t ie = ie_def(rp, col, est, n_gpu, rem, U, v);
            if (ie > 0 && ie < ia) score++;
        }
        if (score >= bestScore) { bestScore = score; bestU = U; }
    }
    return bestU;
}

static int check_ticks(int32_t n, const int32_t *a) {
    for (int64_t i = 0; i < 2 * (int64_t)n; i++)
        if (a[i] < 1 || a[i] > ORC_MAX_TICK) return ORC_E_RANGE;
    return ORC_OK;
}

/* IA and IE of every task at a given remaining in-degree (NULL = initial
 * in-degrees) and unit time (0 = the search above).  Input CSR must be
 * canonical. */
int orc_attributes(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *est, int32_t n_gpu,
                   const int32_t *rem_in, int32_t unit_time, int32_t *ia, int32_t *ie, int32_t *U_used) {
    if (n < 0 || unit_time < 0) return ORC_E_INVAL;
    if (check_ticks(n, est)) return ORC_E_RANGE;
    int32_t *rem = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!rem) return ORC_E_NOMEM;
    if (rem_in) memcpy(rem, rem_in, sizeof(int32_t) * (size_t)n);
    else
        for (int32_t e = 0; e < rp[n]; e++) rem[col[e]]++;
    int64_t U = unit_time > 0 ? unit_time : auto_unit_time(n, rp, col, est, n_gpu, rem);
    for (int32_t v = 0; v < n; v++) {
        ia[v] = rp[v + 1] - rp[v];
        ie[v] = ie_def(rp, col, est, n_gpu, rem, U, v);
    }
    *U_used = (int32_t)U;
    free(rem);
    return ORC_OK;
}

/* ------------------------------------------------ transitive attributes */

/* A topological order (Kahn, from the tasks without predecessors). */
static int topo_order(int32_t n, const int32_t *rp, const int32_t *col, int32_t *order) {
    int32_t *left = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!left) return ORC_E_NOMEM;
    for (int32_t e = 0; e < rp[n]; e++) left[col[e]]++;
    int32_t head = 0, tail = 0;
    for (int32_t v = 0; v < n; v++)
        if (left[v] == 0) order[tail++] = v;
    while (head < tail) {
        int32_t v = order[head++];
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (--left[col[e]] == 0) order[tail++] = col[e];
    }
    free(left);
    return tail == n ? ORC_OK : ORC_E_CYCLE;
}

/* Transitive reading of the two attributes (Section 4.3: the source of a
 * fully connected DAG scores the number of its tasks; Section 4.2: with a
 * large unit time IE converges to IA; Section 7: IE looks at a time window
 * after the task).  With D(v) = v and every task reachable from v:
 *   IA_T(v)    = |D(v)|;
 *   EF_v(d)    = the longest tau-weighted path from v to d, both ends
 *                included -- d's earliest finish when v starts at time 0
 *                and workers are unlimited;
 *   IE_T(v; U) = #{d in D(v) : EF_v(d) <= U}.
 * Both are computed once on the whole DAG (offline, Section 4.3), one
 * forward pass per source v over a topological order.  With unit_time == 0
 * U is chosen on the ladder U = 2^j, j = 0..J, 2^J the first power of two
 * at least the DAG's longest path (where every IE_T has reached IA_T): the U
 * with the most tasks whose IE_T is neither 0 nor IA_T, the larger U on a
 * tie.  The longest path must stay below 2^30 ticks (ORC_E_RANGE). */
int orc_transitive(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *est, int32_t n_gpu,
                   int32_t unit_time, int32_t *ia, int32_t *ie, int32_t *U_used, int64_t *longest) {
    if (n < 0 || unit_time < 0) return ORC_E_INVAL;
    if (check_ticks(n, est)) return ORC_E_RANGE;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t *EF = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    /* within[v][j]: members of D(v) whose finish from v's start is <= 2^j */
    int32_t *within = (int32_t *)calloc((size_t)n * 32 + 1, sizeof(int32_t));
    int rc = ORC_OK;
    if (!order || !pos || !EF || !within) { rc = ORC_E_NOMEM; goto out; }
    if ((rc = topo_order(n, rp, col, order))) goto out;
    for (int32_t i = 0; i < n; i++) pos[order[i]] = i;
    int64_t cp = 0;
    for (int32_t v = 0; v < n; v++) {
        memset(EF, 0, sizeof(int64_t) * (size_t)n);
        EF[v] = tau_of(est, n_gpu, v);
        int32_t members = 0, in_u = 0;
        for (int32_t i = pos[v]; i < n; i++) {
            int32_t u = order[i];
            if (EF[u] == 0) continue;  /* not reachable from v */
            members++;
            if (EF[u] > cp) cp = EF[u];
            if (unit_time > 0 && EF[u] <= unit_time) in_u++;
            for (int j = 0; j < 32; j++)
                if (EF[u] <= ((int64_t)1 << j)) within[(int64_t)v * 32 + j]++;
            for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
                int32_t s = col[e];
                int64_t f = EF[u] + tau_of(est, n_gpu, s);
                if (f > EF[s]) EF[s] = f;
            }
        }
        ia[v] = members;
        ie[v] = in_u;
    }
    if (longest) *longest = cp;
    if (cp >= ORC_MAX_PATH) { rc = ORC_E_RANGE; goto out; }
    int64_t U = unit_time;
    if (unit_time == 0) {
        /* rungs 2^0 .. 2^J, 2^J the first power of two >= the longest path;
           score = tasks with 0 < IE_T < IA_T; the larger U on a tie */
        int J = 0;
        while (((int64_t)1 << J) < cp) J++;
        int64_t bestScore = -1;
        int bestJ = 0;
        for (int j = 0; j <= J; j++) {
            int64_t score = 0;
            for (int32_t v = 0; v < n; v++) {
                const int32_t w = within[(int64_t)v * 32 + j];
                if (w > 0 && w < ia[v]) score++;
            }
            if (score >= bestScore) { bestScore = score; bestJ = j; }
        }
        U = (int64_t)1 << bestJ;
        for (int32_t v = 0; v < n; v++) ie[v] = within[(int64_t)v * 32 + bestJ];
    }
    if (U_used) *U_used = (int32_t)U;
out:
    free(order); free(pos); free(EF); free(within);
    return rc;
}

/* ------------------------------------------------------------ regulator */

typedef struct {
    int64_t peak, prev_n, prev_t, cnt;
    int32_t mode;
    int64_t s_inc, s_dec, dec_step, c, k_num, k_den;
} orc_reg;

/* Parameter defaults (the paper names the parameters but prints no values):
 * task window s_inc = ceil(W/4), s_dec = ceil(W/2), dec_step = s_dec,
 * c = floor(s_dec/2), expected slope k_inc = W / mean(tau). */
static void reg_init(orc_reg *r, const orc_params *p, int32_t W, int64_t tau_bar) {
    r->peak = r->prev_n = r->prev_t = r->cnt = 0;
    r->mode = M_ABILITY;  /* Section 3: the run starts by favouring high ability */
    int64_t s_inc = (W + 3) / 4, s_dec = (W + 1) / 2;
    if (s_inc < 1) s_inc = 1;
    if (s_dec < 1) s_dec = 1;
    r->s_inc = p->s_inc > 0 ? p->s_inc : s_inc;
    r->s_dec = p->s_dec > 0 ? p->s_dec : s_dec;
    r->dec_step = p->dec_step > 0 ? p->dec_step : r->s_dec;
    r->c = p->c >= 0 ? p->c : r->s_dec / 2;
    if (p->k_num > 0 && p->k_den > 0) { r->k_num = p->k_num; r->k_den = p->k_den; }
    else { r->k_num = W; r->k_den = tau_bar; }
}

/* One observation of Nready = N at time t (Section 4.4 pseudocode), with
 * these readings: the peak follows every observation; the state logic runs
 * only when Nready moved by at least the task window since the last time it
 * ran, and otherwise the pop rule is unchanged; "num_nready" is the current
 * Nready; the slope is the Nready change over the elapsed time since the last
 * trigger (compared to k_inc by cross-multiplication, zero elapsed time being
 * an infinite slope); the decrement count is reset while ascending and
 * increased by one by updateDecrementCount; the stable state behaves like the
 * descending one; when no branch applies the current rule is kept. */
static void reg_step(orc_reg *r, int64_t t, int64_t N) {
    if (N > r->peak) r->peak = N;
    int64_t dn = N - r->prev_n;
    if ((dn < 0 ? -dn : dn) < r->s_inc) return;
    int64_t dt = t - r->prev_t;
    r->prev_n = N;
    r->prev_t = t;
    if (N >= r->peak - r->dec_step) {              /* ascending */
        r->cnt = 0;
        if (dn >= r->s_inc) {
            if (dt == 0 || dn * r->k_den > r->k_num * dt) r->mode = M_ABILITY;
            else if (dn * r->k_den < r->k_num * dt) r->mode = M_EFI;
        }
    } else {                                       /* stable / descending */
        if (N > r->peak - r->s_dec * r->cnt) r->mode = M_ABILITY;
        else if (N <= r->peak - r->s_dec * (r->cnt + 1) + r->c) {
            r->mode = M_EFI_LOC;
            if (N <= r->peak - r->s_dec * (r->cnt + 1)) r->cnt += 1;
        }
    }
}

/* Run the regulator alone over a sequence of observations. */
int orc_regulate_seq(int32_t steps, const int64_t *t, const int32_t *N, const orc_params *p, int32_t W,
                     int64_t tau_bar, int32_t *mode, int32_t *cnt, int32_t *peak) {
    orc_reg r;
    reg_init(&r, p, W, tau_bar);
    for (int32_t i = 0; i < steps; i++) {
        reg_step(&r, t[i], N[i]);
        mode[i] = r.mode;
        cnt[i] = (int32_t)r.cnt;
        peak[i] = (int32_t)r.peak;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ simulation */

typedef struct { int32_t v, ie; } hent;
typedef struct { hent *a; int64_t len, cap; } heap;

typedef struct {
    const int32_t *ia, *ie, *seq;
    int order;  /* 0: ability first, 1: efficiency first, 2: push order, 3: upward rank */
    const int64_t *rank;
} hctx;

/* Pop priority (Section 4.4 pop rules; ties fall back to FIFO, Section 4.1):
 * ability rule (IA, IE, earlier push), efficiency rule (IE, IA, earlier
 * push), FIFO (earlier push); the HEFT baseline of Section 6 compares the
 * upward rank (then earlier push).  Returns 1 when a outranks b. */
static int outranks_r(int order, int64_t r_a, int64_t r_b, int32_t ia_a, int32_t ie_a, int32_t sq_a, int32_t ia_b,
                      int32_t ie_b, int32_t sq_b);
static int outranks(int order, int32_t ia_a, int32_t ie_a, int32_t sq_a, int32_t ia_b, int32_t ie_b, int32_t sq_b) {
    if (order == 0) {
        if (ia_a != ia_b) return ia_a > ia_b;
        if (ie_a != ie_b) return ie_a > ie_b;
    } else if (order == 1) {
        if (ie_a != ie_b) return ie_a > ie_b;
        if (ia_a != ia_b) return ia_a > ia_b;
    }
    return sq_a < sq_b;
}
static int outranks_r(int order, int64_t r_a, int64_t r_b, int32_t ia_a, int32_t ie_a, int32_t sq_a, int32_t ia_b,
                      int32_t ie_b, int32_t sq_b) {
    if (order == 3 && r_a != r_b) return r_a > r_b;
    if (order == 3) return sq_a < sq_b;
    return outranks(order, ia_a, ie_a, sq_a, ia_b, ie_b, sq_b);
}

static int hless(const hctx *c, hent x, hent y) {  /* x below y in the max-heap */
    return outranks_r(c->order, c->rank ? c->rank[y.v] : 0, c->rank ? c->rank[x.v] : 0, c->ia[y.v], y.ie,
                      c->seq[y.v], c->ia[x.v], x.ie, c->seq[x.v]);
}

/* HEFT upward rank (Topcuoglu, Hariri and Wu 2002), with no communication
 * cost (no data model here): rank(v) = mean cost of v over the machine's
 * workers + the largest rank of its successors.  Kept multiplied by the
 * worker count W to stay integer (the order is unchanged):
 *   R(v) = n_cpu * est_cpu(v) + n_gpu * est_gpu(v) + max over successors R(s).
 * Successors first: a Kahn order from the sinks (reverse topological). */
static int upward_rank(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *est, int32_t n_cpu,
                       int32_t n_gpu, int64_t *R) {
    int32_t *left = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *prp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *pcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int rc = ORC_OK;
    if (!left || !order || !prp || !pcol || !fill) { rc = ORC_E_NOMEM; goto out; }
    for (int32_t e = 0; e < rp[n]; e++) prp[col[e] + 1]++;
    for (int32_t v = 0; v < n; v++) prp[v + 1] += prp[v];
    memcpy(fill, prp, sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; v++)
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) pcol[fill[col[e]]++] = v;
    int32_t head = 0, tail = 0;
    for (int32_t v = 0; v < n; v++) {
        left[v] = rp[v + 1] - rp[v];
        if (left[v] == 0) order[tail++] = v;
    }
    while (head < tail) {
        int32_t v = order[head++];
        int64_t best = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (R[col[e]] > best) best = R[col[e]];
        R[v] = (int64_t)n_cpu * est[2 * (int64_t)v] + (int64_t)n_gpu * est[2 * (int64_t)v + 1] + best;
        for (int32_t e = prp[v]; e < prp[v + 1]; e++)
            if (--left[pcol[e]] == 0) order[tail++] = pcol[e];
    }
    if (tail != n) rc = ORC_E_CYCLE;
out:
    free(left); free(order); free(prp); free(pcol); free(fill);
    return rc;
}

static int hpush(heap *h, const hctx *c, hent x) {
    if (h->len == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 16;
        hent *na = (hent *)realloc(h->a, sizeof(hent) * (size_t)nc);
        if (!na) return ORC_E_NOMEM;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->len++;
    h->a[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(c, h->a[p], h->a[i])) break;
        hent t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
    return ORC_OK;
}

static hent hpop(heap *h, const hctx *c) {
    hent top = h->a[0];
    h->a[0] = h->a[--h->len];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        if (l < h->len && hless(c, h->a[b], h->a[l])) b = l;
        if (r < h->len && hless(c, h->a[b], h->a[r])) b = r;
        if (b == i) break;
        hent t = h->a[b]; h->a[b] = h->a[i]; h->a[i] = t;
        i = b;
    }
    return top;
}

typedef struct {
    int32_t *a;
    int64_t len, cap;
} ivec;

static int ivec_push(ivec *q, int32_t x) {
    if (q->len == q->cap) {
        int64_t nc = q->cap ? 2 * q->cap : 16;
        int32_t *na = (int32_t *)realloc(q->a, sizeof(int32_t) * (size_t)nc);
        if (!na) return ORC_E_NOMEM;
        q->a = na;
        q->cap = nc;
    }
    q->a[q->len++] = x;
    return ORC_OK;
}

enum { ST_WAIT = 0, ST_QUEUED = 1, ST_RUN = 2, ST_DONE = 3 };

/* Data model (the paper names DMDA's data-transfer term, Section 2, and a
 * data-locality pop rule, Section 4.4, without formulas; this reading keeps
 * both to integer ticks).  Memory node of worker w: 0 (host) for the CPU
 * workers, 1 + (w - n_cpu) for GPU worker w.  Task u leaves one output item of
 * data_kib[u] KiB on the node of the worker that ran it, its home; items are
 * not replicated.  A consumer on another node moves it in
 * xc(u) = ceil(1024 data_kib[u] / bw) ticks. */
static int node_of(int32_t w, int32_t n_cpu) { return w < n_cpu ? 0 : 1 + (w - n_cpu); }

static int64_t xfer_in(const orc_params *p, const int32_t *prp, const int32_t *pcol, const int32_t *home,
                       int32_t v, int node) {
    int64_t x = 0;
    for (int32_t e = prp[v]; e < prp[v + 1]; e++) {
        int32_t u = pcol[e];
        if (home[u] != node) x += ((int64_t)1024 * p->data_kib[u] + p->data_bw - 1) / p->data_bw;
    }
    return x;
}

/*
 * Simulate one DAG (canonical CSR) on n_cpu CPU workers (kind 0, ids
 * 0..n_cpu-1) and n_gpu GPU workers (kind 1).  Integer time; one iteration
 * per event time:
 *   1. push every newly ready task, in ascending id, to the worker with the
 *      least expected termination time: the worker's expected free time
 *      (now, or the running task's start plus its estimate if later) plus the
 *      estimates queued on it plus the task's own estimate; ties to the
 *      lowest worker id (DMDA, Section 2; no transfer cost is modelled);
 *   2. observe Nready = tasks waiting in all queues (running tasks excluded)
 *      with the regulator (INSPIRIT policy only);
 *   3. every idle worker, in ascending id, pops the top task of its own queue
 *      under the current rule, with IE evaluated at the current remaining
 *      in-degrees; the task runs for its true duration;
 *   4. stop when every task has completed; otherwise advance to the earliest
 *      finish time and complete every task finishing then, releasing its
 *      successors' dependencies (Section 2).
 * Decisions use est, time advances with dur.  Returns ORC_E_HANG when more
 * than max_events iterations would be needed.
 * With the data model (data_bw > 0): the push cost adds X(v, w), the transfer
 * ticks of v's inputs whose home is not w's node (DMDA's transfer penalty);
 * the queue's expected length still grows by the estimate alone, the
 * transfers starting at the push and overlapping other work, so v's inputs
 * arrive at arr(v) = t + X(v, chosen w).  A task popped at t starts at
 * max(t, arr(v)).  The efficiency-with-locality rule takes the tasks whose
 * inputs have arrived first, then the efficiency order.  X above 2^20 ticks
 * is ORC_E_RANGE.
 */
static int simulate(int32_t n, const int32_t *rp, const int32_t *col, int32_t n_cpu, int32_t n_gpu,
                    const int32_t *dur, const int32_t *est, const orc_params *p, int variant, int32_t *worker,
                    int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                    orc_trace *trace, int32_t trace_cap, int32_t *n_events, int32_t *U_out) {
    int32_t W = n_cpu + n_gpu;
    int rc = ORC_OK;
    if (n == 0) {
        *makespan = 0;
        if (n_events) *n_events = 0;
        if (U_out) *U_out = 1;
        return ORC_OK;
    }
    int64_t max_events = p->max_events > 0 ? p->max_events : (int64_t)n + 1;

    int32_t *rem = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *ia = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *ie = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *seq = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int8_t *state = (int8_t *)calloc((size_t)n, 1);
    int32_t *qw = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *newly = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *run = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    int64_t *exp_end = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    int64_t *qest = (int64_t *)calloc((size_t)W, sizeof(int64_t));
    ivec *Q = (ivec *)calloc((size_t)W, sizeof(ivec));
    heap *H = (heap *)calloc((size_t)W * 2, sizeof(heap));
    int32_t *prp = NULL, *pcol = NULL, *touched = NULL;
    int32_t *done_now = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    int64_t *R = p->policy == POL_RANK ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
    const int data = p->data_bw > 0;
    int64_t *arr = data ? (int64_t *)calloc((size_t)n, sizeof(int64_t)) : NULL;
    int32_t *home = data ? (int32_t *)calloc((size_t)n, sizeof(int32_t)) : NULL;
    if (!rem || !ia || !ie || !seq || !state || !qw || !newly || !run || !exp_end || !qest || !Q || !H || !done_now ||
        (p->policy == POL_RANK && !R) || (data && (!arr || !home))) {
        rc = ORC_E_NOMEM;
        goto out;
    }
    if (R && (rc = upward_rank(n, rp, col, est, n_cpu, n_gpu, R))) goto out;
    for (int32_t e = 0; e < rp[n]; e++) rem[col[e]]++;
    int32_t U;
    /* direct attributes follow the remaining in-degrees; transitive ones are
       fixed for the whole run */
    const int ie_static = p->attr_mode == 1;
    if (ie_static) rc = orc_transitive(n, rp, col, est, n_gpu, p->unit_time, ia, ie, &U, NULL);
    else rc = orc_attributes(n, rp, col, est, n_gpu, rem, p->unit_time, ia, ie, &U);
    if (rc) goto out;
    if (U_out) *U_out = U;
    int64_t tau_sum = 0;
    for (int32_t v = 0; v < n; v++) tau_sum += tau_of(est, n_gpu, v);
    int64_t tau_bar = tau_sum / n;
    if (tau_bar < 1) tau_bar = 1;
    orc_reg reg;
    reg_init(&reg, p, W, tau_bar);

    if (variant == ORC_HEAP || data) {
        /* predecessor lists: a successor's last unfinished predecessor; inputs */
        prp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        pcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
        touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!prp || !pcol || !touched) { rc = ORC_E_NOMEM; goto out; }
        for (int32_t e = 0; e < rp[n]; e++) prp[col[e] + 1]++;
        for (int32_t v = 0; v < n; v++) prp[v + 1] += prp[v];
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!fill) { rc = ORC_E_NOMEM; goto out; }
        memcpy(fill, prp, sizeof(int32_t) * (size_t)n);
        for (int32_t v = 0; v < n; v++)
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) pcol[fill[col[e]]++] = v;
        free(fill);
    }
    for (int32_t w = 0; w < W; w++) run[w] = -1;

    int32_t n_new = 0;
    for (int32_t v = 0; v < n; v++)
        if (rem[v] == 0) newly[n_new++] = v;
    int64_t t = 0, nready = 0;
    int32_t seqctr = 0, done = 0;
    int64_t events = 0;
    int mode_fixed = p->policy == POL_FIFO ? M_FIFO : p->policy == POL_ABILITY ? M_ABILITY
                   : p->policy == POL_EFI ? M_EFI : p->policy == POL_RANK ? M_RANK
                   : p->policy == POL_LOCALITY ? M_EFI_LOC : -1;
    /* keys that never change while queued: push order, upward rank */
    int static_key = mode_fixed == M_FIFO || mode_fixed == M_RANK;

    for (;;) {
        if (++events > max_events) { rc = ORC_E_HANG; goto out; }
        /* 1. push */
        for (int32_t i = 0; i < n_new; i++) {
            int32_t v = newly[i], best = -1;
            int64_t bestc = 0, bestx = 0;
            for (int32_t w = 0; w < W; w++) {
                int k = w < n_cpu ? 0 : 1;
                int64_t B = t;
                if (run[w] >= 0 && exp_end[w] > t) B = exp_end[w];
                int64_t x = data ? xfer_in(p, prp, pcol, home, v, node_of(w, n_cpu)) : 0;
                int64_t c = B + qest[w] + est[2 * (int64_t)v + k] + x;
                if (best < 0 || c < bestc) { best = w; bestc = c; bestx = x; }
            }
            if (bestx > ORC_MAX_TICK) { rc = ORC_E_RANGE; goto out; }
            if (data) arr[v] = t + bestx;
            int k = best < n_cpu ? 0 : 1;
            seq[v] = seqctr++;
            state[v] = ST_QUEUED;
            qw[v] = best;
            qest[best] += est[2 * (int64_t)v + k];
            nready++;
            if (variant == ORC_PLAIN) {
                if (ivec_push(&Q[best], v)) { rc = ORC_E_NOMEM; goto out; }
            } else {
                hctx c0 = {ia, ie, seq, mode_fixed == M_FIFO ? 2 : mode_fixed == M_RANK ? 3 : 0, R},
                     c1 = {ia, ie, seq, 1, R};
                if (hpush(&H[2 * best], &c0, (hent){v, ie[v]})) { rc = ORC_E_NOMEM; goto out; }
                if (!static_key && hpush(&H[2 * best + 1], &c1, (hent){v, ie[v]})) { rc = ORC_E_NOMEM; goto out; }
            }
        }
        /* 2. regulate */
        int64_t observed = nready;
        if (p->policy == POL_INSPIRIT) reg_step(&reg, t, nready);
        int mode = mode_fixed >= 0 ? mode_fixed : reg.mode;
        int order = mode == M_RANK ? 3 : mode == M_FIFO ? 2 : mode == M_ABILITY ? 0 : 1;
        /* 3. pop */
        int32_t popped = 0;
        for (int32_t w = 0; w < W; w++) {
            if (run[w] >= 0) continue;
            int k = w < n_cpu ? 0 : 1;
            int32_t v = -1, v_ie = 0;
            /* efficiency with locality: inputs already on the node first */
            const int loc = data && mode == M_EFI_LOC;
            if (variant == ORC_PLAIN) {
                if (Q[w].len == 0) continue;
                int64_t bi = -1;
                int32_t b_ie = 0;
                for (int64_t i = 0; i < Q[w].len; i++) {
                    int32_t x = Q[w].a[i];
                    int32_t x_ie = ie_static ? ie[x] : ie_def(rp, col, est, n_gpu, rem, U, x);
                    int32_t y = bi < 0 ? x : Q[w].a[bi];
                    int here_x = loc && arr[x] <= t, here_y = loc && arr[y] <= t;
                    if (bi < 0 || here_x > here_y ||
                        (here_x == here_y && outranks_r(order, R ? R[x] : 0, R ? R[y] : 0, ia[x], x_ie, seq[x],
                                                        ia[y], b_ie, seq[y]))) {
                        bi = i;
                        b_ie = x_ie;
                    }
                }
                v = Q[w].a[bi];
                v_ie = b_ie;
                memmove(Q[w].a + bi, Q[w].a + bi + 1, sizeof(int32_t) * (size_t)(Q[w].len - bi - 1));
                Q[w].len--;
            } else {
                heap *h = &H[2 * w + (order == 1 ? 1 : 0)];
                hctx c = {ia, ie, seq, order, R};
                if (loc) {
                    /* the best queued task whose inputs have arrived, by a
                       scan of the heap's live entries (it stays in the heap
                       and is skipped once running) */
                    for (int64_t i = 0; i < h->len; i++) {
                        hent x = h->a[i];
                        if (state[x.v] != ST_QUEUED || x.ie != ie[x.v] || arr[x.v] > t) continue;
                        if (v < 0 || outranks(1, ia[x.v], x.ie, seq[x.v], ia[v], ie[v], seq[v])) v = x.v;
                    }
                }
                while (v < 0 && h->len > 0) {
                    hent top = hpop(h, &c);
                    if (state[top.v] == ST_QUEUED && (order >= 2 || top.ie == ie[top.v])) { v = top.v; break; }
                }
                if (v < 0) continue;
                v_ie = ie[v];
            }
            state[v] = ST_RUN;
            run[w] = v;
            int64_t s0 = data && arr[v] > t ? arr[v] : t;  /* waits for its inputs */
            start[v] = s0;
            finish[v] = s0 + dur[2 * (int64_t)v + k];
            exp_end[w] = s0 + est[2 * (int64_t)v + k];
            if (data) home[v] = node_of(w, n_cpu);
            qest[w] -= est[2 * (int64_t)v + k];
            worker[v] = w;
            if (ie_at_pop) ie_at_pop[v] = v_ie;
            if (mode_at_pop) mode_at_pop[v] = (int8_t)mode;
            nready--;
            popped++;
        }
        if (trace && events <= trace_cap) {
            orc_trace *r = &trace[events - 1];
            r->t = t;
            r->nready = (int32_t)observed;
            r->mode = mode;
            r->cnt = (int32_t)reg.cnt;
            r->peak = (int32_t)reg.peak;
            r->pushed = n_new;
            r->popped = popped;
        }
        /* 4. stop or advance */
        if (done == n) break;
        int64_t tn = -1;
        for (int32_t w = 0; w < W; w++)
            if (run[w] >= 0 && (tn < 0 || finish[run[w]] < tn)) tn = finish[run[w]];
        if (tn < 0) { rc = ORC_E_HANG; goto out; }
        t = tn;
        int32_t nd = 0;
        for (int32_t w = 0; w < W; w++)
            if (run[w] >= 0 && finish[run[w]] == t) {
                done_now[nd++] = run[w];
                state[run[w]] = ST_DONE;
                run[w] = -1;
                done++;
            }
        n_new = 0;
        int32_t nt = 0;
        for (int32_t i = 0; i < nd; i++) {
            int32_t v = done_now[i];
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t s = col[e];
                if (variant == ORC_HEAP && rem[s] >= 2) touched[nt++] = s;  /* may repeat */
                if (--rem[s] == 0) newly[n_new++] = s;
            }
        }
        qsort(newly, (size_t)n_new, sizeof(int32_t), cmp_i32);
        if (variant == ORC_HEAP && !ie_static) {
            /* successors that dropped to one remaining predecessor this event */
            qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
            for (int32_t i = 0; i < nt; i++) {
                int32_t s = touched[i];
                if ((i > 0 && touched[i - 1] == s) || rem[s] != 1) continue;
                int32_t u = -1;
                for (int32_t e = prp[s]; e < prp[s + 1]; e++)
                    if (state[pcol[e]] != ST_DONE) { u = pcol[e]; break; }
                if ((int64_t)tau_of(est, n_gpu, u) + tau_of(est, n_gpu, s) > U) continue;
                ie[u]++;
                if (state[u] == ST_QUEUED && !static_key) {
                    hctx c0 = {ia, ie, seq, 0, R}, c1 = {ia, ie, seq, 1, R};
                    if (hpush(&H[2 * qw[u]], &c0, (hent){u, ie[u]}) ||
                        hpush(&H[2 * qw[u] + 1], &c1, (hent){u, ie[u]})) { rc = ORC_E_NOMEM; goto out; }
                }
            }
        }
    }
    *makespan = t;
    if (n_events) *n_events = (int32_t)events;

out:
    free(rem); free(ia); free(ie); free(seq); free(state); free(qw); free(newly); free(run);
    free(exp_end); free(qest); free(done_now); free(prp); free(pcol); free(touched); free(R); free(arr); free(home);
    if (Q) for (int32_t w = 0; w < W; w++) free(Q[w].a);
    if (H) for (int32_t w = 0; w < 2 * W; w++) free(H[w].a);
    free(Q);
    free(H);
    return rc;
}

static int check_params(int32_t n, int32_t n_cpu, int32_t n_gpu, const int32_t *dur, const int32_t *est,
                        const orc_params *p) {
    if (n_cpu < 0 || n_gpu < 0 || p->policy < 0 || p->policy > 5 || p->unit_time < 0 || p->max_events < 0 ||
        p->attr_mode < 0 || p->attr_mode > 1 || p->data_bw < 0 || (p->data_bw > 0 && !p->data_kib))
        return ORC_E_INVAL;
    if (p->data_bw > 0)
        for (int32_t v = 0; v < n; v++)
            if (p->data_kib[v] < 0 || p->data_kib[v] > ORC_MAX_TICK) return ORC_E_RANGE;
    int32_t W = n_cpu + n_gpu;
    if (W < 1 || W > ORC_MAX_W) return ORC_E_RANGE;
    if (n > ORC_MAX_N) return ORC_E_RANGE;
    if (p->k_num > ORC_MAX_TICK || p->k_den > ORC_MAX_TICK) return ORC_E_RANGE;
    if (check_ticks(n, dur) || check_ticks(n, est)) return ORC_E_RANGE;
    return ORC_OK;
}

/* Schedule one DAG given as a user CSR (canonicalised here).  Outputs are
 * indexed by task id; trace (nullable) receives one record per event up to
 * trace_cap. */
int orc_schedule(int32_t n, const int32_t *rp, const int32_t *col, int32_t n_cpu, int32_t n_gpu,
                 const int32_t *dur, const int32_t *est, const orc_params *p, int32_t variant, int32_t *worker,
                 int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop, int8_t *mode_at_pop,
                 orc_trace *trace, int32_t trace_cap, int32_t *n_events, int32_t *U_used) {
    if (n < 0) return ORC_E_INVAL;
    int rc = check_params(n, n_cpu, n_gpu, dur, est, p);
    if (rc) return rc;
    int32_t *crp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *ccol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[n] > 0 ? rp[n] : 1));
    if (!crp || !ccol) { free(crp); free(ccol); return ORC_E_NOMEM; }
    rc = orc_canon(n, rp, col, crp, ccol);
    if (!rc)
        rc = simulate(n, crp, ccol, n_cpu, n_gpu, dur, est, p, variant, worker, start, finish, makespan,
                      ie_at_pop, mode_at_pop, trace, trace_cap, n_events, U_used);
    free(crp);
    free(ccol);
    return rc;
}

/* ---------------------------------------------------------------- batch */

typedef struct {
    int32_t B;
    const int64_t *toff, *eoff;
    const int32_t *rp, *col, *n_cpu, *n_gpu, *dur, *est;
    const orc_params *p;
    int32_t variant;
    int32_t *worker, *ie_at_pop, *status;
    int64_t *start, *finish, *makespan;
    int8_t *mode_at_pop;
    int32_t next;
    pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg) {
    batch_job *j = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int32_t b = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (b >= j->B) break;
        int64_t t0 = j->toff[b], e0 = j->eoff[b];
        int32_t n = (int32_t)(j->toff[b + 1] - t0);
        orc_params pb = *j->p;
        if (pb.data_kib) pb.data_kib += t0;
        j->status[b] = orc_schedule(n, j->rp + t0 + b, j->col + e0, j->n_cpu[b], j->n_gpu[b], j->dur + 2 * t0,
                                    j->est + 2 * t0, &pb, j->variant, j->worker + t0, j->start + t0,
                                    j->finish + t0, j->makespan + b, j->ie_at_pop ? j->ie_at_pop + t0 : NULL,
                                    j->mode_at_pop ? j->mode_at_pop + t0 : NULL, NULL, 0, NULL, NULL);
    }
    return NULL;
}

/* Schedule B independent DAGs laid out back to back (task_off/edge_off are
 * prefix sums; DAG b's local row pointer starts at row_ptr[task_off[b] + b])
 * on n_threads host threads.  Per-DAG status codes go to status[b]. */
int orc_schedule_batch(int32_t B, const int64_t *task_off, const int64_t *edge_off, const int32_t *row_ptr,
                       const int32_t *col, const int32_t *n_cpu, const int32_t *n_gpu, const int32_t *dur,
                       const int32_t *est, const orc_params *p, int32_t variant, int32_t n_threads,
                       int32_t *worker, int64_t *start, int64_t *finish, int64_t *makespan, int32_t *ie_at_pop,
                       int8_t *mode_at_pop, int32_t *status) {
    batch_job j = {B, task_off, edge_off, row_ptr, col, n_cpu, n_gpu, dur, est, p, variant,
                   worker, ie_at_pop, status, start, finish, makespan, mode_at_pop, 0, PTHREAD_MUTEX_INITIALIZER};
    if (n_threads < 1) n_threads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    if (!th) return ORC_E_NOMEM;
    for (int32_t i = 0; i < n_threads; i++) pthread_create(&th[i], NULL, batch_worker, &j);
    for (int32_t i = 0; i < n_threads; i++) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&j.mu);
    for (int32_t b = 0; b < B; b++)
        if (status[b]) return status[b];
    return ORC_OK;
}

/* ----------------------------------------------------------- brute force */

typedef struct {
    int32_t n, W, n_cpu;
    const int32_t *rp, *col, *dur;
    int32_t npred[16];
    int64_t fin[16], avail[64], best;
} bf_ctx;

static void bf_rec(bf_ctx *c, uint32_t placed, int64_t cur) {
    if (cur >= c->best) return;
    if (placed == (1u << c->n) - 1) { c->best = cur; return; }
    for (int32_t v = 0; v < c->n; v++) {
        if (placed & (1u << v) || c->npred[v]) continue;
        int64_t ready = 0;
        for (int32_t u = 0; u < c->n; u++)
            if (placed & (1u << u))
                for (int32_t e = c->rp[u]; e < c->rp[u + 1]; e++)
                    if (c->col[e] == v && c->fin[u] > ready) ready = c->fin[u];
        for (int32_t w = 0; w < c->W; w++) {
            int k = w < c->n_cpu ? 0 : 1;
            /* identical workers with the same free time are interchangeable */
            int dup = 0;
            for (int32_t x = (k ? c->n_cpu : 0); x < w; x++)
                if (c->avail[x] == c->avail[w]) { dup = 1; break; }
            if (dup) continue;
            int64_t s = c->avail[w] > ready ? c->avail[w] : ready;
            int64_t f = s + c->dur[2 * v + k];
            int64_t saved = c->avail[w];
            c->avail[w] = f;
            c->fin[v] = f;
            for (int32_t e = c->rp[v]; e < c->rp[v + 1]; e++) c->npred[c->col[e]]--;
            bf_rec(c, placed | (1u << v), cur > f ? cur : f);
            for (int32_t e = c->rp[v]; e < c->rp[v + 1]; e++) c->npred[c->col[e]]++;
            c->avail[w] = saved;
        }
    }
}

/* Minimum makespan over all schedules (each task on one worker for its true
 * duration, no overlap on a worker, precedence respected), by exhaustive
 * search over the order in which tasks are placed and the worker each goes
 * to, every task starting as early as its worker and predecessors allow.
 * Every optimal schedule is reproduced by placing its tasks in start order,
 * so the search is exact.  n <= 12 and W <= 8 (canonical CSR). */
int orc_brute_opt(int32_t n, const int32_t *rp, const int32_t *col, int32_t n_cpu, int32_t n_gpu,
                  const int32_t *dur, int64_t *opt) {
    int32_t W = n_cpu + n_gpu;
    if (n < 0 || n > 12 || W < 1 || W > 8) return ORC_E_RANGE;
    bf_ctx c;
    memset(&c, 0, sizeof c);
    c.n = n; c.W = W; c.n_cpu = n_cpu; c.rp = rp; c.col = col; c.dur = dur;
    c.best = INT64_MAX;
    for (int32_t e = 0; e < rp[n]; e++) c.npred[col[e]]++;
    bf_rec(&c, 0, 0);
    *opt = n == 0 ? 0 : c.best;
    return ORC_OK;
}
