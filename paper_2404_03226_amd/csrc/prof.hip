// Opt-in kernel timing: HIP events recorded on the caller's stream around
// each library launch, summed per kernel name on request.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace insp {
namespace {

struct Rec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};

struct Prof {
    std::mutex mu;
    int on = 0;  // 0 off, 1 every scope, 2 outermost scopes only
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<std::string, std::pair<double, int64_t>>> done;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void settle() {
        for (Rec &r : pending) {
            float ms = 0.f;
            if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                bool found = false;
                for (auto &d : done)
                    if (d.first == r.name) {
                        d.second.first += ms;
                        d.second.second += 1;
                        found = true;
                    }
                if (!found) done.push_back({r.name, {ms, 1}});
            }
            if (r.a) pool.push_back(r.a);
            if (r.b) pool.push_back(r.b);
        }
        pending.clear();
    }
};

Prof &prof() {
    static Prof p;
    return p;
}

}  // namespace

// Marks are not recorded while this thread captures a graph.
static thread_local int t_suspended = 0;
// Nesting depth of this thread's scopes (mode 2 records the outermost only).
static thread_local int t_depth = 0;

void prof_suspend(bool on) { t_suspended += on ? 1 : -1; }

void prof_mark(hipStream_t st, const char *kernel, bool begin) {
    const int depth = begin ? ++t_depth : t_depth--;
    if (t_suspended) return;
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (p.on == 0 || (p.on == 2 && depth != 1)) return;
    if (begin) {
        Rec r;
        r.name = kernel;
        r.a = p.get();
        if (r.a) (void)hipEventRecord(r.a, st);
        p.pending.push_back(r);
    } else {
        for (auto it = p.pending.rbegin(); it != p.pending.rend(); ++it)
            if (it->name == kernel && !it->b) {
                it->b = p.get();
                if (it->b) (void)hipEventRecord(it->b, st);
                break;
            }
    }
}

}  // namespace insp

using namespace insp;

extern "C" int insp_profile_enable(int on) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!on) {
        for (Rec &r : p.pending) {
            if (r.a) p.pool.push_back(r.a);
            if (r.b) p.pool.push_back(r.b);
        }
        p.pending.clear();
        p.done.clear();
    }
    p.on = on == 2 ? 2 : (on != 0 ? 1 : 0);
    return INSP_OK;
}

extern "C" int insp_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.settle();
    double ms = 0;
    int64_t n = 0;
    const char *k = kernel ? kernel : "";
    for (auto &d : p.done)
        if (d.first.compare(0, strlen(k), k) == 0) {
            ms += d.second.first;
            n += d.second.second;
        }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    return INSP_OK;
}
