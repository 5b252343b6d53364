// Host runtime pieces shared by the launchers:
//  * the second stream (and its two events) that a closure uses to overlap
//    the next round's pivot and panels with the bulk of the current update;
//  * kernel timing for the closures (a tracing aid behind sr_profile_enable /
//    sr_profile_read): while enabled, every launch of a closure phase is
//    bracketed by a pair of hipEvents recorded on the launch's own stream,
//    and the algorithmic work of the launch (semiring updates) is noted.
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

#include "sr_internal.h"

namespace sr {
namespace {

struct Rec {
    hipEvent_t start, stop;
    int kind, phase;
    double units;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local hipEvent_t t_start = nullptr;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// One second stream (with its two events) per (device, caller stream): two
// closures enqueued on different caller streams then overlap each other as
// well.  The table is small and never shrinks; each entry is locked while a
// closure enqueues its fork/join sequence.
struct AuxEntry {
    int device;
    hipStream_t caller;
    Aux aux;
    std::mutex mu;
};
constexpr int kMaxAux = 64;
std::mutex g_aux_table_mu;
AuxEntry g_aux_table[kMaxAux];
int g_aux_count = 0;

}  // namespace

Aux *aux_acquire(hipStream_t caller, bool create) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    AuxEntry *entry = nullptr;
    {
        std::lock_guard<std::mutex> g(g_aux_table_mu);
        for (int i = 0; i < g_aux_count; i++)
            if (g_aux_table[i].device == dev && g_aux_table[i].caller == caller) {
                entry = &g_aux_table[i];
                break;
            }
        if (!entry) {
            // none yet: create one, unless the caller may not create streams
            // (then the closure runs its phases in order on its own stream)
            if (!create || g_aux_count == kMaxAux) return nullptr;  // table full: no lookahead
            Aux a{};
            // default priority: the two streams must not differ in priority
            // The events only order the two streams of one device, so a
            // device-scope release is enough (no system-scope cache flush).
            const unsigned evf = hipEventDisableTiming | hipEventReleaseToDevice;
            if (hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&a.ev_main, evf) != hipSuccess ||
                hipEventCreateWithFlags(&a.ev_aux[0], evf) != hipSuccess ||
                hipEventCreateWithFlags(&a.ev_aux[1], evf) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            a.device = dev;
            a.slot = g_aux_count;
            entry = &g_aux_table[g_aux_count++];
            entry->device = dev;
            entry->caller = caller;
            entry->aux = a;
        }
    }
    entry->mu.lock();
    return &entry->aux;
}

void aux_release(Aux *a) {
    if (a) g_aux_table[a->slot].mu.unlock();
}

bool prof_on() {
    std::lock_guard<std::mutex> g(g_mu);
    return g_on;
}

void prof_begin(hipStream_t st) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_on) return;
    t_start = get_event();
    if (t_start) (void)hipEventRecord(t_start, st);
}

void prof_end(hipStream_t st, int kind, int phase, double units) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_on || !t_start) return;
    hipEvent_t stop = get_event();
    if (!stop) return;
    (void)hipEventRecord(stop, st);
    g_recs.push_back(Rec{t_start, stop, kind, phase, units});
    t_start = nullptr;
}

int prof_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_on = on != 0;
    return 0;
}

int prof_read(int kind, int phase, double *ms, int64_t *launches, double *units) {
    std::vector<Rec> mine, rest;
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (const Rec &r : g_recs) (r.kind == kind && r.phase == phase ? mine : rest).push_back(r);
        g_recs.swap(rest);
    }
    double total = 0.0, u = 0.0;
    int64_t n = 0;
    hipError_t err = hipSuccess;
    for (const Rec &r : mine) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) err = e;
        total += t;
        u += r.units;
        n++;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (const Rec &r : mine) {
            g_pool.push_back(r.start);
            g_pool.push_back(r.stop);
        }
    }
    if (ms) *ms = total;
    if (launches) *launches = n;
    if (units) *units = u;
    return err == hipSuccess ? 0 : -1;
}

}  // namespace sr
