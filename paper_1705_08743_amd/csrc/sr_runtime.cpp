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

constexpr int kMaxDevices = 64;
std::mutex g_aux_mu[kMaxDevices];
Aux g_aux[kMaxDevices];
bool g_aux_ready[kMaxDevices];

}  // namespace

Aux *aux_acquire() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    g_aux_mu[dev].lock();
    if (!g_aux_ready[dev]) {
        Aux a{};
        // default priority: the two streams must not differ in priority
        if (hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&a.ev_main, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&a.ev_aux, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            g_aux_mu[dev].unlock();
            return nullptr;
        }
        a.device = dev;
        g_aux[dev] = a;
        g_aux_ready[dev] = true;
    }
    return &g_aux[dev];
}

void aux_release(Aux *a) {
    if (a) g_aux_mu[a->device].unlock();
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
