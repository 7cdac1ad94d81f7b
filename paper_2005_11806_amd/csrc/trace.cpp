// Per-kernel HIP-event timing of a plan's launches (psv_trace_* in psv.h).
#include <cstdio>
#include <map>
#include <string>

#include "internal.hpp"

namespace psv {

// The events only time launches: recording them without the default
// system-scope fence keeps them from writing back and invalidating the caches
// between a kernel and the next, which would slow the next kernel and count in
// its time. Waiting on them still waits for the work before them.
hipEvent_t Trace::get() {
    if (next == pool.size()) {
        hipEvent_t e;
        PSV_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        pool.push_back(e);
    }
    return pool[next++];
}

void Trace::release_all() {
    recs.clear();
    next = 0;
}

TraceScope::TraceScope(const Plan& p, const char* name, hipStream_t s)
    : t_(p.trace.on ? &p.trace : nullptr), s_(s), idx_(0) {
    if (!t_) return;
    TraceRec r{name, t_->get(), t_->get()};
    PSV_HIP(hipEventRecord(r.a, s_));
    idx_ = t_->recs.size();
    t_->recs.push_back(r);
}

TraceScope::~TraceScope() {
    if (t_) (void)hipEventRecord(t_->recs[idx_].b, s_);
}

// Synchronises on the last event and writes {"name": [launches, total_ms], ...}.
std::string trace_summary(Plan& p) {
    std::map<std::string, std::pair<long, double>> acc;
    for (auto& r : p.trace.recs) {
        PSV_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        PSV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        auto& e = acc[r.name];
        e.first += 1;
        e.second += ms;
    }
    std::string out = "{";
    bool first = true;
    for (auto& kv : acc) {
        char buf[256];
        std::snprintf(buf, sizeof(buf), "%s\"%s\": [%ld, %.9g]", first ? "" : ", ", kv.first.c_str(),
                      kv.second.first, kv.second.second);
        out += buf;
        first = false;
    }
    out += "}";
    p.trace.release_all();
    return out;
}

void trace_free(Plan& p) {
    for (hipEvent_t e : p.trace.pool) (void)hipEventDestroy(e);
    p.trace.pool.clear();
    p.trace.release_all();
}

}  // namespace psv
