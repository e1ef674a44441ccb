// Optional per-phase timing with HIP events recorded on the caller's stream
// around each group of kernels (binning, build, project, m2p, adjoints).
// Off by default; when on, every phase costs two event records.
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace p2m {

namespace {

struct Rec {
    int phase;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<Rec> g_recs;
double g_total_ms[PH_COUNT];
long long g_count[PH_COUNT];

const char* kNames[PH_COUNT] = {"bin",       "build",      "project",    "m2p",        "m2p_bwd",
                                "project_bwd", "build_bwd", "build_fast", "build_slow", "weights",
                                "k_weights",   "k_weights_rd"};

hipEvent_t take() {
    if (g_pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
}

// Resolve finished records into the totals (caller holds the lock).
void drain(bool wait) {
    std::vector<Rec> keep;
    for (Rec& r : g_recs) {
        if (!wait && hipEventQuery(r.b) == hipErrorNotReady) {
            keep.push_back(r);
            continue;
        }
        (void)hipEventSynchronize(r.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_total_ms[r.phase] += ms;
            g_count[r.phase] += 1;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.swap(keep);
}

}  // namespace

PhaseTimer::PhaseTimer(int phase, hipStream_t st) : phase_(phase), st_(st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    a_ = take();
    b_ = take();
    if (a_ && b_) (void)hipEventRecord(a_, st_);
}

PhaseTimer::~PhaseTimer() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, st_);
    g_recs.push_back(Rec{phase_, a_, b_});
    if (g_recs.size() > 4096) drain(false);
}

}  // namespace p2m

extern "C" {

int p2m_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(p2m::g_mu);
    p2m::drain(true);
    for (int i = 0; i < p2m::PH_COUNT; ++i) {
        p2m::g_total_ms[i] = 0.0;
        p2m::g_count[i] = 0;
    }
    p2m::g_on = on != 0;
    return P2M_OK;
}

int p2m_profile_read(const char* phase, double* total_ms, int64_t* count) {
    std::lock_guard<std::mutex> lk(p2m::g_mu);
    p2m::drain(true);
    for (int i = 0; i < p2m::PH_COUNT; ++i) {
        if (phase && !std::strcmp(phase, p2m::kNames[i])) {
            if (total_ms) *total_ms = p2m::g_total_ms[i];
            if (count) *count = p2m::g_count[i];
            return P2M_OK;
        }
    }
    p2m::set_error("unknown profile phase '%s'", phase ? phase : "(null)");
    return P2M_EINVAL;
}

}  // extern "C"
