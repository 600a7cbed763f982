// Opt-in per-kernel timing: when enabled, every launcher brackets its kernel with a
// pair of HIP events recorded on the launch stream.  Durations are resolved when the
// totals are read (after the caller synchronised), so timing adds two event records
// per launch and no synchronisation.
#include <cstdlib>
#include <mutex>
#include <vector>

#include "pdep_internal.h"

namespace pdep {

namespace {

struct Pending {
    int kid;
    hipEvent_t a, b;
    double bytes, flops;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    unsigned mask = ~0u;   // kernel classes that are timed while on
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[K_COUNT] = {0};
    long long count[K_COUNT] = {0};
    double bytes[K_COUNT] = {0};
    double flops[K_COUNT] = {0};

    hipEvent_t ev() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        PDEP_HIP(hipEventCreate(&e));
        return e;
    }
    void resolve() {
        for (auto& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                total_ms[p.kid] += ms;
                count[p.kid] += 1;
                bytes[p.kid] += p.bytes;
                flops[p.kid] += p.flops;
            } else {
                (void)hipGetLastError();
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};

Profiler& prof() {
    static Profiler p;
    return p;
}

const char* kNames[K_COUNT] = {"sphere_to_sticks", "slab_hv",    "sticks_to_sphere", "slab_inv_store",
                               "slab_fwd_product", "slab_density", "gemm_ahb",      "gemm_update",
                               "row_dots",         "cg_update",    "misc",          "slab_hv_fp64",
                               "sphere_to_sticks_fp64", "sticks_to_sphere_fp64", "gemm_ahb_fp64",
                               "gemm_update_fp64"};

}  // namespace

namespace {
thread_local int g_suspended = 0;   // ProfSuspend scopes open on this thread
}

bool profiling_on() { return prof().on && g_suspended == 0; }

ProfSuspend::ProfSuspend() { ++g_suspended; }
ProfSuspend::~ProfSuspend() { --g_suspended; }

ProfScope::ProfScope(int kid, hipStream_t s, double bytes, double flops)
    : kid_(kid), s_(s), bytes_(bytes), flops_(flops) {
    Profiler& p = prof();
    if (!p.on || !((p.mask >> kid) & 1u) || g_suspended > 0) return;
    std::lock_guard<std::mutex> g(p.mu);
    a_ = p.ev();
    b_ = p.ev();
    PDEP_HIP(hipEventRecord(a_, s_));
    active_ = true;
}

ProfScope::~ProfScope() {
    if (!active_) return;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (hipEventRecord(b_, s_) != hipSuccess) {
        (void)hipGetLastError();
        p.pool.push_back(a_);
        p.pool.push_back(b_);
        return;
    }
    p.pending.push_back({kid_, a_, b_, bytes_, flops_});
}

bool verbose() {
    static const bool v = std::getenv("PDEP_VERBOSE") != nullptr;
    return v;
}

}  // namespace pdep

extern "C" {

int pdep_profile_enable(int on) {
    pdep::Profiler& p = pdep::prof();
    std::lock_guard<std::mutex> g(p.mu);
    try {
        p.resolve();
    } catch (...) {
    }
    p.on = on != 0;
    return PDEP_OK;
}

int pdep_profile_set_classes(unsigned mask) {
    pdep::Profiler& p = pdep::prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.mask = mask;
    return PDEP_OK;
}

int pdep_profile_read(int reset, double* total_ms, long long* launches, double* bytes, double* flops,
                      int max_kernels) {
    pdep::Profiler& p = pdep::prof();
    std::lock_guard<std::mutex> g(p.mu);
    try {
        p.resolve();
    } catch (...) {
        return PDEP_EDEVICE;
    }
    for (int k = 0; k < pdep::K_COUNT && k < max_kernels; ++k) {
        if (total_ms) total_ms[k] = p.total_ms[k];
        if (launches) launches[k] = p.count[k];
        if (bytes) bytes[k] = p.bytes[k];
        if (flops) flops[k] = p.flops[k];
    }
    if (reset)
        for (int k = 0; k < pdep::K_COUNT; ++k) {
            p.total_ms[k] = 0.0;
            p.count[k] = 0;
            p.bytes[k] = 0.0;
            p.flops[k] = 0.0;
        }
    return PDEP_OK;
}

const char* pdep_profile_kernel_name(int k) {
    return (k >= 0 && k < pdep::K_COUNT) ? pdep::kNames[k] : "";
}

}  // extern "C"
