// Kernel-class timing (see prof.h).
#include <mutex>

#include "prof.h"

namespace pomm {

namespace {

// Events outlive handles: a released profiler returns its events here and the next
// one takes them back, so that profiled setups do not create and destroy thousands
// of events each.
std::mutex g_event_mu;
std::vector<hipEvent_t>& event_store() {
    static std::vector<hipEvent_t> v;
    return v;
}

}  // namespace

const char* prof_kind_name(int k) {
    switch (k) {
        case PK_SPECTRAL: return "spectral_apply";
        case PK_SPP_SOLVE: return "spp_solve_gemm";
        case PK_SPP_SETUP: return "spp_setup";
        case PK_ARNOLDI: return "arnoldi";
        case PK_GMRES_AUX: return "gmres_aux";
        case PK_OMM: return "omm_outer";
        case PK_SPP_STENCIL: return "spp_solve_level0";
        default: return "?";
    }
}

Profiler*& current_profiler() {
    static thread_local Profiler* p = nullptr;
    return p;
}

hipEvent_t Profiler::get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    {
        std::lock_guard<std::mutex> lock(g_event_mu);
        auto& st = event_store();
        if (!st.empty()) {
            hipEvent_t e = st.back();
            st.pop_back();
            return e;
        }
    }
    hipEvent_t e;
    POMM_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::collect() {
    if (recs.empty()) return;
    POMM_HIP(hipStreamSynchronize(stream));
    for (auto& r : recs) {
        float ms = 0.f;
        POMM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        stats.ms[r.kind] += ms;
        stats.bytes[r.kind] += r.bytes;
        stats.flops[r.kind] += r.flops;
        stats.launches[r.kind] += r.nlaunch;
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
}

void Profiler::reset() {
    collect();
    stats = ProfStats{};
}

void Profiler::release() {
    if (stream) (void)hipStreamSynchronize(stream);
    std::lock_guard<std::mutex> lock(g_event_mu);
    auto& st = event_store();
    for (auto& r : recs) {
        st.push_back(r.a);
        st.push_back(r.b);
    }
    recs.clear();
    st.insert(st.end(), pool.begin(), pool.end());
    pool.clear();
}

ProfScope::ProfScope(int kind_, double bytes_, double flops_, hipStream_t s_, int nlaunch_)
    : p(current_profiler()), kind(kind_), bytes(bytes_), flops(flops_), nlaunch(nlaunch_), s(s_) {
    if (p && p->on && ((p->mask >> kind) & 1u)) {
        a = p->get_event();
        POMM_HIP(hipEventRecord(a, s));
    } else {
        p = nullptr;
    }
}

ProfScope::~ProfScope() {
    if (!p) return;
    hipEvent_t b = p->get_event();
    if (hipEventRecord(b, s) != hipSuccess) return;
    p->recs.push_back(Profiler::Rec{a, b, kind, bytes, flops, nlaunch});
}

}  // namespace pomm
