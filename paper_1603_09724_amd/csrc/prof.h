// Kernel-class timing with HIP events on the launching stream.
//
// When a handle enables profiling, every launch site wraps its kernel in a
// ProfScope that records an event before and after the launch together with
// the algorithmic bytes and flops of that launch.  collect() waits for the
// stream and accumulates elapsed time per kernel class, so a caller gets the
// average launch duration and the achieved rate of each class.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace pomm {

enum ProfKind : int {
    PK_SPECTRAL = 0,   // FFT-based applies (H.X, (H - z) z, Q G b, shifted-Laplacian inverse)
    PK_SPP_SOLVE,      // block cyclic reduction solve GEMMs
    PK_SPP_SETUP,      // stencils, assembly, factorization GEMMs and inversions
    PK_ARNOLDI,        // Gram-Schmidt + Givens step
    PK_GMRES_AUX,      // residual, cycle update, flags, pole sum
    PK_OMM,            // Gram products, gradient GEMM, quartic, updates, reductions
    PK_SPP_STENCIL,    // first level of the block cyclic reduction solve: tridiagonal solves, stencil products
    PK_COUNT
};

const char* prof_kind_name(int k);

struct ProfStats {
    double ms[PK_COUNT] = {0};
    double bytes[PK_COUNT] = {0};
    double flops[PK_COUNT] = {0};
    long long launches[PK_COUNT] = {0};
};

struct Profiler {
    bool on = false;
    unsigned mask = ~0u;   // classes recorded while on
    hipStream_t stream = nullptr;
    struct Rec {
        hipEvent_t a, b;
        int kind;
        double bytes, flops;
        int nlaunch;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    ProfStats stats;
    hipEvent_t get_event();
    void collect();
    void reset();
    void release();
};

// The profiler the current API call reports to (null when profiling is off).
Profiler*& current_profiler();

struct ProfScope {
    Profiler* p;
    hipEvent_t a = nullptr;
    int kind;
    double bytes, flops;
    int nlaunch;
    ProfScope(int kind_, double bytes_, double flops_, hipStream_t s, int nlaunch_ = 1);
    ~ProfScope();
    hipStream_t s;
};

}  // namespace pomm
