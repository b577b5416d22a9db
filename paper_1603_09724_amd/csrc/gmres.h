// Batched restarted GMRES for the rough shifted solves of the Fermi-pole
// preconditioner (Section 3.1, eqs. direct and lst; settings of Section 4).
//
// S = p * N independent systems (H - z_j) y = g_c, system s = j*N + c, all
// advanced in lockstep with per-system convergence masks.  Right
// preconditioning (A M^{-1} u = r, y = y0 + M^{-1} u), modified Gram-Schmidt
// Arnoldi, Givens rotations, the true residual recomputed at every restart,
// initial guess y0 = g (the right-hand side itself, as in the paper).
#pragma once

#include <complex>
#include <vector>

#include "common.h"
#include "spectral.h"
#include "spp.h"

namespace pomm {

struct GmresWork {
    int S = 0, n = 0, N = 0, p = 0, restart = 0;
    // complex128 state
    cplx<double>* Vb = nullptr;   // (restart+1) x S x n basis
    cplx<double>* Xs = nullptr;   // S x n solutions
    cplx<double>* W = nullptr;    // S x n operator outputs
    cplx<double>* U = nullptr;    // S x n (= SPP rhs buffer)
    cplx<double>* Z = nullptr;    // S x n (= SPP solution buffer)
    cplx<double>* work = nullptr; // S x n multi-pass FFT scratch (large grids)
    cplx<double>* Hh = nullptr;   // S x (restart+1) x restart
    cplx<double>* cs = nullptr;   // S x restart
    cplx<double>* sn = nullptr;
    cplx<double>* g = nullptr;    // S x (restart+1)
    double* bnorm = nullptr;      // S
    int* active = nullptr;        // S: in the current cycle's Arnoldi process
    int* done = nullptr;          // S: converged
    int* kcyc = nullptr;          // S: steps taken this cycle
    int* pole_active = nullptr;   // p
    int* counter = nullptr;       // device: active systems after a step
    unsigned long long* steps = nullptr;  // device: Arnoldi steps (all systems)
    int* counter_host = nullptr;  // pinned
    cplx<double>* pole_z = nullptr;   // p poles (device)
    cplx<double>* pole_w = nullptr;   // p weights (device)
};

void gmres_alloc(GmresWork& w, int n, int N, int p, int restart, bool multipass);
void gmres_free(GmresWork& w);

struct PrecondConfig {
    int inner = 0;           // 0 = SPP, 1 = PP
    double rtol = 1e-5;
    int restart = 15;
    int cycles = 5;
    double l = 0.0;          // <V>
};

// PG (n x ncols, complex128) = sum_j w_j Y_j, (H - z_j) Y_j = G, ncols <= N.
void fermi_precondition(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg,
                        const double* V_dev, const cplx<double>* G, cplx<double>* PG, int ncols, hipStream_t s);

}  // namespace pomm
