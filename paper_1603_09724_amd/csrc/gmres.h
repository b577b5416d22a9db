// Batched restarted GMRES for the rough shifted solves of the Fermi-pole
// preconditioner (Section 3.1, eqs. direct and lst; settings of Section 4).
//
// S = p * N independent systems (H - z_j) y = g_c, system s = j*N + c, all
// advanced in lockstep with per-system convergence masks.  Right
// preconditioning (A M^{-1} u = r, y = y0 + M^{-1} u, stop on the true
// residual relative to ||g||) or left preconditioning (GMRES on M^{-1} A, stop
// on the preconditioned residual relative to its initial value: for a stiff
// operator in single precision the true residual carries round-off of size
// eps ||A|| ||y|| that M^{-1} damps).  Modified Gram-Schmidt Arnoldi, Givens
// rotations, the residual recomputed at every restart, initial guess y0 = g
// (the right-hand side itself, as in the paper).
#pragma once

#include <complex>
#include <vector>

#include "common.h"
#include "spectral.h"
#include "spp.h"

namespace pomm {

struct GmresWork {
    int S = 0, n = 0, N = 0, p = 0, restart = 0;
    bool fp32 = false;            // Krylov vectors in complex64 (else complex128)
    // Krylov vectors at the working precision (complex64 or complex128)
    void* Vb = nullptr;           // (restart+1) x S x n basis
    void* Xs = nullptr;           // S x n solutions
    void* W = nullptr;            // S x n operator outputs
    void* U = nullptr;            // S x n (= SPP rhs buffer)
    void* Z = nullptr;            // S x n (= SPP solution buffer)
    cplx<double>* work = nullptr; // S x n complex128 multi-pass FFT scratch (large grids)
    // small per-system state, always complex128
    cplx<double>* Hh = nullptr;   // S x (restart+1) x restart
    cplx<double>* cs = nullptr;   // S x restart
    cplx<double>* sn = nullptr;
    cplx<double>* g = nullptr;    // S x (restart+1)
    cplx<double>* ys = nullptr;   // S x restart: the final cycle's least-squares solutions
    double* bnorm = nullptr;      // S
    int* active = nullptr;        // S: in the current cycle's Arnoldi process
    int* done = nullptr;          // S: converged
    int* kcyc = nullptr;          // S: steps taken this cycle
    int* pole_active = nullptr;   // p
    int* counter = nullptr;       // device: per-pole active counts (p)
    unsigned long long* steps = nullptr;  // device: Arnoldi steps (all systems)
    int* counter_host = nullptr;  // pinned
    cplx<double>* pole_z = nullptr;   // p poles (device)
    cplx<double>* pole_w = nullptr;   // p weights (device)
};

void gmres_alloc(GmresWork& w, int n, int N, int p, int restart, bool multipass, bool fp32);
void gmres_free(GmresWork& w);

struct PrecondConfig {
    int inner = 0;           // 0 = SPP, 1 = PP
    double rtol = 1e-5;
    int restart = 15;
    int cycles = 5;
    bool left = false;       // left preconditioning (M^{-1} A); else right (A M^{-1})
    bool verify = true;      // recompute the residual before accepting convergence
    double l = 0.0;          // <V>
};

// PG (n x ncols, complex128) = sum_j w_j Y_j, (H - z_j) Y_j = G, ncols <= N.
// The solves run at the workspace precision (V_dev / V32_dev is the potential
// in that precision); G is read and PG accumulated in complex128.
void fermi_precondition(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg,
                        const double* V_dev, const float* V32_dev, const cplx<double>* G, cplx<double>* PG,
                        int ncols, hipStream_t s);

// Y (n x ncols, complex128) = M_pole^{-1} B: the inner preconditioner of one
// pole (SPP: P_j^{-1} Q G_j B; PP: the Fourier diagonal), at the workspace
// precision.  Uses the GMRES workspace as staging.
void inner_apply(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg, int pole,
                 const cplx<double>* B, cplx<double>* Y, int ncols, hipStream_t s);

}  // namespace pomm
