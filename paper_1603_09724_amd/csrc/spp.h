// Sparsifying preconditioner (Section 3.2) for the shifted systems (H - z_j) y = b.
//
// Per pole z_j, with l = <V> and G_j = (-Laplacian/2 + l - z_j)^{-1}:
//   * stencil q_j on the 3x3 neighbourhood minimizing ||q^T G_j(a, a^c)||
//     (so that Q G_j is essentially supported on the stencil);
//   * t_s = (Q G_j)(0, s) and the sparse matrix P_j(i, i+s) = q_s + t_s (V_{i+s} - l) (eq. P);
//   * the preconditioner M_j^{-1} b = P_j^{-1} (Q G_j b), with Q G_j applied in
//     Fourier space and P_j^{-1} by an exact sparse direct factorization.
//
// Direct solver: P_j is block cyclic-tridiagonal over the m grid lines (each
// line couples to its two neighbours through the 3x3 stencil).  Block cyclic
// reduction eliminates every other line per level (all levels batched over
// lines and poles on the GPU, dense line blocks, complex GEMMs); the last one
// or three lines are solved with a dense inverse.  On the first level the line
// blocks are still the sparse stencil: the diagonal blocks are cyclic
// tridiagonal (solved by a bordered tridiagonal LU, O(m) per column) and the
// couplings are applied as stencil products.
#pragma once

#include <complex>
#include <vector>

#include "common.h"
#include "dense.h"
#include "spectral.h"

namespace pomm {

struct SppLevel {
    int step = 1;
    std::vector<int> odd, even;
    size_t off_ainv = 0, off_f = 0, off_g = 0, off_alpha = 0, off_gamma = 0;  // per level, x (pole stride)
};

enum SppPhase : int { PH_GEMM = 0, PH_STENCIL_FWD = 1, PH_STENCIL_BWD = 2, PH_TRI_FWD = 3, PH_TRI_BWD = 4 };

struct Spp {
    int m = 0, b = 0, p = 0, N = 0, n = 0;
    double l = 0.0;                  // <V>
    std::vector<SppLevel> levels;
    std::vector<int> final_lines;
    // The solve stops the reduction at level cut_level, once at most 8 lines (cut_lines)
    // are left, and applies the inverse of their reduced system, fcut (p blocks of order
    // mc m, column major, mc = cut_lines.size()), computed at setup from the remaining
    // levels and the final inverse applied to the identity.  cut_level = levels.size():
    // the factored final is used as it is.
    int cut_level = 0;
    std::vector<int> cut_lines;
    cplx<double>* fcut = nullptr;
    cplx<float>* fcut32 = nullptr;
    size_t off_final = 0;            // (mf*b)^2 per pole
    size_t fac_elems = 0;            // all factors, all poles
    std::vector<size_t> level_base; // element offset of each level region
    size_t final_base = 0;
    cplx<double>* fac = nullptr;     // factors (complex128)
    cplx<float>* fac32 = nullptr;    // complex64 copy for the mixed-precision solve
    cplx<double>* mult = nullptr;    // Q G_j in Fourier space, p x n
    cplx<float>* mult32 = nullptr;
    std::vector<std::complex<double>> q, t;   // p x 9
    std::vector<double> farfield;    // ||q^T G(a, a^c)|| per pole
    // solve task lists for the fixed rhs/solution buffers
    GemmTask<double>* tasks64 = nullptr;
    GemmTask<float>* tasks32 = nullptr;
    std::vector<int> task_begin;     // per phase (fwd levels, final, bwd levels)
    std::vector<int> task_count;
    std::vector<int> phase_kind;       // PH_GEMM, PH_STENCIL_FWD, PH_STENCIL_BWD
    std::vector<double> phase_flops;   // all poles active
    std::vector<double> phase_bytes;
    // level-0 line blocks (cyclic tridiagonal): bordered-LU factors per (pole, odd line),
    // tri_stride(m) entries each (see spp.hip)
    cplx<double>* tri = nullptr;
    cplx<float>* tri32 = nullptr;
    bool pcr = false;                  // power-of-two m: cyclic-reduction multipliers in tri

    // complex64 solve with split products (gemm_split): factor blocks as fp16 tiles in place
    // of fac32 (split_planes 4: hi and lo; 2: hi alone), and their task list
    bool split = false;
    int split_planes = 4;
    int split_variant = -1;        // gemm_split workgroup shape (-1: chosen per launch)
    void* fac16 = nullptr;
    SplitTask* tasks16 = nullptr;

    cplx<double>* qs_d = nullptr;      // stencils q and t on the device (level-0 sparse products)
    cplx<double>* ts_d = nullptr;
    const double* V = nullptr;         // device potential (owned by the caller)
    cplx<double>* R = nullptr;       // rhs buffer (n x p*N), destroyed by the solve
    cplx<double>* X = nullptr;       // solution buffer (n x p*N)
    cplx<float>* R32 = nullptr;
    cplx<float>* X32 = nullptr;
};

// Build stencils, P_j and their factorization for poles z (unshifted frame).
// V is the device potential (FP64).  R/X: complex128 solve buffers (n x p*N,
// system s = pole*N + column), fixed for the lifetime of the preconditioner;
// null when only the complex64 solve is wanted.  R32/X32: the complex64
// buffers, used when want32 (factors are then also kept in complex64, or, with
// split_planes 4 or 2, as fp16 hi/lo or hi tiles for the split-product GEMM; 0: not split).
void spp_setup(Spp& sp, const SpectralPlan& plan, const double* V_dev, double l,
               const std::vector<std::complex<double>>& z, int N, cplx<double>* R, cplx<double>* X,
               cplx<float>* R32, cplx<float>* X32, bool want32, int split_planes, hipStream_t s);
void spp_free(Spp& sp);

// X = P_j^{-1} R for every pole (all N columns of a pole at once).  R is
// overwritten.  pole_active (device, p ints) gates whole poles; may be null.
template <typename T>
void spp_solve(const Spp& sp, const int* pole_active, int active_poles, hipStream_t s);

// Largest pole count per (grid side) that the factor storage allows; bytes per pole.
size_t spp_bytes_per_pole(int m, bool want32);

}  // namespace pomm
