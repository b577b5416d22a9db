// Spectral apply: out = post( F^{-1}( mult(k) . F(in) ) ) for a batch of
// columns on the periodic grid.  This is the H.X apply of Section 4.1
// (kinetic symbol |k|^2/2 in Fourier space, V in real space) and, with other
// multipliers, the Fourier-diagonal parts of the GMRES operator and of the
// sparsifying preconditioner (Q G b, Section 3.2).
#pragma once

#include "common.h"
#include "fft.h"

namespace pomm {

enum MultMode : int {
    MULT_KINETIC = 0,       // |k|^2/2
    MULT_TABLE = 1,         // mult_tab[group * n + kflat]
    MULT_INV_SHIFTED = 2,   // 1/(|k|^2/2 + c_group)
};
enum PostMode : int {
    POST_NONE = 0,          // out = t
    POST_SHIFTED_H = 1,     // out = t + (V - s_group) * in   (s real sigma or complex pole)
    POST_RESIDUAL = 2,      // out = rhs_col - (t + (V - s_group) * in): the residual b - (H - z) x
};

template <typename T>
struct SpecArgs {
    const cplx<T>* in = nullptr;
    long ld_in = 0;
    cplx<T>* out = nullptr;
    long ld_out = 0;
    int ncols = 0;
    int cols_per_group = 1;        // group = column / cols_per_group (the pole index)
    int mult_mode = MULT_KINETIC;
    const cplx<T>* mult_tab = nullptr;   // MULT_TABLE: per group, n entries (order: spectral_table_reorder)
    const cplx<double>* group_c = nullptr;  // MULT_INV_SHIFTED: per group constant
    int post_mode = POST_NONE;
    const T* V = nullptr;          // POST_SHIFTED_H: potential (n reals)
    const cplx<double>* post_shift = nullptr;  // per group shift; null -> real `sigma`
    double sigma = 0.0;
    const cplx<double>* rhs = nullptr;  // POST_RESIDUAL: column (col % cols_per_group) at rhs + c * ld_rhs
    long ld_rhs = 0;
    // Chained second apply (register kernel only, spectral_chain_available): the result of
    // the first is not written but transformed again with the table multiplier chain_tab
    // (no post step) and written to chain_out (ld_out).
    const cplx<T>* chain_tab = nullptr;
    cplx<T>* chain_out = nullptr;
    // POST_SHIFTED_H on the register kernel (spectral_reg_available, no chain): the output is
    // comb_a h + comb_b comb instead of h, comb laid out as out (it may be out itself; it is
    // not read when comb_b == 0)
    const cplx<T>* comb = nullptr;
    double comb_a = 1.0, comb_b = 0.0;
    const int* col_mask = nullptr; // columns with col_mask[col] == 0 are skipped (left untouched)
    int active_hint = -1;          // columns expected to be active (profiling counts only); -1 = ncols
};

struct SpectralPlan {
    int dim = 2, m = 0, n = 0;
    RadixPlan plan{};
    int pitch = 0;              // LDS row pitch of the fused 2D kernel
    size_t fused_lds64 = 0, fused_lds32 = 0;   // bytes; 0 = does not fit
    int fused_threads = 0;
    int lines_per_block = 0;    // multi-pass kernel
    void* tw64 = nullptr;       // device twiddles exp(-2 pi i t/m), complex128
    void* tw32 = nullptr;       // complex64
    size_t lds_limit = 0;
};

void spectral_plan_init(SpectralPlan& sp, int dim, int m, size_t lds_limit);
void spectral_plan_free(SpectralPlan& sp);

// `work` must hold n*ncols elements when the column does not fit the fused
// kernel (multi-pass path); it may be null otherwise.
template <typename T>
void spectral_apply(const SpectralPlan& sp, const SpecArgs<T>& a, cplx<T>* work, hipStream_t s);

template <typename T>
bool spectral_needs_work(const SpectralPlan& sp);

// MULT_TABLE tables: natural FFT order (k1 + m k2) in, kernel order out (the
// register kernel reads its multipliers in register-slot order; other kernels
// use the natural order and get a copy).  ntab tables of n entries each.
template <typename T>
void spectral_table_reorder(const SpectralPlan& sp, const cplx<T>* in, cplx<T>* out, int ntab, hipStream_t s);
template <typename T>
bool spectral_table_reordered(const SpectralPlan& sp);

// Register/transposition kernel for 2D m in {32, 64, 128} (spectral_reg.hip).
template <typename T>
bool spectral_reg_available(const SpectralPlan& sp);
template <typename T>
void spectral_reg_apply(const SpectralPlan& sp, const SpecArgs<T>& a, hipStream_t s);
// Whether spectral_apply takes SpecArgs::chain_tab (two applies in one pass over the data).
template <typename T>
bool spectral_chain_available(const SpectralPlan& sp);

}  // namespace pomm
