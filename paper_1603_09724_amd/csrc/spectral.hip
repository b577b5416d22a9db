// Spectral apply kernels (see spectral.h).
//
// Fused path (2D, column fits in LDS): one workgroup per column loads it once
// from HBM into LDS, runs the forward 2D FFT (axis-0 lines, then axis-1
// lines), multiplies by the Fourier multiplier, runs the inverse 2D FFT and
// writes the post-processed result once: one HBM read and one write per
// column element (plus V and, for POST_SHIFTED_H, a re-read of the input).
//
// Multi-pass path (3D, or FP64 128^2 whose 256 KB column exceeds LDS): one
// kernel per axis pass over batches of lines; the last axis does forward,
// multiply and inverse in one pass.
#include "spectral.h"
#include "prof.h"

#include <cmath>
#include <vector>

namespace pomm {

namespace {

constexpr int kEPT = 16;   // FFT elements per thread

template <typename T>
__device__ __forceinline__ cplx<T> mult_value(const SpecArgs<T>& a, int group, int kflat, int k1, int k2, int k3) {
    if (a.mult_mode == MULT_KINETIC) {
        return mk<T>((T)(0.5 * (double)(k1 * k1 + k2 * k2 + k3 * k3)), (T)0);
    } else if (a.mult_mode == MULT_TABLE) {
        return a.mult_tab[kflat];  // the kernels offset mult_tab to the column's group
    } else {
        const cplx<double> c = a.group_c[group];
        const double re = 0.5 * (double)(k1 * k1 + k2 * k2 + k3 * k3) + c.re, im = c.im;
        const double d = re * re + im * im;
        return mk<T>((T)(re / d), (T)(-im / d));
    }
}

template <typename T>
__device__ __forceinline__ cplx<T> post_value(const SpecArgs<T>& a, int group, cplx<T> t, const cplx<T>* xin,
                                              long j, int col) {
    if (a.post_mode == POST_NONE) return t;
    const cplx<T> x = xin[j];
    double sre = a.sigma, sim = 0.0;
    if (a.post_shift) {
        sre = a.post_shift[group].re;
        sim = a.post_shift[group].im;
    }
    const T vr = a.V[j] - (T)sre;
    const T vi = -(T)sim;
    const cplx<T> h = mk<T>(t.re + vr * x.re - vi * x.im, t.im + vr * x.im + vi * x.re);
    if (a.post_mode == POST_RESIDUAL) {
        const cplx<double> b = a.rhs[(long)(col % a.cols_per_group) * a.ld_rhs + j];
        return mk<T>((T)(b.re - (double)h.re), (T)(b.im - (double)h.im));
    }
    return h;
}

// ---------------------------------------------------------------- fused 2D
template <typename T>
__global__ void __launch_bounds__(1024) spectral2d_fused(SpecArgs<T> a, RadixPlan plan, const cplx<T>* __restrict__ twg,
                                                         long tab_ld, int pitch) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    const int m = plan.m;
    cplx<T>* buf = tw + m;
    const int n = m * m;
    const int col = blockIdx.x;
    if (a.col_mask && a.col_mask[col] == 0) return;
    const int group = col / a.cols_per_group;
    for (int t = threadIdx.x; t < m; t += blockDim.x) tw[t] = twg[t];
    const cplx<T>* x = a.in + (long)col * a.ld_in;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int j2 = j / m, j1 = j - j2 * m;
        buf[j2 * pitch + j1] = x[j];
    }
    __syncthreads();
    const LineSet rows{m, pitch, 1}, cols{m, 1, pitch};
    lds_fft<kEPT, false>(buf, rows, plan, tw);
    lds_fft<kEPT, false>(buf, cols, plan, tw);
    SpecArgs<T> aa = a;
    if (a.mult_mode == MULT_TABLE) aa.mult_tab = a.mult_tab + (long)group * tab_ld;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int j2 = j / m, j1 = j - j2 * m;
        const cplx<T> f = mult_value(aa, group, j, freq_of(j1, m), freq_of(j2, m), 0);
        cplx<T>& b = buf[j2 * pitch + j1];
        b = b * f;
    }
    __syncthreads();
    lds_fft<kEPT, true>(buf, cols, plan, tw);
    lds_fft<kEPT, true>(buf, rows, plan, tw);
    const T inv_n = (T)(1.0 / (double)n);
    cplx<T>* y = a.out + (long)col * a.ld_out;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int j2 = j / m, j1 = j - j2 * m;
        const cplx<T> t = inv_n * buf[j2 * pitch + j1];
        y[j] = post_value(a, group, t, x, j, col);
    }
}

// ---------------------------------------------------------------- multi-pass
enum PassMode : int { PASS_FWD = 0, PASS_FWD_MULT_INV = 1, PASS_INV = 2, PASS_INV_POST = 3 };

// Lines of `axis` of column blockIdx.y; this block handles lines
// [blockIdx.x*L, blockIdx.x*L + L) in the order described in line_base().
__device__ __forceinline__ long line_base(int dim, int m, int axis, int line) {
    if (axis == 0) return (long)line * m;                     // line = j2 + m j3
    const int j1 = line % m, rest = line / m;
    if (dim == 2) return j1;                                   // axis 1
    if (axis == 1) return j1 + (long)m * m * rest;             // rest = j3
    return j1 + (long)m * rest;                                // axis 2, rest = j2
}

template <typename T>
__global__ void __launch_bounds__(256) spectral_lines(SpecArgs<T> a, RadixPlan plan, const cplx<T>* __restrict__ twg,
                                                      long tab_ld, int dim, int axis, int mode, int L, int pitch,
                                                      const cplx<T>* __restrict__ src, long ld_src,
                                                      cplx<T>* __restrict__ dst, long ld_dst) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
    const int m = plan.m;
    cplx<T>* buf = tw + m;
    const int col = blockIdx.y;
    if (a.col_mask && a.col_mask[col] == 0) return;
    const int group = col / a.cols_per_group;
    const int line0 = blockIdx.x * L;
    long stride = 1;
    for (int i = 0; i < axis; ++i) stride *= m;
    for (int t = threadIdx.x; t < m; t += blockDim.x) tw[t] = twg[t];
    const cplx<T>* xs = src + (long)col * ld_src;
    const int total = L * m;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int l, e;
        if (axis == 0) { l = idx / m; e = idx - l * m; }
        else { e = idx / L; l = idx - e * L; }
        buf[l * pitch + e] = xs[line_base(dim, m, axis, line0 + l) + e * stride];
    }
    __syncthreads();
    const LineSet ls{L, pitch, 1};
    if (mode == PASS_FWD || mode == PASS_FWD_MULT_INV) lds_fft<kEPT, false>(buf, ls, plan, tw);
    if (mode == PASS_FWD_MULT_INV) {
        SpecArgs<T> aa = a;
        if (a.mult_mode == MULT_TABLE) aa.mult_tab = a.mult_tab + (long)group * tab_ld;
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int l = idx / m, e = idx - l * m;
            const int line = line0 + l;
            const long flat = line_base(dim, m, axis, line) + e * stride;
            // frequency coordinates of this element: all axes have been transformed
            const int c1 = (int)(flat % m), c2 = (int)((flat / m) % m), c3 = dim == 3 ? (int)(flat / ((long)m * m)) : 0;
            const cplx<T> f = mult_value(aa, group, (int)flat, freq_of(c1, m), freq_of(c2, m),
                                         dim == 3 ? freq_of(c3, m) : 0);
            buf[l * pitch + e] = buf[l * pitch + e] * f;
        }
        __syncthreads();
    }
    if (mode != PASS_FWD) lds_fft<kEPT, true>(buf, ls, plan, tw);
    cplx<T>* yd = dst + (long)col * ld_dst;
    long n = 1;
    for (int i = 0; i < dim; ++i) n *= m;
    const T scale = (T)(1.0 / (double)n);
    const cplx<T>* xin = a.in + (long)col * a.ld_in;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int l, e;
        if (axis == 0) { l = idx / m; e = idx - l * m; }
        else { e = idx / L; l = idx - e * L; }
        const long flat = line_base(dim, m, axis, line0 + l) + e * stride;
        cplx<T> t = buf[l * pitch + e];
        if (mode == PASS_INV_POST) t = post_value(a, group, scale * t, xin, flat, col);
        yd[flat] = t;
    }
}

template <typename T>
const cplx<T>* tw_of(const SpectralPlan& sp) {
    if constexpr (sizeof(T) == 8) return reinterpret_cast<const cplx<T>*>(sp.tw64);
    else return reinterpret_cast<const cplx<T>*>(sp.tw32);
}

}  // namespace

void spectral_plan_init(SpectralPlan& sp, int dim, int m, size_t lds_limit) {
    POMM_CHECK(dim == 2 || dim == 3, 1, "dim must be 2 or 3");
    POMM_CHECK(m >= 8 && m <= 128 && m % 2 == 0, 1, "m must be even, 8..128");
    sp.dim = dim;
    sp.m = m;
    sp.n = 1;
    for (int i = 0; i < dim; ++i) sp.n *= m;
    // radix plan: 4s, then a 3, then a 2
    int r = m, ns = 0;
    while (r % 4 == 0 && r > 1) { sp.plan.radix[ns++] = 4; r /= 4; }
    if (r % 3 == 0) { sp.plan.radix[ns++] = 3; r /= 3; }
    if (r % 2 == 0) { sp.plan.radix[ns++] = 2; r /= 2; }
    POMM_CHECK(r == 1, 1, "grid side must be 2^a * 3^b with b <= 1");
    sp.plan.m = m;
    sp.plan.nstages = ns;
    sp.lds_limit = lds_limit;
    sp.pitch = m + 1;
    if (dim == 2) {
        const size_t need64 = (size_t)(m + (size_t)m * sp.pitch) * 16;
        const size_t need32 = (size_t)(m + (size_t)m * sp.pitch) * 8;
        sp.fused_lds64 = need64 <= lds_limit ? need64 : 0;
        sp.fused_lds32 = need32 <= lds_limit ? need32 : 0;
        int th = (sp.n + kEPT - 1) / kEPT;
        th = ((th + 63) / 64) * 64;
        sp.fused_threads = th > 1024 ? 1024 : th;
    }
    // multi-pass: L lines per block with L*m = 2048 elements (256 threads x 8)
    sp.lines_per_block = 2048 / m;
    if (sp.lines_per_block < 1) sp.lines_per_block = 1;
    while ((sp.n / m) % sp.lines_per_block) sp.lines_per_block /= 2;
    std::vector<double> t64(2 * m);
    std::vector<float> t32(2 * m);
    for (int t = 0; t < m; ++t) {
        // exp(-2 pi i t/m) with exact values at the quarter points
        const double ang = -2.0 * M_PI * (double)t / (double)m;
        double c = std::cos(ang), s = std::sin(ang);
        if (4 * t == m) { c = 0; s = -1; }
        if (2 * t == m) { c = -1; s = 0; }
        if (4 * t == 3 * m) { c = 0; s = 1; }
        t64[2 * t] = c;
        t64[2 * t + 1] = s;
        t32[2 * t] = (float)c;
        t32[2 * t + 1] = (float)s;
    }
    POMM_HIP(hipMalloc(&sp.tw64, 16 * m));
    POMM_HIP(hipMalloc(&sp.tw32, 8 * m));
    POMM_HIP(hipMemcpy(sp.tw64, t64.data(), 16 * m, hipMemcpyHostToDevice));
    POMM_HIP(hipMemcpy(sp.tw32, t32.data(), 8 * m, hipMemcpyHostToDevice));
}

void spectral_plan_free(SpectralPlan& sp) {
    if (sp.tw64) (void)hipFree(sp.tw64);
    if (sp.tw32) (void)hipFree(sp.tw32);
    sp.tw64 = sp.tw32 = nullptr;
}

template <typename T>
bool spectral_needs_work(const SpectralPlan& sp) {
    if (spectral_reg_available<T>(sp)) return false;
    const size_t fused = sizeof(T) == 8 ? sp.fused_lds64 : sp.fused_lds32;
    return !(sp.dim == 2 && fused > 0);
}

template <typename T>
bool spectral_chain_available(const SpectralPlan& sp) {
    return spectral_reg_available<T>(sp);
}

template <typename T>
void spectral_apply(const SpectralPlan& sp, const SpecArgs<T>& a, cplx<T>* work, hipStream_t s) {
    if (a.ncols <= 0) return;
    POMM_CHECK(!a.chain_tab || spectral_chain_available<T>(sp), 1, "chained spectral apply not available here");
    POMM_CHECK(!a.comb || spectral_reg_available<T>(sp), 1, "combined epilogue not available here");
    // algorithmic traffic: read the input, write the output, read V once; 10 n log2 n flops per column
    const double act = a.active_hint >= 0 ? a.active_hint : a.ncols;
    const double bytes = act * 2.0 * sizeof(cplx<T>) * sp.n + (a.post_mode != POST_NONE ? sizeof(T) * sp.n : 0) +
                         (a.post_mode == POST_RESIDUAL ? act * sizeof(cplx<double>) * sp.n : 0);
    const double flops = (a.chain_tab ? 2.0 : 1.0) * act * 10.0 * sp.n * std::log2((double)sp.n);
    ProfScope prof(PK_SPECTRAL, bytes, flops, s, spectral_needs_work<T>(sp) ? (sp.dim == 2 ? 3 : 5) : 1);
    const cplx<T>* tw = tw_of<T>(sp);
    const long tab_ld = sp.n;
    if (spectral_reg_available<T>(sp)) {
        spectral_reg_apply<T>(sp, a, s);
        return;
    }
    if (!spectral_needs_work<T>(sp)) {
        const size_t lds = sizeof(T) == 8 ? sp.fused_lds64 : sp.fused_lds32;
        hipLaunchKernelGGL(spectral2d_fused<T>, dim3(a.ncols), dim3(sp.fused_threads), lds, s, a, sp.plan, tw,
                           tab_ld, sp.pitch);
        check_launch("spectral2d_fused");
        return;
    }
    POMM_CHECK(work != nullptr, 1, "spectral_apply: multi-pass path needs a work buffer");
    const int L = sp.lines_per_block, m = sp.m;
    const int pitch = m + 1;
    const size_t lds = sizeof(cplx<T>) * ((size_t)m + (size_t)L * pitch);
    const int lines = sp.n / m;
    dim3 grid(lines / L, a.ncols);
    const int threads = ((L * m / kEPT + 63) / 64) * 64;
    const long ldw = sp.n;
    auto pass = [&](int axis, int mode, const cplx<T>* src, long lds_, cplx<T>* dst, long ldd) {
        hipLaunchKernelGGL(spectral_lines<T>, grid, dim3(threads), lds, s, a, sp.plan, tw, tab_ld, sp.dim, axis, mode, L,
                           pitch, src, lds_, dst, ldd);
        check_launch("spectral_lines");
    };
    if (sp.dim == 2) {
        pass(0, PASS_FWD, a.in, a.ld_in, work, ldw);
        pass(1, PASS_FWD_MULT_INV, work, ldw, work, ldw);
        pass(0, PASS_INV_POST, work, ldw, a.out, a.ld_out);
    } else {
        pass(0, PASS_FWD, a.in, a.ld_in, work, ldw);
        pass(1, PASS_FWD, work, ldw, work, ldw);
        pass(2, PASS_FWD_MULT_INV, work, ldw, work, ldw);
        pass(1, PASS_INV, work, ldw, work, ldw);
        pass(0, PASS_INV_POST, work, ldw, a.out, a.ld_out);
    }
}

template void spectral_apply<double>(const SpectralPlan&, const SpecArgs<double>&, cplx<double>*, hipStream_t);
template void spectral_apply<float>(const SpectralPlan&, const SpecArgs<float>&, cplx<float>*, hipStream_t);
template bool spectral_chain_available<double>(const SpectralPlan&);
template bool spectral_chain_available<float>(const SpectralPlan&);
template bool spectral_needs_work<double>(const SpectralPlan&);
template bool spectral_needs_work<float>(const SpectralPlan&);

}  // namespace pomm
