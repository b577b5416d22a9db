// Fused 2D spectral apply for m = 16*R2 (m in {32, 64, 128}), one workgroup per column.
//
// Each thread holds 16 complex values.  A line FFT of length m = 16*R2 is a
// four-step transform across the R2 threads of the line: thread t2 holds
// x[t2 + R2 k] (k < 16), takes a 16-point DFT in registers, multiplies by
// w_m^{t2 k16}, exchanges through a wave-local LDS transpose so that it owns
// k16 in [t2 G, t2 G + G) (G = 16/R2) for every t2, and finishes with R2-point
// DFTs: X[k16 + 16 k2].  The inverse runs the same steps backwards from that
// frequency layout.  The 2D transform is: row FFTs, a block transpose through
// LDS to a column layout, column FFT, Fourier multiplier, inverse column FFT,
// block transpose back, inverse row FFTs, epilogue.  All index arithmetic is
// compile time except the thread id.  Exchanges move one real component per round,
// or whole complex values in one round for FP32 128x128 (complex_exchange).
#include <algorithm>

#include "prof.h"
#include "spectral.h"

namespace pomm {

namespace {

// cos and sin of 2 pi e/16
__device__ constexpr double kC16[16] = {1.0, 0.92387953251128676, 0.70710678118654752, 0.38268343236508977,
                                        0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128676,
                                        -1.0, -0.92387953251128676, -0.70710678118654752, -0.38268343236508977,
                                        0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128676};
__device__ constexpr double kS16[16] = {0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128676,
                                        1.0, 0.92387953251128676, 0.70710678118654752, 0.38268343236508977,
                                        0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128676,
                                        -1.0, -0.92387953251128676, -0.70710678118654752, -0.38268343236508977};

// a * w16^e with w16 = exp(-2 pi i/16) (forward) or its conjugate (INV)
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> rot16(cplx<T> a, int e) {
    const T c = (T)kC16[e & 15];
    const T s = INV ? (T)kS16[e & 15] : -(T)kS16[e & 15];
    return mk<T>(a.re * c - a.im * s, a.re * s + a.im * c);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>& a, cplx<T>& b, cplx<T>& c, cplx<T>& d) {
    const cplx<T> s0 = a + c, s1 = a - c, s2 = b + d, s3 = b - d;
    const cplx<T> is3 = mk<T>(-s3.im, s3.re);
    a = s0 + s2;
    c = s0 - s2;
    if (INV) {
        b = s1 + is3;
        d = s1 - is3;
    } else {
        b = s1 - is3;
        d = s1 + is3;
    }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4v(cplx<T>* v) { dft4<T, INV>(v[0], v[1], v[2], v[3]); }

// 8-point: radix 2 over two 4-point halves (even / odd inputs)
template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    o1 = rot16<T, INV>(o1, 2);
    o2 = rot16<T, INV>(o2, 4);
    o3 = rot16<T, INV>(o3, 6);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
}

// 16-point: input n = 4 n1 + n2 in natural order; output X[k1 + 4 k2] left in
// register v[4 k1 + k2], i.e. X[k] sits in v[P16(k)] (callers index through P16).
__host__ __device__ constexpr int P16(int k) { return 4 * (k & 3) + (k >> 2); }

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T>* v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<T, INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // now v[4 k1 + n2] = Y[n2][k1]
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) v[4 * k1 + n2] = rot16<T, INV>(v[4 * k1 + n2], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<T, INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // now v[4 k1 + k2] = X[k1 + 4 k2]
}

template <int R, typename T, bool INV>
__device__ __forceinline__ void dft_r(cplx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 4) dft4v<T, INV>(v);
    else dft8<T, INV>(v);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T& comp(cplx<T>& a, int c) { return c ? a.im : a.re; }

// Exchange slot access: with CX the slot holds a whole complex value (LDS viewed as
// cplx<T>), otherwise component c of it.
template <bool CX, typename T>
__device__ __forceinline__ void xput(T* base, int idx, const cplx<T>& v, int c) {
    if constexpr (CX) reinterpret_cast<cplx<T>*>(base)[idx] = v;
    else base[idx] = c ? v.im : v.re;
}
template <bool CX, typename T>
__device__ __forceinline__ void xget(const T* base, int idx, cplx<T>& v, int c) {
    if constexpr (CX) v = reinterpret_cast<const cplx<T>*>(base)[idx];
    else (c ? v.im : v.re) = base[idx];
}

// CX: exchanges move whole complex values in one round; otherwise one real component
// per round (half the LDS, so FP64 128 x 128 fits and smaller sizes keep several
// workgroups per CU).  Measured per size: one round pays off only for FP32 128 x 128,
// which runs one workgroup per CU either way.
template <typename T, int R2>
constexpr bool complex_exchange() { return sizeof(T) == 4 && R2 == 8; }

template <typename T, int R2>
struct RegFFT {
    static constexpr bool CX = complex_exchange<T, R2>();
    static constexpr int NC = CX ? 1 : 2;        // exchange rounds
    static constexpr int EW = CX ? 2 : 1;        // T words per exchanged element
    static constexpr int m = 16 * R2;
    static constexpr int G = 16 / R2;
    static constexpr int LPW = 64 / R2;          // lines per wave
    static constexpr int WROW = R2 + 1;          // padded k16 row of the wave transpose
    static constexpr int WLINE = 16 * WROW + 1;  // padded line
    static constexpr int NLR = m + R2;           // line pitch of the natural-order staging (R2 mod 32 banks)
    static constexpr int WREG = LPW * WLINE > LPW * NLR ? LPW * WLINE : LPW * NLR;   // per-wave region (T elements)

    // Staging index of local element lane + 64 i: (loc / m) NLR + loc % m = loc + (loc / m) R2,
    // with (lane + 64 i) / m = lane / m + 64 i / m since m divides 64 or 64 divides m.
    static __device__ __forceinline__ int nat_base(int lane) { return lane + (lane / m) * R2; }
    static constexpr int nat_off(int i) { return 64 * i + ((64 * i) / m) * R2; }

    // Natural order (lane l holds local element l + 64 i of the wave's LPW lines) to the
    // line-FFT layout (thread (line_w, t2) holds x[t2 + R2 k] of its line), component-wise.
    static __device__ __forceinline__ void to_lines(cplx<T>* v, T* wreg, int lane, int line_w, int t2) {
        const int nb = nat_base(lane);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wave_sync();
#pragma unroll
            for (int i = 0; i < 16; ++i) xput<CX>(wreg, nb + nat_off(i), v[i], c);
            wave_sync();
#pragma unroll
            for (int k = 0; k < 16; ++k) xget<CX>(wreg, line_w * NLR + t2 + R2 * k, v[k], c);
        }
    }
    // Inverse of to_lines, from v[P16(k)] = y[t2 + R2 k] back to natural order in v[i].
    static __device__ __forceinline__ void to_natural(cplx<T>* v, T* wreg, int lane, int line_w, int t2) {
        const int nb = nat_base(lane);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wave_sync();
#pragma unroll
            for (int k = 0; k < 16; ++k) xput<CX>(wreg, line_w * NLR + t2 + R2 * k, v[P16(k)], c);
            wave_sync();
#pragma unroll
            for (int i = 0; i < 16; ++i) xget<CX>(wreg, nb + nat_off(i), v[i], c);
        }
    }

    // forward line FFT: v[k] = x[t2 + R2 k]  ->  v[q R2 + k2] = X[t2 G + q + 16 k2]
    static __device__ __forceinline__ void fwd(cplx<T>* v, T* wreg, int line_w, int t2, const cplx<T>* twl) {
        dft16<T, false>(v);
#pragma unroll
        for (int k16 = 1; k16 < 16; ++k16) v[P16(k16)] = v[P16(k16)] * twl[t2 * k16];
        const int base = line_w * WLINE;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wave_sync();
#pragma unroll
            for (int k16 = 0; k16 < 16; ++k16) xput<CX>(wreg, base + k16 * WROW + t2, v[P16(k16)], c);
            wave_sync();
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int s = 0; s < R2; ++s) xget<CX>(wreg, base + (t2 * G + q) * WROW + s, v[q * R2 + s], c);
        }
#pragma unroll
        for (int q = 0; q < G; ++q) dft_r<R2, T, false>(v + q * R2);
    }

    // inverse line FFT (unnormalized) from the layout fwd produces back to v[P16(j)] = x[t2 + R2 j]
    static __device__ __forceinline__ void inv(cplx<T>* v, T* wreg, int line_w, int t2, const cplx<T>* twl) {
#pragma unroll
        for (int q = 0; q < G; ++q) dft_r<R2, T, true>(v + q * R2);
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int s = 1; s < R2; ++s) v[q * R2 + s] = v[q * R2 + s] * conj(twl[s * (t2 * G + q)]);
        const int base = line_w * WLINE;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wave_sync();
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int s = 0; s < R2; ++s) xput<CX>(wreg, base + (t2 * G + q) * WROW + s, v[q * R2 + s], c);
            wave_sync();
#pragma unroll
            for (int k16 = 0; k16 < 16; ++k16) xget<CX>(wreg, base + k16 * WROW + t2, v[k16], c);
        }
        dft16<T, true>(v);
    }
};

template <typename T>
__device__ __forceinline__ cplx<T> reg_mult(const SpecArgs<T>& a, const cplx<T>* tab, int group, int kflat, int k1,
                                            int k2) {
    if (a.mult_mode == MULT_KINETIC) return mk<T>((T)(0.5 * (double)(k1 * k1 + k2 * k2)), (T)0);
    if (a.mult_mode == MULT_TABLE) return tab[kflat];
    const cplx<double> c = a.group_c[group];
    const double re = 0.5 * (double)(k1 * k1 + k2 * k2) + c.re, im = c.im;
    const double d = re * re + im * im;
    return mk<T>((T)(re / d), (T)(-im / d));
}

// Global I/O order: natural (coalesced, one more wave-local exchange each way) where
// the kernel is limited by memory-request rate (small lines), strided line order where
// it is limited by LDS throughput (long FP64 lines and m = 128); measured per size.
template <typename T, int R2>
constexpr bool natural_io() { return sizeof(T) * R2 <= 16; }

// The plain FP32 kernel at m <= 64 fits 4 waves per SIMD (at most 128 VGPRs): asked for
// explicitly, since the allocator otherwise takes a few registers more and drops a wave.
template <typename T>
constexpr int reg_min_waves(int R2, bool plain) { return plain && sizeof(T) == 4 && R2 <= 4 ? 4 : 1; }

template <typename T, int R2, bool CHAIN, bool RESID, bool COMB = false>
__global__ void __launch_bounds__(16 * R2 * R2, reg_min_waves<T>(R2, !CHAIN && !RESID && !COMB)) spectral2d_reg(SpecArgs<T> a, const cplx<T>* __restrict__ twg,
                                                               long tab_ld) {
    using F = RegFFT<T, R2>;
    constexpr int m = F::m, G = F::G, PB = m + R2, TPC = 16 * R2 * R2;
    constexpr bool NAT = natural_io<T, R2>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* twl = reinterpret_cast<cplx<T>*>(smem_raw);     // m twiddles
    T* lds = reinterpret_cast<T*>(twl + m);                   // transposes (block and per-wave, time shared)
    const int col = blockIdx.x;
    if (a.col_mask && a.col_mask[col] == 0) return;
    const int group = col / a.cols_per_group;
    const int t = threadIdx.x, line = t / R2, t2 = t % R2;
    const int lane = t & 63, wave = t >> 6, line_w = lane / R2;
    T* wreg = lds + wave * F::WREG * F::EW;
    for (int i = t; i < m; i += blockDim.x) twl[i] = twg[i];

    // this wave's LPW lines are 1024 consecutive elements of the column: coalesced loads,
    // then the wave-local exchange to the line-FFT layout
    const long wbase = (long)wave * 1024;
    const cplx<T>* x = a.in + (long)col * a.ld_in + wbase;
    cplx<T> v[16];
    if constexpr (NAT) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = x[lane + 64 * i];
        F::to_lines(v, wreg, lane, line_w, t2);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = x[(t2 + R2 * k) + m * line_w];
    }

    // 2D transform of the column in v (row `line`: v[k] = x[t2 + R2 k]) with multiplier
    // `mode` (table `tab` in register order): forward rows, block transpose, forward
    // columns, multiplier, inverse columns, transpose back, inverse rows; on return
    // v[P16(k)] = y[t2 + R2 k] unnormalized.
    auto transform = [&](int mode, const cplx<T>* tab) {
        __syncthreads();
        // rows: thread (line = row r) -> X_row[r][k1 = t2 G + q + 16 k2] in v[q R2 + k2]
        F::fwd(v, wreg, line_w, t2, twl);
        // block transpose to columns: thread (line = column c) holds rows j2 = t2 + R2 k
#pragma unroll
        for (int c = 0; c < F::NC; ++c) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2)
                    xput<F::CX>(lds, line * PB + (t2 * G + q + 16 * k2), v[q * R2 + k2], c);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; ++k) xget<F::CX>(lds, (t2 + R2 * k) * PB + line, v[k], c);
        }
        __syncthreads();
        // columns: forward, Fourier multiplier at (k1 = freq(line), k2 = freq(kappa)), inverse
        F::fwd(v, wreg, line_w, t2, twl);
        const int k1 = freq_of(line, m);
        if (mode == MULT_KINETIC) {
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int kap = freq_of(t2 * G + q + 16 * k2, m);
                    v[q * R2 + k2] = (T)(0.5 * (double)(k1 * k1 + kap * kap)) * v[q * R2 + k2];
                }
        } else if (mode == MULT_TABLE) {
            // table in register order (spectral_table_reorder): slot s of thread t at s * TPC + t
            const cplx<T>* tb = tab + (long)group * tab_ld + t;
#pragma unroll
            for (int sl = 0; sl < 16; ++sl) v[sl] = v[sl] * tb[sl * TPC];
        } else {
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int kappa = t2 * G + q + 16 * k2;
                    v[q * R2 + k2] =
                        v[q * R2 + k2] * reg_mult<T>(a, (const cplx<T>*)nullptr, group, 0, k1, freq_of(kappa, m));
                }
        }
        F::inv(v, wreg, line_w, t2, twl);
        // block transpose back: thread (line = row r) holds Y[r][k1 = t2 G + q + 16 k2]
#pragma unroll
        for (int c = 0; c < F::NC; ++c) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; ++k) xput<F::CX>(lds, (t2 + R2 * k) * PB + line, v[P16(k)], c);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2)
                    xget<F::CX>(lds, line * PB + (t2 * G + q + 16 * k2), v[q * R2 + k2], c);
        }
        __syncthreads();
        F::inv(v, wreg, line_w, t2, twl);
    };

    transform(a.mult_mode, a.mult_tab);
    // epilogue: y = v / n (+ (V - s) x, or b - that); element of slot i at local offset
    // off(i).  Plain: stored at once; chained: kept in registers for the second transform.
    if constexpr (NAT) F::to_natural(v, wreg, lane, line_w, t2);
    auto off = [&](int i) { return NAT ? lane + 64 * i : (t2 + R2 * i) + m * line_w; };
    auto slot = [&](int i) { return NAT ? i : P16(i); };
    const T inv_n = (T)(1.0 / ((double)m * m));
    cplx<T>* yo = a.out + (long)col * a.ld_out + wbase;
    auto emit = [&](int i, cplx<T> val) {
        if constexpr (CHAIN) v[slot(i)] = val;
        else yo[off(i)] = val;
    };
    if (a.post_mode != POST_NONE) {
        double sre = a.sigma, sim = 0.0;
        if (a.post_shift) {
            sre = a.post_shift[group].re;
            sim = a.post_shift[group].im;
        }
        const T vi = -(T)sim;
        const T* Vw = a.V + wbase;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int j = off(i);
            const cplx<T> r = inv_n * v[slot(i)];
            const cplx<T> xv = x[j];
            const T vr = Vw[j] - (T)sre;
            const cplx<T> h = mk<T>(r.re + vr * xv.re - vi * xv.im, r.im + vr * xv.im + vi * xv.re);
            if constexpr (RESID) {   // residual b - (H - z) x, in double from the complex128 b
                const cplx<double> bj = a.rhs[(long)(col % a.cols_per_group) * a.ld_rhs + wbase + j];
                emit(i, mk<T>((T)(bj.re - (double)h.re), (T)(bj.im - (double)h.im)));
            } else if constexpr (COMB) {   // comb_a h + comb_b comb
                const T ca = (T)a.comb_a, cb = (T)a.comb_b;
                cplx<T> o = mk<T>(ca * h.re, ca * h.im);
                if (cb != (T)0) {
                    const cplx<T> pv = a.comb[(long)col * a.ld_out + wbase + j];
                    o = mk<T>(o.re + cb * pv.re, o.im + cb * pv.im);
                }
                emit(i, o);
            } else {
                emit(i, h);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) emit(i, inv_n * v[slot(i)]);
    }
    if constexpr (CHAIN) {
        // second transform on the result, still in registers: slot(i) holds the element at
        // off(i), the offsets of the input load, so it re-enters in the input layout
        if constexpr (!NAT) {
            cplx<T> tmp[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) tmp[i] = v[P16(i)];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = tmp[i];
        } else {
            F::to_lines(v, wreg, lane, line_w, t2);
        }
        transform(MULT_TABLE, a.chain_tab);
        if constexpr (NAT) F::to_natural(v, wreg, lane, line_w, t2);
        cplx<T>* y2 = a.chain_out + (long)col * a.ld_out + wbase;
#pragma unroll
        for (int i = 0; i < 16; ++i) y2[off(i)] = inv_n * v[slot(i)];
    }
}

template <typename T, int R2>
size_t reg_lds_bytes() {
    using F = RegFFT<T, R2>;
    constexpr int m = F::m;
    const size_t block = (size_t)m * (m + R2);
    const size_t waves = (size_t)(16 * R2 * R2 / 64) * F::WREG;
    return sizeof(cplx<T>) * m + sizeof(T) * F::EW * (block > waves ? block : waves);
}

template <typename T, int R2, bool CHAIN, bool RESID, bool COMB = false>
void launch_reg_k(const SpectralPlan& sp, const SpecArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
    const size_t lds = reg_lds_bytes<T, R2>();
    static const bool attr_set = [lds] {   // once per process, thread-safe
        (void)hipFuncSetAttribute((const void*)spectral2d_reg<T, R2, CHAIN, RESID, COMB>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((spectral2d_reg<T, R2, CHAIN, RESID, COMB>), dim3(a.ncols), dim3(16 * R2 * R2), lds, s, a,
                       tw, (long)sp.n);
    check_launch("spectral2d_reg");
}

template <typename T, int R2>
void launch_reg(const SpectralPlan& sp, const SpecArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
    const bool resid = a.post_mode == POST_RESIDUAL;
    if (a.comb) {
        POMM_CHECK(a.post_mode == POST_SHIFTED_H && !a.chain_tab, 1, "comb needs the plain shifted-H epilogue");
        launch_reg_k<T, R2, false, false, true>(sp, a, tw, s);
        return;
    }
    if (a.chain_tab) {
        if (resid) launch_reg_k<T, R2, true, true>(sp, a, tw, s);
        else launch_reg_k<T, R2, true, false>(sp, a, tw, s);
    } else {
        if (resid) launch_reg_k<T, R2, false, true>(sp, a, tw, s);
        else launch_reg_k<T, R2, false, false>(sp, a, tw, s);
    }
}

// out[s * TPC + t] = in[line + m * (t2 G + s / R2 + 16 (s % R2))] with line = t / R2, t2 = t % R2:
// the Fourier multiplier of register slot s of thread t in the column phase above.
template <typename T, int R2>
__global__ void table_reorder_kernel(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, int ntab) {
    constexpr int m = 16 * R2, G = 16 / R2, TPC = 16 * R2 * R2, n = m * m;
    const long total = (long)ntab * n;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long tb = e / n;
        const int o = (int)(e - tb * n), sl = o / TPC, t = o - sl * TPC;
        const int line = t / R2, t2 = t % R2;
        out[e] = in[tb * n + line + m * (t2 * G + sl / R2 + 16 * (sl % R2))];
    }
}

}  // namespace

template <typename T>
bool spectral_table_reordered(const SpectralPlan& sp) {
    return spectral_reg_available<T>(sp);
}

template <typename T>
void spectral_table_reorder(const SpectralPlan& sp, const cplx<T>* in, cplx<T>* out, int ntab, hipStream_t s) {
    const long total = (long)ntab * sp.n;
    if (!spectral_table_reordered<T>(sp)) {
        POMM_HIP(hipMemcpyAsync(out, in, sizeof(cplx<T>) * total, hipMemcpyDeviceToDevice, s));
        return;
    }
    const unsigned blocks = (unsigned)std::min<long>(4096, (total + 255) / 256);
    if (sp.m == 32) hipLaunchKernelGGL((table_reorder_kernel<T, 2>), dim3(blocks), dim3(256), 0, s, in, out, ntab);
    else if (sp.m == 64) hipLaunchKernelGGL((table_reorder_kernel<T, 4>), dim3(blocks), dim3(256), 0, s, in, out, ntab);
    else hipLaunchKernelGGL((table_reorder_kernel<T, 8>), dim3(blocks), dim3(256), 0, s, in, out, ntab);
    check_launch("table_reorder");
}

template <typename T>
bool spectral_reg_available(const SpectralPlan& sp) {
    if (sp.dim != 2) return false;
    size_t lds = 0;
    if (sp.m == 32) lds = reg_lds_bytes<T, 2>();
    else if (sp.m == 64) lds = reg_lds_bytes<T, 4>();
    else if (sp.m == 128) lds = reg_lds_bytes<T, 8>();
    else return false;
    return lds <= sp.lds_limit;
}

template <typename T>
void spectral_reg_apply(const SpectralPlan& sp, const SpecArgs<T>& a, hipStream_t s) {
    const cplx<T>* tw = sizeof(T) == 8 ? reinterpret_cast<const cplx<T>*>(sp.tw64)
                                       : reinterpret_cast<const cplx<T>*>(sp.tw32);
    if (sp.m == 32) launch_reg<T, 2>(sp, a, tw, s);
    else if (sp.m == 64) launch_reg<T, 4>(sp, a, tw, s);
    else launch_reg<T, 8>(sp, a, tw, s);
}

template bool spectral_reg_available<double>(const SpectralPlan&);
template bool spectral_reg_available<float>(const SpectralPlan&);
template void spectral_reg_apply<double>(const SpectralPlan&, const SpecArgs<double>&, hipStream_t);
template void spectral_reg_apply<float>(const SpectralPlan&, const SpecArgs<float>&, hipStream_t);
template bool spectral_table_reordered<double>(const SpectralPlan&);
template bool spectral_table_reordered<float>(const SpectralPlan&);
template void spectral_table_reorder<double>(const SpectralPlan&, const cplx<double>*, cplx<double>*, int, hipStream_t);
template void spectral_table_reorder<float>(const SpectralPlan&, const cplx<float>*, cplx<float>*, int, hipStream_t);

}  // namespace pomm
