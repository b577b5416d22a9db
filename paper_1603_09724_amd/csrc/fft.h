// Device-side Stockham FFT on lines held in LDS.
//
// A set of `nlines` lines of length m sits in LDS at buf[line*ls + elem*es].
// One call of stockham_stage<R> performs one radix-R Stockham autosort pass
// over all lines with the whole workgroup: butterfly b = (line, j),
// j in [0, m/R), reads the R inputs j + r*m/R, twiddles them by
// exp(-+2 pi i (j mod Ns) r / (Ns R)), takes the length-R DFT and writes the
// outputs to (j / Ns)*Ns*R + (j mod Ns) + r*Ns, where Ns is the product of
// the radices of the earlier passes.  After all passes the lines hold their
// DFT in natural order.  Reads complete before a barrier and writes follow
// it, so the pass is in place.
#pragma once

#include "common.h"

namespace pomm {

constexpr int kMaxStages = 8;

struct RadixPlan {
    int m;
    int nstages;
    int radix[kMaxStages];
};

// Forward DFT of length R in registers (sign -1); INV uses sign +1.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
    if constexpr (R == 2) {
        cplx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R == 3) {
        // omega = exp(-+2 pi i/3) = -1/2 -+ i sqrt(3)/2
        const T s3 = (T)0.86602540378443864676;
        cplx<T> a = v[0], b = v[1], c = v[2];
        cplx<T> t = b + c, d = b - c;
        cplx<T> m1 = a - (T)0.5 * t;
        // -+ i*s3*d
        cplx<T> rot = INV ? mk<T>(-s3 * d.im, s3 * d.re) : mk<T>(s3 * d.im, -s3 * d.re);
        v[0] = a + t;
        v[1] = m1 + rot;
        v[2] = m1 - rot;
    } else if constexpr (R == 4) {
        cplx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cplx<T> s0 = a + c, s1 = a - c, s2 = b + d, s3 = b - d;
        // forward: X1 = s1 - i s3, X3 = s1 + i s3 ; inverse swaps the sign
        cplx<T> is3 = mk<T>(-s3.im, s3.re);  // i*s3
        v[0] = s0 + s2;
        v[2] = s0 - s2;
        if (INV) {
            v[1] = s1 + is3;
            v[3] = s1 - is3;
        } else {
            v[1] = s1 - is3;
            v[3] = s1 + is3;
        }
    } else {
        static_assert(R == 2 || R == 3 || R == 4, "unsupported radix");
    }
}

struct LineSet {
    int nlines;
    int ls;  // line stride (elements)
    int es;  // element stride (elements)
};

// One radix-R pass.  tw[t] = exp(-2 pi i t/m) for t in [0, m).
// SLOTS >= ceil(nlines*m/R / blockDim.x).
template <int R, int SLOTS, bool INV, typename T>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, const LineSet ls, const int m, const int Ns,
                                               const cplx<T>* tw) {
    const int mR = m / R;
    const int total = ls.nlines * mR;
    const int twstep = m / (Ns * R);
    cplx<T> v[SLOTS][R];
    int dst[SLOTS], lb[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int b = threadIdx.x + s * blockDim.x;
        dst[s] = -1;
        if (b < total) {
            const int line = b / mR, j = b - line * mR;
            const cplx<T>* base = buf + line * ls.ls;
#pragma unroll
            for (int r = 0; r < R; ++r) v[s][r] = base[(j + r * mR) * ls.es];
            const int k = j % Ns;
            const int step = k * twstep;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cplx<T> t = tw[(step * r) % m];
                if (INV) t.im = -t.im;
                v[s][r] = v[s][r] * t;
            }
            dft_small<R, INV>(v[s]);
            dst[s] = (j / Ns) * Ns * R + k;
            lb[s] = line * ls.ls;
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        if (dst[s] >= 0) {
            cplx<T>* base = buf + lb[s];
#pragma unroll
            for (int r = 0; r < R; ++r) base[(dst[s] + r * Ns) * ls.es] = v[s][r];
        }
    }
    __syncthreads();
}

// Full FFT of every line in `ls` (all passes of `plan`).  EPT is the number of
// line elements per thread (nlines*m <= EPT*blockDim.x).
template <int EPT, bool INV, typename T>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, const LineSet ls, const RadixPlan& plan, const cplx<T>* tw) {
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        const int R = plan.radix[s];
        if (R == 4)
            stockham_stage<4, (EPT + 3) / 4, INV>(buf, ls, plan.m, Ns, tw);
        else if (R == 2)
            stockham_stage<2, (EPT + 1) / 2, INV>(buf, ls, plan.m, Ns, tw);
        else
            stockham_stage<3, (EPT + 2) / 3, INV>(buf, ls, plan.m, Ns, tw);
        Ns *= R;
    }
}

__host__ __device__ inline int freq_of(int j, int m) { return j < m / 2 ? j : j - m; }

}  // namespace pomm
