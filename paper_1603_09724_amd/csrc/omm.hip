// Kernels of the outer OMM iteration (see omm.h).
//
// E_omm(X) = tr A - 1/2 tr(S A) with S = X*X and A = X*H_sigma X (eq. omm).
// Along X + a D: S(a) = S0 + a S1 + a^2 S2, A(a) = A0 + a A1 + a^2 A2 with
// S1 = C + C*, A1 = B + B* (C = X*D, B = X*HD; H Hermitian gives D*HX = B*),
// so E(a) is a quartic whose coefficients are traces of N x N products.
#include "omm.h"

namespace pomm {

namespace {

constexpr int kRedBlocks = 256;

__device__ double quartic_val(const double* c, double a) {
    return c[0] + a * (c[1] + a * (c[2] + a * (c[3] + a * c[4])));
}

// Real roots of the cubic E'(a) = c1 + 2 c2 a + 3 c3 a^2 + 4 c4 a^3 (c4 > 0), each
// polished by Newton steps; returns the count.
__device__ int cubic_real_roots(const double* c, double* r) {
    const double A = 3.0 * c[3] / (4.0 * c[4]);
    const double B = 2.0 * c[2] / (4.0 * c[4]);
    const double C = c[1] / (4.0 * c[4]);
    // a = t - A/3:  t^3 + p t + q = 0
    const double p = B - A * A / 3.0;
    const double q = 2.0 * A * A * A / 27.0 - A * B / 3.0 + C;
    const double disc = 0.25 * q * q + p * p * p / 27.0;
    int cnt = 0;
    if (disc > 0.0) {
        const double sq = sqrt(disc);
        const double u = cbrt(-0.5 * q + sq), v = cbrt(-0.5 * q - sq);
        r[cnt++] = u + v - A / 3.0;
    } else {
        const double rr = sqrt(fmax(-p / 3.0, 0.0));
        double arg = rr > 0.0 ? (-0.5 * q) / (rr * rr * rr) : 0.0;
        arg = fmin(1.0, fmax(-1.0, arg));
        const double phi = acos(arg);
        for (int k = 0; k < 3; ++k) r[cnt++] = 2.0 * rr * cos((phi - 2.0 * M_PI * k) / 3.0) - A / 3.0;
    }
    for (int i = 0; i < cnt; ++i) {
        double a = r[i];
        for (int it = 0; it < 3; ++it) {
            const double f = c[1] + a * (2.0 * c[2] + a * (3.0 * c[3] + a * 4.0 * c[4]));
            const double df = 2.0 * c[2] + a * (6.0 * c[3] + a * 12.0 * c[4]);
            if (df == 0.0) break;
            const double an = a - f / df;
            if (!isfinite(an)) break;
            a = an;
        }
        r[i] = a;
    }
    return cnt;
}

__global__ void __launch_bounds__(256) quartic_kernel(cplx<double>* __restrict__ gr, int N, OmmScalars* __restrict__ sc) {
    __shared__ double red[4];
    const long NN = (long)N * N;
    cplx<double>* S0 = gr;
    cplx<double>* A0 = gr + NN;
    const cplx<double>* Cm = gr + 2 * NN;
    const cplx<double>* S2 = gr + 3 * NN;
    const cplx<double>* Bm = gr + 4 * NN;
    const cplx<double>* A2 = gr + 5 * NN;
    // partial sums of the trace terms
    double t[12] = {0};
    for (long e = threadIdx.x; e < NN; e += blockDim.x) {
        const int a = (int)(e % N), b = (int)(e / N);
        const long ab = a + (long)b * N, ba = b + (long)a * N;
        // X[a,b] * Y[b,a] products (real parts)
        const cplx<double> s0ab = S0[ab], a0ba = A0[ba], a2ba = A2[ba], s2ab = S2[ab];
        const cplx<double> s1ab = Cm[ab] + conj(Cm[ba]);
        const cplx<double> a1ba = Bm[ba] + conj(Bm[ab]);
        t[0] += (s0ab * a0ba).re;   // tr(S0 A0)
        t[1] += (s0ab * a1ba).re;   // tr(S0 A1)
        t[2] += (s1ab * a0ba).re;   // tr(S1 A0)
        t[3] += (s0ab * a2ba).re;   // tr(S0 A2)
        t[4] += (s1ab * a1ba).re;   // tr(S1 A1)
        t[5] += (s2ab * a0ba).re;   // tr(S2 A0)
        t[6] += (s1ab * a2ba).re;   // tr(S1 A2)
        t[7] += (s2ab * a1ba).re;   // tr(S2 A1)
        t[8] += (s2ab * a2ba).re;   // tr(S2 A2)
        if (a == b) {
            t[9] += A0[ab].re;                 // tr A0
            t[10] += 2.0 * Bm[ab].re;          // tr A1
            t[11] += A2[ab].re;                // tr A2
        }
    }
    for (int i = 0; i < 12; ++i) t[i] = block_sum(t[i], red);
    __shared__ double alpha_s;
    if (threadIdx.x == 0) {
        double c[5];
        c[0] = t[9] - 0.5 * t[0];
        c[1] = t[10] - 0.5 * (t[1] + t[2]);
        c[2] = t[11] - 0.5 * (t[3] + t[4] + t[5]);
        c[3] = -0.5 * (t[6] + t[7]);
        c[4] = -0.5 * t[8];
        for (int i = 0; i < 5; ++i) sc->c[i] = c[i];
        double alpha = 0.0;
        int bad = !(c[4] > 0.0) || !isfinite(c[4]) || !isfinite(c[1]);
        if (!bad) {
            double r[3];
            const int cnt = cubic_real_roots(c, r);
            double best = 0.0, bestE = 0.0;
            bool have = false;
            for (int i = 0; i < cnt; ++i) {
                if (!isfinite(r[i])) continue;
                const double e = quartic_val(c, r[i]);
                if (!have || e < bestE || (e == bestE && fabs(r[i]) < fabs(best))) {
                    have = true;
                    best = r[i];
                    bestE = e;
                }
            }
            if (have) alpha = best;
            else bad = 1;
        }
        sc->breakdown = bad;
        sc->alpha = alpha;
        sc->energy = quartic_val(c, alpha);
        alpha_s = alpha;
    }
    __syncthreads();
    const double al = alpha_s, al2 = al * al;
    for (long e = threadIdx.x; e < NN; e += blockDim.x) {
        const int a = (int)(e % N), b = (int)(e / N);
        const long ba = b + (long)a * N;
        const cplx<double> s1 = Cm[e] + conj(Cm[ba]);
        const cplx<double> a1 = Bm[e] + conj(Bm[ba]);
        S0[e] = S0[e] + al * s1 + al2 * S2[e];
        A0[e] = A0[e] + al * a1 + al2 * A2[e];
    }
}

__global__ void __launch_bounds__(256) energy_kernel(const cplx<double>* __restrict__ gr, int N, OmmScalars* __restrict__ sc) {
    __shared__ double red[4];
    const long NN = (long)N * N;
    const cplx<double>* S0 = gr;
    const cplx<double>* A0 = gr + NN;
    double tsa = 0, ta = 0;
    for (long e = threadIdx.x; e < NN; e += blockDim.x) {
        const int a = (int)(e % N), b = (int)(e / N);
        tsa += (S0[a + (long)b * N] * A0[b + (long)a * N]).re;
        if (a == b) ta += A0[e].re;
    }
    tsa = block_sum(tsa, red);
    ta = block_sum(ta, red);
    if (threadIdx.x == 0) sc->energy = ta - 0.5 * tsa;
}

__global__ void step_update_kernel(cplx<double>* __restrict__ X, cplx<double>* __restrict__ HX,
                                   const cplx<double>* __restrict__ D, const cplx<double>* __restrict__ HD, long count,
                                   const OmmScalars* __restrict__ sc) {
    const double a = sc->alpha;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        X[i] = X[i] + a * D[i];
        HX[i] = HX[i] + a * HD[i];
    }
}

// parts[b] = sum over this block's grid-stride range of f0, parts[kRedBlocks + b] of f1
__global__ void __launch_bounds__(256) norms_partial_kernel(const cplx<double>* __restrict__ G,
                                                            const cplx<double>* __restrict__ HX, long count,
                                                            double* __restrict__ parts) {
    __shared__ double red[4];
    double a = 0, b = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        a += norm2(G[i]);
        b += norm2(HX[i]);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = a;
        parts[kRedBlocks + blockIdx.x] = b;
    }
}

__global__ void norms_final_kernel(const double* __restrict__ parts, OmmScalars* __restrict__ sc) {
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int i = 0; i < kRedBlocks; ++i) { a += parts[i]; b += parts[kRedBlocks + i]; }
        sc->gnorm2 = a;
        sc->hxnorm2 = b;
    }
}

// G = -PG;  partial Re<G, G - Gp> and Re<Gp, Gp>
__global__ void __launch_bounds__(256) pr_partial_kernel(const cplx<double>* __restrict__ PG,
                                                         const cplx<double>* __restrict__ Gp, long count,
                                                         double* __restrict__ parts) {
    __shared__ double red[4];
    double a = 0, b = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        const cplx<double> g = mk<double>(-PG[i].re, -PG[i].im);
        const cplx<double> gp = Gp[i];
        a += (cmulc(g, g - gp)).re;
        b += norm2(gp);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = a;
        parts[kRedBlocks + blockIdx.x] = b;
    }
}

__global__ void pr_final_kernel(const double* __restrict__ parts, OmmScalars* __restrict__ sc) {
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int i = 0; i < kRedBlocks; ++i) { a += parts[i]; b += parts[kRedBlocks + i]; }
        sc->dot_gdg = a;
        sc->dot_gpgp = b;
        const double beta = b > 0.0 ? a / b : 0.0;
        sc->beta = beta > 0.0 ? beta : 0.0;
    }
}

__global__ void direction_kernel(const cplx<double>* __restrict__ PG, cplx<double>* __restrict__ Gp,
                                 cplx<double>* __restrict__ D, long count, int first, const OmmScalars* __restrict__ sc) {
    const double beta = first ? 0.0 : sc->beta;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        const cplx<double> g = mk<double>(-PG[i].re, -PG[i].im);
        D[i] = first ? g : g + beta * D[i];
        Gp[i] = g;
    }
}

}  // namespace

void quartic_step(cplx<double>* grams, int N, OmmScalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(quartic_kernel, dim3(1), dim3(256), 0, s, grams, N, sc);
    check_launch("quartic");
}

void energy_from_grams(const cplx<double>* grams, int N, OmmScalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(256), 0, s, grams, N, sc);
    check_launch("energy");
}

void step_update(cplx<double>* X, cplx<double>* HX, const cplx<double>* D, const cplx<double>* HD, long count,
                 const OmmScalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(step_update_kernel, dim3(1024), dim3(256), 0, s, X, HX, D, HD, count, sc);
    check_launch("step_update");
}

void grad_norms(const cplx<double>* G, const cplx<double>* HX, long count, double* parts, OmmScalars* sc,
                hipStream_t s) {
    hipLaunchKernelGGL(norms_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, G, HX, count, parts);
    check_launch("norms_partial");
    hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(64), 0, s, parts, sc);
    check_launch("norms_final");
}

void cg_direction(const cplx<double>* PG, cplx<double>* Gp, cplx<double>* D, long count, int first, double* parts,
                  OmmScalars* sc, hipStream_t s) {
    if (!first) {
        hipLaunchKernelGGL(pr_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, PG, Gp, count, parts);
        check_launch("pr_partial");
        hipLaunchKernelGGL(pr_final_kernel, dim3(1), dim3(64), 0, s, parts, sc);
        check_launch("pr_final");
    }
    hipLaunchKernelGGL(direction_kernel, dim3(1024), dim3(256), 0, s, PG, Gp, D, count, first, sc);
    check_launch("direction");
}

}  // namespace pomm
