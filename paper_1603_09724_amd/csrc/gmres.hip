// Batched restarted GMRES and the Fermi-pole preconditioner (see gmres.h).
#include "gmres.h"
#include "prof.h"

namespace pomm {

namespace {

constexpr int kArnThreads = 1024;
constexpr int kArnEPT = 16;   // n <= 16384 on 2D grids: the working vector stays in registers

// x_s = g_c (the initial guess is the right-hand side); columns c >= ncols are parked as done.
template <typename T>
__global__ void init_solution_kernel(const cplx<double>* __restrict__ G, int n, int N, int ncols,
                                     cplx<T>* __restrict__ Xs, int* __restrict__ done, int* __restrict__ todo,
                                     int* __restrict__ active, int* __restrict__ kcyc) {
    const int s = blockIdx.y;
    const int c = s % N;
    if (c >= ncols) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { done[s] = 1; todo[s] = 0; active[s] = 0; kcyc[s] = 0; }
        return;
    }
    const cplx<double>* b = G + (long)c * n;
    cplx<T>* x = Xs + (long)s * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = ccast<T>(b[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) { done[s] = 0; todo[s] = 1; active[s] = 0; kcyc[s] = 0; }
}

// Right preconditioning: r = b - W with W = (H - z) x, reference norm ||b||.
// Left preconditioning (left = 1): W already holds M^{-1}(b - (H - z) x) and the
// reference norm is its value in the first cycle.  Converged systems are
// retired; the rest start a cycle with v_0 = r / ||r||.
template <typename T>
__global__ void __launch_bounds__(kArnThreads) residual_kernel(
    const cplx<double>* __restrict__ G, const cplx<T>* __restrict__ W, int n, int N, int restart, double rtol,
    int cycle, int left, cplx<T>* __restrict__ V0, long vstride, cplx<double>* __restrict__ g,
    double* __restrict__ bnorm, int* __restrict__ done, int* __restrict__ todo, int* __restrict__ active,
    int* __restrict__ kcyc) {
    __shared__ double red[kArnThreads / 64];
    const int s = blockIdx.x;
    if (done[s]) return;
    const cplx<double>* b = G + (long)(s % N) * n;
    const cplx<T>* w = W + (long)s * n;
    // the residual stays in registers (n <= kArnThreads * kArnEPT): one read, one write
    cplx<double> r[kArnEPT];
    double rr = 0.0, bb = 0.0;
#pragma unroll
    for (int e = 0; e < kArnEPT; ++e) {
        const int i = threadIdx.x + e * kArnThreads;
        r[e] = mk<double>(0, 0);
        if (i < n) {
            if (left) {
                r[e] = ccast<double>(w[i]);
            } else {
                const cplx<double> bi = b[i];
                r[e] = bi - ccast<double>(w[i]);
                if (cycle == 0) bb += norm2(bi);
            }
            rr += norm2(r[e]);
        }
    }
    rr = block_sum(rr, red);
    if (cycle == 0 && !left) bb = block_sum(bb, red);
    const double beta = sqrt(rr);
    const double bn = cycle == 0 ? (left ? beta : sqrt(bb)) : bnorm[s];
    const bool conv = beta <= rtol * bn;
    if (conv) {
        __syncthreads();
        if (threadIdx.x == 0) {
            done[s] = 1;
            todo[s] = 0;
            active[s] = 0;
            kcyc[s] = 0;
            if (cycle == 0) bnorm[s] = bn;
        }
        return;
    }
    const double inv = 1.0 / beta;
    cplx<T>* v = V0 + (long)s * n;
#pragma unroll
    for (int e = 0; e < kArnEPT; ++e) {
        const int i = threadIdx.x + e * kArnThreads;
        if (i < n) v[i] = ccast<T>(inv * r[e]);
    }
    if (threadIdx.x == 0) {
        if (cycle == 0) bnorm[s] = bn;
        cplx<double>* gs = g + (long)s * (restart + 1);
        gs[0] = mk<double>(beta, 0.0);
        for (int i = 1; i <= restart; ++i) gs[i] = mk<double>(0, 0);
        active[s] = 1;
        kcyc[s] = 0;
    }
}

// Thread 0 of an Arnoldi step: apply the previous rotations to the new Hessenberg
// column hcol[0..j+1], compute and apply the new one, update the residual estimate and
// retire the system when it meets rtol, fills the cycle or breaks down.
__device__ __forceinline__ void arnoldi_givens(cplx<double>* hcol, int j, int restart, double rtol, double hn,
                                               const double* __restrict__ bnorm, cplx<double>* __restrict__ Hh,
                                               cplx<double>* __restrict__ cs, cplx<double>* __restrict__ sn,
                                               cplx<double>* __restrict__ g, int* __restrict__ active,
                                               int* __restrict__ kcyc, unsigned long long* __restrict__ steps, int s) {
    cplx<double>* H = Hh + (long)s * (restart + 1) * restart;   // H[i + (restart+1)*col]
    cplx<double>* c = cs + (long)s * restart;
    cplx<double>* sv = sn + (long)s * restart;
    cplx<double>* gs = g + (long)s * (restart + 1);
    hcol[j + 1] = mk<double>(hn, 0.0);
    for (int i = 0; i < j; ++i) {   // previous rotations
        const cplx<double> a = hcol[i], b = hcol[i + 1];
        hcol[i] = c[i] * a + sv[i] * b;
        hcol[i + 1] = conj(c[i]) * b - conj(sv[i]) * a;
    }
    const cplx<double> a = hcol[j], b = hcol[j + 1];
    const double den = sqrt(norm2(a) + norm2(b));
    cplx<double> cj, sj;
    if (den == 0.0) { cj = mk<double>(1, 0); sj = mk<double>(0, 0); }
    else { cj = (1.0 / den) * conj(a); sj = (1.0 / den) * conj(b); }
    c[j] = cj;
    sv[j] = sj;
    hcol[j] = mk<double>(den, 0.0);
    hcol[j + 1] = mk<double>(0, 0);
    for (int i = 0; i <= j + 1 && i <= restart; ++i) H[i + (long)(restart + 1) * j] = hcol[i];
    const cplx<double> gj = gs[j];
    gs[j + 1] = mk<double>(0, 0) - conj(sj) * gj;
    gs[j] = cj * gj;
    kcyc[s] = j + 1;
    atomicAdd(steps, 1ull);
    const double res = sqrt(norm2(gs[j + 1]));
    if (res <= rtol * bnorm[s] || j + 1 == restart || hn == 0.0) active[s] = 0;
}

// One Arnoldi step j for every active system: modified Gram-Schmidt of
// w = A v_j against v_0..v_j, h_{j+1,j} = ||w||, v_{j+1} = w/h, Givens update
// of column j and the residual estimate |g_{j+1}|.
template <typename T>
__global__ void __launch_bounds__(kArnThreads) arnoldi_kernel(
    const cplx<T>* __restrict__ Wv, cplx<T>* __restrict__ Vb, long vstride, int n, int j, int restart,
    double rtol, const double* __restrict__ bnorm, cplx<double>* __restrict__ Hh, cplx<double>* __restrict__ cs,
    cplx<double>* __restrict__ sn, cplx<double>* __restrict__ g, int* __restrict__ active, int* __restrict__ kcyc,
    unsigned long long* __restrict__ steps) {
    __shared__ double red[kArnThreads / 64];
    __shared__ double red2[2][kArnThreads / 64];
    __shared__ cplx<double> hcol[34];
    const int s = blockIdx.x;
    if (!active[s]) return;
    cplx<T> w[kArnEPT];
    const cplx<T>* wsrc = Wv + (long)s * n;
#pragma unroll
    for (int e = 0; e < kArnEPT; ++e) {
        const int i = threadIdx.x + e * kArnThreads;
        w[e] = i < n ? wsrc[i] : mk<T>(0, 0);
    }
    // modified Gram-Schmidt (real and imaginary parts of each dot reduced together)
    for (int i = 0; i <= j; ++i) {
        const cplx<T>* v = Vb + (long)i * vstride + (long)s * n;
        cplx<T> vl[kArnEPT];
        double hr = 0, hi = 0;
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) {
            const int idx = threadIdx.x + e * kArnThreads;
            vl[e] = idx < n ? v[idx] : mk<T>(0, 0);
            const cplx<T> p = cmulc(vl[e], w[e]);
            hr += (double)p.re;
            hi += (double)p.im;
        }
        block_sum2(hr, hi, red2);
        const cplx<double> h = mk<double>(hr, hi);
        const cplx<T> ht = ccast<T>(h);
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) w[e] = w[e] - ht * vl[e];
        if (threadIdx.x == 0) hcol[i] = h;
    }
    double nn = 0;
#pragma unroll
    for (int e = 0; e < kArnEPT; ++e) nn += (double)norm2(w[e]);
    nn = block_sum(nn, red);
    const double hn = sqrt(nn);
    if (hn > 0.0) {
        const T inv = (T)(1.0 / hn);
        cplx<T>* vn = Vb + (long)(j + 1) * vstride + (long)s * n;
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) {
            const int idx = threadIdx.x + e * kArnThreads;
            if (idx < n) vn[idx] = inv * w[e];
        }
    }
    if (threadIdx.x == 0) arnoldi_givens(hcol, j, restart, rtol, hn, bnorm, Hh, cs, sn, g, active, kcyc, steps, s);
}

// The same step for complex64 with the working vector in LDS (n <= 16384: 128 KiB):
// each thread owns elements threadIdx.x + e * kArnThreads of w, so the updates need no
// synchronization, and the registers hold only the basis vector being projected out
// and the next one, which is requested before the reduction of the current dot.
__global__ void __launch_bounds__(kArnThreads) arnoldi_lds_kernel(
    const cplx<float>* __restrict__ Wv, cplx<float>* __restrict__ Vb, long vstride, int n, int j, int restart,
    double rtol, const double* __restrict__ bnorm, cplx<double>* __restrict__ Hh, cplx<double>* __restrict__ cs,
    cplx<double>* __restrict__ sn, cplx<double>* __restrict__ g, int* __restrict__ active, int* __restrict__ kcyc,
    unsigned long long* __restrict__ steps) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<float>* wl = reinterpret_cast<cplx<float>*>(smem_raw);   // n entries
    __shared__ double red[kArnThreads / 64];
    __shared__ double red2[2][kArnThreads / 64];
    __shared__ cplx<double> hcol[34];
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int t = threadIdx.x;
    const cplx<float>* wsrc = Wv + (long)s * n;
    for (int i = t; i < n; i += kArnThreads) wl[i] = wsrc[i];
    auto load_v = [&](int i, cplx<float>(&dst)[kArnEPT]) {
        const cplx<float>* v = Vb + (long)i * vstride + (long)s * n;
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) {
            const int idx = t + e * kArnThreads;
            dst[e] = v[idx < n ? idx : n - 1];
        }
    };
    cplx<float> vl[kArnEPT];
    load_v(0, vl);
    for (int i = 0; i <= j; ++i) {
        double hr = 0, hi = 0;
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) {
            const int idx = t + e * kArnThreads;
            if (idx < n) {
                const cplx<float> p = cmulc(vl[e], wl[idx]);
                hr += (double)p.re;
                hi += (double)p.im;
            }
        }
        cplx<float> vn[kArnEPT];
        load_v(i < j ? i + 1 : i, vn);   // requested before the reduction
        block_sum2(hr, hi, red2);
        const cplx<double> h = mk<double>(hr, hi);
        const cplx<float> ht = ccast<float>(h);
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) {
            const int idx = t + e * kArnThreads;
            if (idx < n) wl[idx] = wl[idx] - ht * vl[e];
        }
        if (t == 0) hcol[i] = h;
#pragma unroll
        for (int e = 0; e < kArnEPT; ++e) vl[e] = vn[e];
    }
    double nn = 0;
#pragma unroll
    for (int e = 0; e < kArnEPT; ++e) {
        const int idx = t + e * kArnThreads;
        if (idx < n) nn += (double)norm2(wl[idx]);
    }
    nn = block_sum(nn, red);
    const double hn = sqrt(nn);
    if (hn > 0.0) {
        const float inv = (float)(1.0 / hn);
        cplx<float>* vn = Vb + (long)(j + 1) * vstride + (long)s * n;
        for (int i = t; i < n; i += kArnThreads) vn[i] = inv * wl[i];
    }
    if (t == 0) arnoldi_givens(hcol, j, restart, rtol, hn, bnorm, Hh, cs, sn, g, active, kcyc, steps, s);
}

// flag[p] = any(mask[p*N + c] != 0); counts[p] = number of nonzero masks (if counts).
__global__ void pole_flags_kernel(const int* __restrict__ mask, int N, int* __restrict__ flag, int* __restrict__ counts) {
    const int p = blockIdx.x;
    int cnt = 0;
    for (int c = threadIdx.x; c < N; c += blockDim.x) cnt += mask[p * N + c] != 0;
    cnt = wave_sum(cnt);
    if (threadIdx.x == 0) {
        flag[p] = cnt > 0;
        if (counts) counts[p] = cnt;
    }
}

// u = sum_i y_i v_i with R y = g (k x k upper triangular from the Givens QR).
// U = sum_i y_i v_i (ACC = 0) or U += sum_i y_i v_i (ACC = 1) for the systems that stepped,
// y from the cycle's triangular least-squares system.
template <typename T, bool ACC>
__global__ void __launch_bounds__(kArnThreads) cycle_update_kernel(const cplx<T>* __restrict__ Vb, long vstride, int n,
                                                           int restart, const cplx<double>* __restrict__ Hh,
                                                           const cplx<double>* __restrict__ g,
                                                           const int* __restrict__ kcyc, cplx<T>* __restrict__ U) {
    __shared__ cplx<double> y[33];
    __shared__ cplx<double> Hs[33 * 32];   // the k stepped columns of the Hessenberg matrix, then g
    const int s = blockIdx.x;   // one workgroup per system: y is solved once
    const int k = kcyc[s];
    if (k == 0) return;
    {   // staged by all threads: the back substitution then reads LDS, not a chain of loads
        const cplx<double>* H = Hh + (long)s * (restart + 1) * restart;
        const int hk = (restart + 1) * k;
        for (int e = threadIdx.x; e < hk; e += blockDim.x) Hs[e] = H[e];
        if (threadIdx.x < k) y[threadIdx.x] = g[(long)s * (restart + 1) + threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            cplx<double> acc = y[i];
            for (int c = i + 1; c < k; ++c) acc = acc - Hs[i + (restart + 1) * c] * y[c];
            y[i] = cdiv(acc, Hs[i + (restart + 1) * i]);
        }
    }
    __syncthreads();
    cplx<T>* u = U + (long)s * n;
    for (long r = threadIdx.x; r < n; r += blockDim.x) {
        cplx<double> acc = ACC ? ccast<double>(u[r]) : cplx<double>{0, 0};
        for (int i = 0; i < k; ++i) acc = acc + y[i] * ccast<double>(Vb[(long)i * vstride + (long)s * n + r]);
        u[r] = ccast<T>(acc);
    }
}

// y of every system that stepped this cycle, into ys (S x restart): the back substitution of
// cycle_update_kernel, in the same order
__global__ void cycle_solve_kernel(const cplx<double>* __restrict__ Hh, const cplx<double>* __restrict__ g,
                                   const int* __restrict__ kcyc, int restart, int S, cplx<double>* __restrict__ ys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int k = kcyc[s];
    const cplx<double>* H = Hh + (long)s * (restart + 1) * restart;
    cplx<double>* y = ys + (long)s * restart;
    for (int i = k - 1; i >= 0; --i) {
        cplx<double> acc = g[(long)s * (restart + 1) + i];
        for (int c = i + 1; c < k; ++c) acc = acc - H[i + (restart + 1) * c] * y[c];
        y[i] = cdiv(acc, H[i + (restart + 1) * i]);
    }
}

// PG = sum_j w_j x_j per column with the final cycle's left update x_j + sum_{i<k} y_i v_i
// folded in (x is not written back).  Each x is rounded to the working precision as the
// update would store it, so PG is bitwise the unfused update followed by pole_sum_kernel.
template <typename T>
__global__ void cycle_pole_sum_kernel(const cplx<T>* __restrict__ Xs, const cplx<T>* __restrict__ Vb, long vstride,
                                      const cplx<double>* __restrict__ ys, const int* __restrict__ kcyc, int restart,
                                      const cplx<double>* __restrict__ wts, int n, int N, int p, int ncols,
                                      cplx<double>* __restrict__ PG) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int c = (int)(idx / n);
    const long r = idx - (long)c * n;
    cplx<double> acc = {0, 0};
    for (int j = 0; j < p; ++j) {
        const long sn = (long)j * N + c;
        const int k = kcyc[sn];
        cplx<double> u = ccast<double>(Xs[sn * n + r]);
        for (int i = 0; i < k; ++i) u = u + ys[sn * restart + i] * ccast<double>(Vb[(long)i * vstride + sn * n + r]);
        acc = acc + wts[j] * ccast<double>(ccast<T>(u));
    }
    PG[idx] = acc;
}

template <typename T>
__global__ void axpy_masked_kernel(cplx<T>* __restrict__ Xs, const cplx<T>* __restrict__ Z, int n,
                                   const int* __restrict__ kcyc) {
    const int s = blockIdx.y;
    if (kcyc[s] == 0) return;
    for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (long)gridDim.x * blockDim.x)
        Xs[(long)s * n + r] = Xs[(long)s * n + r] + Z[(long)s * n + r];
}

// PG[:, c] = sum_j w_j Xs[j*N + c]   (fixed pole order, FP64 accumulation)
template <typename T>
__global__ void pole_sum_kernel(const cplx<T>* __restrict__ Xs, const cplx<double>* __restrict__ wts, int n, int N,
                                int p, int ncols, cplx<double>* __restrict__ PG) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int c = (int)(idx / n);
    const long r = idx - (long)c * n;
    cplx<double> acc = {0, 0};
    for (int j = 0; j < p; ++j) acc = acc + wts[j] * ccast<double>(Xs[((long)j * N + c) * n + r]);
    PG[idx] = acc;
}

// out[i] = in[i] converted (columns are contiguous: count = n * ncols)
template <typename Tin, typename Tout>
__global__ void copy_cast_kernel(const cplx<Tin>* __restrict__ in, cplx<Tout>* __restrict__ out, long count) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        out[i] = ccast<Tout>(in[i]);
}

__global__ void one_pole_flags_kernel(int* __restrict__ col_mask, int* __restrict__ pole_active, int S, int N, int p,
                                      int pole, int ncols) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        col_mask[s] = (s / N == pole && s % N < ncols) ? 1 : 0;
        if (s < p) pole_active[s] = s == pole ? 1 : 0;
    }
}

}  // namespace

void gmres_alloc(GmresWork& w, int n, int N, int p, int restart, bool multipass, bool fp32) {
    POMM_CHECK(restart >= 1 && restart <= 32, 1, "gmres_restart must be in 1..32");
    POMM_CHECK(n <= kArnThreads * kArnEPT, 8, "GMRES kernels support n <= 16384 (2D grids up to 128^2)");
    w.S = p * N;
    w.n = n;
    w.N = N;
    w.p = p;
    w.restart = restart;
    w.fp32 = fp32;
    const size_t vec = (size_t)w.S * n;
    const size_t esz = fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    POMM_HIP(dev_alloc(&w.Vb, esz * vec * (restart + 1)));
    POMM_HIP(dev_alloc(&w.Xs, esz * vec));
    POMM_HIP(dev_alloc(&w.W, esz * vec));
    POMM_HIP(dev_alloc(&w.U, esz * vec));
    POMM_HIP(dev_alloc(&w.Z, esz * vec));
    if (multipass) POMM_HIP(dev_alloc(&w.work, sizeof(cplx<double>) * vec));
    POMM_HIP(dev_alloc(&w.Hh, sizeof(cplx<double>) * w.S * (restart + 1) * restart));
    POMM_HIP(dev_alloc(&w.cs, sizeof(cplx<double>) * w.S * restart));
    POMM_HIP(dev_alloc(&w.sn, sizeof(cplx<double>) * w.S * restart));
    POMM_HIP(dev_alloc(&w.g, sizeof(cplx<double>) * w.S * (restart + 1)));
    POMM_HIP(dev_alloc(&w.ys, sizeof(cplx<double>) * w.S * restart));
    POMM_HIP(dev_alloc(&w.bnorm, sizeof(double) * w.S));
    POMM_HIP(dev_alloc(&w.active, sizeof(int) * w.S));
    POMM_HIP(dev_alloc(&w.done, sizeof(int) * w.S * 2));   // done, then todo
    POMM_HIP(dev_alloc(&w.kcyc, sizeof(int) * w.S));
    POMM_HIP(dev_alloc(&w.pole_active, sizeof(int) * p));
    POMM_HIP(dev_alloc(&w.counter, sizeof(int) * p));
    POMM_HIP(dev_alloc(&w.steps, sizeof(unsigned long long)));
    POMM_HIP(hipMemsetAsync(w.steps, 0, sizeof(unsigned long long), alloc_stream()));
    POMM_HIP(hipHostMalloc(&w.counter_host, sizeof(int) * p));
    POMM_HIP(dev_alloc(&w.pole_z, sizeof(cplx<double>) * p * 2));   // z, then (l - z) for PP
    POMM_HIP(dev_alloc(&w.pole_w, sizeof(cplx<double>) * p));
}

void gmres_free(GmresWork& w) {
    for (void* ptr : {w.Vb, w.Xs, w.W, w.U, w.Z, (void*)w.work, (void*)w.Hh,
                      (void*)w.cs, (void*)w.sn, (void*)w.g, (void*)w.ys, (void*)w.bnorm, (void*)w.active, (void*)w.done,
                      (void*)w.kcyc, (void*)w.pole_active, (void*)w.counter, (void*)w.steps, (void*)w.pole_z,
                      (void*)w.pole_w})
        if (ptr) (void)dev_free(ptr);
    if (w.counter_host) (void)hipHostFree(w.counter_host);
    w = GmresWork{};
}

namespace {

template <typename T>
void precondition_t(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg,
                    const T* V_dev, const cplx<double>* G, cplx<double>* PG, int ncols, hipStream_t s) {
    const int n = w.n, N = w.N, S = w.S, p = w.p, restart = w.restart;
    cplx<T>* const Vb = static_cast<cplx<T>*>(w.Vb);
    cplx<T>* const Xs = static_cast<cplx<T>*>(w.Xs);
    cplx<T>* const W = static_cast<cplx<T>*>(w.W);
    cplx<T>* const U = static_cast<cplx<T>*>(w.U);
    cplx<T>* const Z = static_cast<cplx<T>*>(w.Z);
    cplx<T>* const work = reinterpret_cast<cplx<T>*>(w.work);
    POMM_CHECK(ncols >= 1 && ncols <= N, 1, "ncols must be in 1..N");
    POMM_CHECK(cfg.restart == restart, 1, "restart differs from the allocated workspace");
    const bool use_spp = cfg.inner == 0;
    POMM_CHECK(!use_spp || spp != nullptr, 1, "sparsifying preconditioner not set up");
    int* todo = w.done + S;
    const long vstride = (long)S * n;
    const unsigned gx = cdiv_u(n, 256) > 64 ? 64 : cdiv_u(n, 256);
    const double vec_bytes = (double)sizeof(cplx<T>) * n;
    int act_sys = ncols * p, act_poles = p;   // host view of the active sets (profiling and skip)

    {
        ProfScope prof(PK_GMRES_AUX, 2.0 * vec_bytes * act_sys, 0.0, s);
        hipLaunchKernelGGL(init_solution_kernel<T>, dim3(gx, S), dim3(256), 0, s, G, n, N, ncols, Xs, w.done, todo,
                           w.active, w.kcyc);
        check_launch("init_solution");
    }

    // (H - z_j) applied to a batch of S vectors, or with rhs the residual G - (H - z_j) in
    auto apply_shifted_h = [&](const cplx<T>* in, cplx<T>* out, const int* mask, int active,
                               const cplx<double>* rhs = nullptr) {
        SpecArgs<T> a;
        a.in = in;
        a.ld_in = n;
        a.out = out;
        a.ld_out = n;
        a.ncols = S;
        a.cols_per_group = N;
        a.mult_mode = MULT_KINETIC;
        a.post_mode = rhs ? POST_RESIDUAL : POST_SHIFTED_H;
        a.rhs = rhs;
        a.ld_rhs = n;
        a.V = V_dev;
        a.post_shift = w.pole_z;
        a.col_mask = mask;
        a.active_hint = active;
        spectral_apply<T>(plan, a, work, s);
    };
    // Z = M_j^{-1} in (in must not be U when SPP is used)
    auto apply_minv = [&](const cplx<T>* in, const int* mask, const int* pflags, int active, int apoles) {
        SpecArgs<T> a;
        a.in = in;
        a.ld_in = n;
        a.ld_out = n;
        a.ncols = S;
        a.cols_per_group = N;
        a.col_mask = mask;
        a.active_hint = active;
        if (use_spp) {
            a.out = U;   // Q G_j in = right-hand side of P_j
            a.mult_mode = MULT_TABLE;
            if constexpr (sizeof(T) == 8) a.mult_tab = spp->mult;
            else a.mult_tab = spp->mult32;
            spectral_apply<T>(plan, a, work, s);
            spp_solve<T>(*spp, pflags, apoles, s);   // U -> Z
        } else {
            a.out = Z;
            a.mult_mode = MULT_INV_SHIFTED;
            a.group_c = w.pole_z + p;   // l - z_j
            spectral_apply<T>(plan, a, work, s);
        }
    };
    // Z = M_j^{-1} (H - z_j) in, or with rhs Z = M_j^{-1} (rhs - (H - z_j) in) (left side).
    // With the sparsifying preconditioner both Fourier-diagonal steps run as one chained
    // spectral pass over the data (H - z_j, then Q G_j), followed by the sparse solve.
    const bool chain = use_spp && spectral_chain_available<T>(plan);
    auto apply_minv_a = [&](const cplx<T>* in, const int* mask, const int* pflags, int active, int apoles,
                            const cplx<double>* rhs) {
        if (!chain) {
            apply_shifted_h(in, W, mask, active, rhs);
            apply_minv(W, mask, pflags, active, apoles);
            return;
        }
        SpecArgs<T> a;
        a.in = in;
        a.ld_in = n;
        a.ld_out = n;
        a.ncols = S;
        a.cols_per_group = N;
        a.mult_mode = MULT_KINETIC;
        a.post_mode = rhs ? POST_RESIDUAL : POST_SHIFTED_H;
        a.rhs = rhs;
        a.ld_rhs = n;
        a.V = V_dev;
        a.post_shift = w.pole_z;
        a.col_mask = mask;
        a.active_hint = active;
        if constexpr (sizeof(T) == 8) a.chain_tab = spp->mult;
        else a.chain_tab = spp->mult32;
        a.chain_out = U;   // Q G_j (b - (H - z_j) x) = right-hand side of P_j
        spectral_apply<T>(plan, a, work, s);
        spp_solve<T>(*spp, pflags, apoles, s);   // U -> Z
    };
    auto read_counters = [&]() {   // per-pole active counts of the last counted flags()
        POMM_HIP(hipMemcpyAsync(w.counter_host, w.counter, sizeof(int) * p, hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        act_sys = act_poles = 0;
        for (int j = 0; j < p; ++j) {
            act_sys += w.counter_host[j];
            act_poles += w.counter_host[j] > 0;
        }
    };
    auto flags = [&](const int* mask, bool count) {
        ProfScope prof(PK_GMRES_AUX, 4.0 * S, 0.0, s);
        hipLaunchKernelGGL(pole_flags_kernel, dim3(p), dim3(64), 0, s, mask, N, w.pole_active,
                           count ? w.counter : nullptr);
        check_launch("pole_flags");
    };

    const bool left = cfg.left;
    bool fold_update = false;   // the final left update is left to the pole sum
    for (int cyc = 0; cyc < cfg.cycles; ++cyc) {
        if (left) {   // Z = M^{-1} (b - (H - z) x)
            if (cyc == 0) flags(todo, false);
            apply_minv_a(Xs, todo, w.pole_active, act_sys, act_poles, G);
        } else {
            apply_shifted_h(Xs, W, todo, act_sys);
        }
        {
            ProfScope prof(PK_GMRES_AUX, 3.0 * vec_bytes * act_sys, 8.0 * n * act_sys, s);
            hipLaunchKernelGGL(residual_kernel<T>, dim3(S), dim3(kArnThreads), 0, s, G, left ? Z : W, n, N, restart, cfg.rtol,
                               cyc, left ? 1 : 0, Vb, vstride, w.g, w.bnorm, w.done, todo, w.active, w.kcyc);
            check_launch("residual");
        }
        flags(w.active, true);
        read_counters();
        if (act_sys == 0) break;   // every system converged
        // every system active now takes at least one step this cycle: these are the
        // counts of the kcyc > 0 systems of the update below
        const int cyc_sys = act_sys, cyc_poles = act_poles;
        bool all_converged = false;   // every system's Arnoldi residual estimate met rtol
        for (int j = 0; j < restart; ++j) {
            // next Krylov vector: A M^{-1} v_j (right) or M^{-1} A v_j (left)
            const cplx<T>* kv;
            if (left) {
                apply_minv_a(Vb + (long)j * vstride, w.active, w.pole_active, act_sys, act_poles, nullptr);
                kv = Z;
            } else {
                apply_minv(Vb + (long)j * vstride, w.active, w.pole_active, act_sys, act_poles);
                apply_shifted_h(Z, W, w.active, act_sys);
                kv = W;
            }
            {
                ProfScope prof(PK_ARNOLDI, vec_bytes * act_sys * (j + 3), 16.0 * n * act_sys * (j + 2), s);
                if constexpr (sizeof(T) == 4) {   // complex64: the working vector in LDS
                    static const bool attr_set = [] {   // once per process, thread-safe
                        (void)hipFuncSetAttribute((const void*)arnoldi_lds_kernel,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)(sizeof(cplx<float>) * kArnThreads * kArnEPT));
                        return true;
                    }();
                    (void)attr_set;
                    hipLaunchKernelGGL(arnoldi_lds_kernel, dim3(S), dim3(kArnThreads), sizeof(cplx<float>) * n, s, kv,
                                       Vb, vstride, n, j, restart, cfg.rtol, w.bnorm, w.Hh, w.cs, w.sn, w.g, w.active,
                                       w.kcyc, w.steps);
                } else {
                    hipLaunchKernelGGL(arnoldi_kernel<T>, dim3(S), dim3(kArnThreads), 0, s, kv, Vb, vstride, n, j,
                                       restart, cfg.rtol, w.bnorm, w.Hh, w.cs, w.sn, w.g, w.active, w.kcyc, w.steps);
                }
                check_launch("arnoldi");
            }
            flags(w.active, true);
            read_counters();
            if (act_sys == 0) {
                all_converged = true;
                break;
            }
        }
        // x += M^{-1} (sum_i y_i v_i) (right) or x += sum_i y_i v_i (left), for the systems
        // that stepped this cycle
        act_sys = cyc_sys;
        act_poles = cyc_poles;
        // no cycle follows: accepted estimates, or the last cycle allowed
        const bool final_cycle = (all_converged && !cfg.verify) || cyc == cfg.cycles - 1;
        if (left && final_cycle) {   // the update is folded into the pole sum below
            fold_update = true;
            break;
        }
        if (left) {   // x += sum_i y_i v_i in one pass
            ProfScope prof(PK_GMRES_AUX, vec_bytes * act_sys * (restart / 2 + 2), 8.0 * n * act_sys * restart / 2, s);
            hipLaunchKernelGGL((cycle_update_kernel<T, true>), dim3(S), dim3(kArnThreads), 0, s, Vb, vstride, n,
                               restart, w.Hh, w.g, w.kcyc, Xs);
            check_launch("cycle_update");
        } else {      // x += M^{-1} (sum_i y_i v_i)
            flags(w.kcyc, false);   // pole gates of the update's M^{-1}
            {
                ProfScope prof(PK_GMRES_AUX, vec_bytes * act_sys * (restart / 2 + 1), 8.0 * n * act_sys * restart / 2,
                               s);
                hipLaunchKernelGGL((cycle_update_kernel<T, false>), dim3(S), dim3(kArnThreads), 0, s, Vb, vstride,
                                   n, restart, w.Hh, w.g, w.kcyc, W);
                check_launch("cycle_update");
            }
            apply_minv(W, w.kcyc, w.pole_active, act_sys, act_poles);
            ProfScope prof(PK_GMRES_AUX, 3.0 * vec_bytes * act_sys, 2.0 * n * act_sys, s);
            hipLaunchKernelGGL(axpy_masked_kernel<T>, dim3(gx, S), dim3(256), 0, s, Xs, Z, n, w.kcyc);
            check_launch("axpy_masked");
        }
        // without verification the Arnoldi estimates are accepted: no residual check follows
        if (all_converged && !cfg.verify) break;
        // the systems that did not converge stay in todo for the next residual check:
        // exactly the set that entered this cycle (act_sys, act_poles)
        if (left) flags(todo, false);   // pole gates of the next residual's M^{-1}
    }
    if (fold_update) {   // read x and the cycle's basis once, write only PG
        ProfScope prof(PK_GMRES_AUX, vec_bytes * (ncols * p + (double)act_sys * (restart / 2)) + 16.0 * n * ncols,
                       8.0 * n * ncols * p + 8.0 * n * act_sys * restart / 2, s, 2);
        hipLaunchKernelGGL(cycle_solve_kernel, dim3(cdiv_u(S, 256)), dim3(256), 0, s, w.Hh, w.g, w.kcyc, restart, S,
                           w.ys);
        check_launch("cycle_solve");
        hipLaunchKernelGGL(cycle_pole_sum_kernel<T>, dim3(cdiv_u((size_t)n * ncols, 256)), dim3(256), 0, s, Xs, Vb,
                           vstride, w.ys, w.kcyc, restart, w.pole_w, n, N, p, ncols, PG);
        check_launch("cycle_pole_sum");
        return;
    }
    {
        ProfScope prof(PK_GMRES_AUX, vec_bytes * ncols * (p + 1), 8.0 * n * ncols * p, s);
        hipLaunchKernelGGL(pole_sum_kernel<T>, dim3(cdiv_u((size_t)n * ncols, 256)), dim3(256), 0, s, Xs, w.pole_w, n,
                           N, p, ncols, PG);
        check_launch("pole_sum");
    }
}

}  // namespace

void fermi_precondition(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg,
                        const double* V_dev, const float* V32_dev, const cplx<double>* G, cplx<double>* PG,
                        int ncols, hipStream_t s) {
    if (w.fp32) precondition_t<float>(plan, spp, w, cfg, V32_dev, G, PG, ncols, s);
    else precondition_t<double>(plan, spp, w, cfg, V_dev, G, PG, ncols, s);
}

namespace {

template <typename T>
void inner_apply_t(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg, int pole,
                   const cplx<double>* B, cplx<double>* Y, int ncols, hipStream_t s) {
    const int n = w.n, N = w.N, S = w.S, p = w.p;
    cplx<T>* const W = static_cast<cplx<T>*>(w.W);
    cplx<T>* const U = static_cast<cplx<T>*>(w.U);
    cplx<T>* const Z = static_cast<cplx<T>*>(w.Z);
    const long off = (long)pole * N * n, cnt = (long)n * ncols;
    hipLaunchKernelGGL(one_pole_flags_kernel, dim3(cdiv_u(S, 256)), dim3(256), 0, s, w.active, w.pole_active, S, N, p,
                       pole, ncols);
    check_launch("one_pole_flags");
    hipLaunchKernelGGL((copy_cast_kernel<double, T>), dim3(1024), dim3(256), 0, s, B, W + off, cnt);
    check_launch("copy_cast");
    SpecArgs<T> a;
    a.in = W;
    a.ld_in = n;
    a.ld_out = n;
    a.ncols = S;
    a.cols_per_group = N;
    a.col_mask = w.active;
    a.active_hint = ncols;
    const cplx<T>* result;
    if (cfg.inner == 0) {
        a.out = U;
        a.mult_mode = MULT_TABLE;
        if constexpr (sizeof(T) == 8) a.mult_tab = spp->mult;
        else a.mult_tab = spp->mult32;
        spectral_apply<T>(plan, a, reinterpret_cast<cplx<T>*>(w.work), s);
        spp_solve<T>(*spp, w.pole_active, 1, s);
        result = Z;
    } else {
        a.out = U;
        a.mult_mode = MULT_INV_SHIFTED;
        a.group_c = w.pole_z + p;
        spectral_apply<T>(plan, a, reinterpret_cast<cplx<T>*>(w.work), s);
        result = U;
    }
    hipLaunchKernelGGL((copy_cast_kernel<T, double>), dim3(1024), dim3(256), 0, s, result + off, Y, cnt);
    check_launch("copy_cast");
}

}  // namespace

void inner_apply(const SpectralPlan& plan, const Spp* spp, GmresWork& w, const PrecondConfig& cfg, int pole,
                 const cplx<double>* B, cplx<double>* Y, int ncols, hipStream_t s) {
    POMM_CHECK(pole >= 0 && pole < w.p, 1, "pole index out of range");
    POMM_CHECK(ncols >= 1 && ncols <= w.N, 1, "ncols must be in 1..N");
    POMM_CHECK(cfg.inner != 0 || spp != nullptr, 1, "sparsifying preconditioner not set up");
    if (w.fp32) inner_apply_t<float>(plan, spp, w, cfg, pole, B, Y, ncols, s);
    else inner_apply_t<double>(plan, spp, w, cfg, pole, B, Y, ncols, s);
}

}  // namespace pomm
