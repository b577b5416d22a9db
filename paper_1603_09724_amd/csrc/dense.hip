// Dense complex kernels (see dense.h).
#include "dense.h"

namespace pomm {

namespace {

// ------------------------------------------------------------------ Gram
// parts[(p*chunks + c)*N*N + a + b*N] = sum_{r in chunk c} conj(P[r,a]) Q[r,b]
// One workgroup of 256 threads per (64 x 64 output tile, row chunk, product): the chunk's
// rows pass through LDS 16 at a time, and thread (tx, ty) accumulates the 4 x 4 outputs
// (ty + 16 i, tx + 16 j), so that each pair of LDS reads feeds two complex multiply-adds.
constexpr int kGT = 64, kGK = 16;

__global__ void __launch_bounds__(256) gram_partial_kernel(const cplx<double>* const* __restrict__ Ps,
                                                           const cplx<double>* const* __restrict__ Qs, int n, int N,
                                                           int rows_per_chunk, int chunks,
                                                           cplx<double>* __restrict__ parts) {
    const int tiles = (N + kGT - 1) / kGT;
    const int ta = blockIdx.x % tiles, tb = blockIdx.x / tiles;
    const int c = blockIdx.y, p = blockIdx.z;
    const cplx<double>* P = Ps[p];
    const cplx<double>* Q = Qs[p];
    const int a0 = ta * kGT, b0 = tb * kGT;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    __shared__ cplx<double> Pl[kGK][kGT + 1];
    __shared__ cplx<double> Ql[kGK][kGT + 1];
    cplx<double> acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = {0, 0};
    const int r_begin = c * rows_per_chunk;
    const int r_end = min(n, r_begin + rows_per_chunk);
    for (int r0 = r_begin; r0 < r_end; r0 += kGK) {
        // 16 rows x 64 columns of each operand: thread e = tid + 256 q takes row e % 16 of
        // column e / 16 (a wave reads 4 runs of 16 consecutive rows)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            const int rr = e & (kGK - 1), cc = e / kGK;
            const int gr = r0 + rr;
            cplx<double> pv = {0, 0}, qv = {0, 0};
            if (gr < r_end) {
                if (a0 + cc < N) pv = P[gr + (long)(a0 + cc) * n];
                if (b0 + cc < N) qv = Q[gr + (long)(b0 + cc) * n];
            }
            Pl[rr][cc] = pv;
            Ql[rr][cc] = qv;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kGK; ++rr) {
            cplx<double> pa[4], qb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                pa[i] = Pl[rr][ty + 16 * i];
                qb[i] = Ql[rr][tx + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = acc[i][j] + cmulc(pa[i], qb[j]);
        }
        __syncthreads();
    }
    cplx<double>* out = parts + ((long)p * chunks + c) * N * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = a0 + ty + 16 * i, b = b0 + tx + 16 * j;
            if (a < N && b < N) out[a + (long)b * N] = acc[i][j];
        }
}

__global__ void gram_reduce_kernel(const cplx<double>* __restrict__ parts, int N, int chunks, int nprod,
                                   cplx<double>* __restrict__ out) {
    const long NN = (long)N * N;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NN * nprod) return;
    const long p = idx / NN, e = idx - p * NN;
    cplx<double> s = {0, 0};
    for (int c = 0; c < chunks; ++c) s = s + parts[(p * chunks + c) * NN + e];
    out[p * NN + e] = s;
}

// ------------------------------------------------------------------ inverse
// In-place Gauss-Jordan with row pivoting on one matrix per block (global memory).
template <typename T>
__global__ void __launch_bounds__(256) invert_kernel(cplx<T>* mats, long stride, int n, int* pivs) {
    cplx<T>* a = mats + (long)blockIdx.x * stride;
    int* perm = pivs + (long)blockIdx.x * n;
    __shared__ double rv[256];
    __shared__ int ri[256];
    __shared__ cplx<T> rowk[384];
    __shared__ cplx<T> colk[384];
    __shared__ int piv_s;
    const int tid = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        // pivot: argmax_{i >= k} |a[i][k]|, ties to the smaller index
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < n; i += blockDim.x) {
            const double v = (double)norm2(a[i + (long)k * n]);
            if (v > best) { best = v; bi = i; }
        }
        rv[tid] = best;
        ri[tid] = bi;
        __syncthreads();
        for (int off = blockDim.x / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double o = rv[tid + off];
                const int oi = ri[tid + off];
                if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) { rv[tid] = o; ri[tid] = oi; }
            }
            __syncthreads();
        }
        if (tid == 0) { piv_s = ri[0]; perm[k] = ri[0]; }
        __syncthreads();
        const int p = piv_s;
        if (p != k)
            for (int j = tid; j < n; j += blockDim.x) {
                cplx<T> t = a[k + (long)j * n];
                a[k + (long)j * n] = a[p + (long)j * n];
                a[p + (long)j * n] = t;
            }
        __syncthreads();
        const cplx<T> pivinv = cdiv(mk<T>(1, 0), a[k + (long)k * n]);
        // scaled pivot row (with a_kk replaced by 1 before scaling) and the multipliers
        for (int j = tid; j < n; j += blockDim.x) {
            const cplx<T> v = (j == k) ? mk<T>(1, 0) : a[k + (long)j * n];
            rowk[j] = v * pivinv;
            colk[j] = (j == k) ? mk<T>(0, 0) : a[j + (long)k * n];
        }
        __syncthreads();
        for (long e = tid; e < (long)n * n; e += blockDim.x) {
            const int i = (int)(e % n), j = (int)(e / n);
            if (i == k) {
                a[e] = rowk[j];
            } else {
                const cplx<T> base = (j == k) ? mk<T>(0, 0) : a[e];
                a[e] = base - colk[i] * rowk[j];
            }
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k)
            for (int i = tid; i < n; i += blockDim.x) {
                cplx<T> t = a[i + (long)k * n];
                a[i + (long)k * n] = a[i + (long)p * n];
                a[i + (long)p * n] = t;
            }
        __syncthreads();
    }
}

}  // namespace

template <typename T>
void gemm_batched(const GemmTask<T>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                  hipStream_t s, int active_hint) {
    if (ntasks <= 0) return;
    // every task built by this library has a real alpha
    if constexpr (sizeof(T) == 8) gemm_mfma_f64(tasks_dev, ntasks, M, Nc, K, gate_flags, s, active_hint);
    else gemm_mfma_f32(tasks_dev, ntasks, M, Nc, K, gate_flags, s, active_hint);
}

GramPlan gram_plan(int n, int N) {
    GramPlan g;
    g.n = n;
    g.N = N;
    const int tiles = ((N + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
    int chunks = 1024 / (tiles * 6) + 1;   // aim for ~1k blocks over 6 products
    const int maxc = (n + 127) / 128;      // at least 128 rows per chunk
    if (chunks > maxc) chunks = maxc;
    if (chunks < 1) chunks = 1;
    g.chunks = chunks;
    return g;
}

size_t gram_parts_elems(const GramPlan& g, int nprod) { return (size_t)nprod * g.chunks * g.N * g.N; }

void gram_products(const GramPlan& g, const cplx<double>* const* Ps, const cplx<double>* const* Qs, int nprod,
                   cplx<double>* parts, cplx<double>* out, hipStream_t s) {
    const int tiles = ((g.N + kGT - 1) / kGT) * ((g.N + kGT - 1) / kGT);
    int rpc = (g.n + g.chunks - 1) / g.chunks;
    rpc = ((rpc + kGK - 1) / kGK) * kGK;
    hipLaunchKernelGGL(gram_partial_kernel, dim3(tiles, g.chunks, nprod), dim3(256), 0, s, Ps, Qs, g.n, g.N, rpc,
                       g.chunks, parts);
    check_launch("gram_partial");
    const long tot = (long)g.N * g.N * nprod;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(cdiv_u(tot, 256)), dim3(256), 0, s, parts, g.N, g.chunks, nprod, out);
    check_launch("gram_reduce");
}

// Register-resident Gauss-Jordan for n <= 128: one workgroup of 128 G threads per
// matrix, thread t holds row r = t % 128 of columns g + G i (g = t / 128,
// i = 0..128/G - 1).  Partial pivoting without row exchanges: the pivot of step k is
// the unused row p_k with the largest |a(p_k, k)| (ties to the smaller row);
// after n steps the register image X satisfies A^{-1}(k, p_j) = X(p_k, j),
// which the final store applies.  G = 8 spreads a matrix over a whole CU (for
// batches that fill the chip); smaller G puts several matrices on a CU and takes
// fewer waves into each step's barriers (for small batches, where the chain of 128
// dependent steps is the cost).
template <typename T, int G = 8>
__global__ void __launch_bounds__(128 * G) invert_reg_kernel(cplx<T>* mats, long stride, int n) {
    constexpr int RI = 128 / G;
    cplx<T>* a = mats + (long)blockIdx.x * stride;
    const int tid = threadIdx.x, r = tid & 127, g = tid >> 7, lane = tid & 63, wave = tid >> 6;
    __shared__ cplx<T> rowp[2][128], colk[2][128];
    __shared__ int perm[128], invp[128];
    __shared__ int used[128];
    __shared__ double bv[2];
    __shared__ int bi[2];
    cplx<T> x[RI];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int c = g + G * i;
        x[i] = (r < n && c < n) ? a[r + (long)c * n] : mk<T>(0, 0);
    }
    if (tid < 128) used[tid] = tid < n ? 0 : 1;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int buf = k & 1, kg = k % G, ki = k / G;
        cplx<T> xk = x[0];
#pragma unroll
        for (int i = 1; i < RI; ++i)
            if (i == ki) xk = x[i];
        if (g == kg) {   // the two waves holding column k: argmax over the unused rows
            double v = used[r] ? -1.0 : (double)norm2(xk);
            int idx = r;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(v, off);
                const int oi = __shfl_xor(idx, off);
                if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
            }
            if (lane == 0) { bv[wave & 1] = v; bi[wave & 1] = idx; }
            colk[buf][r] = xk;
        }
        __syncthreads();
        const int p = (bv[0] > bv[1] || (bv[0] == bv[1] && bi[0] < bi[1])) ? bi[0] : bi[1];
        if (r == p) {
#pragma unroll
            for (int i = 0; i < RI; ++i) rowp[buf][g + G * i] = x[i];
            if (g == 0) { perm[k] = p; used[p] = 1; }
        }
        __syncthreads();
        const cplx<T> pinv = cdiv(mk<T>(1, 0), rowp[buf][k]);
        // one branch-free update for every element: x - sc rp, times pinv on the pivot row
        // (whose x is rp: sc = 0 there); column k is set afterwards (-sc, pinv on the pivot row)
        const bool isp = r == p;
        const cplx<T> sc = isp ? mk<T>(0, 0) : colk[buf][r] * pinv;
        const cplx<T> f = isp ? pinv : mk<T>(1, 0);
#pragma unroll
        for (int i = 0; i < RI; ++i) x[i] = f * (x[i] - sc * rowp[buf][g + G * i]);
        if (g == kg) {
            const cplx<T> xkn = isp ? pinv : mk<T>(0, 0) - sc;
#pragma unroll
            for (int i = 0; i < RI; ++i)
                if (i == ki) x[i] = xkn;
        }
    }
    __syncthreads();
    if (tid < 128) invp[tid] = 0;
    __syncthreads();
    if (tid < n && perm[tid] < n) invp[perm[tid]] = tid;
    __syncthreads();
    if (r < n) {   // (a NaN input can leave the permutation incomplete: never store outside the matrix)
        const int ro = invp[r];
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int c = g + G * i;
            if (c < n && perm[c] < n) a[ro + (long)perm[c] * n] = x[i];
        }
    }
}

template <typename T>
void invert_batched(cplx<T>* mats, long stride, int n, int count, int* piv, hipStream_t s) {
    if (count <= 0) return;
    POMM_CHECK(n <= 384, 1, "invert_batched: order above 384");
    if (n <= 128) {
        // complex64 batches above one matrix per CU: two half-CU workgroups per CU (measured
        // at order 128: 1.03 against 1.34 ms for 960 matrices, 0.54 against 0.69 for 480;
        // a whole CU per matrix stays faster up to 256 matrices)
        if (sizeof(T) == 4 && count > 256)
            hipLaunchKernelGGL((invert_reg_kernel<T, 4>), dim3(count), dim3(512), 0, s, mats, stride, n);
        else
            hipLaunchKernelGGL((invert_reg_kernel<T, 8>), dim3(count), dim3(1024), 0, s, mats, stride, n);
    } else {
        hipLaunchKernelGGL(invert_kernel<T>, dim3(count), dim3(256), 0, s, mats, stride, n, piv);
    }
    check_launch("invert_batched");
}

template void gemm_batched<double>(const GemmTask<double>*, int, int, int, int, const int*, hipStream_t, int);
template void gemm_batched<float>(const GemmTask<float>*, int, int, int, int, const int*, hipStream_t, int);
template void invert_batched<double>(cplx<double>*, long, int, int, int*, hipStream_t);
template void invert_batched<float>(cplx<float>*, long, int, int, int*, hipStream_t);

}  // namespace pomm
