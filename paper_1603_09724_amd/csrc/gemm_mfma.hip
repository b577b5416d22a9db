// Batched multi-term complex GEMM on the matrix cores (v_mfma_f64_16x16x4f64 for
// complex128, v_mfma_f32_16x16x4f32 for complex64).
//
// Same task semantics as gemm_batched (dense.h): C = beta C + sum_t alpha_t A_t B_t
// with real alpha_t.  A complex product is four real MFMA products:
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
//
// A workgroup of W waves computes a (16 W) x 64 tile of one task; wave w owns
// 16 rows and all 64 columns (four 16 x 16 MFMA blocks for the real and four
// for the imaginary part).  The factor operand A is never shared between
// waves, so each lane loads its MFMA fragments straight from global memory
// into registers, one K chunk ahead of the chunk being multiplied (unconditional
// loads from clamped addresses, masked where they are used).  The
// right-hand-side chunk (KC x 64) is shared by all waves and staged through a
// double-buffered LDS tile, one barrier per chunk.
// MFMA operand layout (16x16x4, one block): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element v holds D[l/16 + 4 v][l%16] for the f64
// instruction and D[4 (l/16) + v][l%16] for the f32 one (both checked on gfx950).
#include "dense.h"

namespace pomm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef f64x4 acc;
    static constexpr int KC = 16;   // K chunk per pipeline stage
    __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
    typedef f32x4 acc;
    static constexpr int KC = 32;
    __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

// Loads and stores through the global address space (the operand pointers come
// from the task table, so the compiler cannot infer it).
template <typename T>
__device__ __forceinline__ cplx<T> gload(const cplx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2*)p;
    return cplx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gstore(cplx<T>* p, cplx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    *(__attribute__((address_space(1))) v2*)p = v2{v.re, v.im};
}

// T: the operands' type in memory; TC: the type of the products (TC = float with T = double
// reads complex128 operands, multiplies in complex64 on the fp32 matrix cores and writes
// complex128 results).
template <typename T, int W, typename TC = T>
__global__ void __launch_bounds__(64 * W) gemm_mfma_kernel(const GemmTask<T>* __restrict__ tasks, int M, int Nc, int K,
                                                           const int* __restrict__ gate_flags) {
    typedef Mfma<TC> F;
    typedef typename F::acc acc_t;
    constexpr int NT = 64 * W, KC = F::KC, KK = KC / 4, BP = KC + 1, BL = KC * 64 / NT;
    const GemmTask<T>& task = tasks[blockIdx.y];
    if (gate_flags && task.gate >= 0 && gate_flags[task.gate] == 0) return;
    const int rtiles = (M + 16 * W - 1) / (16 * W);
    const int rt = blockIdx.x % rtiles, ct = blockIdx.x / rtiles;
    const int col0 = ct * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wrow = rt * 16 * W + wave * 16;
    const bool live = wrow < M;   // uniform per wave
    __shared__ cplx<TC> Bs[2][64][BP];   // [buffer][column][k]
    acc_t cr[4], ci[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cr[j] = acc_t{0, 0, 0, 0};
        ci[j] = acc_t{0, 0, 0, 0};
    }
    const int nch = (K + KC - 1) / KC;
    const int total = task.nterms * nch;   // pipeline stages: (term, K chunk)
    cplx<T> an[KK], bst[BL];
    TC alpha_n = 1;
    // Loads are unconditional, from addresses clamped into the operands, and
    // out-of-range values are masked where they are used: the loads of the next
    // stage then stay in flight while this one is multiplied.
    const int ra = wrow + li < M ? wrow + li : M - 1;
    auto load_a = [&](int q) {
        const int t = q / nch, kc = q - t * nch;
        const cplx<T>* A = task.t[t].A;
        const int lda = task.t[t].lda;
        alpha_n = (TC)task.t[t].alpha_re;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const int k = kc * KC + kk * 4 + lk;
            an[kk] = gload(A + ra + (long)(k < K ? k : K - 1) * lda);
        }
    };
    auto load_b = [&](int q) {
        const int t = q / nch, kc = q - t * nch;
        const cplx<T>* B = task.t[t].B;
        const int ldb = task.t[t].ldb;
#pragma unroll
        for (int e = 0; e < BL; ++e) {
            const int idx = tid + NT * e;
            const int c = idx / KC, k = idx - c * KC;
            const int gk = kc * KC + k, gc = col0 + c;
            bst[e] = gload(B + (gk < K ? gk : K - 1) + (long)(gc < Nc ? gc : Nc - 1) * ldb);
        }
    };
    auto store_b = [&](int buf, int q) {
        const int kc = q % nch;
#pragma unroll
        for (int e = 0; e < BL; ++e) {
            const int idx = tid + NT * e;
            const int c = idx / KC, k = idx - c * KC;
            const bool ok = kc * KC + k < K && col0 + c < Nc;
            Bs[buf][c][k] = ok ? ccast<TC>(bst[e]) : mk<TC>(0, 0);
        }
    };
    load_a(0);
    load_b(0);
    store_b(0, 0);
    __syncthreads();
    for (int q = 0; q < total; ++q) {
        const int buf = q & 1;
        cplx<T> ac[KK];
        const TC alpha = alpha_n;
        const int kc = q % nch;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) ac[kk] = an[kk];
        // next stage in flight while this one is multiplied (the last stage is requested
        // again at the end, so that the wait counts stay static)
        load_a(q + 1 < total ? q + 1 : q);
        load_b(q + 1 < total ? q + 1 : q);
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const bool ok = wrow + li < M && kc * KC + kk * 4 + lk < K;
                const TC ar = ok ? alpha * (TC)ac[kk].re : TC(0), ai = ok ? alpha * (TC)ac[kk].im : TC(0), nai = -ai;
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    const cplx<TC> b = Bs[buf][jb * 16 + li][kk * 4 + lk];
                    cr[jb] = F::op(ar, b.re, cr[jb]);
                    cr[jb] = F::op(nai, b.im, cr[jb]);
                    ci[jb] = F::op(ar, b.im, ci[jb]);
                    ci[jb] = F::op(ai, b.re, ci[jb]);
                }
            }
        }
        if (q + 1 < total) store_b(buf ^ 1, q + 1);
        __syncthreads();
    }
    if (!live) return;
    const T beta = (T)task.beta;
    // the old values of C are all requested before any is used (one memory latency,
    // not one per element)
    cplx<T> old[4][4];
    if (task.beta != 0.0) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wrow + F::row(lk, v), c = col0 + jb * 16 + li;
                const int rc = r < M ? r : M - 1, cc = c < Nc ? c : Nc - 1;
                old[jb][v] = gload(task.C + rc + (long)cc * task.ldc);
            }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = wrow + F::row(lk, v);
            const int c = col0 + jb * 16 + li;
            if (r >= M || c >= Nc) continue;
            cplx<T> val = mk<T>((T)cr[jb][v], (T)ci[jb][v]);
            if (task.beta != 0.0) val = val + beta * old[jb][v];
            gstore(task.C + r + (long)c * task.ldc, val);
        }
}

template <typename T, int W, typename TC = T>
void launch_w(const GemmTask<T>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags, hipStream_t s) {
    const int tiles = ((Nc + 63) / 64) * ((M + 16 * W - 1) / (16 * W));
    for (int t0 = 0; t0 < ntasks; t0 += 65535) {   // grid.y is limited to 65535
        const int cnt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, W, TC>), dim3(tiles, cnt), dim3(64 * W), 0, s, tasks_dev + t0, M, Nc, K,
                           gate_flags);
        check_launch("gemm_mfma");
    }
}

template <typename T, typename TC = T>
void launch_mfma(const GemmTask<T>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags, hipStream_t s,
                 int active_hint) {
    if (ntasks <= 0) return;
    // waves per workgroup: cover the rows, but keep >= ~1k workgroups doing work for
    // small batches (measured on the sparse-solve phases: 8 waves from ~1k tasks up)
    const long busy = active_hint >= 0 ? active_hint : ntasks;
    int w = 8;
    while (w > 1 && 16 * (w / 2) >= M) w /= 2;
    if (w == 8 && busy * ((Nc + 63) / 64) < 1024) w = 4;
    switch (w) {
        case 8: launch_w<T, 8, TC>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        case 4: launch_w<T, 4, TC>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        case 2: launch_w<T, 2, TC>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        default: launch_w<T, 1, TC>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
    }
}

}  // namespace

void gemm_mfma_f64(const GemmTask<double>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s, int active_hint) {
    launch_mfma<double>(tasks_dev, ntasks, M, Nc, K, gate_flags, s, active_hint);
}

void gemm_mfma_f32(const GemmTask<float>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s, int active_hint) {
    launch_mfma<float>(tasks_dev, ntasks, M, Nc, K, gate_flags, s, active_hint);
}

void gemm_mfma_f64_c32(const GemmTask<double>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                       hipStream_t s, int active_hint) {
    launch_mfma<double, float>(tasks_dev, ntasks, M, Nc, K, gate_flags, s, active_hint);
}

}  // namespace pomm
