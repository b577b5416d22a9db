// Batched multi-term complex GEMM on the matrix cores (v_mfma_f64_16x16x4f64 for
// complex128, v_mfma_f32_16x16x4f32 for complex64).
//
// Same task semantics as gemm_batched_kernel (dense.hip): C = beta C + sum_t alpha_t A_t B_t
// with real alpha_t.  A complex product is four real MFMA products on
// de-interleaved operands: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
// Block tile MT x 64 (MT = 128 or 64), MT/16 waves, each a 32 x 32 sub-tile of
// 2 x 2 MFMA blocks (16 x 16); K staged through LDS in chunks of 16 (four MFMA
// k-steps).  A 128-row tile covers a whole grid line block, so its
// right-hand-side tile is loaded once.
// MFMA operand layout (16x16x4, one block): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element v holds D[l/16 + 4 v][l%16] for the f64
// instruction and D[4 (l/16) + v][l%16] for the f32 one (both checked on gfx950).
#include "dense.h"

namespace pomm {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 64, kMK = 16;

// One 16x16x4 block product per precision, and the accumulator row of element v
// for lane group lk = lane/16 (the two instructions differ here).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef f64x4 acc;
    static constexpr int kPad = 1;   // LDS row padding (elements)
    __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
    typedef f32x4 acc;
    static constexpr int kPad = 16;
    __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

template <typename T, int MT>
__global__ void __launch_bounds__(MT * 4) gemm_mfma_kernel(const GemmTask<T>* __restrict__ tasks, int M, int Nc, int K,
                                                           const int* __restrict__ gate_flags) {
    typedef Mfma<T> F;
    typedef typename F::acc acc_t;
    constexpr int NTH = MT * 4, kMT = MT, kLP = MT + F::kPad, kBP = kNT + F::kPad;
    const GemmTask<T>& task = tasks[blockIdx.y];
    if (gate_flags && task.gate >= 0 && gate_flags[task.gate] == 0) return;
    const int tilesM = (M + kMT - 1) / kMT;
    const int tm = blockIdx.x % tilesM, tn = blockIdx.x / tilesM;
    const int row0 = tm * kMT, col0 = tn * kNT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    __shared__ T Ar[kMK][kLP], Ai[kMK][kLP], Br[kMK][kBP], Bi[kMK][kBP];
    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cr[i][j] = acc_t{0, 0, 0, 0};
            ci[i][j] = acc_t{0, 0, 0, 0};
        }
    for (int t = 0; t < task.nterms; ++t) {
        const GemmTerm<T> term = task.t[t];
        const T alpha = (T)term.alpha_re;
        for (int k0 = 0; k0 < K; k0 += kMK) {
            // A tile: MT rows x 16 k, element (r, k) at A[r + k*lda]
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tid + NTH * q;
                const int r = e % kMT, k = e / kMT;
                const int gr = row0 + r, gk = k0 + k;
                cplx<T> v = {0, 0};
                if (gr < M && gk < K) v = term.A[gr + (long)gk * term.lda];
                Ar[k][r] = alpha * v.re;
                Ai[k][r] = alpha * v.im;
            }
            // B tile: 16 k x 64 cols, element (k, c) at B[k + c*ldb]
#pragma unroll
            for (int q = 0; q < 1024 / NTH; ++q) {
                const int e = tid + NTH * q;
                const int k = e & 15, c = e >> 4;
                const int gk = k0 + k, gc = col0 + c;
                cplx<T> v = {0, 0};
                if (gk < K && gc < Nc) v = term.B[gk + (long)gc * term.ldb];
                Br[k][c] = v.re;
                Bi[k][c] = v.im;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kMK; kk += 4) {
                T ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    ar[ib] = Ar[kk + lk][wr + ib * 16 + li];
                    ai[ib] = Ai[kk + lk][wr + ib * 16 + li];
                    nai[ib] = -ai[ib];
                }
#pragma unroll
                for (int jb = 0; jb < 2; ++jb) {
                    br[jb] = Br[kk + lk][wc + jb * 16 + li];
                    bi[jb] = Bi[kk + lk][wc + jb * 16 + li];
                }
#pragma unroll
                for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb) {
                        cr[ib][jb] = F::op(ar[ib], br[jb], cr[ib][jb]);
                        cr[ib][jb] = F::op(nai[ib], bi[jb], cr[ib][jb]);
                        ci[ib][jb] = F::op(ar[ib], bi[jb], ci[ib][jb]);
                        ci[ib][jb] = F::op(ai[ib], br[jb], ci[ib][jb]);
                    }
            }
            __syncthreads();
        }
    }
    const T beta = (T)task.beta;
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + wr + ib * 16 + F::row(lk, v);
                const int c = col0 + wc + jb * 16 + li;
                if (r >= M || c >= Nc) continue;
                cplx<T>* p = task.C + r + (long)c * task.ldc;
                cplx<T> val = mk<T>(cr[ib][jb][v], ci[ib][jb][v]);
                if (task.beta != 0.0) val = val + beta * (*p);
                *p = val;
            }
}

template <typename T>
void launch_mfma(const GemmTask<T>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags, hipStream_t s) {
    if (ntasks <= 0) return;
    const bool wide = M > 64;
    const int MT = wide ? 128 : 64;
    const int tiles = ((M + MT - 1) / MT) * ((Nc + kNT - 1) / kNT);
    for (int t0 = 0; t0 < ntasks; t0 += 65535) {
        const int cnt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
        if (wide)
            hipLaunchKernelGGL((gemm_mfma_kernel<T, 128>), dim3(tiles, cnt), dim3(512), 0, s, tasks_dev + t0, M, Nc, K,
                               gate_flags);
        else
            hipLaunchKernelGGL((gemm_mfma_kernel<T, 64>), dim3(tiles, cnt), dim3(256), 0, s, tasks_dev + t0, M, Nc, K,
                               gate_flags);
        check_launch("gemm_mfma");
    }
}

}  // namespace

void gemm_mfma_f64(const GemmTask<double>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s) {
    launch_mfma<double>(tasks_dev, ntasks, M, Nc, K, gate_flags, s);
}

void gemm_mfma_f32(const GemmTask<float>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s) {
    launch_mfma<float>(tasks_dev, ntasks, M, Nc, K, gate_flags, s);
}

}  // namespace pomm
