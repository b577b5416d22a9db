// Dense complex kernels: batched multi-term GEMM, split-K Gram products and
// batched Gauss-Jordan inversion.
#pragma once

#include "common.h"

namespace pomm {

constexpr int kMaxTerms = 8;   // terms per GEMM task

template <typename T>
struct GemmTerm {
    const cplx<T>* A;   // M x K, column major, lda
    const cplx<T>* B;   // K x Nc, column major, ldb
    int lda, ldb;
    double alpha_re, alpha_im;
};

template <typename T>
struct GemmTask {
    cplx<T>* C;         // M x Nc, column major, ldc
    int ldc;
    int nterms;         // 1..kMaxTerms
    double beta;        // real; 0 means C is not read
    int gate;           // index into the gate flags (skip the task when flags[gate] == 0), -1 = always
    GemmTerm<T> t[kMaxTerms];
};

// C = beta C + sum_t alpha_t A_t B_t for every task; tasks in device memory.
// active_hint: tasks expected to pass the gate (launch shape only); -1 = all.
template <typename T>
void gemm_batched(const GemmTask<T>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                  hipStream_t s, int active_hint = -1);

// Matrix-core paths of gemm_batched (MFMA f64 / f32); alpha_t must be real.
void gemm_mfma_f64(const GemmTask<double>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s, int active_hint);
void gemm_mfma_f32(const GemmTask<float>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                   hipStream_t s, int active_hint);
// complex128 operands and results, complex64 products on the fp32 matrix cores
void gemm_mfma_f64_c32(const GemmTask<double>* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                       hipStream_t s, int active_hint);

// Split-product GEMM (gemm_split.hip): complex64 right-hand sides and results, the
// factor operand as fp16 hi/lo tiles (4 planes: three fp16 products per real product)
// or as fp16 hi tiles alone (2 planes: two products), on the matrix cores, fp32
// accumulation.  C = beta C + sum_t alpha_t A_t B_t.
struct SplitTerm {
    const void* A;             // split block of split_block_bytes(M, K, planes) bytes (split_blocks)
    const cplx<float>* B;      // K x Nc, column major, ldb; 16-byte aligned, ldb even
    int ldb;
    float alpha;               // real; includes the block's power-of-two scale
};
struct SplitTask {
    cplx<float>* C;            // M x Nc, column major, ldc
    int ldc;
    int nterms;                // 1..kMaxTerms
    float beta;                // real; 0 means C is not read
    int gate;                  // as GemmTask::gate
    SplitTerm t[kMaxTerms];
};
size_t split_block_bytes(int M, int K, int planes);
// K must be a multiple of 8, planes 2 or 4.  Split `count` complex128 blocks src[i] (M x K, column
// major, lda[i]) into dst[i]; expo[i] receives e with block = 2^e * (stored block).  Pointer arrays
// in device memory.
void split_blocks(const cplx<double>* const* src_dev, const int* lda_dev, void* const* dst_dev, int count, int M, int K,
                  int planes, int* expo_dev, hipStream_t s);
// variant: workgroup shape, W waves per 16-row group times KSPLIT groups that share the
// K stages (0: 4x1, 1: 4x2, 2: 2x4, 3: 8x1, 4: 2x2; -1: chosen from the busy tile count)
void gemm_split(const SplitTask* tasks_dev, int ntasks, int M, int Nc, int K, int planes, const int* gate_flags,
                hipStream_t s, int active_hint, int variant = -1);

// Gram products: out[p] (N x N, column major) = P_p^H Q_p over n rows, for
// `nprod` pairs given as device pointer arrays Ps/Qs (each n x N, ld = n).
// `parts` workspace: nprod * chunks * N * N complex; fixed-order reduction.
struct GramPlan {
    int n = 0, N = 0, chunks = 0;
};
GramPlan gram_plan(int n, int N);
size_t gram_parts_elems(const GramPlan& g, int nprod);
void gram_products(const GramPlan& g, const cplx<double>* const* Ps, const cplx<double>* const* Qs, int nprod,
                   cplx<double>* parts, cplx<double>* out, hipStream_t s);

// In-place inversion of `count` matrices of order n (column major, ld = n),
// consecutive in memory with stride `stride` elements; partial pivoting.
// `piv` workspace: count * n ints.
template <typename T>
void invert_batched(cplx<T>* mats, long stride, int n, int count, int* piv, hipStream_t s);

}  // namespace pomm
