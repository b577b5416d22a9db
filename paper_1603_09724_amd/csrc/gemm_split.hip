// Batched multi-term complex GEMM for complex64 data with fp16 split products on the
// matrix cores (v_mfma_f32_16x16x32_f16, fp32 accumulation).
//
// A real number x is carried as 2^e (h + l) with h = fp16(x 2^-e), l = fp16(x 2^-e - h)
// and a power-of-two scale 2^e that puts the largest magnitude of its group in
// [2^14, 2^15).  The product of two such numbers is taken as h_a h_b + h_a l_b + l_a h_b:
// the dropped l_a l_b is 2^-22 of the product, so that a split product is about as
// accurate as a complex64 one, at the fp16 matrix rate (16 times the fp32 one per
// product, three products instead of one).  A complex product is four real ones:
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
//
// The factor operand A is fixed for the lifetime of a solver: it is split once
// (split_blocks) into tiles in MFMA fragment order with one scale per block, folded
// into the term's alpha.  The right-hand-side operand B (complex64 in HBM) is split
// when it is staged into LDS, with one scale per column and K chunk, so every chunk
// is multiplied into a fresh accumulator and added to the result with its scale.
//
// MFMA operand layout (16x16x32 f16, one block): lane l supplies A[l%16][8(l/16)+e]
// and B[8(l/16)+e][l%16], e = 0..7; accumulator element v holds D[4(l/16)+v][l%16].
//
// With one plane per part (PL = 2) the factor is kept as h alone: the block product is
// then that of the factor rounded once to fp16 (relative error 2^-12 per element, a fixed
// matrix), times the right-hand side split as above; two fp16 products per real product
// and half the factor bytes.  The solve stays a fixed linear operator.
//
// Split block layout: tiles of 16 rows x 32 k, tile (rt, kt) at (rt KT + kt) * PL KiB,
// KT = ceil(K/32) rounded up to even; inside a tile PL planes of 1 KiB (PL = 4: hi re,
// lo re, hi im, lo im; PL = 2: hi re, hi im), each 64 lanes x 8 halves in the fragment
// order above; rows >= M and k >= K are zero.  K must be a multiple of 8 (whole 8-deep
// groups of B).
#include "dense.h"

namespace pomm {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kPlaneBytes = 1024;

// k tiles stored per 16-row tile: ceil(K/32) rounded up to even, so that a 64-deep
// stage never reads past the block (the padding tiles are zero)
__host__ __device__ __forceinline__ int split_ktiles(int K) { return ((K + 63) / 64) * 2; }

__device__ __forceinline__ f4 mfma(h8 a, h8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }

// 2^k as a float, -126 <= k <= 127
__device__ __forceinline__ float pow2f(int k) { return __uint_as_float((unsigned)(k + 127) << 23); }

// Scale exponent s for a group whose largest magnitude is mx: mx 2^s in [2^14, 2^15)
// (s clamped to [-126, 126]; a zero or subnormal maximum gives s = 0).
__device__ __forceinline__ int group_shift(float mx) {
    const int be = (int)((__float_as_uint(mx) >> 23) & 0xff);
    if (be == 0) return 0;
    const int s = 14 - (be - 127);
    return s > 126 ? 126 : (s < -126 ? -126 : s);
}

// ---- setup: split one complex128 block per workgroup
__global__ void __launch_bounds__(256) split_blocks_kernel(const cplx<double>* const* __restrict__ src,
                                                           const int* __restrict__ lda, void* const* __restrict__ dst,
                                                           int M, int K, int planes, int* __restrict__ expo) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const cplx<double>* A = src[b];
    const int ld = lda[b];
    double mx = 0;
    for (long e = threadIdx.x; e < (long)M * K; e += blockDim.x) {
        const int r = (int)(e % M), k = (int)(e / M);
        const cplx<double> v = A[r + (long)k * ld];
        mx = fmax(mx, fmax(fabs(v.re), fabs(v.im)));
    }
    // block max (values are >= 0, so a max over lanes then waves)
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int ex = 0;
    if (mx > 0) {
        (void)frexp(mx, &ex);   // mx < 2^ex
        ex -= 15;               // stored = block 2^-ex < 2^15
    }
    if (threadIdx.x == 0) expo[b] = ex;
    // thread (tile, lane): the 8 values of its fragment slot, every plane (the lanes of a
    // wave read 4 runs of 16 consecutive rows and write 1 KiB per plane)
    const int RT = (M + 15) / 16, KT = split_ktiles(K);
    h8* out = static_cast<h8*>(dst[b]);
    for (int idx = threadIdx.x; idx < RT * KT * 64; idx += blockDim.x) {
        const int tile = idx / 64, lane = idx % 64;
        const int rt = tile / KT, kt = tile % KT;
        const int r = rt * 16 + lane % 16, k0 = kt * 32 + 8 * (lane / 16);
        h8 pl[4];
#pragma unroll
        for (int el = 0; el < 8; ++el) {
            const int k = k0 + el;
            double xr = 0, xi = 0;
            if (r < M && k < K) {
                const cplx<double> v = A[r + (long)k * ld];
                xr = ldexp(v.re, -ex);
                xi = ldexp(v.im, -ex);
            }
            const _Float16 hr = (_Float16)(float)xr, hi = (_Float16)(float)xi;
            pl[0][el] = hr;
            pl[1][el] = (_Float16)(float)(xr - (double)hr);
            pl[2][el] = hi;
            pl[3][el] = (_Float16)(float)(xi - (double)hi);
        }
        if (planes == 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) out[((size_t)tile * 4 + q) * 64 + lane] = pl[q];
        } else {   // hi re, hi im
            out[((size_t)tile * 2) * 64 + lane] = pl[0];
            out[((size_t)tile * 2 + 1) * 64 + lane] = pl[2];
        }
    }
}

// ---- the product kernel
// A workgroup is KSPLIT groups of W waves.  Wave w of group g owns 16 rows (row strip w)
// and the 64 columns of the tile, and takes the pipeline stages (term, 32-deep K chunk)
// q = g, g + KSPLIT, ...; the groups' partial results are summed through LDS in a fixed
// order at the end.  KSPLIT > 1 shortens the chain of stages of one workgroup, for
// launches with too few tiles to fill the chip.  Each group stages its right-hand-side
// chunk through its own double-buffered LDS area (one barrier per round of stages).
// Global loads are unconditional, from addresses clamped into the operands, and
// out-of-range data is masked only where it is used, so that the loads of the next
// stage stay in flight while this one is multiplied.
template <int W, int KSPLIT>
struct SplitSmem {
    h8 Bs[KSPLIT][2][4][4][64];   // [group][buffer][column block][plane][lane]
    float invs[KSPLIT][2][64];    // per column: 2^-s of the chunk's scale
};

template <int W, int KSPLIT, int PL>
__global__ void __launch_bounds__(64 * W * KSPLIT) gemm_split_kernel(const SplitTask* __restrict__ tasks, int ntasks,
                                                                     int M, int Nc, int K,
                                                                     const int* __restrict__ gate_flags) {
    constexpr int NT = 64 * W, NG = 4, ITEMS = 64 * NG;   // staging threads per group, 8-deep groups per chunk
    constexpr int IPT = (ITEMS + NT - 1) / NT;            // staging items per thread
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef float v2 __attribute__((ext_vector_type(2)));
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs by linear id,
    // so id L runs on XCD L % 8; the tiles of one task are given ids 8 apart (same XCD, so
    // the task's right-hand side is read into one L2), tasks padded to a multiple of 8.
    const int rtiles = (M + 16 * W - 1) / (16 * W);
    const int tiles = rtiles * ((Nc + 63) / 64);
    const int L = blockIdx.x, xcd = L & 7, r8 = L >> 3;
    const int ti = (r8 / tiles) * 8 + xcd, tile = r8 % tiles;
    if (ti >= ntasks) return;
    const SplitTask& task = tasks[ti];
    if (gate_flags && task.gate >= 0 && gate_flags[task.gate] == 0) return;
    const int rt = tile % rtiles, ct = tile / rtiles;
    const int col0 = ct * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = wave / W, wg = wave % W, gtid = threadIdx.x - grp * NT;
    const int RT = (M + 15) / 16, KT = (K + 31) / 32, KTP = split_ktiles(K);
    const int wrt = rt * W + wg;     // 16-row tile of this wave
    const bool live = wrt < RT;      // uniform per wave
    const int wrt_c = live ? wrt : RT - 1;
    __shared__ __align__(16) unsigned char smem_raw[sizeof(SplitSmem<W, KSPLIT>) > (KSPLIT - 1) * NT * 32 * 4
                                                        ? sizeof(SplitSmem<W, KSPLIT>)
                                                        : (KSPLIT - 1) * NT * 32 * 4];
    SplitSmem<W, KSPLIT>& sm = *reinterpret_cast<SplitSmem<W, KSPLIT>*>(smem_raw);
    f4 mr[4], mi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        mr[j] = f4{0, 0, 0, 0};
        mi[j] = f4{0, 0, 0, 0};
    }
    const int nch = KT;                    // 32-deep chunks per term
    const int total = task.nterms * nch;   // pipeline stages: (term, K chunk)
    const int rounds = (total + KSPLIT - 1) / KSPLIT;
    h8 an[PL];
    v4 bst[IPT][4];
    float alpha_n = 1;
    auto clampq = [&](int q) { return q < total ? q : total - 1; };
    auto load = [&](int q) {
        const int t = q / nch, kc = q - t * nch;
        alpha_n = task.t[t].alpha;
        const h8* At = static_cast<const h8*>(task.t[t].A) + ((size_t)wrt_c * KTP + (size_t)kc) * (PL * 64);
#pragma unroll
        for (int pl = 0; pl < PL; ++pl) an[pl] = *(const __attribute__((address_space(1))) h8*)(At + pl * 64 + lane);
        const cplx<float>* B = task.t[t].B;
        const int ldb = task.t[t].ldb;
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const int it = gtid + NT * e;
            const int j = it / NG, G = it % NG;
            const int k0 = kc * 32 + 8 * G, gc = col0 + j;
            const int k0c = k0 < K - 8 ? k0 : K - 8, gcc = gc < Nc - 1 ? gc : Nc - 1;
            const cplx<float>* p = B + k0c + (long)gcc * ldb;
#pragma unroll
            for (int u = 0; u < 4; ++u) bst[e][u] = *(const __attribute__((address_space(1))) v4*)(p + 2 * u);
        }
    };
    // split the group's staged chunk of stage q (valid when q < total) into LDS buffer b
    auto store_b = [&](int q, int b) {
        const int kc = q % nch;
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const int it = gtid + NT * e;
            const int j = it / NG, G = it % NG;
            const bool valid = q < total && it < ITEMS && col0 + j < Nc && kc * 32 + 8 * G < K;
            float x[16];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                x[4 * u] = valid ? bst[e][u].x : 0.0f;
                x[4 * u + 1] = valid ? bst[e][u].y : 0.0f;
                x[4 * u + 2] = valid ? bst[e][u].z : 0.0f;
                x[4 * u + 3] = valid ? bst[e][u].w : 0.0f;
            }
            float mx = 0;
#pragma unroll
            for (int u = 0; u < 16; ++u) mx = fmaxf(mx, fabsf(x[u]));
#pragma unroll
            for (int off = 1; off < NG; off <<= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
            const int s = group_shift(mx);
            const float sc = pow2f(s);
            h8 hr, lr, hi, li;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float xr = x[2 * u] * sc, xi = x[2 * u + 1] * sc;
                const _Float16 a = (_Float16)xr, c = (_Float16)xi;
                hr[u] = a;
                lr[u] = (_Float16)(xr - (float)a);
                hi[u] = c;
                li[u] = (_Float16)(xi - (float)c);
            }
            if (it < ITEMS) {
                const int jb = j / 16, slot = G * 16 + j % 16;
                sm.Bs[grp][b][jb][0][slot] = hr;
                sm.Bs[grp][b][jb][1][slot] = lr;
                sm.Bs[grp][b][jb][2][slot] = hi;
                sm.Bs[grp][b][jb][3][slot] = li;
                if (G == 0) sm.invs[grp][b][j] = pow2f(-s);
            }
        }
    };
    // round r: this group's stage q = r KSPLIT + grp from LDS buffer r % 2
    int q = grp;
    load(clampq(q));
    store_b(q, 0);
    __syncthreads();
    for (int r = 0; r < rounds; ++r, q += KSPLIT) {
        const int b = r & 1;
        h8 ac[PL];
#pragma unroll
        for (int pl = 0; pl < PL; ++pl) ac[pl] = an[pl];
        const float alpha = alpha_n;
        // next stage in flight while this one is multiplied (a stage past the end is
        // requested again and masked: unconditional loads keep the wait counts static)
        load(clampq(q + KSPLIT));
        if (live && q < total) {
            f4 cr[4], ci[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                cr[jb] = f4{0, 0, 0, 0};
                ci[jb] = f4{0, 0, 0, 0};
            }
            if constexpr (PL == 4) {
                const h8 nhi = -ac[2], nli = -ac[3];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    const h8 bhr = sm.Bs[grp][b][jb][0][lane], blr = sm.Bs[grp][b][jb][1][lane];
                    const h8 bhi = sm.Bs[grp][b][jb][2][lane], bli = sm.Bs[grp][b][jb][3][lane];
                    cr[jb] = mfma(ac[0], bhr, cr[jb]);
                    ci[jb] = mfma(ac[0], bhi, ci[jb]);
                    cr[jb] = mfma(ac[0], blr, cr[jb]);
                    ci[jb] = mfma(ac[0], bli, ci[jb]);
                    cr[jb] = mfma(ac[1], bhr, cr[jb]);
                    ci[jb] = mfma(ac[1], bhi, ci[jb]);
                    cr[jb] = mfma(nhi, bhi, cr[jb]);
                    ci[jb] = mfma(ac[2], bhr, ci[jb]);
                    cr[jb] = mfma(nhi, bli, cr[jb]);
                    ci[jb] = mfma(ac[2], blr, ci[jb]);
                    cr[jb] = mfma(nli, bhi, cr[jb]);
                    ci[jb] = mfma(ac[3], bhr, ci[jb]);
                }
            } else {   // fp16 factor (hi re, hi im) times the split right-hand side
                const h8 nhi = -ac[1];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    const h8 bhr = sm.Bs[grp][b][jb][0][lane], blr = sm.Bs[grp][b][jb][1][lane];
                    const h8 bhi = sm.Bs[grp][b][jb][2][lane], bli = sm.Bs[grp][b][jb][3][lane];
                    cr[jb] = mfma(ac[0], bhr, cr[jb]);
                    ci[jb] = mfma(ac[0], bhi, ci[jb]);
                    cr[jb] = mfma(ac[0], blr, cr[jb]);
                    ci[jb] = mfma(ac[0], bli, ci[jb]);
                    cr[jb] = mfma(nhi, bhi, cr[jb]);
                    ci[jb] = mfma(ac[1], bhr, ci[jb]);
                    cr[jb] = mfma(nhi, bli, cr[jb]);
                    ci[jb] = mfma(ac[1], blr, ci[jb]);
                }
            }
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const float f = alpha * sm.invs[grp][b][jb * 16 + (lane & 15)];
                mr[jb] += f * cr[jb];
                mi[jb] += f * ci[jb];
            }
        }
        if (r + 1 < rounds) store_b(q + KSPLIT, b ^ 1);
        __syncthreads();
    }
    if constexpr (KSPLIT > 1) {
        // the groups' partial sums, added in group order by group 0
        float* red = reinterpret_cast<float*>(smem_raw);   // [group - 1][wave of group][32][lane]
        if (grp > 0) {
            float* dst = red + ((size_t)(grp - 1) * W + wg) * 32 * 64 + lane;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dst[(jb * 8 + v) * 64] = mr[jb][v];
                    dst[(jb * 8 + 4 + v) * 64] = mi[jb][v];
                }
        }
        __syncthreads();
        if (grp > 0) return;
#pragma unroll
        for (int g = 1; g < KSPLIT; ++g) {
            const float* src = red + ((size_t)(g - 1) * W + wg) * 32 * 64 + lane;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    mr[jb][v] += src[(jb * 8 + v) * 64];
                    mi[jb][v] += src[(jb * 8 + 4 + v) * 64];
                }
        }
    }
    if (!live) return;
    const float beta = task.beta;
    const int li = lane & 15, lk = lane >> 4;
    // the old values of C are all requested before any is used (one memory latency,
    // not one per element)
    v2 old[4][4];
    if (beta != 0.0f) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wrt * 16 + 4 * lk + v, c = col0 + jb * 16 + li;
                const int rc = r < M ? r : M - 1, cc = c < Nc ? c : Nc - 1;
                old[jb][v] = *(const __attribute__((address_space(1))) v2*)(task.C + rc + (long)cc * task.ldc);
            }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = wrt * 16 + 4 * lk + v;
            const int c = col0 + jb * 16 + li;
            if (r >= M || c >= Nc) continue;
            float vr = mr[jb][v], vi = mi[jb][v];
            if (beta != 0.0f) {
                vr += beta * old[jb][v].x;
                vi += beta * old[jb][v].y;
            }
            *(__attribute__((address_space(1))) v2*)(task.C + r + (long)c * task.ldc) = v2{vr, vi};
        }
}

template <int W, int KSPLIT, int PL>
void launch_split(const SplitTask* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags, hipStream_t s) {
    const int tiles = ((Nc + 63) / 64) * ((M + 16 * W - 1) / (16 * W));
    const int chunk = 65536;   // tasks per launch (a multiple of 8)
    for (int t0 = 0; t0 < ntasks; t0 += chunk) {
        const int cnt = ntasks - t0 < chunk ? ntasks - t0 : chunk;
        const unsigned grid = (unsigned)((cnt + 7) / 8 * 8) * (unsigned)tiles;
        hipLaunchKernelGGL((gemm_split_kernel<W, KSPLIT, PL>), dim3(grid), dim3(64 * W * KSPLIT), 0, s, tasks_dev + t0, cnt,
                           M, Nc, K, gate_flags);
        check_launch("gemm_split");
    }
}

}  // namespace

size_t split_block_bytes(int M, int K, int planes) {
    return (size_t)((M + 15) / 16) * split_ktiles(K) * planes * kPlaneBytes;
}

void split_blocks(const cplx<double>* const* src_dev, const int* lda_dev, void* const* dst_dev, int count, int M, int K,
                  int planes, int* expo_dev, hipStream_t s) {
    if (count <= 0) return;
    POMM_CHECK(planes == 2 || planes == 4, 1, "split blocks have 2 or 4 planes");
    hipLaunchKernelGGL(split_blocks_kernel, dim3(count), dim3(256), 0, s, src_dev, lda_dev, dst_dev, M, K, planes,
                       expo_dev);
    check_launch("split_blocks");
}

template <int PL>
void gemm_split_planes(const SplitTask* tasks_dev, int ntasks, int M, int Nc, int K, const int* gate_flags,
                       hipStream_t s, int variant) {
    switch (variant) {
        case 1: launch_split<4, 2, PL>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        case 2: launch_split<2, 4, PL>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        case 3: launch_split<8, 1, PL>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        case 4: launch_split<2, 2, PL>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
        default: launch_split<4, 1, PL>(tasks_dev, ntasks, M, Nc, K, gate_flags, s); break;
    }
}

void gemm_split(const SplitTask* tasks_dev, int ntasks, int M, int Nc, int K, int planes, const int* gate_flags,
                hipStream_t s, int active_hint, int variant) {
    if (ntasks <= 0) return;
    POMM_CHECK(K >= 8 && K % 8 == 0 && Nc >= 1 && M >= 1, 1, "split products need K a multiple of 8");
    POMM_CHECK(planes == 2 || planes == 4, 1, "split blocks have 2 or 4 planes");
    if (variant < 0) {
        // measured per phase on the 128^2 workload: one group of 4 waves per 64 rows while
        // the busy tiles fill the chip, K shared by 2 or 4 groups when they do not
        const long busy = active_hint >= 0 ? active_hint : ntasks;
        const long wg4 = busy * ((M + 63) / 64) * ((Nc + 63) / 64);
        variant = wg4 >= 256 ? 0 : (wg4 >= 128 ? 1 : 2);
    }
    if (planes == 4) gemm_split_planes<4>(tasks_dev, ntasks, M, Nc, K, gate_flags, s, variant);
    else gemm_split_planes<2>(tasks_dev, ntasks, M, Nc, K, gate_flags, s, variant);
}

}  // namespace pomm
