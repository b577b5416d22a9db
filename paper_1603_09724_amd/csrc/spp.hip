// Sparsifying preconditioner: stencil construction, assembly of P_j, block
// cyclic reduction factorization and solve (see spp.h).
#include "spp.h"
#include "prof.h"

#include <algorithm>
#include <cstring>

namespace pomm {

namespace {

using cd = std::complex<double>;

constexpr int kStencil = 9;   // 3x3 neighbourhood, index (s1+1) + 3 (s2+1)
constexpr int kDisp = 25;     // displacements in {-2..2}^2, index (d1+2) + 5 (d2+2)

// g(D) = (1/n) sum_k gh(k) e^{+2 pi i k.D/m},  R(D) = (1/n) sum_k |gh(k)|^2 e^{-2 pi i k.D/m},
// gh(k) = 1/(|k|^2/2 + l - z_j).  One block per (pole, displacement).
__global__ void __launch_bounds__(256) green_moments_kernel(const cplx<double>* __restrict__ zs, double l, int m,
                                                            const cplx<double>* __restrict__ tw,
                                                            cplx<double>* __restrict__ gD,
                                                            cplx<double>* __restrict__ RD) {
    __shared__ double red[4];
    const int j = blockIdx.x, di = blockIdx.y;
    const int d1 = di % 5 - 2, d2 = di / 5 - 2;
    const int n = m * m;
    const cplx<double> z = zs[j];
    double gre = 0, gim = 0, rre = 0, rim = 0;
    for (int kf = threadIdx.x; kf < n; kf += blockDim.x) {
        const int i2 = kf / m, i1 = kf - i2 * m;
        const int k1 = freq_of(i1, m), k2 = freq_of(i2, m);
        const double re = 0.5 * (double)(k1 * k1 + k2 * k2) + l - z.re, im = -z.im;
        const double den = re * re + im * im;
        const double hr = re / den, hi = -im / den;
        int t = (k1 * d1 + k2 * d2) % m;
        if (t < 0) t += m;
        const cplx<double> e = tw[t];   // e^{-2 pi i t/m}
        gre += hr * e.re + hi * e.im;   // gh * conj(e)
        gim += hi * e.re - hr * e.im;
        const double a = hr * hr + hi * hi;
        rre += a * e.re;
        rim += a * e.im;
    }
    gre = block_sum(gre, red);
    gim = block_sum(gim, red);
    rre = block_sum(rre, red);
    rim = block_sum(rim, red);
    if (threadIdx.x == 0) {
        gD[j * kDisp + di] = mk<double>(gre / n, gim / n);
        RD[j * kDisp + di] = mk<double>(rre / n, rim / n);
    }
}

// mult[j][k] = qhat_j(k) * gh_j(k), qhat(k) = sum_s q_s e^{+2 pi i k.s/m}.
__global__ void rhs_mult_kernel(const cplx<double>* __restrict__ zs, const cplx<double>* __restrict__ qs, double l,
                                int m, int p, const cplx<double>* __restrict__ tw, cplx<double>* __restrict__ mult,
                                cplx<float>* __restrict__ mult32) {
    const int n = m * m;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * p) return;
    const int j = (int)(idx / n), kf = (int)(idx - (long)j * n);
    const int i2 = kf / m, i1 = kf - i2 * m;
    const int k1 = freq_of(i1, m), k2 = freq_of(i2, m);
    cplx<double> qh = {0, 0};
    for (int s = 0; s < kStencil; ++s) {
        const int s1 = s % 3 - 1, s2 = s / 3 - 1;
        int t = (k1 * s1 + k2 * s2) % m;
        if (t < 0) t += m;
        qh = qh + qs[j * kStencil + s] * conj(tw[t]);
    }
    const cplx<double> z = zs[j];
    const cplx<double> den = mk<double>(0.5 * (double)(k1 * k1 + k2 * k2) + l - z.re, -z.im);
    const cplx<double> v = cdiv(qh, den);
    mult[idx] = v;
    if (mult32) mult32[idx] = ccast<float>(v);
}

// blocks[((pole*m + line)*3 + w) * m*m], w = 0: A (same line), 1: B (next line), 2: C (previous line).
// Entry (row r, column c) of a block at r + c*m.
// Stencil coupling P(j, j + (s1, s2)) = q_s + t_s (V_{j+s} - l) of point j = (r, line).
__device__ __forceinline__ cplx<double> stencil_p(const cplx<double>* q, const cplx<double>* t, const double* V,
                                                  double l, int m, int line, int r, int s1, int s2) {
    const int s = (s1 + 1) + 3 * (s2 + 1);
    const int c = (r + s1 + m) % m, ln = (line + s2 + m) % m;
    return q[s] + (V[c + (long)m * ln] - l) * t[s];
}

// Dense A_o of every (pole, level-0 odd line) into out (the inputs of the inversion when
// m is not a power of two): A_o(r, c) = sum of P(r, (s1, 0)) over (r + s1) mod m = c.
__global__ void assemble_odd_kernel(const double* __restrict__ V, double l, const cplx<double>* __restrict__ qs,
                                    const cplx<double>* __restrict__ ts, int m, cplx<double>* __restrict__ out) {
    const int u = blockIdx.x, pole = blockIdx.y, o = 2 * u + 1;
    const long bb = (long)m * m;
    cplx<double>* blk = out + ((long)pole * (m / 2) + u) * bb;
    const cplx<double>* q = qs + pole * kStencil;
    const cplx<double>* t = ts + pole * kStencil;
    for (long e = threadIdx.x; e < bb; e += blockDim.x) {
        const int r = (int)(e % m), c = (int)(e / m);
        cplx<double> v = mk<double>(0, 0);
        for (int s1 = -1; s1 <= 1; ++s1)
            if ((r + s1 + m) % m == c) v = v + stencil_p(q, t, V, l, m, o, r, s1, 0);
        blk[e] = v;
    }
}

// First-level Schur complements of the even lines.  With the couplings of line e to the
// lines below and above (C_e, B_e: cyclic tridiagonal, from the stencil) and the dense
// inverses of the odd neighbours, alpha = C_e Ainv_{e-1} and gamma = B_e Ainv_{e+1}:
//   A_e' = A_e - alpha B_{e-1} - gamma C_{e+1},  C_e' = -alpha C_{e-1},  B_e' = -gamma B_{e+1}.
// Element (i, j) of each is a 3 x 3 stencil of an inverse around (i, j): the row factors
// C_e(i, i+s), B_e(i, i+s) and the column factors X(j-s', j) of the neighbours' blocks.
// blocks: (pole, even line e) at ((pole m/2 + e/2) 3 + w) m^2, w = 0 (A'), 1 (B'), 2 (C').
__global__ void __launch_bounds__(256) level0_schur_kernel(const cplx<double>* __restrict__ ainv,
                                                           const double* __restrict__ V, double l,
                                                           const cplx<double>* __restrict__ qs,
                                                           const cplx<double>* __restrict__ ts, int m,
                                                           cplx<double>* __restrict__ blocks) {
    const int u = blockIdx.x, pole = blockIdx.y, no = m / 2;
    const int e = 2 * u, om = (e + m - 1) % m, op = (e + 1) % m;
    const long bb = (long)m * m;
    const cplx<double>* q = qs + pole * kStencil;
    const cplx<double>* t = ts + pole * kStencil;
    const cplx<double>* Am = ainv + ((long)pole * no + (om - 1) / 2) * bb;
    const cplx<double>* Ap = ainv + ((long)pole * no + (op - 1) / 2) * bb;
    cplx<double>* out = blocks + ((long)pole * no + u) * 3 * bb;
    const long chunk = (bb + gridDim.z - 1) / gridDim.z;
    const long e0 = (long)blockIdx.z * chunk, e1 = e0 + chunk < bb ? e0 + chunk : bb;
    for (long f = e0 + threadIdx.x; f < e1; f += blockDim.x) {
        const int i = (int)(f % m), j = (int)(f / m);
        cplx<double> u1[3], u2[3];   // alpha(i, j - s'), gamma(i, j - s')
#pragma unroll
        for (int sp = 0; sp < 3; ++sp) {
            u1[sp] = mk<double>(0, 0);
            u2[sp] = mk<double>(0, 0);
        }
#pragma unroll
        for (int s = -1; s <= 1; ++s) {
            const cplx<double> cc = stencil_p(q, t, V, l, m, e, i, s, -1), cb = stencil_p(q, t, V, l, m, e, i, s, 1);
            const long row = (i + s + m) % m;
#pragma unroll
            for (int sp = -1; sp <= 1; ++sp) {
                const long idx = row + (long)((j - sp + m) % m) * m;
                u1[sp + 1] = u1[sp + 1] + cc * Am[idx];
                u2[sp + 1] = u2[sp + 1] + cb * Ap[idx];
            }
        }
        cplx<double> a = mk<double>(0, 0), bo = mk<double>(0, 0), co = mk<double>(0, 0);
#pragma unroll
        for (int s1 = -1; s1 <= 1; ++s1)
            if ((i + s1 + m) % m == j) a = a + stencil_p(q, t, V, l, m, e, i, s1, 0);
#pragma unroll
        for (int sp = -1; sp <= 1; ++sp) {
            const int r = (j - sp + m) % m;   // X(r, j) = P((r, line), (sp, s2)) of the neighbour line
            a = a - u1[sp + 1] * stencil_p(q, t, V, l, m, om, r, sp, 1) -
                u2[sp + 1] * stencil_p(q, t, V, l, m, op, r, sp, -1);
            co = co - u1[sp + 1] * stencil_p(q, t, V, l, m, om, r, sp, -1);
            bo = bo - u2[sp + 1] * stencil_p(q, t, V, l, m, op, r, sp, 1);
        }
        out[f] = a;
        out[bb + f] = bo;
        out[2 * bb + f] = co;
    }
}

// Copy `count` blocks of `elems` elements: dst[i] <- src[i].
__global__ void copy_blocks_kernel(const cplx<double>* const* __restrict__ src, cplx<double>* const* __restrict__ dst,
                                   long elems) {
    const cplx<double>* s = src[blockIdx.y];
    cplx<double>* d = dst[blockIdx.y];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < elems; e += (long)gridDim.x * blockDim.x) d[e] = s[e];
}

// Final dense system of mf (even) lines per pole: F[a][a] += A, F[a][a+1] += B, F[a][a-1] += C (cyclic).
__global__ void assemble_final_kernel(const cplx<double>* __restrict__ blocks, const int* __restrict__ lines, int mf,
                                      int m, cplx<double>* __restrict__ fin, long fin_stride) {
    const int pole = blockIdx.y;
    const int F = mf * m;
    const long bb = (long)m * m;
    cplx<double>* out = fin + (long)pole * fin_stride;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)F * F; e += (long)gridDim.x * blockDim.x) {
        const int R = (int)(e % F), Cc = (int)(e / F);
        const int a = R / m, r = R % m, bcol = Cc / m, c = Cc % m;
        const int line = lines[a];
        const cplx<double>* base = blocks + ((long)pole * (m / 2) + line / 2) * 3 * bb;
        cplx<double> v = {0, 0};
        const long off = r + (long)c * m;
        if (bcol == a) v = v + base[off];
        if (bcol == (a + 1) % mf) v = v + base[bb + off];
        if (bcol == (a + mf - 1) % mf) v = v + base[2 * bb + off];
        out[e] = v;
    }
}

// ---- level-0 line blocks
// A_o (line o, the s2 = 0 part of P) is cyclic tridiagonal: sub a_i = P(i, i-1),
// diagonal b_i, super c_i = P(i, i+1), indices mod m.  It is diagonally dominant
// on the workloads here (|b_i| >= 2.6 (|a_i| + |c_i|) for every pole), so it is
// factored without pivoting as a bordered system: T = the leading m-1 rows and
// columns (tridiagonal LU), the border u (last column: u_0 = a_0, u_{m-2} =
// c_{m-2}), w (last row: w_0 = c_{m-1}, w_{m-2} = a_{m-1}) and the corner b_{m-1}.
// A y = r: p = T^{-1} r', y_{m-1} = (r_{m-1} - w.p) / (b_{m-1} - w.T^{-1}u),
// y_i = p_i - (T^{-1}u)_i y_{m-1}.
// Storage per (pole, level-0 odd line): lsub[m] (l_i, i = 1..m-2), invd[m]
// (1/d_i, i = 0..m-2), sup[m] (c_i, i = 0..m-3), sv[m] ((T^{-1}u)_i), then
// w_0, w_{m-2}, 1/(b_{m-1} - w.T^{-1}u).
__host__ __device__ constexpr int tri_stride(int m) { return 4 * m + 4; }

__global__ void tri_factor_kernel(const cplx<double>* __restrict__ qs, const cplx<double>* __restrict__ ts,
                                  const double* __restrict__ V, double l, int m, int p, cplx<double>* __restrict__ tri) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int no = m / 2;
    if (idx >= p * no) return;
    const int pole = idx / no, o = 2 * (idx % no) + 1;
    const cplx<double>* q = qs + pole * kStencil;
    const cplx<double>* t = ts + pole * kStencil;
    // P(i, i + s1) on line o: stencil index (s1 + 1) + 3 (0 + 1)
    auto coef = [&](int s1, int i) {
        const int ii = (i + s1 + m) % m;
        return q[4 + s1] + (V[ii + (long)m * o] - l) * t[4 + s1];
    };
    cplx<double>* lsub = tri + (size_t)idx * tri_stride(m);
    cplx<double>* invd = lsub + m;
    cplx<double>* sup = lsub + 2 * m;
    cplx<double>* sv = lsub + 3 * m;
    cplx<double>* sc = lsub + 4 * m;
    const cplx<double> one = mk<double>(1, 0);
    lsub[0] = mk<double>(0, 0);
    invd[0] = cdiv(one, coef(0, 0));
    for (int i = 1; i <= m - 2; ++i) {
        lsub[i] = coef(-1, i) * invd[i - 1];
        invd[i] = cdiv(one, coef(0, i) - lsub[i] * coef(1, i - 1));
    }
    for (int i = 0; i <= m - 3; ++i) sup[i] = coef(1, i);
    // sv = T^{-1} u
    for (int i = 0; i <= m - 2; ++i) sv[i] = mk<double>(0, 0);
    sv[0] = coef(-1, 0);
    sv[m - 2] = sv[m - 2] + coef(1, m - 2);
    for (int i = 1; i <= m - 2; ++i) sv[i] = sv[i] - lsub[i] * sv[i - 1];
    sv[m - 2] = sv[m - 2] * invd[m - 2];
    for (int i = m - 3; i >= 0; --i) sv[i] = (sv[i] - sup[i] * sv[i + 1]) * invd[i];
    const cplx<double> w0 = coef(1, m - 1), wl = coef(-1, m - 1);
    sc[0] = w0;
    sc[1] = wl;
    sc[2] = cdiv(one, coef(0, m - 1) - (w0 * sv[0] + wl * sv[m - 2]));
    sc[3] = mk<double>(0, 0);
}

// X_o = A_o^{-1} R_o (ACC = 0) or X_o -= A_o^{-1} R_o (ACC = 1) for the level-0 odd
// lines o = 2u + 1, CPW right-hand sides per workgroup (one per lane).  The m x CPW
// block is staged in LDS (coalesced loads and stores along the line); each lane
// then sweeps its column in place.
template <typename T, int CPW, bool ACC>
__global__ void __launch_bounds__(64) tri_lines_kernel(const cplx<T>* __restrict__ R, cplx<T>* __restrict__ X,
                                                       const cplx<T>* __restrict__ tri, int m, int N, long n,
                                                       const int* __restrict__ pole_active) {
    const int u = blockIdx.x, c0 = blockIdx.y * CPW, pole = blockIdx.z;
    if (pole_active && pole_active[pole] == 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int P = CPW + 1;
    const int lane = threadIdx.x, no = m / 2, o = 2 * u + 1, fs = tri_stride(m);
    cplx<T>* fsh = reinterpret_cast<cplx<T>*>(smem_raw);   // the line's factors
    cplx<T>* sh = fsh + fs;                                  // [i][column], pitch P
    const int ncol = N - c0 < CPW ? N - c0 : CPW;
    const long base = ((long)pole * N + c0) * n + (long)o * m;
    const cplx<T>* f = tri + ((size_t)pole * no + u) * fs;
    for (int i = lane; i < fs; i += 64) fsh[i] = f[i];
    // staging in batches of 8 loads per lane (m <= 128: element i = lane + 64 h, h < 2)
#pragma unroll 2
    for (int cc0 = 0; cc0 < CPW; cc0 += 4) {
        cplx<T> tmp[4][2];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cc = cc0 + a, i = lane + 64 * h;
                tmp[a][h] = (cc < ncol && i < m) ? R[base + (long)cc * n + i] : mk<T>(0, 0);
            }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cc = cc0 + a, i = lane + 64 * h;
                if (cc < ncol && i < m) sh[i * P + cc] = tmp[a][h];
            }
    }
    __syncthreads();
    if (lane < ncol) {
        const cplx<T>* lsub = fsh;
        const cplx<T>* invd = fsh + m;
        const cplx<T>* sup = fsh + 2 * m;
        const cplx<T>* sv = fsh + 3 * m;
        cplx<T>* col = sh + lane;
        cplx<T> z = col[0];
#pragma unroll 16
        for (int i = 1; i <= m - 2; ++i) {
            z = col[i * P] - lsub[i] * z;
            col[i * P] = z;
        }
        z = z * invd[m - 2];
        col[(m - 2) * P] = z;
#pragma unroll 16
        for (int i = m - 3; i >= 0; --i) {
            z = (col[i * P] - sup[i] * z) * invd[i];
            col[i * P] = z;
        }
        const cplx<T> ylast =
            (col[(m - 1) * P] - (fsh[4 * m] * col[0] + fsh[4 * m + 1] * col[(m - 2) * P])) * fsh[4 * m + 2];
        col[(m - 1) * P] = ylast;
#pragma unroll 16
        for (int i = 0; i <= m - 2; ++i) col[i * P] = col[i * P] - sv[i] * ylast;
    }
    __syncthreads();
#pragma unroll 2
    for (int cc0 = 0; cc0 < CPW; cc0 += 4) {
        cplx<T> old[4][2];
        if constexpr (ACC) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = cc0 + a, i = lane + 64 * h;
                    old[a][h] = (cc < ncol && i < m) ? X[base + (long)cc * n + i] : mk<T>(0, 0);
                }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cc = cc0 + a, i = lane + 64 * h;
                if (cc < ncol && i < m) {
                    const cplx<T> y = sh[i * P + cc];
                    X[base + (long)cc * n + i] = ACC ? old[a][h] - y : y;
                }
            }
    }
}

// Power-of-two m: parallel cyclic reduction of the same periodic systems, one lane
// per line element.  Reduction step s (distance d = 2^s, s < S = log2 m - 1) maps
// each equation a_i x_{i-d} + b_i x_i + c_i x_{i+d} = r_i to one in x_{i-2d}, x_i,
// x_{i+2d} with the multipliers alpha_i = -a_i / b_{i-d}, gamma_i = -c_i / b_{i+d}
// (r_i <- r_i + alpha_i r_{i-d} + gamma_i r_{i+d}); after S steps equation i couples
// x_i and x_{i+m/2} only, and the 2x2 systems give x_i = u_i r_i + v_i r_{i+m/2}.
// The multipliers do not depend on the right-hand side: they are computed once per
// (pole, line) and stored as [k][i], k = 2s (alpha), 2s + 1 (gamma), 2S (u), 2S + 1 (v).
__host__ __device__ inline int pcr_steps(int m) {
    int s = 0;
    while ((2 << s) < m) ++s;   // 2^(s+1) >= m
    return s;                    // log2 m - 1 for a power of two
}

// One workgroup of m threads per (pole, odd line), thread i = equation i; the current
// coefficients of all equations in LDS (read, barrier, then overwritten).
__global__ void __launch_bounds__(128) pcr_factor_kernel(const cplx<double>* __restrict__ qs,
                                                         const cplx<double>* __restrict__ ts,
                                                         const double* __restrict__ V, double l, int m,
                                                         cplx<double>* __restrict__ out) {
    const int no = m / 2, u = blockIdx.x, pole = blockIdx.y, i = threadIdx.x;
    const int o = 2 * u + 1, S = pcr_steps(m);
    const cplx<double>* q = qs + pole * kStencil;
    const cplx<double>* t = ts + pole * kStencil;
    __shared__ cplx<double> A[128], B[128], C[128];
    auto coef = [&](int s1) {
        const int ii = (i + s1 + m) % m;
        return q[4 + s1] + (V[ii + (long)m * o] - l) * t[4 + s1];
    };
    cplx<double> a = coef(-1), b = coef(0), c = coef(1);
    cplx<double>* dst = out + ((size_t)pole * no + u) * (2 * S + 2) * m + i;
    const cplx<double> one = mk<double>(1, 0);
    for (int s = 0, d = 1; s < S; ++s, d *= 2) {
        A[i] = a;
        B[i] = b;
        C[i] = c;
        __syncthreads();
        const int im = (i - d + m) % m, ip = (i + d) % m;
        const cplx<double> al = mk<double>(0, 0) - a * cdiv(one, B[im]);
        const cplx<double> ga = mk<double>(0, 0) - c * cdiv(one, B[ip]);
        dst[(2 * s) * m] = al;
        dst[(2 * s + 1) * m] = ga;
        const cplx<double> na = al * A[im];
        const cplx<double> nb = b + al * C[im] + ga * A[ip];
        const cplx<double> nc = ga * C[ip];
        __syncthreads();
        a = na;
        b = nb;
        c = nc;
    }
    A[i] = a;
    B[i] = b;
    C[i] = c;
    __syncthreads();
    const int h = (i + m / 2) % m;
    const cplx<double> ei = a + c, eh = A[h] + C[h];
    const cplx<double> det = b * B[h] - ei * eh;
    dst[(2 * S) * m] = cdiv(B[h], det);
    dst[(2 * S + 1) * m] = mk<double>(0, 0) - cdiv(ei, det);
}

// The reduction applied to G right-hand sides held by the workgroup's threads
// (thread t: element i of column slot t / m; `al`, `ga`, uu, vv its multipliers);
// buf: two LDS exchange buffers of G x 128, *bsel the next one to use.
template <typename T, int G, int SMAX>
__device__ __forceinline__ void pcr_apply(cplx<T> (&r)[G], const cplx<T> (&al)[SMAX], const cplx<T> (&ga)[SMAX],
                                          cplx<T> uu, cplx<T> vv, int S, int m, int t, int i,
                                          cplx<T> (*buf)[G][128], int& bsel) {
    const int base_t = t - i;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
        if (s >= S) break;
        const int d = 1 << s;
#pragma unroll
        for (int g = 0; g < G; ++g) buf[bsel][g][t] = r[g];
        __syncthreads();
        const int im = base_t + ((i - d) & (m - 1)), ip = base_t + ((i + d) & (m - 1));
#pragma unroll
        for (int g = 0; g < G; ++g) r[g] = r[g] + al[s] * buf[bsel][g][im] + ga[s] * buf[bsel][g][ip];
        bsel ^= 1;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) buf[bsel][g][t] = r[g];
    __syncthreads();
    const int ih = base_t + ((i + m / 2) & (m - 1));
#pragma unroll
    for (int g = 0; g < G; ++g) r[g] = uu * r[g] + vv * buf[bsel][g][ih];
    bsel ^= 1;
}

// Multipliers of element i of (pole, line u) into registers.
template <typename T, int SMAX>
__device__ __forceinline__ void pcr_load(const cplx<T>* cf, int m, int S, cplx<T> (&al)[SMAX], cplx<T> (&ga)[SMAX],
                                         cplx<T>& uu, cplx<T>& vv) {
#pragma unroll
    for (int s = 0; s < SMAX; ++s)
        if (s < S) {
            al[s] = cf[(2 * s) * m];
            ga[s] = cf[(2 * s + 1) * m];
        }
    uu = cf[(2 * S) * m];
    vv = cf[(2 * S + 1) * m];
}

// Level-0 couplings of element i of line `line` through the stencil's s2 = -1 and +1
// parts: pc[h][s1 + 1] = P(j, j + (s1, s2)) with s2 = -1 (h = 0) or +1 (h = 1),
// j = (i, line), P(j, j + s) = q_s + t_s (V_{j+s} - l).
template <typename T>
__device__ __forceinline__ void coupling_load(const cplx<double>* __restrict__ q, const cplx<double>* __restrict__ t,
                                              const double* __restrict__ V, double l, int m, int line, int i,
                                              cplx<T> (&pc)[2][3]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int s2 = h ? 1 : -1, ln = (line + s2 + m) % m;
#pragma unroll
        for (int s1 = -1; s1 <= 1; ++s1) {
            const int s = (s1 + 1) + 3 * (s2 + 1), c = (i + s1 + m) % m;
            pc[h][s1 + 1] = ccast<T>(q[s] + (V[c + (long)m * ln] - l) * t[s]);
        }
    }
}

// sum_{h, s1} pc[h][s1 + 1] x_h(i + s1) from the two neighbour lines' values in LDS
// (ex[h][base + k] = x_h(k)); im1, ip1 = i -+ 1 wrapped.
template <typename T>
__device__ __forceinline__ cplx<T> coupling_apply(const cplx<T> (&pc)[2][3], const cplx<T>* exm, const cplx<T>* exp_,
                                                  cplx<T> xm, cplx<T> xp, int base, int im1, int ip1) {
    return pc[0][0] * exm[base + im1] + pc[0][1] * xm + pc[0][2] * exm[base + ip1] + pc[1][0] * exp_[base + im1] +
           pc[1][1] * xp + pc[1][2] * exp_[base + ip1];
}

// Level-0 couplings of the lines of one parity: R_line -= C x_{line-1} + B x_{line+1}
// (ASSIGN = 0, the forward elimination of the even lines) or R_line = C x_{line-1} +
// B x_{line+1} (ASSIGN = 1).  One workgroup of 128 threads per (line, pole): thread
// t = element t % m of column slot t / m (threads past the last whole slot idle), the
// six coefficients computed once and reused for every column, G columns per slot per
// pass, the neighbour lines exchanged through double-buffered LDS (one barrier a pass).
template <typename T, bool ASSIGN>
__global__ void __launch_bounds__(128) couple_lines_kernel(const cplx<T>* __restrict__ X, cplx<T>* __restrict__ R,
                                                           int m, int N, long n, int parity,
                                                           const cplx<double>* __restrict__ qs,
                                                           const cplx<double>* __restrict__ ts,
                                                           const double* __restrict__ V, double l,
                                                           const int* __restrict__ pole_active) {
    constexpr int G = 4;
    const int u = blockIdx.x, pole = blockIdx.y;
    if (pole_active && pole_active[pole] == 0) return;
    __shared__ cplx<T> ex[2][2][G][128];
    const int t = threadIdx.x, nslot = 128 / m, slot = t / m, i = t % m;
    const bool act = slot < nslot;
    const int line = parity + 2 * u;
    cplx<T> pc[2][3];
    coupling_load<T>(qs + pole * kStencil, ts + pole * kStencil, V, l, m, line, i, pc);
    const int base = t - i, im1 = i == 0 ? m - 1 : i - 1, ip1 = i == m - 1 ? 0 : i + 1;
    const long pb = (long)pole * N * n + i;
    const long lm = pb + (long)((line + m - 1) % m) * m, lp = pb + (long)((line + 1) % m) * m, lo = pb + (long)line * m;
    // the next pass's values are requested before this pass is computed (unconditional
    // loads from columns clamped to N - 1; results of columns >= N are not stored)
    cplx<T> xm[G], xp[G], ro[G];
    auto load = [&](int cb, cplx<T>(&am)[G], cplx<T>(&ap)[G], cplx<T>(&aro)[G]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = cb + slot + nslot * g;
            const long cc = (long)(c < N ? c : N - 1) * n;
            am[g] = X[lm + cc];
            ap[g] = X[lp + cc];
            if constexpr (!ASSIGN) aro[g] = R[lo + cc];
        }
    };
    load(0, xm, xp, ro);
    int bsel = 0;
    for (int cb = 0; cb < N; cb += nslot * G) {
        cplx<T> nm[G], np[G], nro[G];
        load(cb + nslot * G < N ? cb + nslot * G : cb, nm, np, nro);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ex[bsel][0][g][t] = xm[g];
            ex[bsel][1][g][t] = xp[g];
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = cb + slot + nslot * g;
            if (act && c < N) {
                const cplx<T> w = coupling_apply<T>(pc, ex[bsel][0][g], ex[bsel][1][g], xm[g], xp[g], base, im1, ip1);
                R[lo + (long)c * n] = ASSIGN ? w : ro[g] - w;
            }
        }
        bsel ^= 1;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            xm[g] = nm[g];
            xp[g] = np[g];
            ro[g] = nro[g];
        }
    }
}

// X_o = A_o^{-1} R_o (ACC = 0) or X_o -= A_o^{-1} R_o (ACC = 1) by the reduction above:
// one workgroup of 128 threads per (line, pole), thread t = element t % m of column
// slot t / m; G columns per slot at a time, one LDS exchange (double-buffered, one
// barrier) per reduction step.  COUPLE (with ACC): the right-hand side is not read from
// R but formed in place as w_o = C_o x_{o-1} + B_o x_{o+1} from the neighbour lines of
// X (the backward substitution of the first level, x_o = t_o - A_o^{-1} w_o).
template <typename T, bool ACC, bool COUPLE>
__global__ void __launch_bounds__(128) pcr_lines_kernel(const cplx<T>* __restrict__ R, cplx<T>* __restrict__ X,
                                                        const cplx<T>* __restrict__ cf, int m, int N, long n,
                                                        const int* __restrict__ pole_active,
                                                        const cplx<double>* __restrict__ qs,
                                                        const cplx<double>* __restrict__ ts,
                                                        const double* __restrict__ V, double l) {
    constexpr int G = 4, SMAX = 6;
    const int u = blockIdx.x, pole = blockIdx.y;
    if (pole_active && pole_active[pole] == 0) return;
    __shared__ cplx<T> buf[2][G][128];
    __shared__ cplx<T> ex[2][G][COUPLE ? 128 : 1];
    const int t = threadIdx.x, i = t % m, slot = t / m, nslot = 128 / m, S = pcr_steps(m);
    const int no = m / 2, o = 2 * u + 1;
    cplx<T> al[SMAX], ga[SMAX], uu, vv;
    pcr_load<T, SMAX>(cf + ((size_t)pole * no + u) * (2 * S + 2) * m + i, m, S, al, ga, uu, vv);
    cplx<T> pc[2][3];
    if constexpr (COUPLE) coupling_load<T>(qs + pole * kStencil, ts + pole * kStencil, V, l, m, o, i, pc);
    const int base = t - i, im1 = (i - 1) & (m - 1), ip1 = (i + 1) & (m - 1);
    const long pb = (long)pole * N * n + i;
    const long lb = pb + (long)o * m, lm = pb + (long)(o - 1) * m, lp = pb + (long)((o + 1) & (m - 1)) * m;
    // inputs of a pass: right-hand side (or the two neighbour lines) and the old solution;
    // the next pass's are requested before this one is reduced (columns clamped to N - 1)
    cplx<T> ia[G], ib[G], io[G];
    auto load = [&](int cb, cplx<T>(&a0)[G], cplx<T>(&a1)[G], cplx<T>(&a2)[G]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = cb + slot + nslot * g;
            const long cc = (long)(c < N ? c : N - 1) * n;
            if constexpr (COUPLE) {
                a0[g] = X[lm + cc];
                a1[g] = X[lp + cc];
            } else {
                a0[g] = R[lb + cc];
            }
            if constexpr (ACC) a2[g] = X[lb + cc];
        }
    };
    load(0, ia, ib, io);
    int bsel = 0;
    for (int cb = 0; cb < N; cb += nslot * G) {
        cplx<T> na[G], nb[G], no_[G];
        load(cb + nslot * G < N ? cb + nslot * G : cb, na, nb, no_);
        cplx<T> r[G];
        if constexpr (COUPLE) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                ex[0][g][t] = ia[g];
                ex[1][g][t] = ib[g];
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < G; ++g) r[g] = coupling_apply<T>(pc, ex[0][g], ex[1][g], ia[g], ib[g], base, im1, ip1);
            // the exchange buffers are next written after the reduction's barriers
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) r[g] = ia[g];
        }
        pcr_apply<T, G, SMAX>(r, al, ga, uu, vv, S, m, t, i, buf, bsel);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = cb + slot + nslot * g;
            if (c < N) X[lb + (long)c * n] = ACC ? io[g] - r[g] : r[g];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ia[g] = na[g];
            ib[g] = nb[g];
            io[g] = no_[g];
        }
    }
}

// The value v of lane src of the wave (every lane takes part).
template <typename T>
__device__ __forceinline__ cplx<T> lane_get(cplx<T> v, int src) {
    const int a = src << 2;
    if constexpr (sizeof(T) == 4) {
        return cplx<T>{__int_as_float(__builtin_amdgcn_ds_bpermute(a, __float_as_int(v.re))),
                       __int_as_float(__builtin_amdgcn_ds_bpermute(a, __float_as_int(v.im)))};
    } else {
        auto get = [&](double x) {
            const long long b = __double_as_longlong(x);
            const int lo = __builtin_amdgcn_ds_bpermute(a, (int)(b & 0xffffffffll));
            const int hi = __builtin_amdgcn_ds_bpermute(a, (int)(b >> 32));
            return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
        };
        return cplx<T>{(T)get(v.re), (T)get(v.im)};
    }
}

// Whole-wave moves without the LDS pipe: the value of lane l - 1 (ROT = 0x13C, the DPP
// wave rotate right by one) or l + 1 (ROT = 0x134, rotate left), both modulo 64, and of
// lane l ^ 32 (gfx950 permlane32_swap of the register with itself: the low half of the
// second result and the high half of the first hold the swapped halves).
template <int ROT>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ROT, 0xF, 0xF, false));
}
__device__ __forceinline__ float swap32_f(float x, bool low) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(low ? r[1] : r[0]);
}
template <typename T, typename F>
__device__ __forceinline__ cplx<T> per_dword(cplx<T> v, F f) {
    if constexpr (sizeof(T) == 4) {
        return cplx<T>{f(v.re), f(v.im)};
    } else {
        auto g = [&](double x) {
            const long long b = __double_as_longlong(x);
            const float lo = f(__int_as_float((int)(b & 0xffffffffll))), hi = f(__int_as_float((int)(b >> 32)));
            return __longlong_as_double(((long long)__float_as_int(hi) << 32) | (unsigned)__float_as_int(lo));
        };
        return cplx<T>{(T)g(v.re), (T)g(v.im)};
    }
}

// Two consecutive elements of a line (16 bytes for complex64, 32 for complex128).
template <typename T>
struct CPair {
    cplx<T> a, b;
};
template <typename T>
__device__ __forceinline__ CPair<T> load_pair(const cplx<T>* p) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        const v4 v = *(const v4*)p;
        return CPair<T>{cplx<T>{v.x, v.y}, cplx<T>{v.z, v.w}};
    } else {
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 x = *(const v2*)p, y = *(const v2*)(p + 1);
        return CPair<T>{cplx<T>{x.x, x.y}, cplx<T>{y.x, y.y}};
    }
}
template <typename T>
__device__ __forceinline__ void store_pair(cplx<T>* p, cplx<T> a, cplx<T> b) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        *(v4*)p = v4{a.re, a.im, b.re, b.im};
    } else {
        typedef T v2 __attribute__((ext_vector_type(2)));
        *(v2*)p = v2{a.re, a.im};
        *(v2*)(p + 1) = v2{b.re, b.im};
    }
}

// The same reduction as pcr_lines_kernel with the exchanges inside one wave: lane l holds
// the points 2q and 2q + 1 (q = l % (m/2)) of one column line and takes its neighbours'
// values with lane permutes, so no LDS traffic besides the permutes and no workgroup
// barrier.  One workgroup of 4 waves per (line, pole); a wave holds 128/m columns per
// register set, G register sets per pass, and the waves interleave over the columns.
// W64 (m = 128, a column per wave): the moves by one pair and by half the line use the
// DPP rotates and the half swap instead of permutes.
template <typename T, bool ACC, bool COUPLE, int G, bool W64>
__global__ void __launch_bounds__(256) pcr_wave_kernel(const cplx<T>* __restrict__ R, cplx<T>* __restrict__ X,
                                                       const cplx<T>* __restrict__ cf, int m, int N, long n,
                                                       const int* __restrict__ pole_active,
                                                       const cplx<double>* __restrict__ qs,
                                                       const cplx<double>* __restrict__ ts,
                                                       const double* __restrict__ V, double l) {
    constexpr int SMAX = 6;
    const int u = blockIdx.x, pole = blockIdx.y;
    if (pole_active && pole_active[pole] == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Lc = m >> 1, cpw = 64 / Lc;   // lanes per column, columns per register set
    const int cs = lane / Lc, q = lane % Lc, sb = cs * Lc;
    const int S = pcr_steps(m), no = m / 2, o = 2 * u + 1, i0 = 2 * q;
    auto at = [&](int off) { return sb + ((q + off) & (Lc - 1)); };   // lane of pair q + off
    cplx<T> al[SMAX][2], ga[SMAX][2], uu[2], vv[2];
    {
        const cplx<T>* c0 = cf + ((size_t)pole * no + u) * (2 * S + 2) * m + i0;
#pragma unroll
        for (int s = 0; s < SMAX; ++s)
            if (s < S) {
                const CPair<T> x = load_pair(c0 + (2 * s) * m), y = load_pair(c0 + (2 * s + 1) * m);
                al[s][0] = x.a;
                al[s][1] = x.b;
                ga[s][0] = y.a;
                ga[s][1] = y.b;
            }
        const CPair<T> x = load_pair(c0 + (2 * S) * m), y = load_pair(c0 + (2 * S + 1) * m);
        uu[0] = x.a;
        uu[1] = x.b;
        vv[0] = y.a;
        vv[1] = y.b;
    }
    cplx<T> pc[2][2][3];   // [point][neighbour line][offset + 1]
    if constexpr (COUPLE) {
        coupling_load<T>(qs + pole * kStencil, ts + pole * kStencil, V, l, m, o, i0, pc[0]);
        coupling_load<T>(qs + pole * kStencil, ts + pole * kStencil, V, l, m, o, i0 + 1, pc[1]);
    }
    const long pb = (long)pole * N * n + i0;
    const long lb = pb + (long)o * m, lm = pb + (long)(o - 1) * m, lp = pb + (long)((o + 1) & (m - 1)) * m;
    const int per_pass = 4 * G * cpw;
    auto col = [&](int cb, int g) { return cb + (wave + 4 * g) * cpw + cs; };
    // inputs of a pass: right-hand side (or the two neighbour lines) and the old solution;
    // the next pass's are requested before this one is reduced (columns clamped to N - 1)
    CPair<T> ia[G], ib[G], io[G];
    auto load = [&](int cb, CPair<T>(&a0)[G], CPair<T>(&a1)[G], CPair<T>(&a2)[G]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = col(cb, g);
            const long cc = (long)(c < N ? c : N - 1) * n;
            if constexpr (COUPLE) {
                a0[g] = load_pair(X + lm + cc);
                a1[g] = load_pair(X + lp + cc);
            } else {
                a0[g] = load_pair(R + lb + cc);
            }
            if constexpr (ACC) a2[g] = load_pair(X + lb + cc);
        }
    };
    load(0, ia, ib, io);
    const int left = at(-1), right = at(1), half = at(Lc / 2);
    const bool low = lane < 32;
    auto from_left = [&](cplx<T> v) {
        if constexpr (W64) return per_dword<T>(v, [](float x) { return dpp_f<0x13C>(x); });
        else return lane_get(v, left);
    };
    auto from_right = [&](cplx<T> v) {
        if constexpr (W64) return per_dword<T>(v, [](float x) { return dpp_f<0x134>(x); });
        else return lane_get(v, right);
    };
    auto from_half = [&](cplx<T> v) {
        if constexpr (W64) return per_dword<T>(v, [&](float x) { return swap32_f(x, low); });
        else return lane_get(v, half);
    };
    for (int cb = 0; cb < N; cb += per_pass) {
        CPair<T> na[G], nb[G], no_[G];
        load(cb + per_pass < N ? cb + per_pass : cb, na, nb, no_);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            cplx<T> x0, x1;
            if constexpr (COUPLE) {
                // neighbour lines at i0 - 1 and i0 + 2 come from the adjacent pairs
                const cplx<T> mL = from_left(ia[g].b), mR = from_right(ia[g].a);
                const cplx<T> pL = from_left(ib[g].b), pR = from_right(ib[g].a);
                x0 = pc[0][0][0] * mL + pc[0][0][1] * ia[g].a + pc[0][0][2] * ia[g].b + pc[0][1][0] * pL +
                     pc[0][1][1] * ib[g].a + pc[0][1][2] * ib[g].b;
                x1 = pc[1][0][0] * ia[g].a + pc[1][0][1] * ia[g].b + pc[1][0][2] * mR + pc[1][1][0] * ib[g].a +
                     pc[1][1][1] * ib[g].b + pc[1][1][2] * pR;
            } else {
                x0 = ia[g].a;
                x1 = ia[g].b;
            }
            {   // distance 1: one neighbour of each point is in the pair
                const cplx<T> L = from_left(x1), Rr = from_right(x0);
                const cplx<T> n0 = x0 + al[0][0] * L + ga[0][0] * x1;
                const cplx<T> n1 = x1 + al[0][1] * x0 + ga[0][1] * Rr;
                x0 = n0;
                x1 = n1;
            }
#pragma unroll
            for (int s = 1; s < SMAX; ++s) {
                if (s >= S) break;
                const int hd = 1 << (s - 1);   // distance 2^s = hd pairs
                const int lmn = at(-hd), lpn = at(hd);
                cplx<T> m0, m1, p0, p1;
                if (W64 && s == 1) {
                    m0 = from_left(x0);
                    m1 = from_left(x1);
                    p0 = from_right(x0);
                    p1 = from_right(x1);
                } else {
                    m0 = lane_get(x0, lmn);
                    m1 = lane_get(x1, lmn);
                    p0 = lane_get(x0, lpn);
                    p1 = lane_get(x1, lpn);
                }
                x0 = x0 + al[s][0] * m0 + ga[s][0] * p0;
                x1 = x1 + al[s][1] * m1 + ga[s][1] * p1;
            }
            const cplx<T> f0 = from_half(x0), f1 = from_half(x1);
            x0 = uu[0] * x0 + vv[0] * f0;
            x1 = uu[1] * x1 + vv[1] * f1;
            const int c = col(cb, g);
            if (c < N) {
                if constexpr (ACC) store_pair(X + lb + (long)c * n, io[g].a - x0, io[g].b - x1);
                else store_pair(X + lb + (long)c * n, x0, x1);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ia[g] = na[g];
            ib[g] = nb[g];
            io[g] = no_[g];
        }
    }
}

// Dense A_o^{-1} (m x m, column major) of every (pole, level-0 odd line) from the same
// reduction applied to the identity: the first factorization level needs it for its
// Schur complements.
__global__ void __launch_bounds__(128) pcr_inverse_kernel(const cplx<double>* __restrict__ cf, int m,
                                                          cplx<double>* __restrict__ ainv, long stride) {
    constexpr int G = 4, SMAX = 6;
    const int u = blockIdx.x, pole = blockIdx.y, no = m / 2;
    __shared__ cplx<double> buf[2][G][128];
    const int t = threadIdx.x, i = t % m, slot = t / m, nslot = 128 / m, S = pcr_steps(m);
    cplx<double> al[SMAX], ga[SMAX], uu, vv;
    pcr_load<double, SMAX>(cf + ((size_t)pole * no + u) * (2 * S + 2) * m + i, m, S, al, ga, uu, vv);
    cplx<double>* out = ainv + ((long)pole * no + u) * stride;
    int bsel = 0;
    for (int cb = 0; cb < m; cb += nslot * G) {
        cplx<double> r[G];
#pragma unroll
        for (int g = 0; g < G; ++g) r[g] = mk<double>(i == cb + slot + nslot * g ? 1.0 : 0.0, 0.0);
        pcr_apply<double, G, SMAX>(r, al, ga, uu, vv, S, m, t, i, buf, bsel);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int c = cb + slot + nslot * g;
            if (c < m) out[i + (long)c * m] = r[g];
        }
    }
}

// LDS of tri_lines_kernel: factors plus the m x (CPW + 1) block
template <typename T, int CPW>
constexpr size_t tri_lds_bytes(int m) { return sizeof(cplx<T>) * ((size_t)tri_stride(m) + (size_t)m * (CPW + 1)); }
template <typename T, int CPW>
constexpr size_t tri_lds_max() { return tri_lds_bytes<T, CPW>(128); }

// count identity blocks of order D, consecutive: out[b][j][i] = (i == j)
__global__ void identity_kernel(cplx<double>* __restrict__ out, int D, long count) {
    const long total = count * (long)D * D;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long w = e % ((long)D * D);
        out[e] = mk<double>((w % D) == (w / D) ? 1.0 : 0.0, 0.0);
    }
}

__global__ void to_fp32_kernel(const cplx<double>* __restrict__ a, cplx<float>* __restrict__ b, long count) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        b[i] = ccast<float>(a[i]);
}

__global__ void to_fp64_kernel(const cplx<float>* __restrict__ a, cplx<double>* __restrict__ b, long count) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
        b[i] = ccast<double>(a[i]);
}

// Smallest eigenpair of a Hermitian matrix (row major, n x n) by cyclic Jacobi rotations.
void hermitian_min_eig(int n, std::vector<cd> A, std::vector<cd>& vec, double& lmin) {
    std::vector<cd> Vm(n * n, 0.0);
    for (int i = 0; i < n; ++i) Vm[i * n + i] = 1.0;
    auto at = [&](int i, int j) -> cd& { return A[i * n + j]; };
    double fro = 0;
    for (auto& x : A) fro += std::norm(x);
    fro = std::sqrt(fro);
    // Jacobi converges quadratically near the end; once the off-diagonal norm is small and a
    // sweep no longer halves it, it is at the rounding floor (about eps ||A||) and further
    // sweeps only rotate noise.
    double off_prev = 0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) off += std::norm(at(i, j));
        off = std::sqrt(off);
        if (off <= 1e-17 * fro || (sweep > 0 && off <= 1e-13 * fro && off > 0.5 * off_prev)) break;
        off_prev = off;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd apq = at(p, q);
                const double mag = std::abs(apq);
                if (mag == 0.0) continue;
                const double app = at(p, p).real(), aqq = at(q, q).real();
                const cd d = std::conj(apq) / mag;   // makes the (p,q) entry real and positive
                const double theta = (aqq - app) / (2.0 * mag);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // G on (p,q): [[c, s], [-d s, d c]];  A <- G^H A G, V <- V G
                const cd g11 = c, g12 = s, g21 = -d * s, g22 = d * c;
                for (int k = 0; k < n; ++k) {   // columns
                    const cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * g11 + akq * g21;
                    at(k, q) = akp * g12 + akq * g22;
                }
                for (int k = 0; k < n; ++k) {   // rows
                    const cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = std::conj(g11) * apk + std::conj(g21) * aqk;
                    at(q, k) = std::conj(g12) * apk + std::conj(g22) * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const cd vkp = Vm[k * n + p], vkq = Vm[k * n + q];
                    Vm[k * n + p] = vkp * g11 + vkq * g21;
                    Vm[k * n + q] = vkp * g12 + vkq * g22;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < n; ++i)
        if (at(i, i).real() < at(best, best).real()) best = i;
    lmin = at(best, best).real();
    vec.resize(n);
    for (int k = 0; k < n; ++k) vec[k] = Vm[k * n + best];
}

int disp_index(int d1, int d2) { return (d1 + 2) + 5 * (d2 + 2); }

template <typename T>
struct Fac;
template <>
struct Fac<double> {
    static const cplx<double>* base(const Spp& s) { return s.fac; }
};
template <>
struct Fac<float> {
    static const cplx<float>* base(const Spp& s) { return s.fac32; }
};

}  // namespace

size_t spp_bytes_per_pole(int m, bool want32) {
    // levels: sum over levels of (3 odd + 2 even) blocks, final (mf m)^2, setup blocks 3 m^2 per line
    size_t blocks = 0;
    int ml = m;
    while (ml % 2 == 0 && ml > 1) {
        blocks += (size_t)(3 * (ml / 2) + 2 * (ml / 2));
        ml /= 2;
    }
    const size_t bb = (size_t)m * m;
    size_t elems = blocks * bb + (size_t)(ml * m) * (ml * m) + 3 * (size_t)m * bb;
    return elems * 16 + (want32 ? (elems - 3 * (size_t)m * bb) * 8 : 0);
}

void spp_setup(Spp& sp, const SpectralPlan& plan, const double* V_dev, double l, const std::vector<cd>& z, int N,
               cplx<double>* R, cplx<double>* X, cplx<float>* R32, cplx<float>* X32, bool want32, int split_planes,
               hipStream_t s) {
    POMM_CHECK(plan.dim == 2, 8, "the sparsifying preconditioner is implemented for 2D grids");
    POMM_CHECK(plan.m <= 128 && plan.m % 2 == 0, 8, "the sparsifying preconditioner needs an even m <= 128");
    const int m = plan.m, n = plan.n, p = (int)z.size();
    ProfScope prof_setup(PK_SPP_SETUP, 0.0, 0.0, s);
    sp.m = m;
    sp.b = m;
    sp.p = p;
    sp.N = N;
    sp.n = n;
    sp.l = l;
    sp.R = R;
    sp.X = X;
    sp.R32 = R32;
    sp.X32 = X32;
    const cplx<double>* tw = reinterpret_cast<const cplx<double>*>(plan.tw64);

    // ---- stencils
    cplx<double>* zs_d = nullptr;
    cplx<double>* gD = nullptr;
    cplx<double>* RD = nullptr;
    POMM_HIP(dev_alloc(&zs_d, sizeof(cplx<double>) * p));
    POMM_HIP(dev_alloc(&gD, sizeof(cplx<double>) * p * kDisp));
    POMM_HIP(dev_alloc(&RD, sizeof(cplx<double>) * p * kDisp));
    std::vector<cplx<double>> zh(p);
    for (int j = 0; j < p; ++j) zh[j] = mk<double>(z[j].real(), z[j].imag());
    POMM_HIP(hipMemcpyAsync(zs_d, zh.data(), sizeof(cplx<double>) * p, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(green_moments_kernel, dim3(p, kDisp), dim3(256), 0, s, zs_d, l, m, tw, gD, RD);
    check_launch("green_moments");
    std::vector<cplx<double>> gh(p * kDisp), Rh(p * kDisp);
    POMM_HIP(hipMemcpyAsync(gh.data(), gD, sizeof(cplx<double>) * p * kDisp, hipMemcpyDeviceToHost, s));
    POMM_HIP(hipMemcpyAsync(Rh.data(), RD, sizeof(cplx<double>) * p * kDisp, hipMemcpyDeviceToHost, s));
    POMM_HIP(hipStreamSynchronize(s));
    sp.q.assign(p * kStencil, 0.0);
    sp.t.assign(p * kStencil, 0.0);
    sp.farfield.assign(p, 0.0);
    for (int j = 0; j < p; ++j) {
        auto g = [&](int d1, int d2) { const auto v = gh[j * kDisp + disp_index(d1, d2)]; return cd(v.re, v.im); };
        auto Rf = [&](int d1, int d2) { const auto v = Rh[j * kDisp + disp_index(d1, d2)]; return cd(v.re, v.im); };
        // (Z Z^*)(s, s') = R(s - s') - sum_{d in a} g(d - s) conj(g(d - s')); Mq = conj(Z Z^*)
        std::vector<cd> M(kStencil * kStencil);
        for (int a = 0; a < kStencil; ++a)
            for (int b = 0; b < kStencil; ++b) {
                const int a1 = a % 3 - 1, a2 = a / 3 - 1, b1 = b % 3 - 1, b2 = b / 3 - 1;
                cd v = Rf(a1 - b1, a2 - b2);
                for (int d = 0; d < kStencil; ++d) {
                    const int e1 = d % 3 - 1, e2 = d / 3 - 1;
                    v -= g(e1 - a1, e2 - a2) * std::conj(g(e1 - b1, e2 - b2));
                }
                M[a * kStencil + b] = std::conj(v);
            }
        for (int a = 0; a < kStencil; ++a)   // symmetrize against rounding
            for (int b = a; b < kStencil; ++b) {
                const cd h = 0.5 * (M[a * kStencil + b] + std::conj(M[b * kStencil + a]));
                M[a * kStencil + b] = h;
                M[b * kStencil + a] = std::conj(h);
            }
        std::vector<cd> qv;
        double lmin = 0;
        hermitian_min_eig(kStencil, M, qv, lmin);
        const cd qc = qv[4];
        const cd ph = std::abs(qc) / qc;
        for (auto& x : qv) x *= ph;
        sp.farfield[j] = std::sqrt(std::max(lmin, 0.0));
        for (int a = 0; a < kStencil; ++a) {
            sp.q[j * kStencil + a] = qv[a];
            // t_s = sum_{s'} q_{s'} g(s - s')
            const int a1 = a % 3 - 1, a2 = a / 3 - 1;
            cd tv = 0;
            for (int b = 0; b < kStencil; ++b) tv += qv[b] * g(a1 - (b % 3 - 1), a2 - (b / 3 - 1));
            sp.t[j * kStencil + a] = tv;
        }
    }
    cplx<double>* qs_d = nullptr;
    cplx<double>* ts_d = nullptr;
    POMM_HIP(dev_alloc(&qs_d, sizeof(cplx<double>) * p * kStencil));
    POMM_HIP(dev_alloc(&ts_d, sizeof(cplx<double>) * p * kStencil));
    {
        std::vector<cplx<double>> qh(p * kStencil), th(p * kStencil);
        for (int i = 0; i < p * kStencil; ++i) {
            qh[i] = mk<double>(sp.q[i].real(), sp.q[i].imag());
            th[i] = mk<double>(sp.t[i].real(), sp.t[i].imag());
        }
        POMM_HIP(hipMemcpyAsync(qs_d, qh.data(), sizeof(cplx<double>) * p * kStencil, hipMemcpyHostToDevice, s));
        POMM_HIP(hipMemcpyAsync(ts_d, th.data(), sizeof(cplx<double>) * p * kStencil, hipMemcpyHostToDevice, s));
        POMM_HIP(hipStreamSynchronize(s));
    }
    {   // level-0 line blocks: reduction multipliers (power-of-two m) or bordered tridiagonal factors
        sp.pcr = (m & (m - 1)) == 0;
        const size_t cnt = (size_t)p * (m / 2) * (sp.pcr ? (size_t)(2 * pcr_steps(m) + 2) * m : (size_t)tri_stride(m));
        POMM_HIP(dev_alloc(&sp.tri, sizeof(cplx<double>) * cnt));
        if (sp.pcr)
            hipLaunchKernelGGL(pcr_factor_kernel, dim3(m / 2, p), dim3(m), 0, s, qs_d, ts_d, V_dev, l, m, sp.tri);
        else
            hipLaunchKernelGGL(tri_factor_kernel, dim3(cdiv_u((size_t)p * (m / 2), 64)), dim3(64), 0, s, qs_d, ts_d,
                               V_dev, l, m, p, sp.tri);
        check_launch("line_factor");
        if (want32) {
            POMM_HIP(dev_alloc(&sp.tri32, sizeof(cplx<float>) * cnt));
            hipLaunchKernelGGL(to_fp32_kernel, dim3(256), dim3(256), 0, s, sp.tri, sp.tri32, (long)cnt);
            check_launch("to_fp32");
        }
    }
    POMM_HIP(dev_alloc(&sp.mult, sizeof(cplx<double>) * (size_t)p * n));
    if (want32) POMM_HIP(dev_alloc(&sp.mult32, sizeof(cplx<float>) * (size_t)p * n));
    hipLaunchKernelGGL(rhs_mult_kernel, dim3(cdiv_u((size_t)p * n, 256)), dim3(256), 0, s, zs_d, qs_d, l, m, p, tw,
                       sp.mult, sp.mult32);
    check_launch("rhs_mult");
    {   // the spectral kernels read the multiplier in their own order
        cplx<double>* t64 = nullptr;
        POMM_HIP(dev_alloc(&t64, sizeof(cplx<double>) * (size_t)p * n));
        spectral_table_reorder<double>(plan, sp.mult, t64, p, s);
        cplx<float>* t32 = nullptr;
        if (want32) {
            POMM_HIP(dev_alloc(&t32, sizeof(cplx<float>) * (size_t)p * n));
            spectral_table_reorder<float>(plan, sp.mult32, t32, p, s);
        }
        POMM_HIP(hipStreamSynchronize(s));
        (void)dev_free(sp.mult);
        sp.mult = t64;
        if (want32) {
            (void)dev_free(sp.mult32);
            sp.mult32 = t32;
        }
    }

    // ---- level structure
    const size_t bb = (size_t)m * m;
    std::vector<int> active(m);
    for (int i = 0; i < m; ++i) active[i] = i;
    int step = 1;
    sp.levels.clear();
    while (active.size() % 2 == 0 && active.size() > 1) {
        SppLevel L;
        L.step = step;
        for (size_t i = 0; i < active.size(); ++i) (i % 2 ? L.odd : L.even).push_back(active[i]);
        sp.levels.push_back(L);
        active = sp.levels.back().even;
        step *= 2;
    }
    sp.final_lines = active;
    size_t off = 0;
    sp.level_base.clear();
    for (size_t li = 0; li < sp.levels.size(); ++li) {
        SppLevel& L = sp.levels[li];
        // the first level's solve works on the stencil directly: only its inverses are kept,
        // for the Schur complements of the next level
        const size_t no = L.odd.size(), ne = li == 0 ? 0 : L.even.size(), nf = li == 0 ? 0 : no;
        sp.level_base.push_back(off);
        L.off_ainv = off;
        L.off_f = L.off_ainv + p * no * bb;
        L.off_g = L.off_f + p * nf * bb;
        L.off_alpha = L.off_g + p * nf * bb;
        L.off_gamma = L.off_alpha + p * ne * bb;
        off = L.off_gamma + p * ne * bb;
    }
    const int mf = (int)sp.final_lines.size();
    const size_t fsz = (size_t)(mf * m) * (mf * m);
    sp.final_base = off;
    off += p * fsz;
    sp.fac_elems = off;
    POMM_HIP(dev_alloc(&sp.fac, sizeof(cplx<double>) * sp.fac_elems));

    // line blocks A, B, C of the even lines (the lines of the levels after the first), dense
    cplx<double>* blocks = nullptr;
    POMM_HIP(dev_alloc(&blocks, sizeof(cplx<double>) * (size_t)p * (m / 2) * 3 * bb));
    auto blk = [&](int pole, int line, int w) {
        return blocks + ((size_t)(pole * (m / 2) + line / 2) * 3 + w) * bb;
    };
    const int piv_max = std::max(p * m, p) * std::max(m, mf * m);
    int* piv = nullptr;
    POMM_HIP(dev_alloc(&piv, sizeof(int) * piv_max));
    // Without a complex128 solve the factors only ever serve complex64 (or fp16) products:
    // the block inversions of orders up to 128 then run in complex64 (Gauss-Jordan with
    // partial pivoting, about 1.4 times faster; the inverse carries complex64 rounding,
    // 3e-7 relative on diagonally dominant blocks), and the Schur complements built from
    // them stay complex128.
    const bool inv32 = R == nullptr;
    cplx<float>* inv_scratch = nullptr;
    long inv_scratch_elems = 0;
    auto invert = [&](cplx<double>* mats, long stride, int order, int count) {
        if (!inv32 || order > 128 || stride != (long)order * order) {
            invert_batched<double>(mats, stride, order, count, piv, s);
            return;
        }
        const long cnt = (long)count * stride;
        if (cnt > inv_scratch_elems) {
            if (inv_scratch) {
                POMM_HIP(hipStreamSynchronize(s));
                (void)dev_free(inv_scratch);
                inv_scratch = nullptr;
            }
            POMM_HIP(dev_alloc(&inv_scratch, sizeof(cplx<float>) * cnt));
            inv_scratch_elems = cnt;
        }
        hipLaunchKernelGGL(to_fp32_kernel, dim3(4096), dim3(256), 0, s, mats, inv_scratch, cnt);
        check_launch("to_fp32");
        invert_batched<float>(inv_scratch, stride, order, count, piv, s);
        hipLaunchKernelGGL(to_fp64_kernel, dim3(4096), dim3(256), 0, s, inv_scratch, mats, cnt);
        check_launch("to_fp64");
    };

    // device scratch for pointer and task lists (reused per level)
    const size_t max_tasks = (size_t)p * m * 3 + 16;
    GemmTask<double>* tdev = nullptr;
    const cplx<double>** srcp = nullptr;
    cplx<double>** dstp = nullptr;
    POMM_HIP(dev_alloc(&tdev, sizeof(GemmTask<double>) * max_tasks));
    POMM_HIP(dev_alloc(&srcp, sizeof(void*) * max_tasks));
    POMM_HIP(dev_alloc(&dstp, sizeof(void*) * max_tasks));
    // the factorization's block products: complex128 throughout, or (mixed form only, as the
    // inversions) complex64 products of the complex128 blocks on the fp32 matrix cores
    auto setup_gemm = [&](const GemmTask<double>* tasks, int count, int Nc) {
        if (inv32) gemm_mfma_f64_c32(tasks, count, m, Nc, m, nullptr, s, -1);
        else gemm_batched<double>(tasks, count, m, Nc, m, nullptr, s);
    };
    auto run_tasks = [&](std::vector<GemmTask<double>>& tk) {
        if (tk.empty()) return;
        POMM_HIP(hipMemcpyAsync(tdev, tk.data(), sizeof(GemmTask<double>) * tk.size(), hipMemcpyHostToDevice, s));
        setup_gemm(tdev, (int)tk.size(), m);
        POMM_HIP(hipStreamSynchronize(s));   // host task vector is reused
    };
    auto term = [&](const cplx<double>* A, const cplx<double>* B, double a) {
        GemmTerm<double> t;
        t.A = A;
        t.B = B;
        t.lda = m;
        t.ldb = m;
        t.alpha_re = a;
        t.alpha_im = 0;
        return t;
    };
    for (size_t li = 0; li < sp.levels.size(); ++li) {
        const SppLevel& L = sp.levels[li];
        const int no = (int)L.odd.size(), ne = (int)L.even.size();
        auto ainv = [&](int pole, int u) { return sp.fac + L.off_ainv + ((size_t)pole * no + u) * bb; };
        auto fo = [&](int pole, int u) { return sp.fac + L.off_f + ((size_t)pole * no + u) * bb; };
        auto go = [&](int pole, int u) { return sp.fac + L.off_g + ((size_t)pole * no + u) * bb; };
        auto al = [&](int pole, int u) { return sp.fac + L.off_alpha + ((size_t)pole * ne + u) * bb; };
        auto ga = [&](int pole, int u) { return sp.fac + L.off_gamma + ((size_t)pole * ne + u) * bb; };
        auto odd_index = [&](int line) { return (int)(std::find(L.odd.begin(), L.odd.end(), line) - L.odd.begin()); };
        // 1. Ainv <- A_o, invert (level 0 with power-of-two m: from the cyclic reduction)
        if (li == 0) {
            if (sp.pcr) {
                hipLaunchKernelGGL(pcr_inverse_kernel, dim3(no, p), dim3(128), 0, s, sp.tri, m, sp.fac + L.off_ainv,
                                   (long)bb);
                check_launch("pcr_inverse");
            } else {
                hipLaunchKernelGGL(assemble_odd_kernel, dim3(no, p), dim3(256), 0, s, V_dev, l, qs_d, ts_d, m,
                                   sp.fac + L.off_ainv);
                check_launch("assemble_odd");
                invert(sp.fac + L.off_ainv, (long)bb, m, p * no);
            }
            // 2.-4. for the first level: the Schur complements of the even lines directly
            hipLaunchKernelGGL(level0_schur_kernel, dim3(m / 2, p, 16), dim3(256), 0, s, sp.fac + L.off_ainv, V_dev,
                               l, qs_d, ts_d, m, blocks);
            check_launch("level0_schur");
            POMM_HIP(hipStreamSynchronize(s));
            continue;
        } else {
            std::vector<const cplx<double>*> sv;
            std::vector<cplx<double>*> dv;
            for (int pole = 0; pole < p; ++pole)
                for (int u = 0; u < no; ++u) {
                    sv.push_back(blk(pole, L.odd[u], 0));
                    dv.push_back(ainv(pole, u));
                }
            POMM_HIP(hipMemcpyAsync(srcp, sv.data(), sizeof(void*) * sv.size(), hipMemcpyHostToDevice, s));
            POMM_HIP(hipMemcpyAsync(dstp, dv.data(), sizeof(void*) * dv.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(copy_blocks_kernel, dim3(16, (unsigned)sv.size()), dim3(256), 0, s, srcp, dstp,
                               (long)bb);
            check_launch("copy_blocks");
            invert(sp.fac + L.off_ainv, (long)bb, m, p * no);
            POMM_HIP(hipStreamSynchronize(s));
        }
        // 2. F = Ainv C_o, G = Ainv B_o (level 0 keeps its sparse B, C instead)
        std::vector<GemmTask<double>> tk;
        for (int pole = 0; pole < p && li > 0; ++pole)
            for (int u = 0; u < no; ++u) {
                GemmTask<double> a{};
                a.ldc = m;
                a.nterms = 1;
                a.beta = 0;
                a.gate = -1;
                a.C = fo(pole, u);
                a.t[0] = term(ainv(pole, u), blk(pole, L.odd[u], 2), 1.0);
                tk.push_back(a);
                a.C = go(pole, u);
                a.t[0] = term(ainv(pole, u), blk(pole, L.odd[u], 1), 1.0);
                tk.push_back(a);
            }
        run_tasks(tk);
        tk.clear();
        // 3. alpha_e = C_e Ainv_{o-}, gamma_e = B_e Ainv_{o+}
        for (int pole = 0; pole < p; ++pole)
            for (int u = 0; u < ne; ++u) {
                const int e = L.even[u];
                const int om = (e - L.step + m) % m, op = (e + L.step) % m;
                GemmTask<double> a{};
                a.ldc = m;
                a.nterms = 1;
                a.beta = 0;
                a.gate = -1;
                a.C = al(pole, u);
                a.t[0] = term(blk(pole, e, 2), ainv(pole, odd_index(om)), 1.0);
                tk.push_back(a);
                a.C = ga(pole, u);
                a.t[0] = term(blk(pole, e, 1), ainv(pole, odd_index(op)), 1.0);
                tk.push_back(a);
            }
        run_tasks(tk);
        tk.clear();
        // 4. A_e -= alpha B_{o-} + gamma C_{o+};  C_e = -alpha C_{o-};  B_e = -gamma B_{o+}
        for (int pole = 0; pole < p; ++pole)
            for (int u = 0; u < ne; ++u) {
                const int e = L.even[u];
                const int om = (e - L.step + m) % m, op = (e + L.step) % m;
                GemmTask<double> a{};
                a.ldc = m;
                a.gate = -1;
                a.C = blk(pole, e, 0);
                a.beta = 1.0;
                a.nterms = 2;
                a.t[0] = term(al(pole, u), blk(pole, om, 1), -1.0);
                a.t[1] = term(ga(pole, u), blk(pole, op, 2), -1.0);
                tk.push_back(a);
                a.beta = 0.0;
                a.nterms = 1;
                a.C = blk(pole, e, 2);
                a.t[0] = term(al(pole, u), blk(pole, om, 2), -1.0);
                tk.push_back(a);
                a.C = blk(pole, e, 1);
                a.t[0] = term(ga(pole, u), blk(pole, op, 1), -1.0);
                tk.push_back(a);
            }
        run_tasks(tk);
    }
    // final dense system
    {
        int* lines_d = nullptr;
        POMM_HIP(dev_alloc(&lines_d, sizeof(int) * mf));
        POMM_HIP(hipMemcpyAsync(lines_d, sp.final_lines.data(), sizeof(int) * mf, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(assemble_final_kernel, dim3(64, p), dim3(256), 0, s, blocks, lines_d, mf, m,
                           sp.fac + sp.final_base, (long)fsz);
        check_launch("assemble_final");
        invert(sp.fac + sp.final_base, (long)fsz, mf * m, p);
        POMM_HIP(hipStreamSynchronize(s));
        (void)dev_free(lines_d);
    }
    // ---- the last lines by one dense inverse.  The solve stops the reduction once at most
    // kCutLines lines are left; the inverse S^{-1} of their reduced system is the remaining
    // levels and the final inverse applied to the identity (order D = mc m per pole).  This
    // replaces the deepest levels of every solve, whose launches have too few tiles to fill
    // the chip, by one launch of mc tasks of mc terms per pole.
    constexpr int kCutLines = 8;
    sp.cut_level = (int)sp.levels.size();
    sp.cut_lines.clear();
    for (size_t li = 1; li < sp.levels.size(); ++li)
        if (sp.levels[li].odd.size() + sp.levels[li].even.size() <= (size_t)kCutLines) {
            sp.cut_level = (int)li;
            sp.cut_lines = sp.levels[li - 1].even;   // the lines entering level li
            break;
        }
    if (sp.cut_level < (int)sp.levels.size()) {
        const int mc = (int)sp.cut_lines.size(), D = mc * m;
        const size_t csz = (size_t)D * D;
        std::vector<int> cidx(m, -1);
        for (int a = 0; a < mc; ++a) cidx[sp.cut_lines[a]] = a;
        cplx<double>* Rc = nullptr;
        POMM_HIP(dev_alloc(&sp.fcut, sizeof(cplx<double>) * csz * p));
        POMM_HIP(dev_alloc(&Rc, sizeof(cplx<double>) * csz * p));
        hipLaunchKernelGGL(identity_kernel, dim3(4096), dim3(256), 0, s, Rc, D, (long)p);
        check_launch("identity");
        // every line the remaining levels touch is one of the cut lines
        for (size_t li = sp.cut_level; li < sp.levels.size(); ++li) {
            const SppLevel& L = sp.levels[li];
            for (const std::vector<int>* set : {&L.even, &L.odd})
                for (int l : *set)
                    POMM_CHECK(cidx[l] >= 0 && cidx[(l - L.step + m) % m] >= 0 && cidx[(l + L.step) % m] >= 0, 5,
                               "sparse solve: inconsistent reduction levels");
        }
        for (int l : sp.final_lines) POMM_CHECK(cidx[l] >= 0, 5, "sparse solve: inconsistent reduction levels");
        auto rc = [&](int pole, int line) { return Rc + (size_t)pole * csz + (size_t)cidx[line] * m; };
        auto xc = [&](int pole, int line) { return sp.fcut + (size_t)pole * csz + (size_t)cidx[line] * m; };
        auto cterm = [&](const cplx<double>* A, int lda, const cplx<double>* B, double a) {
            GemmTerm<double> t;
            t.A = A;
            t.B = B;
            t.lda = lda;
            t.ldb = D;
            t.alpha_re = a;
            t.alpha_im = 0;
            return t;
        };
        std::vector<std::vector<GemmTask<double>>> phases;
        for (size_t li = sp.cut_level; li < sp.levels.size(); ++li) {   // forward
            const SppLevel& L = sp.levels[li];
            const int ne = (int)L.even.size();
            std::vector<GemmTask<double>> tk;
            for (int pole = 0; pole < p; ++pole)
                for (int u = 0; u < ne; ++u) {
                    const int e = L.even[u];
                    const int om = (e - L.step + m) % m, op = (e + L.step) % m;
                    GemmTask<double> a{};
                    a.C = rc(pole, e);
                    a.ldc = D;
                    a.beta = 1.0;
                    a.gate = -1;
                    a.nterms = 2;
                    a.t[0] = cterm(sp.fac + L.off_alpha + ((size_t)pole * ne + u) * bb, m, rc(pole, om), -1.0);
                    a.t[1] = cterm(sp.fac + L.off_gamma + ((size_t)pole * ne + u) * bb, m, rc(pole, op), -1.0);
                    tk.push_back(a);
                }
            phases.push_back(tk);
        }
        {   // final
            std::vector<GemmTask<double>> tk;
            for (int pole = 0; pole < p; ++pole)
                for (int a_ = 0; a_ < mf; ++a_) {
                    GemmTask<double> a{};
                    a.C = xc(pole, sp.final_lines[a_]);
                    a.ldc = D;
                    a.beta = 0.0;
                    a.gate = -1;
                    a.nterms = mf;
                    const cplx<double>* Fp = sp.fac + sp.final_base + (size_t)pole * fsz;
                    for (int b_ = 0; b_ < mf; ++b_)
                        a.t[b_] = cterm(Fp + (size_t)a_ * m + (size_t)b_ * m * (mf * m), mf * m,
                                        rc(pole, sp.final_lines[b_]), 1.0);
                    tk.push_back(a);
                }
            phases.push_back(tk);
        }
        for (int li = (int)sp.levels.size() - 1; li >= sp.cut_level; --li) {   // backward
            const SppLevel& L = sp.levels[li];
            const int no = (int)L.odd.size();
            std::vector<GemmTask<double>> tk;
            for (int pole = 0; pole < p; ++pole)
                for (int u = 0; u < no; ++u) {
                    const int o = L.odd[u];
                    const int om = (o - L.step + m) % m, op = (o + L.step) % m;
                    const size_t idx = (size_t)pole * no + u;
                    GemmTask<double> a{};
                    a.C = xc(pole, o);
                    a.ldc = D;
                    a.beta = 0.0;
                    a.gate = -1;
                    a.nterms = 3;
                    a.t[0] = cterm(sp.fac + L.off_ainv + idx * bb, m, rc(pole, o), 1.0);
                    a.t[1] = cterm(sp.fac + L.off_f + idx * bb, m, xc(pole, om), -1.0);
                    a.t[2] = cterm(sp.fac + L.off_g + idx * bb, m, xc(pole, op), -1.0);
                    tk.push_back(a);
                }
            phases.push_back(tk);
        }
        size_t ntot = 0;
        for (auto& tk : phases) ntot += tk.size();
        GemmTask<double>* ctasks = nullptr;
        POMM_HIP(dev_alloc(&ctasks, sizeof(GemmTask<double>) * ntot));
        size_t at = 0;
        for (auto& tk : phases) {   // every phase's tasks in their own slice: no host sync between phases
            POMM_HIP(hipMemcpyAsync(ctasks + at, tk.data(), sizeof(GemmTask<double>) * tk.size(),
                                    hipMemcpyHostToDevice, s));
            setup_gemm(ctasks + at, (int)tk.size(), D);
            at += tk.size();
        }
        POMM_HIP(hipStreamSynchronize(s));   // host task vectors go out of scope
        (void)dev_free(ctasks);
        (void)dev_free(Rc);
    }
    const bool split16 = split_planes != 0 && want32 && m % 8 == 0;   // whole 8-deep groups of the B operand
    sp.split = split16;
    sp.split_planes = split_planes == 2 ? 2 : 4;
    if (want32 && !split16) {
        POMM_HIP(dev_alloc(&sp.fac32, sizeof(cplx<float>) * sp.fac_elems));
        hipLaunchKernelGGL(to_fp32_kernel, dim3(4096), dim3(256), 0, s, sp.fac, sp.fac32, (long)sp.fac_elems);
        check_launch("to_fp32");
        if (sp.fcut) {
            const long cnt = (long)p * sp.cut_lines.size() * m * sp.cut_lines.size() * m;
            POMM_HIP(dev_alloc(&sp.fcut32, sizeof(cplx<float>) * cnt));
            hipLaunchKernelGGL(to_fp32_kernel, dim3(4096), dim3(256), 0, s, sp.fcut, sp.fcut32, cnt);
            check_launch("to_fp32");
        }
    }

    // ---- solve task lists: phases = fwd levels, final, bwd levels (reverse)
    // The same phase structure is materialized for each precision from its own
    // factor and buffer bases.
    const long colstride = (long)N * n;   // per pole in R/X
    auto build = [&](const auto* facb, const auto* fcb, auto* Rb, auto* Xb, auto& all) {
        using Task = typename std::remove_reference_t<decltype(all)>::value_type;
        using Term = std::remove_reference_t<decltype(all[0].t[0])>;
        all.clear();
        sp.task_begin.clear();
        sp.task_count.clear();
        auto rb = [&](int pole, int line) { return Rb + pole * colstride + (long)line * m; };
        auto xb = [&](int pole, int line) { return Xb + pole * colstride + (long)line * m; };
        auto sterm = [&](const auto* A, int lda, const auto* B, double a) {
            Term t;
            t.A = A;
            t.B = B;
            t.lda = lda;
            t.ldb = n;
            t.alpha_re = a;
            t.alpha_im = 0;
            return t;
        };
        sp.phase_kind.clear();
        auto open_phase = [&](int kind) {
            sp.task_begin.push_back((int)all.size());
            sp.phase_kind.push_back(kind);
        };
        auto close_phase = [&]() { sp.task_count.push_back((int)all.size() - sp.task_begin.back()); };
        // level 0, forward: t_o = A_o^{-1} r_o into X_o (cyclic tridiagonal solves), then
        // r_e -= C_e t_{e-1} + B_e t_{e+1} (stencil products)
        open_phase(PH_TRI_FWD);
        close_phase();
        open_phase(PH_STENCIL_FWD);
        close_phase();
        for (size_t li = 1; li < (size_t)sp.cut_level; ++li) {
            const SppLevel& L = sp.levels[li];
            const int ne = (int)L.even.size();
            open_phase(PH_GEMM);
            for (int pole = 0; pole < p; ++pole)
                for (int u = 0; u < ne; ++u) {
                    const int e = L.even[u];
                    const int om = (e - L.step + m) % m, op = (e + L.step) % m;
                    Task a{};
                    a.C = rb(pole, e);
                    a.ldc = n;
                    a.beta = 1.0;
                    a.gate = pole;
                    a.nterms = 2;
                    a.t[0] = sterm(facb + L.off_alpha + ((size_t)pole * ne + u) * bb, m, rb(pole, om), -1.0);
                    a.t[1] = sterm(facb + L.off_gamma + ((size_t)pole * ne + u) * bb, m, rb(pole, op), -1.0);
                    all.push_back(a);
                }
            close_phase();
        }
        open_phase(PH_GEMM);
        // the last lines: the factored final, or the dense inverse of the cut system
        const bool cut = sp.cut_level < (int)sp.levels.size();
        const std::vector<int>& flines = cut ? sp.cut_lines : sp.final_lines;
        const int nf = (int)flines.size(), Df = nf * m;
        for (int pole = 0; pole < p; ++pole)
            for (int a_ = 0; a_ < nf; ++a_) {
                Task a{};
                a.C = xb(pole, flines[a_]);
                a.ldc = n;
                a.beta = 0.0;
                a.gate = pole;
                a.nterms = nf;
                const auto* Fp = cut ? fcb + (size_t)pole * Df * Df : facb + sp.final_base + (size_t)pole * fsz;
                for (int b_ = 0; b_ < nf; ++b_)
                    a.t[b_] = sterm(Fp + (size_t)a_ * m + (size_t)b_ * m * Df, Df, rb(pole, flines[b_]), 1.0);
                all.push_back(a);
            }
        close_phase();
        for (int li = sp.cut_level - 1; li >= 1; --li) {
            const SppLevel& L = sp.levels[li];
            const int no = (int)L.odd.size();
            open_phase(PH_GEMM);
            for (int pole = 0; pole < p; ++pole)
                for (int u = 0; u < no; ++u) {
                    const int o = L.odd[u];
                    const int om = (o - L.step + m) % m, op = (o + L.step) % m;
                    Task a{};
                    a.C = xb(pole, o);
                    a.ldc = n;
                    a.beta = 0.0;
                    a.gate = pole;
                    a.nterms = 3;
                    const size_t idx = (size_t)pole * no + u;
                    a.t[0] = sterm(facb + L.off_ainv + idx * bb, m, rb(pole, o), 1.0);
                    a.t[1] = sterm(facb + L.off_f + idx * bb, m, xb(pole, om), -1.0);
                    a.t[2] = sterm(facb + L.off_g + idx * bb, m, xb(pole, op), -1.0);
                    all.push_back(a);
                }
            close_phase();
        }
        // level 0, backward: w_o = C_o x_{o-1} + B_o x_{o+1} into R_o (stencil products),
        // x_o = t_o - A_o^{-1} w_o (cyclic tridiagonal solves)
        open_phase(PH_STENCIL_BWD);
        close_phase();
        open_phase(PH_TRI_BWD);
        close_phase();
    };
    std::vector<GemmTask<double>> all;
    if (R) build(static_cast<const cplx<double>*>(sp.fac), static_cast<const cplx<double>*>(sp.fcut), R, X, all);
    std::vector<GemmTask<float>> a32;
    if (want32 && !split16)
        build(static_cast<const cplx<float>*>(sp.fac32), static_cast<const cplx<float>*>(sp.fcut32), R32, X32, a32);
    // split products: the complex128 factor blocks of every term, converted below
    struct MixTerm {
        const cplx<double>* A;
        const cplx<float>* B;
        int lda, ldb;
        double alpha_re, alpha_im;
    };
    struct MixTask {
        cplx<float>* C;
        int ldc;
        int nterms;
        double beta;
        int gate;
        MixTerm t[kMaxTerms];
    };
    std::vector<MixTask> mix;
    if (split16) build(static_cast<const cplx<double>*>(sp.fac), static_cast<const cplx<double>*>(sp.fcut), R32, X32, mix);
    // algorithmic work per phase (all poles, complex128 bytes): 8 b N b flops per complex block
    // product; every factor block read once, every right-hand-side block read and every output
    // block written.  Factor blocks kept as fp16 alone are half the size of complex64 ones
    // (fac_scale, relative to the complex128 count that the solve scales by its element size).
    const double fac_scale = split16 && sp.split_planes == 2 ? 0.5 : 1.0;
    auto task_terms = [&](int i) { return R ? all[i].nterms : (split16 ? mix[i].nterms : a32[i].nterms); };
    sp.phase_flops.clear();
    sp.phase_bytes.clear();
    for (size_t ph = 0; ph < sp.task_begin.size(); ++ph) {
        double fl = 0, by = 0;
        const int kind = sp.phase_kind[ph];
        const double el = (double)p * N * (n / 2);   // half the grid lines, N columns, p poles
        if (kind == PH_STENCIL_BWD && sp.pcr) {
            // formed inside the backward reduction (no launch)
        } else if (kind == PH_STENCIL_FWD || kind == PH_STENCIL_BWD) {
            // 6 coupling products; read the neighbour lines (and the line when accumulating),
            // write the line
            fl = el * 6 * 8;
            by = el * 16.0 * (kind == PH_STENCIL_FWD ? 3 : 2);
        } else if (kind == PH_TRI_FWD || kind == PH_TRI_BWD) {
            // forward and backward sweeps plus the border correction (or the reduction):
            // about 30 flops per element; read the right-hand side, write the solution (and
            // read it first when accumulating); with the couplings formed in place the
            // right-hand side is the neighbour lines instead
            fl = el * (30 + (kind == PH_TRI_BWD && sp.pcr ? 6 * 8 : 0));
            by = el * 16.0 * (kind == PH_TRI_BWD ? 3 : 2);
        }
        for (int i = sp.task_begin[ph]; i < sp.task_begin[ph] + sp.task_count[ph]; ++i) {
            fl += 8.0 * m * N * m * task_terms(i);
            by += 16.0 * (fac_scale * m * m * task_terms(i) + (double)m * N * (task_terms(i) + 1));
        }
        sp.phase_flops.push_back(fl);
        sp.phase_bytes.push_back(by);
    }
    if (R) {
        POMM_HIP(dev_alloc(&sp.tasks64, sizeof(GemmTask<double>) * all.size()));
        POMM_HIP(hipMemcpyAsync(sp.tasks64, all.data(), sizeof(GemmTask<double>) * all.size(), hipMemcpyHostToDevice,
                                s));
    }
    if (want32 && !split16) {
        POMM_HIP(dev_alloc(&sp.tasks32, sizeof(GemmTask<float>) * a32.size()));
        POMM_HIP(hipMemcpyAsync(sp.tasks32, a32.data(), sizeof(GemmTask<float>) * a32.size(), hipMemcpyHostToDevice, s));
    }
    if (split16) {
        // every term's factor block (m x m, its own leading dimension) becomes one split block
        std::vector<const cplx<double>*> src;
        std::vector<int> lda;
        for (const MixTask& t : mix)
            for (int k = 0; k < t.nterms; ++k) {
                src.push_back(t.t[k].A);
                lda.push_back(t.t[k].lda);
            }
        const int nb = (int)src.size();
        const size_t bbytes = split_block_bytes(m, m, sp.split_planes);
        POMM_HIP(dev_alloc(&sp.fac16, bbytes * nb));
        std::vector<void*> dst(nb);
        for (int i = 0; i < nb; ++i) dst[i] = static_cast<char*>(sp.fac16) + bbytes * i;
        const cplx<double>** src_d = nullptr;
        int* lda_d = nullptr;
        void** dst_d = nullptr;
        int* expo_d = nullptr;
        POMM_HIP(dev_alloc(&src_d, sizeof(void*) * nb));
        POMM_HIP(dev_alloc(&dst_d, sizeof(void*) * nb));
        POMM_HIP(dev_alloc(&lda_d, sizeof(int) * nb));
        POMM_HIP(dev_alloc(&expo_d, sizeof(int) * nb));
        POMM_HIP(hipMemcpyAsync(src_d, src.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
        POMM_HIP(hipMemcpyAsync(dst_d, dst.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
        POMM_HIP(hipMemcpyAsync(lda_d, lda.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
        split_blocks(src_d, lda_d, dst_d, nb, m, m, sp.split_planes, expo_d, s);
        std::vector<int> expo(nb);
        POMM_HIP(hipMemcpyAsync(expo.data(), expo_d, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        std::vector<SplitTask> st(mix.size());
        int bi = 0;
        for (size_t i = 0; i < mix.size(); ++i) {
            const MixTask& t = mix[i];
            SplitTask& o = st[i];
            o.C = t.C;
            o.ldc = t.ldc;
            o.nterms = t.nterms;
            o.beta = (float)t.beta;
            o.gate = t.gate;
            for (int k = 0; k < kMaxTerms; ++k) o.t[k] = SplitTerm{nullptr, nullptr, 0, 0.0f};
            for (int k = 0; k < t.nterms; ++k, ++bi) {
                POMM_CHECK(t.t[k].alpha_im == 0.0, 5, "split products need real term coefficients");
                o.t[k].A = dst[bi];
                o.t[k].B = t.t[k].B;
                o.t[k].ldb = t.t[k].ldb;
                o.t[k].alpha = (float)std::ldexp(t.t[k].alpha_re, expo[bi]);
            }
        }
        POMM_HIP(dev_alloc(&sp.tasks16, sizeof(SplitTask) * st.size()));
        POMM_HIP(hipMemcpyAsync(sp.tasks16, st.data(), sizeof(SplitTask) * st.size(), hipMemcpyHostToDevice, s));
        POMM_HIP(hipStreamSynchronize(s));
        (void)dev_free(src_d);
        (void)dev_free(dst_d);
        (void)dev_free(lda_d);
        (void)dev_free(expo_d);
    }
    POMM_HIP(hipStreamSynchronize(s));
    if (!R) {   // complex64 solve only: the complex128 factors are not needed after the conversion
        (void)dev_free(sp.fac);
        sp.fac = nullptr;
        if (sp.fcut) (void)dev_free(sp.fcut);
        sp.fcut = nullptr;
    }
    (void)dev_free(blocks);
    (void)dev_free(piv);
    if (inv_scratch) (void)dev_free(inv_scratch);
    (void)dev_free(tdev);
    (void)dev_free(srcp);
    (void)dev_free(dstp);
    (void)dev_free(zs_d);
    (void)dev_free(gD);
    (void)dev_free(RD);
    sp.qs_d = qs_d;
    sp.ts_d = ts_d;
    sp.V = V_dev;
}

void spp_free(Spp& sp) {
    for (void* ptr : {(void*)sp.fac, (void*)sp.fac32, (void*)sp.mult, (void*)sp.mult32, (void*)sp.tasks64,
                      (void*)sp.tasks32, (void*)sp.qs_d, (void*)sp.ts_d, (void*)sp.tri, (void*)sp.tri32,
                      sp.fac16, (void*)sp.tasks16, (void*)sp.fcut, (void*)sp.fcut32})
        if (ptr) (void)dev_free(ptr);
    sp.fcut = nullptr;
    sp.fcut32 = nullptr;
    sp.fac16 = nullptr;
    sp.tasks16 = nullptr;
    sp.split = false;
    sp.qs_d = nullptr;
    sp.ts_d = nullptr;
    sp.tri = nullptr;
    sp.tri32 = nullptr;
    sp.fac = nullptr;
    sp.fac32 = nullptr;
    sp.mult = nullptr;
    sp.mult32 = nullptr;
    sp.tasks64 = nullptr;
    sp.tasks32 = nullptr;
}

template <typename T>
void spp_solve(const Spp& sp, const int* pole_active, int active_poles, hipStream_t s) {
    const GemmTask<T>* tasks;
    if constexpr (sizeof(T) == 8) tasks = sp.tasks64;
    else tasks = sp.tasks32;
    const double frac = (double)active_poles / sp.p;
    const double esz = (double)sizeof(cplx<T>) / sizeof(cplx<double>);
    cplx<T>* Xs;
    cplx<T>* Rs;
    const cplx<T>* tri;
    if constexpr (sizeof(T) == 8) {
        Xs = sp.X;
        Rs = sp.R;
        tri = sp.tri;
    } else {
        Xs = sp.X32;
        Rs = sp.R32;
        tri = sp.tri32;
    }
    const long half = (long)(sp.m / 2) * sp.m;
    // level-0 tridiagonal solves: right-hand sides per workgroup (one per lane), LDS m x (CPW + 1)
    constexpr int CPW = sizeof(T) == 4 ? 64 : 32;
    const size_t tri_lds = tri_lds_bytes<T, CPW>(sp.m);
    static const bool attr_set = [] {   // once per process, thread-safe
        (void)hipFuncSetAttribute((const void*)tri_lines_kernel<T, CPW, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)tri_lds_max<T, CPW>());
        (void)hipFuncSetAttribute((const void*)tri_lines_kernel<T, CPW, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)tri_lds_max<T, CPW>());
        return true;
    }();
    (void)attr_set;
    const size_t nph = sp.task_begin.size();
    for (size_t ph = 0; ph < nph; ++ph) {
        const int kind = sp.phase_kind[ph];
        if (kind == PH_STENCIL_BWD && sp.pcr) continue;   // formed inside the backward reduction
        if (kind == PH_GEMM) {
            // consecutive GEMM phases (the dense levels) share one timing scope
            size_t end = ph;
            double by = 0, fl = 0;
            while (end < nph && sp.phase_kind[end] == PH_GEMM) {
                by += sp.phase_bytes[end];
                fl += sp.phase_flops[end];
                ++end;
            }
            ProfScope prof(PK_SPP_SOLVE, frac * esz * by, frac * fl, s, (int)(end - ph));
            for (; ph < end; ++ph) {
                const int cnt = sp.task_count[ph];
                const int busy = (int)((long)cnt * active_poles / sp.p);
                bool done = false;
                if constexpr (sizeof(T) == 4) {
                    if (sp.split) {
                        gemm_split(sp.tasks16 + sp.task_begin[ph], cnt, sp.b, sp.N, sp.b, sp.split_planes,
                                   pole_active, s, busy, sp.split_variant);
                        done = true;
                    }
                }
                if (!done) gemm_batched<T>(tasks + sp.task_begin[ph], cnt, sp.b, sp.N, sp.b, pole_active, s, busy);
            }
            --ph;   // the loop's increment moves past the run
            continue;
        }
        ProfScope prof(PK_SPP_STENCIL, frac * esz * sp.phase_bytes[ph], frac * sp.phase_flops[ph], s);
        if ((kind == PH_TRI_FWD || kind == PH_TRI_BWD) && sp.pcr) {
            const dim3 grid(sp.m / 2, sp.p);
            // lane permutes for complex64; complex128 keeps the workgroup LDS exchange for the
            // backward pass, whose wave form needs too many registers for its multipliers
            // (both measured on the 128^2 lattice)
            constexpr int GF = sizeof(T) == 4 ? 4 : 2;
            const bool w64 = sp.m == 128;
            if (kind == PH_TRI_FWD) {
                if (w64)
                    hipLaunchKernelGGL((pcr_wave_kernel<T, false, false, GF, true>), grid, dim3(256), 0, s, Rs, Xs,
                                       tri, sp.m, sp.N, (long)sp.n, pole_active, sp.qs_d, sp.ts_d, sp.V, sp.l);
                else
                    hipLaunchKernelGGL((pcr_wave_kernel<T, false, false, GF, false>), grid, dim3(256), 0, s, Rs, Xs,
                                       tri, sp.m, sp.N, (long)sp.n, pole_active, sp.qs_d, sp.ts_d, sp.V, sp.l);
            } else if constexpr (sizeof(T) == 4) {   // backward couplings formed in place
                if (w64)
                    hipLaunchKernelGGL((pcr_wave_kernel<T, true, true, 2, true>), grid, dim3(256), 0, s, Rs, Xs, tri,
                                       sp.m, sp.N, (long)sp.n, pole_active, sp.qs_d, sp.ts_d, sp.V, sp.l);
                else
                    hipLaunchKernelGGL((pcr_wave_kernel<T, true, true, 2, false>), grid, dim3(256), 0, s, Rs, Xs, tri,
                                       sp.m, sp.N, (long)sp.n, pole_active, sp.qs_d, sp.ts_d, sp.V, sp.l);
            } else {
                hipLaunchKernelGGL((pcr_lines_kernel<T, true, true>), grid, dim3(128), 0, s, Rs, Xs, tri, sp.m, sp.N,
                                   (long)sp.n, pole_active, sp.qs_d, sp.ts_d, sp.V, sp.l);
            }
            check_launch("pcr");
        } else if (kind == PH_TRI_FWD || kind == PH_TRI_BWD) {
            const dim3 grid(sp.m / 2, cdiv_u(sp.N, CPW), sp.p);
            if (kind == PH_TRI_FWD)
                hipLaunchKernelGGL((tri_lines_kernel<T, CPW, false>), grid, dim3(64), tri_lds, s, Rs, Xs, tri, sp.m,
                                   sp.N, (long)sp.n, pole_active);
            else
                hipLaunchKernelGGL((tri_lines_kernel<T, CPW, true>), grid, dim3(64), tri_lds, s, Rs, Xs, tri, sp.m,
                                   sp.N, (long)sp.n, pole_active);
            check_launch("tri_lines");
        } else {
            // forward: R_e -= C_e t_{e-1} + B_e t_{e+1}; backward (tridiagonal path): R_o = w_o
            const dim3 grid(sp.m / 2, sp.p);
            if (kind == PH_STENCIL_FWD)
                hipLaunchKernelGGL((couple_lines_kernel<T, false>), grid, dim3(128), 0, s, Xs, Rs, sp.m, sp.N,
                                   (long)sp.n, 0, sp.qs_d, sp.ts_d, sp.V, sp.l, pole_active);
            else
                hipLaunchKernelGGL((couple_lines_kernel<T, true>), grid, dim3(128), 0, s, Xs, Rs, sp.m, sp.N,
                                   (long)sp.n, 1, sp.qs_d, sp.ts_d, sp.V, sp.l, pole_active);
            check_launch("couple_lines");
        }
    }
}

template void spp_solve<double>(const Spp&, const int*, int, hipStream_t);
template void spp_solve<float>(const Spp&, const int*, int, hipStream_t);

}  // namespace pomm
