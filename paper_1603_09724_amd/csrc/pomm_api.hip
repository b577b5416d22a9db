// C ABI of libpomm (declared in include/pomm.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pomm.h"
#include "common.h"
#include "dense.h"
#include "gmres.h"
#include "omm.h"
#include "poles.h"
#include "prof.h"
#include "spectral.h"
#include "spp.h"

using namespace pomm;

struct omm_ctx {
    hipStream_t stream = nullptr;
    int dim = 2, m = 0, n = 0, N = 0;
    double sigma = 0.0, l = 0.0, vmin = 0.0, vmax = 0.0;
    omm_opts_t opts{};
    omm_spectrum_t spec{};
    std::vector<std::complex<double>> z, w;
    SpectralPlan plan;
    Spp spp;
    bool have_spp = false;
    GmresWork gw;
    double* V = nullptr;
    float* V32 = nullptr;
    // OMM state, n x N complex128 each
    cplx<double>* HX = nullptr;
    cplx<double>* D = nullptr;
    cplx<double>* HD = nullptr;
    cplx<double>* Gr = nullptr;   // gradient G(X)
    cplx<double>* PG = nullptr;   // preconditioned gradient
    cplx<double>* Gp = nullptr;   // previous search gradient
    GramPlan gram;
    cplx<double>* parts = nullptr;
    cplx<double>* grams = nullptr;           // 6 x N x N
    const cplx<double>** gram_P = nullptr;   // device pointer lists (6 each)
    const cplx<double>** gram_Q = nullptr;
    GemmTask<double>* grad_task = nullptr;   // device, one task (X pointer patched per solve)
    OmmScalars* sc = nullptr;
    OmmScalars* sc_host = nullptr;
    double* red = nullptr;
    cplx<double>* bound_X = nullptr;         // X the device lists currently point at
    cplx<double>* outer_tab = nullptr;   // OMM_OUTER_LAPLACE / _TPA symbol (kernel order)
    // precomputed preconditioner U U* (Section 3.3): U n x N, workspace for up to 2N columns
    bool lowrank = false;
    cplx<double>* lr_U = nullptr;
    cplx<double>* lr_Y = nullptr;      // n x 2N: the filtered random block
    cplx<double>* lr_pad = nullptr;    // n x N scratch
    cplx<double>* lr_small = nullptr;  // (2N)^2 + 2 N^2 complex: Grams, triangular inverses, U* G
    cplx<double>* lr_parts = nullptr;
    int* lr_piv = nullptr;
    const cplx<double>** lr_ptrs = nullptr;   // device pointer pairs for the Gram products
    GemmTask<double>* lr_task = nullptr;
    std::string err;
    long long precond_calls = 0;
    Profiler prof;
};

// Routes the launch-site scopes of one API call to the handle's profiler.
struct ProfBind {
    ProfBind(omm_ctx* h) { current_profiler() = h->prof.on ? &h->prof : nullptr; }
    ~ProfBind() { current_profiler() = nullptr; }
};

static thread_local std::string g_setup_error;

static int fail(omm_ctx* h, const Error& e) {
    if (h) h->err = e.what();
    else g_setup_error = e.what();
    return e.code;
}

extern "C" {

void ommDefaultOptions(omm_opts_t* o) {
    if (!o) return;
    o->precision = OMM_FP64;
    o->inner = OMM_INNER_SPP;
    o->poles = OMM_POLES_ELLIPTIC;
    o->npoles = 30;
    o->gmres_rtol = 1e-5;
    o->gmres_restart = 15;
    o->gmres_cycles = 5;
    o->filter_rtol = 1e-5;
    o->tol = 1e-10;
    o->maxit = 4000;
    o->stall = 3;
    o->filter = 1;
    o->pole_tol = 1e-9;
    o->gmres_side = OMM_SIDE_AUTO;
    o->spp_products = OMM_PRODUCTS_SPLIT16;
    o->gmres_verify = 1;
    o->outer = OMM_OUTER_FERMI;
    o->tau = 0.0;
}

const char* ommStatusString(int st) {
    switch (st) {
        case OMM_OK: return "ok";
        case OMM_EINVAL: return "invalid argument";
        case OMM_ENOTNEGDEF: return "shift does not make H negative definite";
        case OMM_ESPECTRUM: return "inconsistent spectral window";
        case OMM_ENOMEM: return "out of device memory";
        case OMM_EHIP: return "HIP runtime error";
        case OMM_ENOCONV: return "iteration cap reached";
        case OMM_EBREAKDOWN: return "line search breakdown";
        case OMM_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* ommLastError(omm_handle_t h) { return h ? h->err.c_str() : g_setup_error.c_str(); }

}  // extern "C"

static void destroy_ctx(omm_ctx* h) {
    if (!h) return;
    AllocBind ab(h->stream);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    h->prof.release();
    gmres_free(h->gw);
    if (h->have_spp) spp_free(h->spp);
    spectral_plan_free(h->plan);
    for (void* p : {(void*)h->V, (void*)h->V32, (void*)h->HX, (void*)h->D, (void*)h->HD, (void*)h->Gr, (void*)h->PG,
                    (void*)h->Gp, (void*)h->parts, (void*)h->grams, (void*)h->gram_P, (void*)h->gram_Q,
                    (void*)h->grad_task, (void*)h->sc, (void*)h->red, (void*)h->lr_U, (void*)h->lr_Y,
                    (void*)h->lr_pad, (void*)h->lr_small, (void*)h->lr_parts, (void*)h->lr_piv, (void*)h->lr_ptrs,
                    (void*)h->lr_task, (void*)h->outer_tab})
        if (p) (void)dev_free(p);
    if (h->sc_host) (void)hipHostFree(h->sc_host);
    delete h;
}

static int setup_estimate_window(const omm_grid_t* grid, const double* V, int N, int n, hipStream_t s,
                                 omm_spectrum_t* spec);

__global__ static void v_to_fp32(const double* a, float* b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

extern "C" int ommSetup(const omm_grid_t* grid, const double* V, int N, double shift, const omm_spectrum_t* spec,
                        const omm_opts_t* opts, void* stream, omm_handle_t* out) {
    omm_ctx* h = nullptr;
    AllocBind ab((hipStream_t)stream);
    try {
        POMM_CHECK(grid && V && out, OMM_EINVAL, "NULL argument");
        *out = nullptr;
        POMM_CHECK(grid->dim == 2 || grid->dim == 3, OMM_EINVAL, "dim must be 2 or 3");
        const int m = grid->m[0];
        for (int i = 1; i < grid->dim; ++i) POMM_CHECK(grid->m[i] == m, OMM_EINVAL, "grid must be cubic (equal m)");
        h = new omm_ctx();
        h->dim = grid->dim;
        h->m = m;
        if (opts) h->opts = *opts;
        else ommDefaultOptions(&h->opts);
        const omm_opts_t& o = h->opts;
        POMM_CHECK(o.precision == OMM_FP64 || o.precision == OMM_MIXED, OMM_EINVAL, "bad precision");
        POMM_CHECK(o.npoles == 0 || (o.npoles >= 2 && o.npoles <= 64 && o.npoles % 2 == 0), OMM_EINVAL,
                   "npoles must be 0 (automatic) or even, 2..64");
        POMM_CHECK(o.npoles != 0 || (o.pole_tol > 0.0 && o.pole_tol < 1.0), OMM_EINVAL, "pole_tol must be in (0, 1)");
        POMM_CHECK(o.gmres_restart >= 1 && o.gmres_restart <= 32, OMM_EINVAL, "gmres_restart must be 1..32");
        POMM_CHECK(o.gmres_cycles >= 1, OMM_EINVAL, "gmres_cycles must be >= 1");
        POMM_CHECK(o.inner == OMM_INNER_SPP || o.inner == OMM_INNER_PP, OMM_EINVAL, "bad inner preconditioner");
        POMM_CHECK(o.poles == OMM_POLES_ELLIPTIC || o.poles == OMM_POLES_CIRCLE, OMM_EINVAL, "bad pole rule");
        POMM_CHECK(o.maxit >= 0 && o.stall >= 0, OMM_EINVAL, "maxit and stall must be >= 0");
        POMM_CHECK(o.gmres_side == OMM_SIDE_AUTO || o.gmres_side == OMM_SIDE_RIGHT || o.gmres_side == OMM_SIDE_LEFT,
                   OMM_EINVAL, "bad gmres_side");
        POMM_CHECK(o.spp_products == OMM_PRODUCTS_SPLIT16 || o.spp_products == OMM_PRODUCTS_FP32 ||
                       o.spp_products == OMM_PRODUCTS_F16,
                   OMM_EINVAL, "bad spp_products");
        POMM_CHECK(o.outer == OMM_OUTER_FERMI || o.outer == OMM_OUTER_LAPLACE || o.outer == OMM_OUTER_TPA, OMM_EINVAL,
                   "bad outer preconditioner");
        POMM_CHECK(o.outer == OMM_OUTER_FERMI || (std::isfinite(o.tau) && o.tau > 0.0), OMM_EINVAL,
                   "the Laplace and TPA preconditioners need tau > 0");
        POMM_CHECK(o.gmres_verify == 0 || o.gmres_verify == 1, OMM_EINVAL, "gmres_verify must be 0 or 1");
        h->stream = (hipStream_t)stream;
        h->prof.stream = h->stream;
        int dev = 0;
        POMM_HIP(hipGetDevice(&dev));
        int lds = 0;
        POMM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        spectral_plan_init(h->plan, h->dim, m, (size_t)lds);
        h->n = h->plan.n;
        const int n = h->n;
        POMM_CHECK(N >= 1 && N < n, OMM_EINVAL, "need 1 <= N < n");
        h->N = N;
        // potential statistics and shift (H - sigma I negative definite, Section 1)
        double vmin = V[0], vmax = V[0], vsum = 0.0;
        for (int i = 0; i < n; ++i) {
            POMM_CHECK(std::isfinite(V[i]), OMM_EINVAL, "V has non-finite entries");
            vmin = std::min(vmin, V[i]);
            vmax = std::max(vmax, V[i]);
            vsum += V[i];
        }
        h->vmin = vmin;
        h->vmax = vmax;
        h->l = vsum / n;
        const double hi = 0.5 * h->dim * (double)(m / 2) * (double)(m / 2) + vmax;
        if (std::isnan(shift)) h->sigma = hi + 1.0;
        else {
            POMM_CHECK(std::isfinite(shift) && shift > hi, OMM_ENOTNEGDEF,
                       "shift must exceed the upper spectral bound " + std::to_string(hi));
            h->sigma = shift;
        }
        omm_spectrum_t estimated{};
        if (!spec) {   // no window given: estimate it on the device
            setup_estimate_window(grid, V, N, n, h->stream, &estimated);
            spec = &estimated;
        }
        h->spec = *spec;
        POMM_CHECK(spec->lo < spec->homo && spec->homo < spec->lumo, OMM_ESPECTRUM, "need lo < homo < lumo");
        POMM_CHECK(spec->lo <= vmin, OMM_ESPECTRUM, "spec.lo must not exceed min V (a lower bound of lambda_1)");
        // poles (unshifted frame); npoles = 0: smallest even p >= 30 meeting pole_tol
        if (h->opts.npoles == 0) {
            int pp = 30;
            if (o.poles == OMM_POLES_ELLIPTIC)
                while (pp < 64 && elliptic_rate(spec->lo, spec->homo, spec->lumo, pp) > o.pole_tol) pp += 2;
            h->opts.npoles = pp;
        }
        if (o.poles == OMM_POLES_ELLIPTIC) elliptic_poles(spec->lo, spec->homo, spec->lumo, o.npoles, h->z, h->w);
        else {
            const double c = spec->lo, rho = 0.5 * (spec->homo + spec->lumo) - spec->lo;
            circle_poles(c, rho, o.npoles, h->z, h->w);
        }
        const int p = o.npoles;
        // device potential
        POMM_HIP(dev_alloc(&h->V, sizeof(double) * n));
        POMM_HIP(hipMemcpyAsync(h->V, V, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        POMM_HIP(dev_alloc(&h->V32, sizeof(float) * n));
        hipLaunchKernelGGL(v_to_fp32, dim3(cdiv_u(n, 256)), dim3(256), 0, h->stream, h->V, h->V32, n);
        check_launch("v_to_fp32");
        // GMRES workspace and pole tables
        const bool mp = spectral_needs_work<double>(h->plan);
        const bool mixed = o.precision == OMM_MIXED;
        gmres_alloc(h->gw, n, N, p, o.gmres_restart, mp, mixed);
        {
            std::vector<cplx<double>> zz(2 * p), ww(p);
            for (int j = 0; j < p; ++j) {
                zz[j] = mk<double>(h->z[j].real(), h->z[j].imag());
                zz[p + j] = mk<double>(h->l - h->z[j].real(), -h->z[j].imag());
                ww[j] = mk<double>(h->w[j].real(), h->w[j].imag());
            }
            POMM_HIP(hipMemcpyAsync(h->gw.pole_z, zz.data(), sizeof(cplx<double>) * 2 * p, hipMemcpyHostToDevice,
                                    h->stream));
            POMM_HIP(hipMemcpyAsync(h->gw.pole_w, ww.data(), sizeof(cplx<double>) * p, hipMemcpyHostToDevice,
                                    h->stream));
            POMM_HIP(hipStreamSynchronize(h->stream));
        }
        if (o.inner == OMM_INNER_SPP) {
            if (mixed)
                spp_setup(h->spp, h->plan, h->V, h->l, h->z, N, nullptr, nullptr, static_cast<cplx<float>*>(h->gw.U),
                          static_cast<cplx<float>*>(h->gw.Z), true,
                          o.spp_products == OMM_PRODUCTS_SPLIT16 ? 4 : (o.spp_products == OMM_PRODUCTS_F16 ? 2 : 0),
                          h->stream);
            else
                spp_setup(h->spp, h->plan, h->V, h->l, h->z, N, static_cast<cplx<double>*>(h->gw.U),
                          static_cast<cplx<double>*>(h->gw.Z), nullptr, nullptr, false, 0, h->stream);
            h->have_spp = true;
        }
        if (o.outer != OMM_OUTER_FERMI) {   // Section 3.1's Fourier-diagonal preconditioner as a table
            std::vector<cplx<double>> tab(n);
            const int d = h->dim;
            for (int e = 0; e < n; ++e) {
                int rest = e;
                double k2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    const int j = rest % m, k = j < m / 2 ? j : j - m;
                    rest /= m;
                    k2 += (double)k * k;
                }
                const double sv = k2 / o.tau;
                double v;
                if (o.outer == OMM_OUTER_LAPLACE) {
                    v = 1.0 / (1.0 + sv);
                } else {
                    const double q = 27.0 + 18.0 * sv + 12.0 * sv * sv + 8.0 * sv * sv * sv;
                    v = q / (q + 16.0 * sv * sv * sv * sv);
                }
                tab[e] = mk<double>(v, 0.0);
            }
            cplx<double>* nat = nullptr;
            POMM_HIP(dev_alloc(&nat, sizeof(cplx<double>) * n));
            POMM_HIP(dev_alloc(&h->outer_tab, sizeof(cplx<double>) * n));
            POMM_HIP(hipMemcpyAsync(nat, tab.data(), sizeof(cplx<double>) * n, hipMemcpyHostToDevice, h->stream));
            spectral_table_reorder<double>(h->plan, nat, h->outer_tab, 1, h->stream);
            POMM_HIP(hipStreamSynchronize(h->stream));
            (void)dev_free(nat);
        }
        // OMM buffers
        const size_t blk = sizeof(cplx<double>) * (size_t)n * N;
        POMM_HIP(dev_alloc(&h->HX, blk));
        POMM_HIP(dev_alloc(&h->D, blk));
        POMM_HIP(dev_alloc(&h->HD, blk));
        POMM_HIP(dev_alloc(&h->Gr, blk));
        POMM_HIP(dev_alloc(&h->PG, blk));
        POMM_HIP(dev_alloc(&h->Gp, blk));
        h->gram = gram_plan(n, N);
        POMM_HIP(dev_alloc(&h->parts, sizeof(cplx<double>) * gram_parts_elems(h->gram, 6)));
        POMM_HIP(dev_alloc(&h->grams, sizeof(cplx<double>) * 6 * N * N));
        POMM_HIP(dev_alloc(&h->gram_P, sizeof(void*) * 6));
        POMM_HIP(dev_alloc(&h->gram_Q, sizeof(void*) * 6));
        POMM_HIP(dev_alloc(&h->grad_task, sizeof(GemmTask<double>)));
        POMM_HIP(dev_alloc(&h->sc, sizeof(OmmScalars)));
        POMM_HIP(hipHostMalloc(&h->sc_host, sizeof(OmmScalars)));
        POMM_HIP(dev_alloc(&h->red, sizeof(double) * 1024));
        POMM_HIP(hipStreamSynchronize(h->stream));
        *out = h;
        return OMM_OK;
    } catch (const Error& e) {
        const int code = fail(nullptr, e);
        destroy_ctx(h);
        return code;
    } catch (const std::bad_alloc&) {
        g_setup_error = "host allocation failed";
        destroy_ctx(h);
        return OMM_ENOMEM;
    }
}

extern "C" int ommDestroy(omm_handle_t h) {
    destroy_ctx(h);
    return OMM_OK;
}

extern "C" int ommGetPoles(omm_handle_t h, double* z, double* w) {
    if (!h || !z || !w) return OMM_EINVAL;
    for (size_t j = 0; j < h->z.size(); ++j) {
        z[2 * j] = h->z[j].real();
        z[2 * j + 1] = h->z[j].imag();
        w[2 * j] = h->w[j].real();
        w[2 * j + 1] = h->w[j].imag();
    }
    return OMM_OK;
}

extern "C" int ommGetStencil(omm_handle_t h, int pole, double* q, double* t) {
    if (!h || !q || !t) return OMM_EINVAL;
    if (!h->have_spp) return OMM_EUNSUPPORTED;
    if (pole < 0 || pole >= (int)h->z.size()) return OMM_EINVAL;
    for (int s = 0; s < 9; ++s) {
        q[2 * s] = h->spp.q[pole * 9 + s].real();
        q[2 * s + 1] = h->spp.q[pole * 9 + s].imag();
        t[2 * s] = h->spp.t[pole * 9 + s].real();
        t[2 * s + 1] = h->spp.t[pole * 9 + s].imag();
    }
    return OMM_OK;
}

extern "C" int ommGetInfo(omm_handle_t h, double* sigma, int* n, int* N, int* npoles) {
    if (!h) return OMM_EINVAL;
    if (sigma) *sigma = h->sigma;
    if (n) *n = h->n;
    if (N) *N = h->N;
    if (npoles) *npoles = (int)h->z.size();
    return OMM_OK;
}

extern "C" int ommGetCounters(omm_handle_t h, long long* gmres_steps, long long* precond_calls) {
    if (!h) return OMM_EINVAL;
    try {
        unsigned long long st = 0;
        POMM_HIP(hipMemcpyAsync(&st, h->gw.steps, sizeof(st), hipMemcpyDeviceToHost, h->stream));
        POMM_HIP(hipStreamSynchronize(h->stream));
        if (gmres_steps) *gmres_steps = (long long)st;
        if (precond_calls) *precond_calls = h->precond_calls;
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

extern "C" int ommApplyH(omm_handle_t h, const void* X, void* HX, int ncols, int prec) {
    if (!h) return OMM_EINVAL;
    ProfBind pb(h);
    try {
        POMM_CHECK(X && HX && ncols >= 1, OMM_EINVAL, "bad arguments");
        POMM_CHECK(prec == OMM_PREC_FP64 || prec == OMM_PREC_FP32, OMM_EINVAL, "bad precision");
        if (prec == OMM_PREC_FP64) {
            SpecArgs<double> a;
            a.in = (const cplx<double>*)X;
            a.ld_in = h->n;
            a.out = (cplx<double>*)HX;
            a.ld_out = h->n;
            a.ncols = ncols;
            a.post_mode = POST_SHIFTED_H;
            a.V = h->V;
            a.sigma = h->sigma;
            const bool mp = spectral_needs_work<double>(h->plan);
            POMM_CHECK(!mp || ncols <= h->gw.S, OMM_EINVAL, "ncols exceeds the scratch of this handle");
            spectral_apply<double>(h->plan, a, h->gw.work, h->stream);
        } else {
            SpecArgs<float> a;
            a.in = (const cplx<float>*)X;
            a.ld_in = h->n;
            a.out = (cplx<float>*)HX;
            a.ld_out = h->n;
            a.ncols = ncols;
            a.post_mode = POST_SHIFTED_H;
            a.V = h->V32;
            a.sigma = h->sigma;
            const bool mp = spectral_needs_work<float>(h->plan);
            POMM_CHECK(!mp || (h->gw.work && ncols <= 2 * h->gw.S), OMM_EINVAL,
                       "ncols exceeds the scratch of this handle");
            spectral_apply<float>(h->plan, a, (cplx<float>*)h->gw.work, h->stream);
        }
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

static PrecondConfig precond_config(const omm_ctx* h, double rtol) {
    PrecondConfig c;
    c.inner = h->opts.inner == OMM_INNER_SPP ? 0 : 1;
    c.rtol = rtol;
    c.restart = h->opts.gmres_restart;
    c.cycles = h->opts.gmres_cycles;
    c.left = h->opts.gmres_side == OMM_SIDE_LEFT ||
             (h->opts.gmres_side == OMM_SIDE_AUTO && h->opts.precision == OMM_MIXED);
    c.l = h->l;
    c.verify = h->opts.gmres_verify != 0;
    return c;
}

// PG = F^{-1} diag(P) F G for the Fourier-diagonal outer preconditioners of Section 3.1
static void outer_apply(omm_ctx* h, const cplx<double>* G, cplx<double>* PG, int ncols) {
    ProfScope prof(PK_OMM, 2.0 * sizeof(cplx<double>) * (double)h->n * ncols, 0.0, h->stream);
    SpecArgs<double> a;
    a.in = G;
    a.ld_in = h->n;
    a.out = PG;
    a.ld_out = h->n;
    a.ncols = ncols;
    a.cols_per_group = ncols;
    a.mult_mode = MULT_TABLE;
    a.mult_tab = h->outer_tab;
    spectral_apply<double>(h->plan, a, h->gw.work, h->stream);
}

// ---- Section 3.3, Algorithm 2: the preconditioner precomputed as U U*

// Columns [0, cols) of the real n x cols block B (ld n) as complex values into out (n x N),
// zero columns after them.
__global__ static void lr_real_block(const double* __restrict__ B, int n, int cols, int N,
                                     cplx<double>* __restrict__ out) {
    const long total = (long)n * N;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
        out[e] = mk<double>(e < (long)n * cols ? B[e] : 0.0, 0.0);
}

// out[:, j] = Y[:, idx[j]] for j < cols (n rows, ld n)
__global__ static void lr_gather(const cplx<double>* __restrict__ Y, int n, const int* __restrict__ idx, int cols,
                                 cplx<double>* __restrict__ out) {
    const long total = (long)n * cols;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e / n), r = (int)(e % n);
        out[e] = Y[r + (long)idx[j] * n];
    }
}

// Columns [0, cols) of G (ld n) into out (n x N), zero columns after them.
__global__ static void lr_pad_block(const cplx<double>* __restrict__ G, int n, int cols, int N,
                                    cplx<double>* __restrict__ out) {
    const long total = (long)n * N;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
        out[e] = e < (long)n * cols ? G[e] : mk<double>(0.0, 0.0);
}

using cd = std::complex<double>;

// Cholesky with diagonal pivoting of the Hermitian c x c matrix G (column major), r steps:
// the column order and R (r x r, upper, column major) of a column-pivoted QR of any Y with
// Y^H Y = G (at step j the pivot is the column of largest remaining norm, ties to the
// smaller index).  Returns false if a pivot is not positive.
static bool pivoted_cholesky(std::vector<cd> G, int c, int r, std::vector<int>& piv, std::vector<cd>& R) {
    piv.resize(c);
    for (int j = 0; j < c; ++j) piv[j] = j;
    std::vector<cd> L((size_t)c * r, 0.0);   // rows of R, in the original column numbering: L[j][col]
    std::vector<double> d(c);
    for (int j = 0; j < c; ++j) d[j] = G[j + (size_t)j * c].real();
    for (int j = 0; j < r; ++j) {
        int best = j;
        for (int l = j + 1; l < c; ++l)
            if (d[piv[l]] > d[piv[best]]) best = l;
        std::swap(piv[j], piv[best]);
        const int pj = piv[j];
        if (!(d[pj] > 0.0)) return false;
        const double rjj = std::sqrt(d[pj]);
        L[(size_t)j * c + pj] = rjj;
        for (int l = j + 1; l < c; ++l) {
            const int pl = piv[l];
            cd v = G[pj + (size_t)pl * c];
            for (int i = 0; i < j; ++i) v -= std::conj(L[(size_t)i * c + pj]) * L[(size_t)i * c + pl];
            v /= rjj;
            L[(size_t)j * c + pl] = v;
            d[pl] -= std::norm(v);
        }
    }
    R.assign((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i <= j; ++i) R[i + (size_t)j * r] = L[(size_t)i * c + piv[j]];
    return true;
}

// Unpivoted Cholesky G = R^H R of the Hermitian r x r matrix G (column major).
static bool cholesky_upper(const std::vector<cd>& G, int r, std::vector<cd>& R) {
    R.assign((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i <= j; ++i) {
            cd v = G[i + (size_t)j * r];
            for (int k = 0; k < i; ++k) v -= std::conj(R[k + (size_t)i * r]) * R[k + (size_t)j * r];
            if (i == j) {
                if (!(v.real() > 0.0)) return false;
                R[i + (size_t)j * r] = std::sqrt(v.real());
            } else {
                R[i + (size_t)j * r] = v / R[i + (size_t)i * r];
            }
        }
    return true;
}

// Inverse of the upper-triangular r x r matrix R (column major) by back substitution.
static std::vector<cd> upper_inverse(const std::vector<cd>& R, int r) {
    std::vector<cd> X((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j) {
        X[j + (size_t)j * r] = 1.0 / R[j + (size_t)j * r];
        for (int i = j - 1; i >= 0; --i) {
            cd v = 0.0;
            for (int k = i + 1; k <= j; ++k) v += R[i + (size_t)k * r] * X[k + (size_t)j * r];
            X[i + (size_t)j * r] = -v / R[i + (size_t)i * r];
        }
    }
    return X;
}

// C (n x cols) = A (n x K) B (K x cols, ld K), one task through the handle's task slot
static void lr_gemm(omm_ctx* h, cplx<double>* C, const cplx<double>* A, const cplx<double>* B, int K, int cols) {
    GemmTask<double> t{};
    t.C = C;
    t.ldc = h->n;
    t.beta = 0.0;
    t.gate = -1;
    t.nterms = 1;
    t.t[0] = GemmTerm<double>{A, B, h->n, K, 1.0, 0.0};
    POMM_HIP(hipMemcpyAsync(h->lr_task, &t, sizeof(t), hipMemcpyHostToDevice, h->stream));
    POMM_HIP(hipStreamSynchronize(h->stream));   // t is a host temporary
    gemm_batched<double>(h->lr_task, 1, h->n, cols, K, nullptr, h->stream);
}

// out (c x c) = P^H Q over the n rows, P and Q n x c
static void lr_gram(omm_ctx* h, const cplx<double>* P, const cplx<double>* Q, int c, cplx<double>* out) {
    const cplx<double>* ptr[2] = {P, Q};
    POMM_HIP(hipMemcpyAsync(h->lr_ptrs, ptr, sizeof(ptr), hipMemcpyHostToDevice, h->stream));
    POMM_HIP(hipStreamSynchronize(h->stream));   // ptr is a host temporary
    gram_products(gram_plan(h->n, c), h->lr_ptrs, h->lr_ptrs + 1, 1, h->lr_parts, out, h->stream);
}

// PG = U (U^H G) for ncols <= N columns of G
static void lowrank_apply(omm_ctx* h, const cplx<double>* G, cplx<double>* PG, int ncols) {
    const int n = h->n, N = h->N;
    ProfScope prof(PK_OMM, sizeof(cplx<double>) * (double)n * (2.0 * N + 2.0 * ncols), 16.0 * n * (double)N * ncols,
                   h->stream, 3);
    const cplx<double>* Gin = G;
    if (ncols < N) {
        hipLaunchKernelGGL(lr_pad_block, dim3(256), dim3(256), 0, h->stream, G, n, ncols, N, h->lr_pad);
        check_launch("lr_pad_block");
        Gin = h->lr_pad;
    }
    cplx<double>* T = h->lr_small;   // N x N
    lr_gram(h, h->lr_U, Gin, N, T);
    lr_gemm(h, PG, h->lr_U, T, N, ncols);
}

extern "C" int ommPrecompute(omm_handle_t h, const double* B, int ncols, double rtol) {
    if (!h) return OMM_EINVAL;
    ProfBind pb(h);
    AllocBind ab(h->stream);
    try {
        if (!B && ncols == 0) {   // back to the pole expansion
            h->lowrank = false;
            return OMM_OK;
        }
        const int n = h->n, N = h->N;
        POMM_CHECK(B != nullptr, OMM_EINVAL, "B is NULL");
        POMM_CHECK(h->opts.outer == OMM_OUTER_FERMI, OMM_EINVAL, "Algorithm 2 needs the Fermi preconditioner");
        POMM_CHECK(ncols >= N && ncols <= 2 * N, OMM_EINVAL, "ncols must be in N..2N");
        hipStream_t s = h->stream;
        if (!h->lr_U) {
            size_t parts = 0;   // the Gram workspace of every column count used: N..2N
            for (int c = N; c <= 2 * N; ++c) parts = std::max(parts, gram_parts_elems(gram_plan(n, c), 1));
            POMM_HIP(dev_alloc(&h->lr_U, sizeof(cplx<double>) * (size_t)n * N));
            POMM_HIP(dev_alloc(&h->lr_Y, sizeof(cplx<double>) * (size_t)n * 2 * N));
            POMM_HIP(dev_alloc(&h->lr_pad, sizeof(cplx<double>) * (size_t)n * N));
            POMM_HIP(dev_alloc(&h->lr_small, sizeof(cplx<double>) * (size_t)6 * N * N));
            POMM_HIP(dev_alloc(&h->lr_parts, sizeof(cplx<double>) * parts));
            POMM_HIP(dev_alloc(&h->lr_piv, sizeof(int) * N));
            POMM_HIP(dev_alloc(&h->lr_ptrs, sizeof(void*) * 2));
            POMM_HIP(dev_alloc(&h->lr_task, sizeof(GemmTask<double>)));
        }
        h->lowrank = false;   // the pole expansion builds Y
        const PrecondConfig cfg = precond_config(h, rtol > 0 ? rtol : h->opts.gmres_rtol);
        // steps 3-4: Y = sum_j w_j Y_j with (H - z_j) Y_j = B, GMRES started from B, N columns a call
        for (int c0 = 0; c0 < ncols; c0 += N) {
            const int cols = std::min(N, ncols - c0);
            hipLaunchKernelGGL(lr_real_block, dim3(256), dim3(256), 0, s, B + (size_t)c0 * n, n, cols, N, h->lr_pad);
            check_launch("lr_real_block");
            fermi_precondition(h->plan, h->have_spp ? &h->spp : nullptr, h->gw, cfg, h->V, h->V32, h->lr_pad,
                               h->lr_Y + (size_t)c0 * n, cols, s);
            ++h->precond_calls;
        }
        // step 5: rank-revealing QR of Y through its Gram matrix: the column order and R of
        // the first N steps of a column-pivoted QR, by pivoted Cholesky of Y^H Y (c x c, host)
        cplx<double>* Gm = h->lr_small;
        lr_gram(h, h->lr_Y, h->lr_Y, ncols, Gm);
        std::vector<cd> Gh((size_t)ncols * ncols);
        POMM_HIP(hipMemcpyAsync(Gh.data(), Gm, sizeof(cd) * Gh.size(), hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        std::vector<int> piv;
        std::vector<cd> R;
        POMM_CHECK(pivoted_cholesky(Gh, ncols, N, piv, R), OMM_ESPECTRUM,
                   "the filtered random block has rank below N");
        const double tiny = 1e-13 * std::abs(R[0]);
        POMM_CHECK(std::abs(R[(N - 1) + (size_t)(N - 1) * N]) > tiny, OMM_ESPECTRUM,
                   "the filtered random block has rank below N");
        std::vector<cd> Ri = upper_inverse(R, N);
        // step 6: U = Y(:, piv[0:N]) R^{-1}; a second Cholesky pass restores orthogonality
        // lost to the Gram matrix's squared condition number
        cplx<double>* Rd = h->lr_small + (size_t)4 * N * N;
        POMM_HIP(hipMemcpyAsync(h->lr_piv, piv.data(), sizeof(int) * N, hipMemcpyHostToDevice, s));
        POMM_HIP(hipMemcpyAsync(Rd, Ri.data(), sizeof(cd) * Ri.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(lr_gather, dim3(256), dim3(256), 0, s, h->lr_Y, n, h->lr_piv, N, h->lr_pad);
        check_launch("lr_gather");
        lr_gemm(h, h->lr_U, h->lr_pad, Rd, N, N);
        lr_gram(h, h->lr_U, h->lr_U, N, Gm);
        std::vector<cd> G2((size_t)N * N);
        POMM_HIP(hipMemcpyAsync(G2.data(), Gm, sizeof(cd) * G2.size(), hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        std::vector<cd> R2;
        POMM_CHECK(cholesky_upper(G2, N, R2), OMM_ESPECTRUM, "orthogonalization failed");
        std::vector<cd> R2i = upper_inverse(R2, N);
        POMM_HIP(hipMemcpyAsync(Rd, R2i.data(), sizeof(cd) * R2i.size(), hipMemcpyHostToDevice, s));
        lr_gemm(h, h->lr_pad, h->lr_U, Rd, N, N);
        std::swap(h->lr_U, h->lr_pad);
        POMM_HIP(hipStreamSynchronize(s));
        h->lowrank = true;
        return OMM_OK;
    } catch (const Error& e) {
        h->lowrank = false;
        return fail(h, e);
    }
}

extern "C" int ommPrecondition(omm_handle_t h, const void* G, void* PG, int ncols, double rtol) {
    if (!h) return OMM_EINVAL;
    ProfBind pb(h);
    try {
        POMM_CHECK(G && PG && G != PG, OMM_EINVAL, "bad pointers");
        POMM_CHECK(ncols >= 1 && ncols <= h->N, OMM_EINVAL, "ncols must be in 1..N");
        if (h->opts.outer != OMM_OUTER_FERMI) {
            outer_apply(h, (const cplx<double>*)G, (cplx<double>*)PG, ncols);
        } else if (h->lowrank) {
            lowrank_apply(h, (const cplx<double>*)G, (cplx<double>*)PG, ncols);
        } else {
            const PrecondConfig cfg = precond_config(h, rtol > 0 ? rtol : h->opts.gmres_rtol);
            fermi_precondition(h->plan, h->have_spp ? &h->spp : nullptr, h->gw, cfg, h->V, h->V32,
                               (const cplx<double>*)G, (cplx<double>*)PG, ncols, h->stream);
        }
        ++h->precond_calls;
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

extern "C" int ommApplyInner(omm_handle_t h, int pole, const void* B, void* Y, int ncols) {
    if (!h) return OMM_EINVAL;
    ProfBind pb(h);
    try {
        POMM_CHECK(B && Y && B != Y, OMM_EINVAL, "bad pointers");
        inner_apply(h->plan, h->have_spp ? &h->spp : nullptr, h->gw, precond_config(h, h->opts.gmres_rtol), pole,
                    (const cplx<double>*)B, (cplx<double>*)Y, ncols, h->stream);
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

// Point the Gram pointer lists and the gradient task at the caller's X.
static void bind_x(omm_ctx* h, cplx<double>* X) {
    if (h->bound_X == X) return;
    const cplx<double>* P[6] = {X, X, X, h->D, X, h->D};
    const cplx<double>* Q[6] = {X, h->HX, h->D, h->D, h->HD, h->HD};
    POMM_HIP(hipMemcpyAsync(h->gram_P, P, sizeof(P), hipMemcpyHostToDevice, h->stream));
    POMM_HIP(hipMemcpyAsync(h->gram_Q, Q, sizeof(Q), hipMemcpyHostToDevice, h->stream));
    // G = 2 G - X A0 - HX S0 with G preloaded with HX
    GemmTask<double> t{};
    t.C = h->Gr;
    t.ldc = h->n;
    t.beta = 2.0;
    t.gate = -1;
    t.nterms = 2;
    const long NN = (long)h->N * h->N;
    t.t[0] = GemmTerm<double>{X, h->grams + NN, h->n, h->N, -1.0, 0.0};
    t.t[1] = GemmTerm<double>{h->HX, h->grams, h->n, h->N, -1.0, 0.0};
    POMM_HIP(hipMemcpyAsync(h->grad_task, &t, sizeof(t), hipMemcpyHostToDevice, h->stream));
    POMM_HIP(hipStreamSynchronize(h->stream));
    h->bound_X = X;
}

extern "C" int ommSolve(omm_handle_t h, void* Xv, omm_info_t* info) {
    if (!h) return OMM_EINVAL;
    ProfBind pb(h);
    try {
        POMM_CHECK(Xv != nullptr, OMM_EINVAL, "X is NULL");
        cplx<double>* X = (cplx<double>*)Xv;
        const int n = h->n, N = h->N;
        const long cnt = (long)n * N;
        const size_t blk = sizeof(cplx<double>) * cnt;
        hipStream_t s = h->stream;
        const omm_opts_t& o = h->opts;
        bind_x(h, X);
        long long steps0 = 0, calls0 = h->precond_calls;
        POMM_HIP(hipMemcpyAsync(&steps0, h->gw.steps, sizeof(steps0), hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        auto apply_h = [&](const cplx<double>* in, cplx<double>* outp) {
            SpecArgs<double> a;
            a.in = in;
            a.ld_in = n;
            a.out = outp;
            a.ld_out = n;
            a.ncols = N;
            a.post_mode = POST_SHIFTED_H;
            a.V = h->V;
            a.sigma = h->sigma;
            spectral_apply<double>(h->plan, a, h->gw.work, s);
        };
        auto precondition = [&](const cplx<double>* G, cplx<double>* PGo, double rtol) {
            if (o.outer != OMM_OUTER_FERMI)   // Section 3.1's comparison preconditioners
                outer_apply(h, G, PGo, N);
            else if (h->lowrank)   // the precomputed U U* (Section 3.3)
                lowrank_apply(h, G, PGo, N);
            else
                fermi_precondition(h->plan, h->have_spp ? &h->spp : nullptr, h->gw, precond_config(h, rtol), h->V,
                                   h->V32, G, PGo, N, s);
            ++h->precond_calls;
        };
        // a8: filter the starting block, X1 = P X0
        if (o.filter && o.outer == OMM_OUTER_FERMI) {
            POMM_HIP(hipMemcpyAsync(h->Gp, X, blk, hipMemcpyDeviceToDevice, s));
            precondition(h->Gp, X, o.filter_rtol);
        }
        const double gram_flops = 8.0 * n * (double)N * N;
        apply_h(X, h->HX);
        {
            ProfScope prof(PK_OMM, 2.0 * blk, 2 * gram_flops, s, 2);
            gram_products(h->gram, h->gram_P, h->gram_Q, 2, h->parts, h->grams, s);   // S0, A0
        }
        const double eps = std::numeric_limits<double>::epsilon();
        double Eprev = 0.0;
        int flat = 0, it = 0, status = OMM_OK, rule = OMM_STOP_MAXIT;
        double E = 0.0, rg = 0.0;
        for (it = 0;; ++it) {
            // a3: G = 2HX - X A0 - HX S0 ; a9: norms and energy
            {
                ProfScope prof(PK_OMM, 4.0 * blk, 2 * gram_flops, s, 5);
                POMM_HIP(hipMemcpyAsync(h->Gr, h->HX, blk, hipMemcpyDeviceToDevice, s));
                gemm_batched<double>(h->grad_task, 1, n, N, N, nullptr, s);
                grad_norms(h->Gr, h->HX, cnt, h->red, h->sc, s);
                energy_from_grams(h->grams, N, h->sc, s);
            }
            POMM_HIP(hipMemcpyAsync(h->sc_host, h->sc, sizeof(OmmScalars), hipMemcpyDeviceToHost, s));
            POMM_HIP(hipStreamSynchronize(s));
            E = h->sc_host->energy;
            rg = std::sqrt(h->sc_host->gnorm2 / h->sc_host->hxnorm2);
            if (it > 0 && std::fabs(E - Eprev) <= 8.0 * eps * std::fabs(E)) ++flat;
            else flat = 0;
            Eprev = E;
            if (!std::isfinite(E) || !std::isfinite(rg)) { status = OMM_EBREAKDOWN; break; }
            if (rg <= o.tol) { rule = OMM_STOP_GRAD; break; }
            if (o.stall && flat >= o.stall) { rule = OMM_STOP_ENERGY; break; }
            if (it == o.maxit) { status = OMM_ENOCONV; rule = OMM_STOP_MAXIT; break; }
            // a6: PG = P G(X);  a5: direction
            precondition(h->Gr, h->PG, o.gmres_rtol);
            {
                ProfScope prof(PK_OMM, 4.0 * blk, 8.0 * cnt, s, 3);
                cg_direction(h->PG, h->Gp, h->D, cnt, it == 0, h->red, h->sc, s);
            }
            // a1: HD ; a2: Gram products ; a4: exact line search ; a5: update
            apply_h(h->D, h->HD);
            {
                ProfScope prof(PK_OMM, 4.0 * blk + 4.0 * blk, 6 * gram_flops, s, 4);
                gram_products(h->gram, h->gram_P, h->gram_Q, 6, h->parts, h->grams, s);
                quartic_step(h->grams, N, h->sc, s);
                step_update(X, h->HX, h->D, h->HD, cnt, h->sc, s);
            }
            POMM_HIP(hipMemcpyAsync(h->sc_host, h->sc, sizeof(OmmScalars), hipMemcpyDeviceToHost, s));
            POMM_HIP(hipStreamSynchronize(s));
            if (h->sc_host->breakdown) { status = OMM_EBREAKDOWN; break; }
        }
        long long steps1 = 0;
        POMM_HIP(hipMemcpyAsync(&steps1, h->gw.steps, sizeof(steps1), hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        if (info) {
            info->iters = it;
            info->status = status;
            info->stop_rule = rule;
            info->energy = E;
            info->rel_grad = rg;
            info->gmres_steps = steps1 - steps0;
            info->precond_calls = h->precond_calls - calls0;
            info->sigma = h->sigma;
        }
        if (status != OMM_OK) h->err = ommStatusString(status);
        if (h->prof.on) h->prof.collect();
        return status;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

extern "C" int ommSolveBatched(omm_handle_t* hs, int count, void* const* Xs, omm_info_t* infos) {
    if (count < 0 || (count > 0 && (!hs || !Xs))) return OMM_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !Xs[i]) return OMM_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return OMM_EINVAL;   // a handle is driven by one thread at a time
    }
    if (count == 0) return OMM_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return OMM_EHIP;
    // one host thread per instance, up to 16: each drives its handle's stream, so the
    // instances' kernels overlap on the device (as far as their streams are distinct)
    const int nthreads = std::min(count, 16);
    std::atomic<int> next{0};
    std::vector<int> status(count, OMM_OK);
    auto worker = [&]() {
        if (hipSetDevice(dev) != hipSuccess) return;
        for (int i = next++; i < count; i = next++) status[i] = ommSolve(hs[i], Xs[i], infos ? &infos[i] : nullptr);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    for (int i = 0; i < count; ++i)
        if (status[i] != OMM_OK) return status[i];
    return OMM_OK;
}

extern "C" int ommSetProfilingClasses(omm_handle_t h, unsigned mask) {
    if (!h) return OMM_EINVAL;
    try {
        h->prof.reset();
        h->prof.mask = mask & ((1u << PK_COUNT) - 1u);
        h->prof.on = h->prof.mask != 0;
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

extern "C" int ommSetProfiling(omm_handle_t h, int on) { return ommSetProfilingClasses(h, on ? ~0u : 0u); }

extern "C" int ommGetProfile(omm_handle_t h, double* ms, double* bytes, double* flops, long long* launches) {
    if (!h) return OMM_EINVAL;
    try {
        h->prof.collect();
        for (int k = 0; k < PK_COUNT; ++k) {
            if (ms) ms[k] = h->prof.stats.ms[k];
            if (bytes) bytes[k] = h->prof.stats.bytes[k];
            if (flops) flops[k] = h->prof.stats.flops[k];
            if (launches) launches[k] = h->prof.stats.launches[k];
        }
        return OMM_OK;
    } catch (const Error& e) {
        return fail(h, e);
    }
}

extern "C" const char* ommProfileClassName(int cls) { return prof_kind_name(cls); }

// ---- spectral window estimate (no handle): Chebyshev-filtered subspace iteration with
// Rayleigh-Ritz on a block of s >= N + 2 columns.  The contour of the pole set needs lo <=
// lambda_1, homo >= lambda_N and lumo <= lambda_{N+1}.  lo = min V (T is positive
// semidefinite); homo and lumo come from the N-th and (N+1)-th Ritz values of the block once
// their residuals are small: the i-th Ritz value of any subspace is at least lambda_i
// (Cauchy interlacing), and an eigenvalue lies within the residual norm of a Ritz value.

// y = a t + b y (b = 0: y = a t, whatever y held), complex128, real a and b
__global__ static void est_axpby(const cplx<double>* __restrict__ t, cplx<double>* __restrict__ y, long total,
                                 double a, double b) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const cplx<double> u = t[e];
        if (b == 0.0) {
            y[e] = mk<double>(a * u.re, a * u.im);
        } else {
            const cplx<double> v = y[e];
            y[e] = mk<double>(a * u.re + b * v.re, a * u.im + b * v.im);
        }
    }
}

// Eigen-decomposition of the real symmetric s x s matrix A (column major) by cyclic Jacobi
// sweeps: eigenvalues ascending in lam, unit eigenvectors in the columns of W in the same
// order.  The first three sweeps rotate only elements above a fifth of the mean off-diagonal
// size; from the fifth on, elements negligible against both diagonal entries are set to zero;
// sweeps stop once the off-diagonal mass is 1e-32 of the whole.
static void symmetric_eig(std::vector<double> A, int s, std::vector<double>& lam, std::vector<double>& W) {
    std::vector<double> U((size_t)s * s, 0.0);
    for (int i = 0; i < s; ++i) U[i + (size_t)i * s] = 1.0;
    auto at = [&](int i, int j) -> double& { return A[i + (size_t)j * s]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int q = 0; q < s; ++q) {
            diag += at(q, q) * at(q, q);
            for (int p = 0; p < q; ++p) off += at(p, q) * at(p, q);
        }
        if (off <= 1e-32 * (diag + 2.0 * off)) break;
        const double thresh = sweep < 3 ? 0.2 * std::sqrt(off) / ((double)s * s) : 0.0;
        for (int p = 0; p < s - 1; ++p)
            for (int q = p + 1; q < s; ++q) {
                const double apq = at(p, q);
                const double g = 100.0 * std::fabs(apq);
                if (sweep > 3 && std::fabs(at(p, p)) + g == std::fabs(at(p, p)) &&
                    std::fabs(at(q, q)) + g == std::fabs(at(q, q))) {
                    at(p, q) = at(q, p) = 0.0;
                    continue;
                }
                if (apq == 0.0 || std::fabs(apq) <= thresh) continue;
                const double tau = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < s; ++k) {   // A <- A G and U <- U G on columns p, q
                    const double x = at(k, p), y = at(k, q);
                    at(k, p) = c * x - sn * y;
                    at(k, q) = sn * x + c * y;
                    const double u = U[k + (size_t)p * s], v = U[k + (size_t)q * s];
                    U[k + (size_t)p * s] = c * u - sn * v;
                    U[k + (size_t)q * s] = sn * u + c * v;
                }
                for (int k = 0; k < s; ++k) {   // A <- G^T A on rows p, q
                    const double x = at(p, k), y = at(q, k);
                    at(p, k) = c * x - sn * y;
                    at(q, k) = sn * x + c * y;
                }
                at(p, q) = at(q, p) = 0.0;
            }
    }
    std::vector<int> ord(s);
    for (int i = 0; i < s; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return at(a, a) < at(b, b); });
    lam.resize(s);
    W.assign((size_t)s * s, 0.0);
    for (int j = 0; j < s; ++j) {
        lam[j] = at(ord[j], ord[j]);
        for (int k = 0; k < s; ++k) W[k + (size_t)j * s] = U[k + (size_t)ord[j] * s];
    }
}

namespace {

struct Estimator {
    hipStream_t s = nullptr;
    SpectralPlan plan;
    int n = 0, cols = 0;
    double* V = nullptr;
    cplx<double>* buf[4] = {nullptr, nullptr, nullptr, nullptr};   // n x cols each
    cplx<double>* work = nullptr;     // multi-pass FFT scratch (large grids)
    cplx<double>* small = nullptr;    // 3 cols^2: Gram, triangular inverse / W, W Theta
    cplx<double>* parts = nullptr;
    const cplx<double>** ptrs = nullptr;
    GemmTask<double>* task = nullptr;
    long applies = 0;

    ~Estimator() {
        if (s) (void)hipStreamSynchronize(s);
        for (void* p : {(void*)V, (void*)buf[0], (void*)buf[1], (void*)buf[2], (void*)buf[3], (void*)work,
                        (void*)small, (void*)parts, (void*)ptrs, (void*)task})
            if (p) (void)dev_free(p);
        spectral_plan_free(plan);
    }
    // out = (H - shift) in, all columns; with comb_a set: out = comb_a (H - shift) in + comb_b out
    // (in the spectral kernel's epilogue where the register kernel serves this grid)
    void happly(const cplx<double>* in, cplx<double>* out, double shift, double comb_a = 0.0, double comb_b = 0.0) {
        SpecArgs<double> a;
        if (comb_a != 0.0) {
            a.comb = out;
            a.comb_a = comb_a;
            a.comb_b = comb_b;
        }
        a.in = in;
        a.ld_in = n;
        a.out = out;
        a.ld_out = n;
        a.ncols = cols;
        a.cols_per_group = cols;
        a.mult_mode = MULT_KINETIC;
        a.post_mode = POST_SHIFTED_H;
        a.V = V;
        a.sigma = shift;
        spectral_apply<double>(plan, a, work, s);
        ++applies;
    }
    // out (cols x cols, device) = P^H Q
    void gram(const cplx<double>* P, const cplx<double>* Q, cplx<double>* out) {
        const cplx<double>* ptr[2] = {P, Q};
        POMM_HIP(hipMemcpyAsync(ptrs, ptr, sizeof(ptr), hipMemcpyHostToDevice, s));
        POMM_HIP(hipStreamSynchronize(s));   // ptr is a host temporary
        gram_products(gram_plan(n, cols), ptrs, ptrs + 1, 1, parts, out, s);
    }
    std::vector<cd> download(const cplx<double>* d) {
        std::vector<cd> h((size_t)cols * cols);
        POMM_HIP(hipMemcpyAsync(h.data(), d, sizeof(cd) * h.size(), hipMemcpyDeviceToHost, s));
        POMM_HIP(hipStreamSynchronize(s));
        return h;
    }
    void upload(cplx<double>* d, const std::vector<cd>& h) {
        POMM_HIP(hipMemcpyAsync(d, h.data(), sizeof(cd) * h.size(), hipMemcpyHostToDevice, s));
        POMM_HIP(hipStreamSynchronize(s));   // h is a host temporary
    }
    // C = A1 M1 + alpha2 A2 M2 (n x cols; M small, device, cols x cols); A2 may be null
    void gemm(cplx<double>* C, const cplx<double>* A1, const cplx<double>* M1, const cplx<double>* A2 = nullptr,
              const cplx<double>* M2 = nullptr, double alpha2 = 0.0) {
        GemmTask<double> t{};
        t.C = C;
        t.ldc = n;
        t.beta = 0.0;
        t.gate = -1;
        t.nterms = A2 ? 2 : 1;
        t.t[0] = GemmTerm<double>{A1, M1, n, cols, 1.0, 0.0};
        if (A2) t.t[1] = GemmTerm<double>{A2, M2, n, cols, alpha2, 0.0};
        POMM_HIP(hipMemcpyAsync(task, &t, sizeof(t), hipMemcpyHostToDevice, s));
        POMM_HIP(hipStreamSynchronize(s));   // t is a host temporary
        gemm_batched<double>(task, 1, n, cols, cols, nullptr, s);
    }
    // Y <- Y R^{-1} with Y^H Y = R^H R, twice (CholeskyQR2); the buffers Y and tmp trade places
    void orthonormalize(cplx<double>*& Y, cplx<double>*& tmp) {
        for (int pass = 0; pass < 2; ++pass) {
            gram(Y, Y, small);
            std::vector<cd> R;
            POMM_CHECK(cholesky_upper(download(small), cols, R), OMM_ESPECTRUM,
                       "the filtered block lost rank (lower the filter degree)");
            upload(small + (size_t)cols * cols, upper_inverse(R, cols));
            gemm(tmp, Y, small + (size_t)cols * cols);
            std::swap(Y, tmp);
        }
    }
    // Rayleigh-Ritz on the orthonormal block Q: Ritz values theta (ascending), Ritz vectors
    // X = Q W and their residual norms |H x_i - theta_i x_i|.  Uses HQ and R as scratch.
    void rayleigh_ritz(const cplx<double>* Q, cplx<double>* X, cplx<double>* HQ, cplx<double>* R,
                       std::vector<double>& theta, std::vector<double>& res) {
        happly(Q, HQ, 0.0);
        gram(Q, HQ, small);
        // H is real symmetric and the start block real, so the whole iteration is real: the
        // Ritz matrix is the real symmetric part of the Gram product (its imaginary parts and
        // asymmetry are rounding)
        const std::vector<cd> G = download(small);
        std::vector<double> Gr((size_t)cols * cols);
        for (int j = 0; j < cols; ++j)
            for (int i = 0; i < cols; ++i)
                Gr[i + (size_t)j * cols] = 0.5 * (G[i + (size_t)j * cols].real() + G[j + (size_t)i * cols].real());
        std::vector<double> Wr;
        symmetric_eig(Gr, cols, theta, Wr);
        std::vector<cd> W((size_t)cols * cols), WT((size_t)cols * cols);
        for (int j = 0; j < cols; ++j)
            for (int i = 0; i < cols; ++i) {
                W[i + (size_t)j * cols] = Wr[i + (size_t)j * cols];
                WT[i + (size_t)j * cols] = Wr[i + (size_t)j * cols] * theta[j];
            }
        upload(small + (size_t)cols * cols, W);
        upload(small + (size_t)2 * cols * cols, WT);
        gemm(X, Q, small + (size_t)cols * cols);
        gemm(R, HQ, small + (size_t)cols * cols, Q, small + (size_t)2 * cols * cols, -1.0);
        gram(R, R, small);
        const std::vector<cd> RR = download(small);
        res.resize(cols);
        for (int j = 0; j < cols; ++j) res[j] = std::sqrt(std::max(0.0, RR[j + (size_t)j * cols].real()));
    }
};

// Chebyshev filter step count that keeps the filtered block's condition near 1e6: the
// polynomial grows like cosh(d acosh|x|) at x = (a0 - c)/e, so d <= acosh(1e6)/acosh|x|.
static int filter_degree(int dmax, double a0, double a, double b) {
    const double e = 0.5 * (b - a), c = 0.5 * (b + a);
    const double x = std::fabs((a0 - c) / e);
    if (!(x > 1.0)) return dmax;
    const double d = std::acosh(1e6) / std::acosh(x);
    return std::max(1, std::min(dmax, (int)d));
}

}  // namespace

// The estimate behind ommEstimateSpectrum (and ommSetup without a window): OMM_OK or
// OMM_ENOCONV; other failures throw.
static int estimate_window(const omm_grid_t* grid, const double* V, int N, const double* B, int ncols, int degree,
                           double tol, int maxit, void* stream, omm_spectrum_t* spec, omm_estimate_info_t* info) {
    {
        POMM_CHECK(grid && V && B && spec, OMM_EINVAL, "NULL argument");
        POMM_CHECK(grid->dim == 2 || grid->dim == 3, OMM_EINVAL, "dim must be 2 or 3");
        const int m = grid->m[0];
        for (int i = 1; i < grid->dim; ++i) POMM_CHECK(grid->m[i] == m, OMM_EINVAL, "grid must be cubic (equal m)");
        if (degree <= 0) degree = 100;
        if (!(tol > 0.0)) tol = 1e-6;
        if (maxit <= 0) maxit = 50;
        POMM_CHECK(degree <= 1000, OMM_EINVAL, "degree must be at most 1000");
        Estimator E;
        E.s = (hipStream_t)stream;
        int dev = 0, lds = 0;
        POMM_HIP(hipGetDevice(&dev));
        POMM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        spectral_plan_init(E.plan, grid->dim, m, (size_t)lds);
        const int n = E.plan.n;
        E.n = n;
        POMM_CHECK(N >= 1 && ncols >= N + 2 && ncols <= n / 2, OMM_EINVAL, "need 1 <= N and N + 2 <= ncols <= n/2");
        E.cols = ncols;
        double vmin = V[0], vmax = V[0];
        for (int i = 0; i < n; ++i) {
            POMM_CHECK(std::isfinite(V[i]), OMM_EINVAL, "V has non-finite entries");
            vmin = std::min(vmin, V[i]);
            vmax = std::max(vmax, V[i]);
        }
        const double hi = 0.5 * grid->dim * (double)(m / 2) * (double)(m / 2) + vmax;   // >= lambda_n
        hipStream_t s = E.s;
        const size_t blk = (size_t)n * ncols;
        POMM_HIP(dev_alloc(&E.V, sizeof(double) * n));
        POMM_HIP(hipMemcpyAsync(E.V, V, sizeof(double) * n, hipMemcpyHostToDevice, s));
        for (auto& b : E.buf) POMM_HIP(dev_alloc(&b, sizeof(cplx<double>) * blk));
        if (spectral_needs_work<double>(E.plan)) POMM_HIP(dev_alloc(&E.work, sizeof(cplx<double>) * blk));
        POMM_HIP(dev_alloc(&E.small, sizeof(cplx<double>) * 3 * (size_t)ncols * ncols));
        POMM_HIP(dev_alloc(&E.parts, sizeof(cplx<double>) * gram_parts_elems(gram_plan(n, ncols), 1)));
        POMM_HIP(dev_alloc(&E.ptrs, sizeof(void*) * 2));
        POMM_HIP(dev_alloc(&E.task, sizeof(GemmTask<double>)));
        cplx<double>* X = E.buf[0];   // Ritz vectors (orthonormal)
        cplx<double>* Y = E.buf[1];   // filter iterate
        cplx<double>* T = E.buf[2];   // (H - c) Y, then scratch
        cplx<double>* U = E.buf[3];   // scratch
        hipLaunchKernelGGL(lr_real_block, dim3(256), dim3(256), 0, s, B, n, ncols, ncols, Y);
        check_launch("lr_real_block");
        std::vector<double> theta, res;
        E.orthonormalize(Y, T);
        E.rayleigh_ritz(Y, X, T, U, theta, res);
        auto converged = [&]() {
            for (int i = 0; i <= N; ++i)
                if (!(res[i] <= tol * std::max(1.0, std::fabs(theta[i])))) return false;
            return true;
        };
        int it = 0;
        for (; it < maxit && !converged(); ++it) {
            // p(H) X, p the Chebyshev polynomial of degree d for [a, b] = [largest Ritz value,
            // upper bound], scaled to 1 at a0 = smallest Ritz value (three-term recurrence
            // with the scaling of Zhou and Saad's filtered subspace iteration)
            const double b = hi, a0 = theta[0];
            const double a = std::min(theta[ncols - 1], b - 1e-3 * (b - a0));
            const int d = filter_degree(degree, a0, a, b);
            const double e = 0.5 * (b - a), c = 0.5 * (b + a);
            double sigma = e / (a0 - c);
            const double tau = 2.0 / sigma;
            const bool fused = spectral_reg_available<double>(E.plan);
            if (fused) {
                E.happly(X, Y, c, sigma / e, 0.0);
            } else {
                E.happly(X, T, c);
                hipLaunchKernelGGL(est_axpby, dim3(1024), dim3(256), 0, s, T, Y, (long)blk, sigma / e, 0.0);
                check_launch("est_axpby");
            }
            for (int k = 2; k <= d; ++k) {
                const double sn = 1.0 / (tau - sigma);
                if (fused) {   // X <- (2 sn/e) (H - c) Y - sigma sn X in the spectral epilogue
                    E.happly(Y, X, c, 2.0 * sn / e, -sigma * sn);
                } else {
                    E.happly(Y, T, c);
                    hipLaunchKernelGGL(est_axpby, dim3(1024), dim3(256), 0, s, T, X, (long)blk, 2.0 * sn / e,
                                       -sigma * sn);
                    check_launch("est_axpby");
                }
                std::swap(X, Y);
                sigma = sn;
            }
            E.orthonormalize(Y, T);
            E.rayleigh_ritz(Y, X, T, U, theta, res);
        }
        spec->lo = vmin;
        spec->homo = theta[N - 1];
        spec->lumo = theta[N] - res[N];
        POMM_HIP(hipStreamSynchronize(s));
        if (info) {
            info->iters = it;
            info->applies = (int)E.applies;
            info->converged = converged() ? 1 : 0;
            info->res_homo = res[N - 1];
            info->res_lumo = res[N];
        }
        POMM_CHECK(spec->lumo > spec->homo, OMM_ESPECTRUM, "no gap between the N-th and (N+1)-th Ritz values");
        return converged() ? OMM_OK : OMM_ENOCONV;
    }
}

extern "C" int ommEstimateSpectrum(const omm_grid_t* grid, const double* V, int N, const double* B, int ncols,
                                   int degree, double tol, int maxit, void* stream, omm_spectrum_t* spec,
                                   omm_estimate_info_t* info) {
    AllocBind ab((hipStream_t)stream);
    try {
        return estimate_window(grid, V, N, B, ncols, degree, tol, maxit, stream, spec, info);
    } catch (const Error& e) {
        return fail(nullptr, e);
    }
}

// Start block of the window estimate inside ommSetup: entries uniform in [-1, 1) from the
// SplitMix64 generator (Steele, Lea and Flood) of state seed + (e + 1) * 0x9E3779B97F4A7C15.
__global__ static void start_block_kernel(double* __restrict__ B, long total, unsigned long long seed) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        unsigned long long z = seed + (unsigned long long)(e + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        B[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

static int setup_estimate_window(const omm_grid_t* grid, const double* V, int N, int n, hipStream_t s,
                                 omm_spectrum_t* spec) {
    const int cols = std::min(N + 8, n / 2);
    POMM_CHECK(N + 2 <= cols, OMM_EINVAL, "the window estimate needs N + 2 <= n/2");
    struct Buf {
        double* p = nullptr;
        ~Buf() {
            if (p) (void)dev_free(p);
        }
    } B;
    POMM_HIP(dev_alloc(&B.p, sizeof(double) * (size_t)n * cols));
    hipLaunchKernelGGL(start_block_kernel, dim3(1024), dim3(256), 0, s, B.p, (long)n * cols, 1603ull);
    check_launch("start_block");
    const int rc = estimate_window(grid, V, N, B.p, cols, 0, 0.0, 0, s, spec, nullptr);
    POMM_CHECK(rc == OMM_OK, OMM_ESPECTRUM, "the spectral window estimate did not converge");
    return OMM_OK;
}

extern "C" int ommGetSpectrum(omm_handle_t h, omm_spectrum_t* spec) {
    if (!h || !spec) return OMM_EINVAL;
    *spec = h->spec;
    return OMM_OK;
}
