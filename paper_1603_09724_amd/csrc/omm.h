// Kernels of the outer OMM iteration (Algorithm 1 with an exact quartic line search).
#pragma once

#include "common.h"

namespace pomm {

// Device scalar block shared by the OMM kernels.
struct OmmScalars {
    double c[5];        // quartic coefficients of E(X + a D)
    double alpha;       // line-search step
    double energy;      // E_omm of the current X
    double gnorm2;      // ||G(X)||_F^2
    double hxnorm2;     // ||H_sigma X||_F^2
    double dot_gdg;     // Re <G, G - G_prev>
    double dot_gpgp;    // Re <G_prev, G_prev>
    double beta;
    int breakdown;      // 1: leading coefficient <= 0 or not finite
    int pad;
};

// grams: 6 consecutive N x N matrices S0 = X*X, A0 = X*HX, C = X*D, S2 = D*D,
// B = X*HD, A2 = D*HD.  Computes c0..c4, the minimizing alpha, E(alpha), and
// replaces S0, A0 by S(alpha), A(alpha).
void quartic_step(cplx<double>* grams, int N, OmmScalars* sc, hipStream_t s);

// E = tr A0 - 1/2 tr(S0 A0) from the first two Gram matrices.
void energy_from_grams(const cplx<double>* grams, int N, OmmScalars* sc, hipStream_t s);

// X += alpha D and HX += alpha HD (alpha from sc).
void step_update(cplx<double>* X, cplx<double>* HX, const cplx<double>* D, const cplx<double>* HD, long count,
                 const OmmScalars* sc, hipStream_t s);

// ||G||^2 and ||HX||^2 into sc (deterministic two-stage reduction; parts >= 2*256 doubles).
void grad_norms(const cplx<double>* G, const cplx<double>* HX, long count, double* parts, OmmScalars* sc,
                hipStream_t s);

// Polak-Ribiere: G = -PG; if first: D = G, else beta = max(0, Re<G, G-Gp>/Re<Gp,Gp>), D = G + beta D.  Gp <- G.
void cg_direction(const cplx<double>* PG, cplx<double>* Gp, cplx<double>* D, long count, int first, double* parts,
                  OmmScalars* sc, hipStream_t s);

}  // namespace pomm
