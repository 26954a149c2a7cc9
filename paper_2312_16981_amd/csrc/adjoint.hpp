// Recording of the forward run and the reverse sweep of the adjoint of the
// frozen-tally macroscopic map (adjoint.hip).
//
// Per recorded step the forward run stores what its macroscopic solve was
// given besides the opacity: the static source Q (which holds rho^n, the wave
// flux and the net particle flux), rho^h, the sampled flags that choose
// C4 - e^{-s} or C4 in the wave flux (Remark 3), and the converged T^{n+1}.
// The reverse sweep differentiates, step by step from the last, the map
// (rho^n, T^n, kappa) -> (rho^{n+1}, T^{n+1}) with those particle results
// held fixed: a transposed source iteration for the cotangent mu of T^{n+1},
// then the cotangents of Q, lambda, sigma, D_f (harmonic face opacity and C2)
// and A (C4 or W), accumulated into dJ/dkappa, and the cotangent of rho^n.
#pragma once
#include <hip/hip_runtime.h>
#include "common.hpp"
#include "device_math.hpp"

namespace ugk {

struct AdjResid {
    unsigned long long dmu, mu;     // max |mu^{k+1} - mu^k|, max |mu^{k+1}| as IEEE bits
};

enum { ADJ_CONV = 0, ADJ_ERR = 1, ADJ_CGU = 2, ADJ_MAXK = 3, ADJ_N_STATUS = 4 };

struct Adj {
    // record: step r occupies [r * n_cg, (r+1) * n_cg) and [r * ncell, (r+1) * ncell)
    double* rQ;
    double* rRhoh;
    uint8_t* rSamp;
    double* rT;
    // reverse sweep
    double* phi;          // [n_cg] phi_g(T^{n+1})
    double* dphi;         // [n_cg] d phi_g / dT at T^{n+1}
    double* rbar;         // [n_cg] cotangent of rho^{n+1}
    double* rbar_next;    // [n_cg] cotangent of rho^n
    double* mu0;          // [ncell] iterates of the transposed source iteration
    double* mu1;
    double* Tbar;         // [ncell] cotangent of T^{n+1}
    double* grad;         // [n_cg] dJ/dkappa, accumulated over steps
    double* c4d;          // [n_cg] dC4/ds
    double* wd;           // [n_cg] dW/ds
    double* Dlx;          // [x-face slots] dD_f/dsigma of the cell on the low side
    double* Dhx;          //                and of the cell on the high side
    double* Dly;          // [y-face slots]
    double* Dhy;
    AdjResid* res;        // [n_inst][RES_SLOTS][RES_SUB]
    int* conv;            // [n_inst] sweeps at convergence, 0 while running
    unsigned long long* status;   // ADJ_CONV: converged instances, ADJ_ERR: non-finite seen,
                                  // ADJ_CGU: (cell, group) updates of the converged sweeps,
                                  // ADJ_MAXK: most sweeps an instance needed
};

hipError_t set_head_series_adj(const HeadSeries& hs);
void launch_rec_store(const Dev& D, const Consts& K, const Adj& A, int r, hipStream_t st);
void launch_adj_coef(const Dev& D, const Consts& K, const Adj& A, hipStream_t st);
void launch_adj_face(const Dev& D, const Consts& K, const Adj& A, int inst, int axis, int64_t nslots,
                     hipStream_t st);
void launch_adj_prep(const Dev& D, const Consts& K, const Adj& A, int r, hipStream_t st);
// sweep k of the transposed iteration followed by its convergence decision
void launch_adj_sweep(const Dev& D, const Consts& K, const Adj& A, int k, hipStream_t st);
void launch_adj_grad(const Dev& D, const Consts& K, const Adj& A, int r, hipStream_t st);

}  // namespace ugk
