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

// Status words: ADJ_CONV converged instances of the reverse step in progress
// (cleared by its set-up), ADJ_ERR non-finite value seen, ADJ_CGU (cell, group)
// updates of the converged sweeps so far, ADJ_MAXK most sweeps any reverse step
// needed so far, ADJ_DONE reverse steps completed (the gate of the next one).
enum { ADJ_CONV = 0, ADJ_ERR = 1, ADJ_CGU = 2, ADJ_MAXK = 3, ADJ_DONE = 4, ADJ_N_STATUS = 5 };

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
    int* stepk;           // [record steps] most sweeps an instance needed in that step
    unsigned long long* status;   // ADJ_* words
};

hipError_t set_head_series_adj(const HeadSeries& hs);
void launch_rec_store(const Dev& D, const Consts& K, const Adj& A, int r, hipStream_t st);
void launch_adj_coef(const Dev& D, const Consts& K, const Adj& A, hipStream_t st);
void launch_adj_face(const Dev& D, const Consts& K, const Adj& A, int inst, int axis, int64_t nslots,
                     hipStream_t st);
// The launches of reverse step q (recorded step r = nrec - 1 - q) carry q as
// their gate: they run only when q reverse steps are done (GATE_OFF: always),
// so reverse steps can be enqueued ahead and the ones behind a step that did
// not converge return at once.
void launch_adj_prep(const Dev& D, const Consts& K, const Adj& A, int r, uint32_t gate, hipStream_t st);
// sweeps k0..k1-1 of the transposed iteration, each one's convergence decided
// before the next (in the next sweep for a single instance, else by a decide
// launch after every sweep)
void launch_adj_sweeps(const Dev& D, const Consts& K, const Adj& A, int k0, int k1, int r, uint32_t gate,
                       hipStream_t st);
void launch_adj_decide(const Dev& D, const Consts& K, const Adj& A, int k, int r, uint32_t gate, hipStream_t st);
// the cotangents of step r once its iteration converged (a single instance's
// convergence after last_sweep is decided here), and the step counted done
void launch_adj_grad(const Dev& D, const Consts& K, const Adj& A, int r, uint32_t gate, int last_sweep,
                     hipStream_t st);

}  // namespace ugk
