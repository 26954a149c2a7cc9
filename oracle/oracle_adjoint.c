/*
 * FP64 CPU oracle -- adjoint of the frozen-tally macroscopic map, and the
 * replay of that map with a new opacity.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper has no adjoint; the differentiated map is this reading of it.  A
 * recorded forward run hands, per step, three particle-phase results to the
 * macroscopic solve: the net particle flux w^{fr,p} (Eq. wfrpFormula), the
 * survivor density rho^p entering the step, and which cell-groups sampled
 * particles (the choice between C4 - e^{-s} and C4 in the wave flux, Remark 3).
 * Holding those fixed, one step is a smooth map of (rho^n, T^n, kappa):
 *
 *   sigma = kappa S_g,  s = lambda = c sigma dt / eps^2            (Sec. 3 group opacity)
 *   rho^h = rho^n - rho^p
 *   F^w   = (c / 4 eps)(A_L rho^h_L - A_R rho^h_R),  A = W(s) or C4(s)   (Sec. 2.2, Remark 3)
 *   Q     = rho^n + (dt/V) sum_f S_f F^w_in + w^{fr,p}/V            (Eq. macroSysFinal, explicit part)
 *   b(T)  = Q + (dt/V) sum_f S_f D_f (phi_nb(T) - phi(T)),  D_f = -(c^2/3eps^2) C2(s_f)/h
 *   T^{n+1} = T^n + (dt/(eps^2 C_v)) sum_g sigma (b - phi)/(1 + lambda)   at its fixed point
 *   rho^{n+1} = (b + lambda phi)/(1 + lambda)                        (Appendix B)
 *
 * with phi = phi_g(T^{n+1}) and T held fixed in pinned cells.  The replay runs
 * this map forward by the source iteration (Algorithm 2) to a fixed point
 * converged to rounding; the adjoint runs it backward: per step, a transposed
 * source iteration for the cotangent mu of T^{n+1},
 *
 *   bbar   = w sigma/(1+lambda) mu + rbar/(1+lambda)          (w = dt/(eps^2 C_v), 0 if pinned)
 *   phibar = -w sigma/(1+lambda) mu + lambda/(1+lambda) rbar + (dt/V) L bbar
 *   mu     = Tbar + sum_g phi_g'(T^{n+1}) phibar
 *
 * (L: the same face operator as in b, which is symmetric).  The local part of
 * the last line is -d mu with d = w sum_g sigma phi_g'/(1+lambda), the
 * contraction factor of the literal sweep: where d > 1 (stiff coupling) the
 * plain iteration of that line diverges exactly as the literal forward sweep
 * does.  Both the replay and the transposed iteration therefore take the
 * diagonally preconditioned form of the linearized sweep (a local Newton step,
 * same fixed point):
 *
 *   forward:  T^{k+1} = T^k + (T^n - T^k + w sum_g sigma (b - phi)/(1+lambda)) / (1 + d)
 *   reverse:  mu^{k+1} = mu^k + (Tbar + sum_g phi_g' phibar(mu^k) - mu^k) / (1 + d)
 *
 * whose iteration matrices are similar to each other's transposes.  Then the cotangents
 * of Q, lambda, sigma, D_f (through the harmonic face opacity and C2), A (through
 * C4 or W) and rho^n.  Everything is written per (cell, group) and per face
 * exactly as the forward step states it; no step is fused or reordered.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

#define XLO 0
#define XHI 1
#define YLO 2
#define YHI 3

typedef struct { int nb; int side; double S; double h; } face_t;

/* The 2*dim faces of cell i: neighbour (-1 outside), side, area, centre distance. */
static int faces_of(const ora_params* P, double dx, double dy, int i, face_t f[4])
{
    int nx = P->nx, ny = P->ny, ix = i % nx, iy = i / nx;
    int n = 0;
    f[n].nb = ix > 0 ? i - 1 : -1; f[n].side = XLO; f[n].S = dy; f[n].h = dx; n++;
    f[n].nb = ix < nx - 1 ? i + 1 : -1; f[n].side = XHI; f[n].S = dy; f[n].h = dx; n++;
    if (P->dim == 2) {
        f[n].nb = iy > 0 ? i - nx : -1; f[n].side = YLO; f[n].S = dx; f[n].h = dy; n++;
        f[n].nb = iy < ny - 1 ? i + nx : -1; f[n].side = YHI; f[n].S = dx; f[n].h = dy; n++;
    }
    return n;
}

/* kappa-dependent coefficients of the macroscopic map. */
typedef struct {
    int nc, G;
    size_t ncg;
    double V, dx, dy;
    double* sig;     /* [ncg] group opacity                 */
    double* s;       /* [ncg] c sigma dt / eps^2 = lambda    */
    double* sf;      /* [ncg*4] face opacity per cell face   */
    double* D;       /* [ncg*4] face coefficient D_f >= 0    */
    double* phib;    /* [4*G] Planckian ghost phi per side   */
} coefs;

static void coefs_free(coefs* M)
{
    free(M->sig); free(M->s); free(M->sf); free(M->D); free(M->phib);
}

static void coefs_build(const ora_sim* sim, const double* kappa, coefs* M)
{
    const ora_params* P = ora__params(sim);
    const double* simpson = ora__simpson(sim);
    const int G = P->G;
    M->nc = P->nx * P->ny;
    M->G = G;
    M->ncg = (size_t)M->nc * G;
    M->V = ora__V(sim);
    M->dx = ora__dx(sim);
    M->dy = ora__dy(sim);
    M->sig = (double*)calloc(M->ncg, sizeof(double));
    M->s = (double*)calloc(M->ncg, sizeof(double));
    M->sf = (double*)calloc(M->ncg * 4, sizeof(double));
    M->D = (double*)calloc(M->ncg * 4, sizeof(double));
    M->phib = (double*)calloc((size_t)4 * G, sizeof(double));
    const double ks = P->c * P->dt / (P->eps * P->eps);
    for (int i = 0; i < M->nc; ++i)
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            M->sig[k] = kappa[k] * simpson[g];
            M->s[k] = P->c * M->sig[k] * P->dt / (P->eps * P->eps);
        }
    for (int i = 0; i < M->nc; ++i) {
        face_t f[4];
        int nf = faces_of(P, M->dx, M->dy, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            for (int q = 0; q < nf; ++q) {
                double a = M->sig[k];
                double sfq = a;
                if (f[q].nb >= 0) {
                    double b = M->sig[(size_t)f[q].nb * G + g];
                    sfq = (a + b > 0.0) ? 2.0 * (a * b) / (a + b) : 0.0;   /* harmonic mean */
                }
                M->sf[k * 4 + q] = sfq;
                double c2 = P->dt * ora_coef_c2_over_dt(ks * sfq);
                M->D[k * 4 + q] = -(P->c * P->c / (3.0 * P->eps * P->eps)) * c2 / f[q].h;
            }
        }
    }
    for (int side = 0; side < 4; ++side)
        for (int g = 0; g < G; ++g)
            M->phib[side * G + g] = P->bc[side] == ORA_BC_PLANCK
                ? ora_phi_group(P->bcT[side], P->nu[g], P->nu[g + 1], P->a, P->c) : 0.0;
}

/* Static source Q of one recorded step with the (replayed) rho^n and the
 * frozen particle results of that step. */
static void frozen_source(const ora_sim* sim, const coefs* M, const ora_rec_step* r,
                          const double* rho_n, double* Q)
{
    const ora_params* P = ora__params(sim);
    const int G = M->G;
    const double cq = P->c / (4.0 * P->eps);
    for (int i = 0; i < M->nc; ++i) {
        face_t f[4];
        int nf = faces_of(P, M->dx, M->dy, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            double Ak = r->sampled[k] ? ora_coef_w(M->s[k]) : ora_coef_c4(M->s[k]);
            double uk = Ak * (rho_n[k] - r->rhop[k]);
            double fin = 0.0;        /* sum_f S_f F^w_in */
            for (int q = 0; q < nf; ++q) {
                double un;
                if (f[q].nb >= 0) {
                    size_t kn = (size_t)f[q].nb * G + g;
                    double An = r->sampled[kn] ? ora_coef_w(M->s[kn]) : ora_coef_c4(M->s[kn]);
                    un = An * (rho_n[kn] - r->rhop[kn]);
                } else if (P->bc[f[q].side] == ORA_BC_REFLECT) {
                    continue;
                } else {
                    un = ora_coef_c4(M->s[k]) * M->phib[f[q].side * G + g];
                }
                fin += f[q].S * cq * (un - uk);
            }
            Q[k] = rho_n[k] + (P->dt / M->V) * fin + r->wnet[k] / M->V;
        }
    }
}

/* Ghost phi beyond a domain face (reflective: mirror of the interior). */
static double ghost(const ora_params* P, const coefs* M, int side, int g, double interior)
{
    if (P->bc[side] == ORA_BC_REFLECT) return interior;
    return M->phib[side * M->G + g];
}

/* b = Q + (dt/V) sum_f S_f D_f (phi_nb - phi) for every (cell, group). */
static void apply_b(const ora_sim* sim, const coefs* M, const double* Q, const double* phi, double* b)
{
    const ora_params* P = ora__params(sim);
    const int G = M->G;
    for (int i = 0; i < M->nc; ++i) {
        face_t f[4];
        int nf = faces_of(P, M->dx, M->dy, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            double lap = 0.0;
            for (int q = 0; q < nf; ++q) {
                double pn = f[q].nb >= 0 ? phi[(size_t)f[q].nb * G + g] : ghost(P, M, f[q].side, g, phi[k]);
                lap += f[q].S * M->D[k * 4 + q] * (pn - phi[k]);
            }
            b[k] = Q[k] + (P->dt / M->V) * lap;
        }
    }
}

/* Fixed point of the source iteration of one frozen step, iterated until the
 * changes of rho and T are at rounding level (max 1000 sweeps). */
static int frozen_solve(const ora_sim* sim, const coefs* M, const double* Q, const double* Tn,
                        double* rho_out, double* T_out)
{
    const ora_params* P = ora__params(sim);
    const double* cv = ora__cv(sim);
    const unsigned char* pinned = ora__pinned(sim);
    const int G = M->G;
    double* phi = (double*)malloc(sizeof(double) * M->ncg);
    double* b = (double*)malloc(sizeof(double) * M->ncg);
    double* Tk = (double*)malloc(sizeof(double) * M->nc);
    for (int i = 0; i < M->nc; ++i) Tk[i] = Tn[i];
    for (size_t k = 0; k < M->ncg; ++k) rho_out[k] = 0.0;
    int status = ORA_ENOCONV;
    for (int it = 0; it < 1000; ++it) {
        for (int i = 0; i < M->nc; ++i)
            for (int g = 0; g < G; ++g)
                phi[(size_t)i * G + g] = ora_phi_group(Tk[i], P->nu[g], P->nu[g + 1], P->a, P->c);
        apply_b(sim, M, Q, phi, b);
        double drho = 0.0, mrho = 0.0, dT = 0.0, mT = 0.0;
        int bad = 0;
        for (int i = 0; i < M->nc; ++i) {
            double sum = 0.0, dsum = 0.0;
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double lam = M->s[k];
                sum += M->sig[k] * (b[k] - phi[k]) / (1.0 + lam);
                dsum += M->sig[k] * ora_dphi_group(Tk[i], P->nu[g], P->nu[g + 1], P->a, P->c) / (1.0 + lam);
            }
            /* linearized emission phi + phi' (T^{k+1} - T^k): one local Newton step */
            const double w = P->dt / (P->eps * P->eps * cv[i]);
            double Tnew = pinned[i] ? Tn[i] : Tk[i] + (Tn[i] - Tk[i] + w * sum) / (1.0 + w * dsum);
            const double dTi = Tnew - Tk[i];
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double lam = M->s[k];
                double pe = phi[k] + ora_dphi_group(Tk[i], P->nu[g], P->nu[g + 1], P->a, P->c) * dTi;
                double r = (b[k] + lam * pe) / (1.0 + lam);
                double dr = fabs(r - rho_out[k]);
                if (dr > drho || dr != dr) drho = dr;
                if (fabs(r) > mrho) mrho = fabs(r);
                rho_out[k] = r;
            }
            if (!(Tnew > 0.0) || !isfinite(Tnew)) bad = 1;
            double dd = fabs(Tnew - Tk[i]);
            if (dd > dT || dd != dd) dT = dd;
            if (Tnew > mT) mT = Tnew;
            T_out[i] = Tnew;
        }
        if (bad) { status = ORA_ENONFINITE; break; }
        for (int i = 0; i < M->nc; ++i) Tk[i] = T_out[i];
        /* rounding level; past 60 sweeps a stall within 1e-14 is accepted */
        const double lim = it >= 60 ? 1e-14 : 4e-16;
        if (it > 0 && drho <= lim * mrho && dT <= lim * mT) { status = ORA_OK; break; }
    }
    free(phi); free(b); free(Tk);
    return status;
}

int ora_replay_frozen(ora_sim* s, const double* kappa, double* T_final)
{
    int nrec = ora__nrec(s);
    if (nrec == 0 || !ora__kappa_rec(s)) return ORA_EINVAL;
    coefs M;
    coefs_build(s, kappa, &M);
    double* rho = (double*)malloc(sizeof(double) * M.ncg);
    double* rho1 = (double*)malloc(sizeof(double) * M.ncg);
    double* T = (double*)malloc(sizeof(double) * M.nc);
    double* T1 = (double*)malloc(sizeof(double) * M.nc);
    double* Q = (double*)malloc(sizeof(double) * M.ncg);
    const ora_rec_step* r0 = ora__rec(s, 0);
    memcpy(rho, r0->rho, sizeof(double) * M.ncg);
    memcpy(T, r0->T, sizeof(double) * M.nc);
    int st = ORA_OK;
    for (int n = 0; n < nrec && st == ORA_OK; ++n) {
        frozen_source(s, &M, ora__rec(s, n), rho, Q);
        st = frozen_solve(s, &M, Q, T, rho1, T1);
        memcpy(rho, rho1, sizeof(double) * M.ncg);
        memcpy(T, T1, sizeof(double) * M.nc);
    }
    if (st == ORA_OK) memcpy(T_final, T, sizeof(double) * M.nc);
    free(rho); free(rho1); free(T); free(T1); free(Q);
    coefs_free(&M);
    return st;
}

/* One transposed sweep:  given mu (cotangent of T^{n+1}), form bbar and phibar. */
static void transposed_terms(const ora_sim* sim, const coefs* M, const double* w, const double* mu,
                             const double* rbar, double* bbar, double* phibar)
{
    const ora_params* P = ora__params(sim);
    const int G = M->G;
    for (int i = 0; i < M->nc; ++i)
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            double lam = M->s[k];
            bbar[k] = w[i] * M->sig[k] / (1.0 + lam) * mu[i] + rbar[k] / (1.0 + lam);
        }
    for (int i = 0; i < M->nc; ++i) {
        face_t f[4];
        int nf = faces_of(P, M->dx, M->dy, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            double lam = M->s[k];
            double lt = 0.0;     /* (L^T bbar)_k, L symmetric */
            for (int q = 0; q < nf; ++q) {
                if (f[q].nb >= 0) lt += f[q].S * M->D[k * 4 + q] * (bbar[(size_t)f[q].nb * G + g] - bbar[k]);
                else if (P->bc[f[q].side] != ORA_BC_REFLECT) lt -= f[q].S * M->D[k * 4 + q] * bbar[k];
            }
            phibar[k] = -w[i] * M->sig[k] / (1.0 + lam) * mu[i] + lam / (1.0 + lam) * rbar[k]
                        + (P->dt / M->V) * lt;
        }
    }
}

/* (cell, group) updates of the transposed iterations of the last ora_adjoint call. */
static long long g_last_updates = 0;
long long ora_adjoint_updates(void) { return g_last_updates; }

int ora_adjoint(ora_sim* s, const double* dJdT, double* grad_kappa)
{
    g_last_updates = 0;
    const int nrec = ora__nrec(s);
    const double* kappa = ora__kappa_rec(s);
    if (nrec == 0 || !kappa) return ORA_EINVAL;
    const ora_params* P = ora__params(s);
    const double* cv = ora__cv(s);
    const double* simpson = ora__simpson(s);
    const unsigned char* pinned = ora__pinned(s);
    coefs M;
    coefs_build(s, kappa, &M);
    const int G = M.G, nc = M.nc;
    const size_t ncg = M.ncg;
    const double ks = P->c * P->dt / (P->eps * P->eps);
    const double cq = P->c / (4.0 * P->eps);
    const double dscale = -(P->c * P->c / (3.0 * P->eps * P->eps)) * P->dt * ks;   /* dD/dsf * h / C2' */

    double* w = (double*)malloc(sizeof(double) * nc);
    for (int i = 0; i < nc; ++i) w[i] = pinned[i] ? 0.0 : P->dt / (P->eps * P->eps * cv[i]);
    double* rbar = (double*)calloc(ncg, sizeof(double));     /* cotangent of rho^{n+1} */
    double* rbar_n = (double*)calloc(ncg, sizeof(double));
    double* Tbar = (double*)malloc(sizeof(double) * nc);      /* cotangent of T^{n+1}   */
    double* mu = (double*)malloc(sizeof(double) * nc);
    double* mu1 = (double*)malloc(sizeof(double) * nc);
    double* dloc = (double*)malloc(sizeof(double) * nc);
    double* bbar = (double*)malloc(sizeof(double) * ncg);
    double* phibar = (double*)malloc(sizeof(double) * ncg);
    double* phi = (double*)malloc(sizeof(double) * ncg);
    double* dphi = (double*)malloc(sizeof(double) * ncg);
    double* Q = (double*)malloc(sizeof(double) * ncg);
    double* b = (double*)malloc(sizeof(double) * ncg);
    double* sbar = (double*)malloc(sizeof(double) * ncg);    /* cotangent of s (= lambda) */
    double* sigbar = (double*)malloc(sizeof(double) * ncg);  /* cotangent of sigma        */
    double* ubar = (double*)malloc(sizeof(double) * ncg);    /* cotangent of A rho^h      */
    memcpy(Tbar, dJdT, sizeof(double) * nc);
    for (size_t k = 0; k < ncg; ++k) grad_kappa[k] = 0.0;
    int status = ORA_OK;

    for (int n = nrec - 1; n >= 0; --n) {
        const ora_rec_step* r = ora__rec(s, n);
        const double* Tn1 = (n + 1 < nrec) ? ora__rec(s, n + 1)->T : ora__T(s);
        /* phi, phi' at the step's fixed point, b there */
        for (int i = 0; i < nc; ++i)
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                phi[k] = ora_phi_group(Tn1[i], P->nu[g], P->nu[g + 1], P->a, P->c);
                dphi[k] = ora_dphi_group(Tn1[i], P->nu[g], P->nu[g + 1], P->a, P->c);
            }
        frozen_source(s, &M, r, r->rho, Q);
        apply_b(s, &M, Q, phi, b);

        /* local diagonal d = w sum_g sigma phi'/(1+lambda) of the transposed map */
        for (int i = 0; i < nc; ++i) {
            double acc = 0.0;
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                acc += M.sig[k] * dphi[k] / (1.0 + M.s[k]);
            }
            dloc[i] = w[i] * acc;
        }
        /* transposed source iteration for mu, preconditioned by 1 + d */
        memcpy(mu, Tbar, sizeof(double) * nc);
        int conv = 0;
        for (int it = 0; it < 1000 && !conv; ++it) {
            transposed_terms(s, &M, w, mu, rbar, bbar, phibar);
            double dm = 0.0, mm = 0.0;
            for (int i = 0; i < nc; ++i) {
                double acc = 0.0;
                for (int g = 0; g < G; ++g) acc += dphi[(size_t)i * G + g] * phibar[(size_t)i * G + g];
                mu1[i] = mu[i] + (Tbar[i] + acc - mu[i]) / (1.0 + dloc[i]);
                double d = fabs(mu1[i] - mu[i]);
                if (d > dm || d != d) dm = d;
                if (fabs(mu1[i]) > mm) mm = fabs(mu1[i]);
            }
            memcpy(mu, mu1, sizeof(double) * nc);
            g_last_updates += (long long)ncg;
            if (!(dm == dm)) break;
            if (dm <= (it >= 60 ? 1e-13 : 1e-15) * mm) conv = 1;
        }
        if (!conv) { status = ORA_ENOCONV; break; }
        transposed_terms(s, &M, w, mu, rbar, bbar, phibar);

        /* cotangents of lambda (= s) and sigma from the two update formulas */
        for (int i = 0; i < nc; ++i)
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double lam = M.s[k];
                double em = (b[k] - phi[k]) / (1.0 + lam);
                sbar[k] = -em / (1.0 + lam) * (w[i] * M.sig[k] * mu[i] + rbar[k]);
                sigbar[k] = w[i] * em * mu[i];
            }
        /* Q-bar = bbar; cotangent of u = A rho^h from sum_f S_f F^w_in */
        for (int i = 0; i < nc; ++i) {
            face_t f[4];
            int nf = faces_of(P, M.dx, M.dy, i, f);
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double acc = 0.0;
                for (int q = 0; q < nf; ++q) {
                    if (f[q].nb >= 0) acc += f[q].S * (bbar[(size_t)f[q].nb * G + g] - bbar[k]);
                    else if (P->bc[f[q].side] != ORA_BC_REFLECT) acc -= f[q].S * bbar[k];
                }
                ubar[k] = (P->dt / M.V) * cq * acc;
            }
        }
        for (int i = 0; i < nc; ++i) {
            face_t f[4];
            int nf = faces_of(P, M.dx, M.dy, i, f);
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double sk = M.s[k];
                double rhoh = r->rho[k] - r->rhop[k];
                double A = r->sampled[k] ? ora_coef_w(sk) : ora_coef_c4(sk);
                double dA = r->sampled[k] ? ora_coef_w_ds(sk) : ora_coef_c4_ds(sk);
                /* A(s) rho^h in this cell's own flux terms */
                sbar[k] += ubar[k] * rhoh * dA;
                /* Planckian ghost inflow C4(s) phi_b */
                for (int q = 0; q < nf; ++q)
                    if (f[q].nb < 0 && P->bc[f[q].side] == ORA_BC_PLANCK)
                        sbar[k] += (P->dt / M.V) * f[q].S * cq * bbar[k] * M.phib[f[q].side * G + g]
                                   * ora_coef_c4_ds(sk);
                /* face coefficients: b_k and b_nb both hold D_f (phi_nb - phi_k) terms */
                double sig_face = 0.0;
                for (int q = 0; q < nf; ++q) {
                    double Dbar;
                    double dsf;      /* d sf / d sigma_k */
                    if (f[q].nb >= 0) {
                        size_t kn = (size_t)f[q].nb * G + g;
                        Dbar = (P->dt / M.V) * f[q].S * (bbar[k] - bbar[kn]) * (phi[kn] - phi[k]);
                        double a = M.sig[k], bb = M.sig[kn];
                        dsf = (a + bb > 0.0) ? 2.0 * bb * bb / ((a + bb) * (a + bb)) : 0.0;
                    } else if (P->bc[f[q].side] == ORA_BC_REFLECT) {
                        continue;
                    } else {
                        Dbar = (P->dt / M.V) * f[q].S * bbar[k] * (M.phib[f[q].side * G + g] - phi[k]);
                        dsf = 1.0;
                    }
                    double dD = dscale * ora_coef_c2_over_dt_ds(ks * M.sf[k * 4 + q]) / f[q].h;
                    sig_face += Dbar * dD * dsf;
                }
                double sig_total = sigbar[k] + ks * sbar[k] + sig_face;
                grad_kappa[k] += simpson[g] * sig_total;
                /* cotangent of rho^n: directly in Q and through rho^h */
                rbar_n[k] = bbar[k] + A * ubar[k];
            }
        }
        memcpy(rbar, rbar_n, sizeof(double) * ncg);
        memcpy(Tbar, mu, sizeof(double) * nc);
    }
    free(w); free(rbar); free(rbar_n); free(Tbar); free(mu); free(mu1); free(dloc); free(bbar); free(phibar);
    free(phi); free(dphi); free(Q); free(b); free(sbar); free(sigbar); free(ubar);
    coefs_free(&M);
    return status;
}
