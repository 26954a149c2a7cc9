/*
 * FP64 CPU oracle -- one UGKWP time step (Algorithm 1 of the paper) for the
 * multigroup radiative transfer system, in 1-D slabs and 2-D Cartesian meshes.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Step n -> n+1, in the order of Algorithm 1:
 *   coefficients    s = c sigma dt / eps^2, e^{-s}, C4, W = C4 - e^{-s}, C2 at faces
 *   wave split      rho^h = rho^n - rho^p;  sample E = e^{-s} rho^h V  (Eq. IhpFormula)
 *                   as N = floor(E / (w_ref V)) particles of weight E/N (Sec. 2.2, omega_k)
 *   free flight     t_f = min(-tau ln eta, dt) for old particles (Eq. particle tf formula),
 *                   t_f = dt for new ones; reset at every interface (Remark 1)
 *   tallies         w^{fr,p} = sum_in - sum_out (Eq. wfrpFormula)
 *   wave flux       F^{fr,wave} with C4 - e^{-s}, or C4 where no particle was
 *                   sampled (Remark 3); zero slopes
 *   implicit solve  Eq. macroSysFinal by source iteration (Appendix B, Algorithm 2)
 *   absorb          collided particles are deleted
 *
 * Readings (the paper is silent or ambiguous here):
 *  - rho is the angle-integrated group intensity; its equilibrium value is
 *    phi_g(T) (4 pi B_g in 3-D, "2 B_g" in Appendix B).  F^eq = C2 (c/eps)^2 (1/3) d phi/dx.
 *  - flights use sigma(nu_k, cell) = kappa_{g,cell} nu_k^-p (Remark 2); the macroscopic
 *    terms use the Simpson group opacity (Sec. 3, group opacity).
 *  - free flight is reset at every interior crossing; a particle ending exactly on
 *    a face stays in its cell; crossing requires t_face < t_rem strictly; an exact
 *    x/y tie crosses x first.
 *  - wave flux uses the start-of-step rho^h and each upwind cell's own s.
 *  - boundary ghosts sit one cell width away: Planckian (phi = rho^h = phi(T_b),
 *    never sampled, sigma of the interior cell), vacuum (0), reflective (mirror;
 *    specular reflection of particles, not tallied).
 *  - source iteration updates T with the explicit emission phi^k of Eq.
 *    macroSysAppendixIte and stops when max|d rho| <= tol max|rho| and
 *    max|dT| <= tol max T over the whole mesh.  The exchange term
 *    sigma (rho^{k+1} - phi^k) is evaluated in the algebraically identical form
 *    sigma (b - phi^k)/(1 + lam), b = Q + (dt/V) sum_f S_f D_f (phi_nb - phi), which
 *    does not cancel in optically thick groups.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

#define XLO 0
#define XHI 1
#define YLO 2
#define YHI 3

struct ora_sim {
    ora_params p;
    double* nu;            /* G+1 edges */
    double* simpson;       /* [G]: Simpson mean of nu^-p over the group */
    int ncell;
    double dx, dy, V;
    int have_opacity, have_material;
    double* kappa;         /* [ncell][G] */
    double* cv; double* T; double* rho; double* rhop; unsigned char* pinned;
    /* particle pool (structure of arrays) */
    int64_t np;
    double *px, *py, *pox, *poy, *pnu, *pw; uint64_t* pid; int32_t* pcell; int32_t* pg;
    uint64_t nbirth;
    int step;
    /* tallies of the last step */
    double *ftx, *fty, *dep, *surv, *start, *wnew, *Q;
    int64_t* nb;
    ora_diag diag;
    /* adjoint recording */
    int recording;
    int nrec, caprec;
    ora_rec_step* rec;
    double *kappa0, *T0rec, *rho0rec;
    /* volumetric source and its switch-off time */
    double *olH, *olchi;          /* Olson's heat capacity per cell (NULL: constant C_v) */
    double* qsrc;
    double q_toff;
    /* tabulated opacity */
    int tab_nmat, tab_nnu, tab_nT;
    int32_t* tab_mat;
    double *tab_lnu, *tab_lT, *tab_lsig;
};

static void* zalloc(size_t n) { void* q = calloc(n ? n : 1, 1); return q; }

static double nupow(double nu, double p)
{
    if (p == 3.0) return 1.0 / (nu * nu * nu);
    return pow(nu, -p);
}

ora_sim* ora_create(const ora_params* p)
{
    if (!p || (p->dim != 1 && p->dim != 2) || p->nx < 1 || p->ny < 1) return NULL;
    if (p->dim == 1 && p->ny != 1) return NULL;
    if (p->G < 1 || !p->nu) return NULL;
    if (p->opacity_stim != 0 && p->opacity_stim != 1) return NULL;
    if (!(p->dt > 0) || !(p->c > 0) || !(p->eps > 0) || !(p->a > 0) || !(p->w_ref > 0)) return NULL;
    if (!(p->x1 > p->x0)) return NULL;
    if (p->dim == 2 && !(p->y1 > p->y0)) return NULL;
    for (int g = 0; g < p->G; ++g) if (!(p->nu[g] > 0) || !(p->nu[g + 1] > p->nu[g])) return NULL;
    ora_sim* s = (ora_sim*)zalloc(sizeof(ora_sim));
    s->p = *p;
    int G = p->G;
    s->nu = (double*)zalloc(sizeof(double) * (G + 1));
    memcpy(s->nu, p->nu, sizeof(double) * (G + 1));
    s->p.nu = s->nu;
    s->simpson = (double*)zalloc(sizeof(double) * G);
    for (int g = 0; g < G; ++g) {
        double nl = s->nu[g], nh = s->nu[g + 1], nm = 0.5 * (nl + nh);
        s->simpson[g] = (nupow(nl, p->nu_power) + 4.0 * nupow(nm, p->nu_power) + nupow(nh, p->nu_power)) / 6.0;
    }
    s->ncell = p->nx * p->ny;
    s->dx = (p->x1 - p->x0) / p->nx;
    s->dy = (p->dim == 2) ? (p->y1 - p->y0) / p->ny : 1.0;
    s->V = s->dx * s->dy;
    size_t ncg = (size_t)s->ncell * G;
    s->kappa = (double*)zalloc(sizeof(double) * ncg);
    s->cv = (double*)zalloc(sizeof(double) * s->ncell);
    s->T = (double*)zalloc(sizeof(double) * s->ncell);
    s->rho = (double*)zalloc(sizeof(double) * ncg);
    s->rhop = (double*)zalloc(sizeof(double) * ncg);
    s->pinned = (unsigned char*)zalloc(s->ncell);
    int64_t cap = p->pool_cap > 0 ? p->pool_cap : 1;
    s->px = (double*)zalloc(sizeof(double) * cap);
    s->py = (double*)zalloc(sizeof(double) * cap);
    s->pox = (double*)zalloc(sizeof(double) * cap);
    s->poy = (double*)zalloc(sizeof(double) * cap);
    s->pnu = (double*)zalloc(sizeof(double) * cap);
    s->pw = (double*)zalloc(sizeof(double) * cap);
    s->pid = (uint64_t*)zalloc(sizeof(uint64_t) * cap);
    s->pcell = (int32_t*)zalloc(sizeof(int32_t) * cap);
    s->pg = (int32_t*)zalloc(sizeof(int32_t) * cap);
    size_t nfx = (size_t)(p->nx + 1) * p->ny, nfy = (size_t)p->nx * (p->ny + 1);
    s->ftx = (double*)zalloc(sizeof(double) * nfx * G * 2);
    s->fty = (double*)zalloc(sizeof(double) * nfy * G * 2);
    s->dep = (double*)zalloc(sizeof(double) * ncg);
    s->surv = (double*)zalloc(sizeof(double) * ncg);
    s->start = (double*)zalloc(sizeof(double) * ncg);
    s->wnew = (double*)zalloc(sizeof(double) * ncg);
    s->Q = (double*)zalloc(sizeof(double) * ncg);
    s->nb = (int64_t*)zalloc(sizeof(int64_t) * ncg);
    return s;
}

static void free_rec(ora_sim* s)
{
    for (int k = 0; k < s->nrec; ++k) {
        free(s->rec[k].rho); free(s->rec[k].T); free(s->rec[k].rhop);
        free(s->rec[k].rhoh); free(s->rec[k].wnet); free(s->rec[k].sampled);
    }
    free(s->rec); s->rec = NULL; s->nrec = 0; s->caprec = 0;
    free(s->kappa0); s->kappa0 = NULL;
}

void ora_destroy(ora_sim* s)
{
    if (!s) return;
    free_rec(s);
    free(s->nu); free(s->simpson); free(s->kappa); free(s->cv); free(s->T); free(s->rho);
    free(s->rhop); free(s->pinned); free(s->px); free(s->py); free(s->pox); free(s->poy);
    free(s->pnu); free(s->pw); free(s->pid); free(s->pcell); free(s->pg); free(s->ftx);
    free(s->fty); free(s->dep); free(s->surv); free(s->start); free(s->wnew); free(s->Q);
    free(s->nb); free(s->olH); free(s->olchi); free(s->qsrc); free(s->tab_mat); free(s->tab_lnu); free(s->tab_lT); free(s->tab_lsig);
    free(s);
}

int ora_set_opacity(ora_sim* s, const double* kappa)
{
    size_t ncg = (size_t)s->ncell * s->p.G;
    for (size_t k = 0; k < ncg; ++k) if (!(kappa[k] >= 0) || !isfinite(kappa[k])) return ORA_EINVAL;
    memcpy(s->kappa, kappa, sizeof(double) * ncg);
    s->have_opacity = 1;
    return ORA_OK;
}

int ora_set_material(ora_sim* s, const double* cv, const double* T0, const double* Tr0,
                     const unsigned char* pinned)
{
    int G = s->p.G;
    for (int i = 0; i < s->ncell; ++i) {
        if (!(cv[i] > 0) || !(T0[i] > 0) || !(Tr0[i] > 0) || !isfinite(cv[i]) || !isfinite(T0[i])
            || !isfinite(Tr0[i])) return ORA_EINVAL;
    }
    for (int i = 0; i < s->ncell; ++i) {
        s->cv[i] = cv[i];
        s->T[i] = T0[i];
        s->pinned[i] = pinned ? pinned[i] : 0;
        for (int g = 0; g < G; ++g)
            s->rho[(size_t)i * G + g] = ora_phi_group(Tr0[i], s->nu[g], s->nu[g + 1], s->p.a, s->p.c);
    }
    memset(s->rhop, 0, sizeof(double) * (size_t)s->ncell * G);
    s->np = 0;
    s->nbirth = 0;
    s->step = 0;
    s->have_material = 1;
    return ORA_OK;
}

int ora_set_source(ora_sim* s, const double* q, double t_off)
{
    size_t ncg = (size_t)s->ncell * s->p.G;
    if (!q) { free(s->qsrc); s->qsrc = NULL; return ORA_OK; }
    for (size_t k = 0; k < ncg; ++k) if (!(q[k] >= 0) || !isfinite(q[k])) return ORA_EINVAL;
    if (!(t_off >= 0)) return ORA_EINVAL;
    if (!s->qsrc) s->qsrc = (double*)malloc(sizeof(double) * ncg);
    memcpy(s->qsrc, q, sizeof(double) * ncg);
    s->q_toff = t_off;
    return ORA_OK;
}

int ora_set_source_planck(ora_sim* s, const double* f, double Ts, double t_off)
{
    if (!f) return ora_set_source(s, NULL, t_off);
    if (!(Ts > 0.0) || !isfinite(Ts)) return ORA_EINVAL;
    const int G = s->p.G;
    const double rate = s->p.c / (s->p.eps * s->p.eps);
    double* q = (double*)malloc(sizeof(double) * (size_t)s->ncell * G);
    if (!q) return ORA_ENOMEM;
    int st = ORA_OK;
    for (int i = 0; i < s->ncell && st == ORA_OK; ++i) {
        if (!(f[i] >= 0.0) || !isfinite(f[i])) st = ORA_EINVAL;
        for (int g = 0; g < G; ++g)
            q[(size_t)i * G + g] = rate * f[i] * ora_phi_group(Ts, s->nu[g], s->nu[g + 1], s->p.a, s->p.c);
    }
    if (st == ORA_OK) st = ora_set_source(s, q, t_off);
    free(q);
    return st;
}

int ora_set_opacity_table(ora_sim* s, int nmat, const int32_t* mat, int nnu, const double* nu, int nT,
                          const double* T, const double* sig)
{
    if (nmat < 1 || nnu < 2 || nT < 2 || !mat || !nu || !T || !sig) return ORA_EINVAL;
    for (int i = 0; i < s->ncell; ++i) if (mat[i] < 0 || mat[i] >= nmat) return ORA_EINVAL;
    for (int k = 0; k + 1 < nnu; ++k) if (!(nu[k] > 0) || !(nu[k + 1] > nu[k])) return ORA_EINVAL;
    for (int k = 0; k + 1 < nT; ++k) if (!(T[k] > 0) || !(T[k + 1] > T[k])) return ORA_EINVAL;
    size_t nt = (size_t)nmat * nT * nnu;
    for (size_t k = 0; k < nt; ++k) if (!(sig[k] > 0) || !isfinite(sig[k])) return ORA_EINVAL;
    free(s->tab_mat); free(s->tab_lnu); free(s->tab_lT); free(s->tab_lsig);
    s->tab_nmat = nmat; s->tab_nnu = nnu; s->tab_nT = nT;
    s->tab_mat = (int32_t*)malloc(sizeof(int32_t) * s->ncell);
    memcpy(s->tab_mat, mat, sizeof(int32_t) * s->ncell);
    s->tab_lnu = (double*)malloc(sizeof(double) * nnu);
    s->tab_lT = (double*)malloc(sizeof(double) * nT);
    s->tab_lsig = (double*)malloc(sizeof(double) * nt);
    for (int k = 0; k < nnu; ++k) s->tab_lnu[k] = log(nu[k]);
    for (int k = 0; k < nT; ++k) s->tab_lT[k] = log(T[k]);
    for (size_t k = 0; k < nt; ++k) s->tab_lsig[k] = log(sig[k]);
    s->have_opacity = 1;
    return ORA_OK;
}

/* Node interval and weight of x among n ascending nodes (clamped at the ends). */
static int tab_locate(const double* nodes, int n, double x, double* frac)
{
    if (x <= nodes[0]) { *frac = 0.0; return 0; }
    if (x >= nodes[n - 1]) { *frac = 1.0; return n - 2; }
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (nodes[mid] <= x) lo = mid; else hi = mid;
    }
    *frac = (x - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
    return lo;
}

double ora_table_sigma(const ora_sim* s, int m, double nu, double T)
{
    double a, b;
    const int i = tab_locate(s->tab_lnu, s->tab_nnu, log(nu), &a);
    const int j = tab_locate(s->tab_lT, s->tab_nT, log(T), &b);
    const double* L = s->tab_lsig + (size_t)m * s->tab_nT * s->tab_nnu;
    const int n = s->tab_nnu;
    const double l00 = L[(size_t)j * n + i], l10 = L[(size_t)j * n + i + 1];
    const double l01 = L[(size_t)(j + 1) * n + i], l11 = L[(size_t)(j + 1) * n + i + 1];
    const double lo = (1.0 - a) * l00 + a * l10, hi = (1.0 - a) * l01 + a * l11;
    return exp((1.0 - b) * lo + b * hi);
}

/* Olson's ionisation fraction (Sec. 3.4): alpha = e^{-chi/T} (sqrt(1 + 4 e^{chi/T})
 * - 1)/2 and dalpha/dT = (chi/T^2)(alpha - 1/sqrt(1 + 4 e^{chi/T})), written with
 * h = e^{-chi/(2T)} (alpha = h (sqrt(h^2 + 4) - h)/2) so that nothing overflows. */
double ora_olson_alpha(double T, double chi, double* dalpha)
{
    const double h = exp(-0.5 * chi / T);
    const double r = sqrt(h * h + 4.0);
    const double alpha = 0.5 * h * (r - h);
    if (dalpha) *dalpha = (chi / (T * T)) * (alpha - h / r);
    return alpha;
}

int ora_set_heat_capacity(ora_sim* s, const double* H, const double* chi)
{
    if (!H) { free(s->olH); free(s->olchi); s->olH = s->olchi = NULL; return ORA_OK; }
    if (!chi) return ORA_EINVAL;
    for (int i = 0; i < s->ncell; ++i)
        if (!(H[i] >= 0.0) || !(chi[i] >= 0.0) || !isfinite(H[i]) || !isfinite(chi[i])) return ORA_EINVAL;
    if (!s->olH) {
        s->olH = (double*)malloc(sizeof(double) * s->ncell);
        s->olchi = (double*)malloc(sizeof(double) * s->ncell);
    }
    memcpy(s->olH, H, sizeof(double) * s->ncell);
    memcpy(s->olchi, chi, sizeof(double) * s->ncell);
    return ORA_OK;
}

/* Heat capacity of cell i at T: the constant C_v of the cell, or Olson's
 * rho C_v = H [1 + alpha + (T + chi) dalpha/dT] (Eq. cvolson, whose a T_keV^3
 * factor is the unit a (1 keV)^3 and is folded into H) where H > 0. */
double ora_heat_capacity(const ora_sim* s, int i, double T)
{
    if (!s->olH || !(s->olH[i] > 0.0)) return s->cv[i];
    double da;
    const double chi = s->olchi[i];
    const double al = ora_olson_alpha(T, chi, &da);
    return s->olH[i] * (1.0 + al + (T + chi) * da);
}

/* Material energy U(T) with dU/dT = C_v (Sec. 2.1's U): C_v T, or for Olson's
 * heat capacity H [T (1 + alpha) + chi alpha], whose derivative is the bracket
 * of Eq. cvolson. */
double ora_material_energy(const ora_sim* s, int i, double T)
{
    if (!s->olH || !(s->olH[i] > 0.0)) return s->cv[i] * T;
    const double chi = s->olchi[i];
    const double al = ora_olson_alpha(T, chi, NULL);
    return s->olH[i] * (T * (1.0 + al) + chi * al);
}

static int olson_cell(const ora_sim* s, int i)
{
    return s->olH != NULL && s->olH[i] > 0.0;
}

/* The temperature of an Olson cell whose material energy is u > 0: U is strictly
 * increasing, so Newton's method from T0 kept inside a bracket [lo, hi] with
 * U(lo) <= u <= U(hi) (bisection when a step leaves it) finds the root; it stops
 * once a step changes T by at most 1e-15 T.  Returns a non-positive value when
 * u <= 0. */
static double olson_temperature(const ora_sim* s, int i, double u, double T0)
{
    if (!(u > 0.0) || !isfinite(u)) return -1.0;
    double lo = 0.0, hi = T0 > 0.0 ? T0 : 1.0;
    for (int n = 0; n < 2100 && ora_material_energy(s, i, hi) < u; ++n) { lo = hi; hi = 2.0 * hi; }
    double T = T0 > lo && T0 < hi ? T0 : 0.5 * (lo + hi);
    for (int n = 0; n < 200; ++n) {
        const double f = ora_material_energy(s, i, T) - u;
        if (f == 0.0) break;
        if (f < 0.0) lo = T; else hi = T;
        double Tn = T - f / ora_heat_capacity(s, i, T);
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        const double d = fabs(Tn - T);
        T = Tn;
        if (d <= 1e-15 * T) break;
    }
    return T;
}

/* kappa of (cell, g) at temperature T: kappa T^-q (Sec. 3.1's sigma0/sqrt(T) for
 * q = 1/2); kappa itself when q = 0. */
static double kappa_at(const ora_sim* s, size_t cg, double T)
{
    return s->p.T_power != 0.0 ? s->kappa[cg] * pow(T, -s->p.T_power) : s->kappa[cg];
}

/* Stimulated-emission factor 1 - e^{-nu/T} (Sec. 3.3), or 1 without it. */
static double stim(const ora_sim* s, double nu, double T)
{
    return s->p.opacity_stim ? -expm1(-nu / T) : 1.0;
}

/* Frequency factor of group g at temperature T: Simpson's mean over the group
 * of nu^-p, times the stimulated-emission factor when that is on. */
static double group_factor(const ora_sim* s, int g, double T)
{
    if (!s->p.opacity_stim) return s->simpson[g];
    const double p = s->p.nu_power, nl = s->nu[g], nh = s->nu[g + 1], nm = 0.5 * (nl + nh);
    return (nupow(nl, p) * stim(s, nl, T) + 4.0 * nupow(nm, p) * stim(s, nm, T)
            + nupow(nh, p) * stim(s, nh, T)) / 6.0;
}

/* Group opacity of (cell, g) at T: Simpson's rule over the group of the
 * tabulated sigma, or kappa(T) times the group factor. */
static double group_sigma(const ora_sim* s, size_t cg, int g, double T)
{
    if (s->tab_lsig) {
        const int m = s->tab_mat[cg / (size_t)s->p.G];
        const double nl = s->nu[g], nh = s->nu[g + 1], nm = 0.5 * (nl + nh);
        return (ora_table_sigma(s, m, nl, T) + 4.0 * ora_table_sigma(s, m, nm, T) + ora_table_sigma(s, m, nh, T)) / 6.0;
    }
    return kappa_at(s, cg, T) * group_factor(s, g, T);
}

/* Opacity seen by a particle of frequency nu in (cell, g) during a step: the
 * cell's temperature T^n. */
static double particle_sigma(const ora_sim* s, size_t cg, double nu, int g)
{
    const double T = s->T[cg / (size_t)s->p.G];
    if (s->tab_lsig) {
        if (s->p.flags & ORA_FLAG_GROUP_SIGMA) return group_sigma(s, cg, g, T);
        return ora_table_sigma(s, s->tab_mat[cg / (size_t)s->p.G], nu, T);
    }
    const double k = kappa_at(s, cg, T);
    if (s->p.flags & ORA_FLAG_GROUP_SIGMA) return k * group_factor(s, g, T);
    return k * nupow(nu, s->p.nu_power) * stim(s, nu, T);
}

/* Harmonic mean face opacity (Appendix B); zero if either side is zero.
 * Written symmetric in (a, b) so both cells of a face see the same value. */
static double harmonic(double a, double b)
{
    if (a + b > 0.0) return 2.0 * (a * b) / (a + b);
    return 0.0;
}

/* Ghost-cell value of phi / rho^h beyond a domain face. */
static double ghost_phi(const ora_sim* s, int side, int g, double interior)
{
    int bc = s->p.bc[side];
    if (bc == ORA_BC_PLANCK) return ora_phi_group(s->p.bcT[side], s->nu[g], s->nu[g + 1], s->p.a, s->p.c);
    if (bc == ORA_BC_REFLECT) return interior;
    return 0.0;
}

/* ---------------- the particle push (A3) ---------------- */

typedef struct { double x, y, ox, oy, nu, w; uint64_t id; int32_t cell, g; } particle;

/* Outcome: 0 survives, 1 collided (absorbed), 2 exited through the domain
 * boundary, 3 a boundary-source particle that never entered the domain.
 * ghost: 0, or 1 + the side beyond which a boundary-source particle was born
 * (in the ghost cell of that side, one cell width deep).  It flies straight and
 * without collisions (it is a new particle) until it reaches the domain face;
 * if that happens within the step, the crossing is tallied like any other and
 * its flight time is drawn in the cell it enters (Remark 1), otherwise it is
 * dropped. */
static int push_1d(ora_sim* s, particle* pp, int is_new, int ghost, double* exit_w, double* in_w,
                   int64_t* ncross)
{
    const ora_params* P = &s->p;
    const int G = P->G, nx = P->nx;
    const double e2c = P->eps * P->eps / P->c, cv = P->c / P->eps, dt = P->dt;
    int ix = pp->cell;
    int g = pp->g;
    double x = pp->x, mu = pp->ox;
    uint32_t d = 0;
    double t = 0.0, t_rem = dt;
    int coll = 0;
    if (ghost) {
        const int right = ghost - 1 == XLO;       /* entering through the low face moves right */
        const double v = cv * mu;
        if (right ? !(v > 0) : !(v < 0)) return 3;
        const double xf = right ? P->x0 : P->x0 + (double)nx * s->dx;   /* the domain faces as the cells' */
        const double te = (xf - x) / v;
        if (!(te < dt)) return 3;
        x = xf;
        t = te;
        ix = right ? 0 : nx - 1;
        const int face = right ? 0 : nx;
        s->ftx[((size_t)face * G + g) * 2 + (right ? 0 : 1)] += pp->w;
        *in_w += pp->w;
        (*ncross)++;
        double sg = particle_sigma(s, (size_t)ix * G + g, pp->nu, g);
        double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
        double a = -(e2c / sg) * log(u);
        coll = a < dt - t;
        t_rem = coll ? a : dt - t;
        is_new = 2;                               /* flight already drawn */
    }
    double sig = particle_sigma(s, (size_t)ix * G + g, pp->nu, g);
    if (is_new == 2) {
        /* a boundary-source particle inside the domain: flight set above */
    } else if (!is_new) {
        double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
        double tau = e2c / sig;
        double a = -tau * log(u);
        coll = a < dt;
        t_rem = coll ? a : dt;
    } else {
        coll = 0;
        t_rem = dt;
    }
    for (;;) {
        double v = cv * mu;
        double xl = P->x0 + (double)ix * s->dx;
        double xr = P->x0 + (double)(ix + 1) * s->dx;
        double tf;
        if (v > 0) tf = (xr - x) / v;
        else if (v < 0) tf = (xl - x) / v;
        else tf = INFINITY;
        if (tf < t_rem) {
            int right = v > 0;
            x = right ? xr : xl;
            t = t + tf;
            int face = right ? ix + 1 : ix;
            int dir = right ? 0 : 1;
            int boundary = right ? (ix == nx - 1) : (ix == 0);
            if (boundary) {
                int side = right ? XHI : XLO;
                if (P->bc[side] == ORA_BC_REFLECT) {
                    mu = -mu;
                    t_rem = t_rem - tf;
                    continue;
                }
                s->ftx[((size_t)face * G + g) * 2 + dir] += pp->w;
                *exit_w += pp->w;
                (*ncross)++;
                pp->x = x; pp->cell = ix; pp->ox = mu;
                return 2;
            }
            s->ftx[((size_t)face * G + g) * 2 + dir] += pp->w;
            (*ncross)++;
            ix += right ? 1 : -1;
            sig = particle_sigma(s, (size_t)ix * G + g, pp->nu, g);
            double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
            double tau = e2c / sig;
            double a = -tau * log(u);
            coll = a < dt - t;
            t_rem = coll ? a : dt - t;
        } else {
            double xn = x + v * t_rem;
            if (xn < xl) xn = xl;
            if (xn > xr) xn = xr;
            x = xn;
            break;
        }
    }
    pp->x = x; pp->cell = ix; pp->ox = mu;
    return coll ? 1 : 0;
}

static int push_2d(ora_sim* s, particle* pp, int is_new, int ghost, double* exit_w, double* in_w,
                   int64_t* ncross)
{
    const ora_params* P = &s->p;
    const int G = P->G, nx = P->nx, ny = P->ny;
    const double e2c = P->eps * P->eps / P->c, cv = P->c / P->eps, dt = P->dt;
    int ix = pp->cell % nx, iy = pp->cell / nx;
    int g = pp->g;
    double x = pp->x, y = pp->y, ox = pp->ox, oy = pp->oy;
    uint32_t d = 0;
    double t = 0.0, t_rem = dt;
    int coll = 0;
    if (ghost) {
        /* the straight line from the ghost cell meets the domain's face plane at
         * time te; it enters if te < dt and the meeting point lies on the domain's
         * side (the cell it enters holds that point) */
        const int side = ghost - 1;
        const double vx = cv * ox, vy = cv * oy;
        const int xside = side == XLO || side == XHI;
        const int lo = side == XLO || side == YLO;
        const double vn = xside ? vx : vy;
        if (lo ? !(vn > 0) : !(vn < 0)) return 3;
        /* the domain's faces and extent as the cells' faces are computed */
        const double xend = P->x0 + (double)nx * s->dx, yend = P->y0 + (double)ny * s->dy;
        const double pf = xside ? (lo ? P->x0 : xend) : (lo ? P->y0 : yend);
        const double te = (pf - (xside ? x : y)) / vn;
        if (!(te < dt)) return 3;
        if (xside) {
            double ye = y + vy * te;
            if (ye < P->y0 || ye > yend) return 3;
            iy = (int)floor((ye - P->y0) / s->dy);
            if (iy > ny - 1) iy = ny - 1;
            if (iy < 0) iy = 0;
            const double yl = P->y0 + (double)iy * s->dy, yr = P->y0 + (double)(iy + 1) * s->dy;
            y = ye < yl ? yl : (ye > yr ? yr : ye);
            x = pf;
            ix = lo ? 0 : nx - 1;
            const int face = iy * (nx + 1) + (lo ? 0 : nx);
            s->ftx[((size_t)face * G + g) * 2 + (lo ? 0 : 1)] += pp->w;
        } else {
            double xe = x + vx * te;
            if (xe < P->x0 || xe > xend) return 3;
            ix = (int)floor((xe - P->x0) / s->dx);
            if (ix > nx - 1) ix = nx - 1;
            if (ix < 0) ix = 0;
            const double xl = P->x0 + (double)ix * s->dx, xr = P->x0 + (double)(ix + 1) * s->dx;
            x = xe < xl ? xl : (xe > xr ? xr : xe);
            y = pf;
            iy = lo ? 0 : ny - 1;
            const int face = (lo ? 0 : ny) * nx + ix;
            s->fty[((size_t)face * G + g) * 2 + (lo ? 0 : 1)] += pp->w;
        }
        t = te;
        *in_w += pp->w;
        (*ncross)++;
        double sg = particle_sigma(s, ((size_t)iy * nx + ix) * G + g, pp->nu, g);
        double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
        double a = -(e2c / sg) * log(u);
        coll = a < dt - t;
        t_rem = coll ? a : dt - t;
        is_new = 2;
    }
    double sig = particle_sigma(s, ((size_t)iy * nx + ix) * G + g, pp->nu, g);
    if (is_new == 2) {
        /* a boundary-source particle inside the domain: flight set above */
    } else if (!is_new) {
        double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
        double tau = e2c / sig;
        double a = -tau * log(u);
        coll = a < dt;
        t_rem = coll ? a : dt;
    } else {
        coll = 0;
        t_rem = dt;
    }
    for (;;) {
        double vx = cv * ox, vy = cv * oy;
        double xl = P->x0 + (double)ix * s->dx, xr = P->x0 + (double)(ix + 1) * s->dx;
        double yl = P->y0 + (double)iy * s->dy, yr = P->y0 + (double)(iy + 1) * s->dy;
        double tx, ty;
        if (vx > 0) tx = (xr - x) / vx;
        else if (vx < 0) tx = (xl - x) / vx;
        else tx = INFINITY;
        if (vy > 0) ty = (yr - y) / vy;
        else if (vy < 0) ty = (yl - y) / vy;
        else ty = INFINITY;
        int xaxis = tx <= ty;
        double tf = xaxis ? tx : ty;
        if (tf < t_rem) {
            t = t + tf;
            int pos, boundary, side;
            size_t bin;
            if (xaxis) {
                pos = vx > 0;
                x = pos ? xr : xl;
                double yn = y + vy * tf;
                if (yn < yl) yn = yl;
                if (yn > yr) yn = yr;
                y = yn;
                boundary = pos ? (ix == nx - 1) : (ix == 0);
                side = pos ? XHI : XLO;
                int face = iy * (nx + 1) + (pos ? ix + 1 : ix);
                bin = ((size_t)face * G + g) * 2 + (pos ? 0 : 1);
            } else {
                pos = vy > 0;
                y = pos ? yr : yl;
                double xn = x + vx * tf;
                if (xn < xl) xn = xl;
                if (xn > xr) xn = xr;
                x = xn;
                boundary = pos ? (iy == ny - 1) : (iy == 0);
                side = pos ? YHI : YLO;
                int face = (pos ? iy + 1 : iy) * nx + ix;
                bin = ((size_t)face * G + g) * 2 + (pos ? 0 : 1);
            }
            double* tally = xaxis ? s->ftx : s->fty;
            if (boundary) {
                if (P->bc[side] == ORA_BC_REFLECT) {
                    if (xaxis) ox = -ox; else oy = -oy;
                    t_rem = t_rem - tf;
                    continue;
                }
                tally[bin] += pp->w;
                *exit_w += pp->w;
                (*ncross)++;
                pp->x = x; pp->y = y; pp->ox = ox; pp->oy = oy; pp->cell = iy * nx + ix;
                return 2;
            }
            tally[bin] += pp->w;
            (*ncross)++;
            if (xaxis) ix += pos ? 1 : -1; else iy += pos ? 1 : -1;
            sig = particle_sigma(s, ((size_t)iy * nx + ix) * G + g, pp->nu, g);
            double u = ora_uniform(P->seed, pp->id, (uint32_t)s->step, ORA_PURPOSE_FLIGHT, d++);
            double tau = e2c / sig;
            double a = -tau * log(u);
            coll = a < dt - t;
            t_rem = coll ? a : dt - t;
        } else {
            double xn = x + vx * t_rem, yn = y + vy * t_rem;
            if (xn < xl) xn = xl;
            if (xn > xr) xn = xr;
            if (yn < yl) yn = yl;
            if (yn > yr) yn = yr;
            x = xn; y = yn;
            break;
        }
    }
    pp->x = x; pp->y = y; pp->ox = ox; pp->oy = oy; pp->cell = iy * nx + ix;
    return coll ? 1 : 0;
}

/* ---------------- the macroscopic part ---------------- */

/* Per-face diffusion coefficient D = -(c/eps)^2 (1/3) C2(s_f) / h >= 0 so that the
 * equilibrium flux through a face with normal +n is -D (phi_next - phi_this). */
static double face_D(const ora_sim* s, double sigf, double h)
{
    const ora_params* P = &s->p;
    double sf = P->c * sigf * P->dt / (P->eps * P->eps);
    double c2 = P->dt * ora_coef_c2_over_dt(sf);
    return -(P->c * P->c / (3.0 * P->eps * P->eps)) * c2 / h;
}

/* Neighbour description for one of the 2*dim faces of a cell. */
typedef struct { int nb; int side; double S; double h; int tx, ty; } nbface;

static int cell_faces(const ora_sim* s, int i, nbface f[4])
{
    const ora_params* P = &s->p;
    int nx = P->nx, ny = P->ny, ix = i % nx, iy = i / nx;
    int n = 0;
    f[n].nb = ix > 0 ? i - 1 : -1; f[n].side = XLO; f[n].S = s->dy; f[n].h = s->dx; n++;
    f[n].nb = ix < nx - 1 ? i + 1 : -1; f[n].side = XHI; f[n].S = s->dy; f[n].h = s->dx; n++;
    if (P->dim == 2) {
        f[n].nb = iy > 0 ? i - nx : -1; f[n].side = YLO; f[n].S = s->dx; f[n].h = s->dy; n++;
        f[n].nb = iy < ny - 1 ? i + nx : -1; f[n].side = YHI; f[n].S = s->dx; f[n].h = s->dy; n++;
    }
    return n;
}

/* Gross particle crossing into / out of (cell i, group g) during the step. */
static void cell_particle_flux(const ora_sim* s, int i, int g, double* in, double* out)
{
    const ora_params* P = &s->p;
    int nx = P->nx, G = P->G, ix = i % nx, iy = i / nx;
    size_t fl = (size_t)iy * (nx + 1) + ix, fr = fl + 1;
    double a_in = s->ftx[(fl * G + g) * 2 + 0] + s->ftx[(fr * G + g) * 2 + 1];
    double a_out = s->ftx[(fl * G + g) * 2 + 1] + s->ftx[(fr * G + g) * 2 + 0];
    if (P->dim == 2) {
        size_t fb = (size_t)iy * nx + ix, ft = (size_t)(iy + 1) * nx + ix;
        a_in += s->fty[(fb * G + g) * 2 + 0] + s->fty[(ft * G + g) * 2 + 1];
        a_out += s->fty[(fb * G + g) * 2 + 1] + s->fty[(ft * G + g) * 2 + 0];
    }
    *in = a_in; *out = a_out;
}

static void rec_push(ora_sim* s, const double* rhoh, const double* wnet, const unsigned char* sampled)
{
    size_t ncg = (size_t)s->ncell * s->p.G;
    if (s->nrec == s->caprec) {
        s->caprec = s->caprec ? 2 * s->caprec : 16;
        s->rec = (ora_rec_step*)realloc(s->rec, sizeof(ora_rec_step) * s->caprec);
    }
    ora_rec_step* r = &s->rec[s->nrec++];
    r->rho = (double*)malloc(sizeof(double) * ncg); memcpy(r->rho, s->rho, sizeof(double) * ncg);
    r->T = (double*)malloc(sizeof(double) * s->ncell); memcpy(r->T, s->T, sizeof(double) * s->ncell);
    r->rhop = (double*)malloc(sizeof(double) * ncg); memcpy(r->rhop, s->rhop, sizeof(double) * ncg);
    r->rhoh = (double*)malloc(sizeof(double) * ncg); memcpy(r->rhoh, rhoh, sizeof(double) * ncg);
    r->wnet = (double*)malloc(sizeof(double) * ncg); memcpy(r->wnet, wnet, sizeof(double) * ncg);
    r->sampled = (unsigned char*)malloc(ncg); memcpy(r->sampled, sampled, ncg);
}

/* ---------------- second-order wave part (Sec. 2.2, the C5 terms) ---------------- */

/* minmod of two undivided differences: 0 when they differ in sign, else the
 * one of smaller magnitude. */
static double minmod(double a, double b)
{
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* Slopes of the wave part rho^h per cell and group along x (and y): MINMOD of
 * the differences to the two neighbours, with the boundary ghost one cell width
 * away (Planckian phi(T_b), vacuum 0, reflective the mirror image), then scaled
 * down where needed so that the linear profile stays non-negative over the
 * cell (|s_x| dx + |s_y| dy <= 2 rho^h); zero where rho^h <= 0. */
static void wave_slopes(const ora_sim* s, const double* rhoh, double* sx, double* sy)
{
    const ora_params* P = &s->p;
    const int G = P->G, nx = P->nx, ny = P->ny;
    for (int i = 0; i < s->ncell; ++i) {
        const int ix = i % nx, iy = i / nx;
        for (int g = 0; g < G; ++g) {
            const size_t k = (size_t)i * G + g;
            const double c0 = rhoh[k];
            double l = ix > 0 ? rhoh[k - G] : ghost_phi(s, XLO, g, c0);
            double r = ix < nx - 1 ? rhoh[k + G] : ghost_phi(s, XHI, g, c0);
            double ax = minmod(c0 - l, r - c0) / s->dx, ay = 0.0;
            if (P->dim == 2) {
                double b = iy > 0 ? rhoh[k - (size_t)nx * G] : ghost_phi(s, YLO, g, c0);
                double t = iy < ny - 1 ? rhoh[k + (size_t)nx * G] : ghost_phi(s, YHI, g, c0);
                ay = minmod(c0 - b, t - c0) / s->dy;
            }
            if (!(c0 > 0.0)) {
                ax = 0.0;
                ay = 0.0;
            } else {
                const double tot = fabs(ax) * s->dx + fabs(ay) * s->dy;
                if (tot > 2.0 * c0) {
                    const double f = 2.0 * c0 / tot;
                    ax = ax * f;
                    ay = ay * f;
                }
            }
            sx[k] = ax;
            if (sy) sy[k] = ay;
        }
    }
}

/* The volumetric source adds to this step (it starts before the switch-off time). */
static int src_on(const ora_sim* s)
{
    return s->qsrc != NULL && (double)s->step * s->p.dt < s->q_toff;
}

/* The wave part's free-transport flux (Sec. 2.2, F^{fr,wave}, with Remark 3's
 * choice of coefficient) and the static source Q = rho^n + (dt/V) sum_f S_f F_in
 * + w^{fr,p}/V of every cell and group, from the wave part rhoh.  Through a face
 * with normal +axis between cells L and R:
 *   F = (c/4eps) [A_L rho^h_L(face) - A_R rho^h_R(face)] + (c^2/6eps^2) [B_L s_L + B_R s_R]
 * where rho^h(face) is the upwind cell's linear profile at the face and s its
 * slope along the axis (angular moments 1/4 and 1/6 of an isotropic intensity
 * over a half sphere), A = C4 - e^{-s} (or C4 unsampled), B = C5 + (dt/2) e^{-s}
 * (or C5 unsampled).  Without slopes the second term and the profile vanish.
 * A Planckian ghost holds phi(T_b) with the interior cell's s, coefficient C4
 * (W when it emitted boundary particles); vacuum 0; a mirror no flux.
 * Returns the energy flowing in through the domain boundary over the step. */
static double wave_source(ora_sim* s, const double* rhoh, const double* sx, const double* sy,
                          const double* A, const double* Bw, const double* sv,
                          const unsigned char* gsamp, const double* wnet, double* Q)
{
    const ora_params* P = &s->p;
    const int G = P->G, nc = s->ncell;
    const double c = P->c, eps = P->eps, dt = P->dt, V = s->V;
    const double cq = c / (4.0 * eps);
    const double cs = c * c * dt / (6.0 * eps * eps);
    double inflow = 0.0;
    for (int i = 0; i < nc; ++i) {
        nbface f[4];
        int nf = cell_faces(s, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            double fsum = 0.0;   /* sum over faces of S * (flux into the cell) */
            for (int q = 0; q < nf; ++q) {
                /* outward sign: the LO faces have inward normal +axis */
                int lo = (f[q].side == XLO || f[q].side == YLO);
                double Fpos;
                if (!sx) {
                    double here = A[k] * rhoh[k];
                    double there;
                    if (f[q].nb >= 0) {
                        size_t kn = (size_t)f[q].nb * G + g;
                        there = A[kn] * rhoh[kn];
                    } else {
                        int bc = P->bc[f[q].side];
                        if (bc == ORA_BC_REFLECT) continue;
                        double Ag = gsamp && gsamp[k * 4 + f[q].side] ? ora_coef_w(sv[k]) : ora_coef_c4(sv[k]);
                        there = (bc == ORA_BC_PLANCK) ? Ag * ghost_phi(s, f[q].side, g, 0.0) : 0.0;
                    }
                    /* flux along +axis through the face: cq (A_left rho^h_left - A_right rho^h_right) */
                    Fpos = lo ? cq * (there - here) : cq * (here - there);
                } else {
                    const int xaxis = f[q].side == XLO || f[q].side == XHI;
                    const double* sl = xaxis ? sx : sy;
                    /* this cell is the right cell of a LO face and the left cell of a HI face */
                    double here = A[k] * (rhoh[k] + (lo ? -0.5 : 0.5) * f[q].h * sl[k]);
                    double hs = Bw[k] * sl[k];
                    double there, ts = 0.0;
                    if (f[q].nb >= 0) {
                        size_t kn = (size_t)f[q].nb * G + g;
                        there = A[kn] * (rhoh[kn] + (lo ? 0.5 : -0.5) * f[q].h * sl[kn]);
                        ts = Bw[kn] * sl[kn];
                    } else {
                        int bc = P->bc[f[q].side];
                        if (bc == ORA_BC_REFLECT) continue;
                        double Ag = gsamp && gsamp[k * 4 + f[q].side] ? ora_coef_w(sv[k]) : ora_coef_c4(sv[k]);
                        there = (bc == ORA_BC_PLANCK) ? Ag * ghost_phi(s, f[q].side, g, 0.0) : 0.0;
                    }
                    Fpos = lo ? cq * (there - here) + cs * (ts + hs) : cq * (here - there) + cs * (hs + ts);
                }
                double Fin = lo ? Fpos : -Fpos;
                fsum += f[q].S * Fin;
                if (f[q].nb < 0) inflow += dt * f[q].S * Fin / c;
            }
            Q[k] = s->rho[k] + (dt / V) * fsum + wnet[k] / V;
            if (src_on(s)) Q[k] = Q[k] + dt * s->qsrc[k];
        }
    }
    return inflow;
}

/* Place a new particle's position along the slope of its cell's wave part:
 * density 1 + bx u + by v over the cell (u, v the offsets from the centre in
 * cell widths), x from its marginal, y from its conditional given x; the same
 * uniform draws as the uniform placement, which a zero slope reproduces. */
static void place_on_slope(double xl, double dx, double yl, double dy, double bx, double by,
                           double U0, double U1, int dim, double* x, double* y)
{
    double ux = 0.0;
    if (bx == 0.0) {
        *x = xl + U0 * dx;
        ux = U0 - 0.5;
    } else {
        ux = ora_linear_offset(bx, U0);
        *x = (xl + 0.5 * dx) + ux * dx;
    }
    if (dim == 2) {
        const double bc = by / (1.0 + bx * ux);
        if (bc == 0.0) *y = yl + U1 * dy;
        else *y = (yl + 0.5 * dy) + ora_linear_offset(bc, U1) * dy;
    }
}

static int step_once(ora_sim* s)
{
    const ora_params* P = &s->p;
    const int G = P->G, nc = s->ncell;
    const size_t ncg = (size_t)nc * G;
    const double V = s->V, dt = P->dt, c = P->c, eps = P->eps;
    ora_diag dg;
    memset(&dg, 0, sizeof(dg));

    /* ---- coefficients (A0) ---- */
    double* sig = (double*)malloc(sizeof(double) * ncg);
    double* sv = (double*)malloc(sizeof(double) * ncg);
    double* es = (double*)malloc(sizeof(double) * ncg);
    double* rhoh = (double*)malloc(sizeof(double) * ncg);
    double* A = (double*)malloc(sizeof(double) * ncg);
    double* wnet = (double*)malloc(sizeof(double) * ncg);
    unsigned char* sampled = (unsigned char*)malloc(ncg);
    double* wsamp = (double*)malloc(sizeof(double) * ncg);
    const int slopes = (P->flags & ORA_FLAG_SLOPES) != 0;
    const int wave_iter = (P->flags & ORA_FLAG_WAVE_ITER) != 0;
    const int bpart = (P->flags & ORA_FLAG_BOUNDARY_PARTICLES) != 0;
    /* slope coefficient B of a sampled cell / 1 (Bw), slopes of rho^h (sx, sy) */
    double* w5samp = slopes ? (double*)malloc(sizeof(double) * ncg) : NULL;
    double* Bw = slopes ? (double*)malloc(sizeof(double) * ncg) : NULL;
    double* sx = slopes ? (double*)malloc(sizeof(double) * ncg) : NULL;
    double* sy = slopes && P->dim == 2 ? (double*)calloc(ncg, sizeof(double)) : NULL;
    /* boundary-source particles: births per (cell, group) and side, and whether
     * the ghost beyond that side sampled any */
    int64_t* ngh = bpart ? (int64_t*)calloc(ncg * 4, sizeof(int64_t)) : NULL;
    unsigned char* gsamp = bpart ? (unsigned char*)calloc(ncg * 4, 1) : NULL;
    for (int i = 0; i < nc; ++i)
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            sig[k] = group_sigma(s, k, g, s->T[i]);
            sv[k] = c * sig[k] * dt / (eps * eps);
            es[k] = exp(-sv[k]);
            wsamp[k] = ora_coef_w(sv[k]);
            if (slopes) w5samp[k] = ora_coef_w5_over_dt(sv[k]);
        }
    /* Thin-thick-joint cells (Sec. 3.2, second case): the sampling fraction
     * e^{-dt/tau_num} with tau_num = tau + C * delta * dt, delta the largest
     * |T^l - T^r| / (T^l + T^r) over the cell's faces across which sigma_g
     * jumps by a factor >= jump (T^n, the temperatures the step starts from).
     * dt/tau_num = s / (1 + s C delta); the wave part of a sampled cell keeps
     * C4(s) - e^{-dt/tau_num} = W(s) - (e^{-dt/tau_num} - e^{-s}) (Remark 3
     * with the larger sampled share). */
    if (P->tau_num_C > 0.0) {
        for (int i = 0; i < nc; ++i) {
            nbface f[4];
            int nf = cell_faces(s, i, f);
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double delta = -1.0;
                for (int q = 0; q < nf; ++q) {
                    if (f[q].nb < 0) continue;
                    size_t kn = (size_t)f[q].nb * G + g;
                    double hi = sig[k] > sig[kn] ? sig[k] : sig[kn];
                    double lo = sig[k] > sig[kn] ? sig[kn] : sig[k];
                    if (!(hi > 0.0) || hi < P->tau_num_jump * lo) continue;
                    double Tl = s->T[i], Tr = s->T[f[q].nb];
                    double d = fabs(Tl - Tr) / (Tl + Tr);
                    if (d > delta) delta = d;
                }
                if (delta < 0.0) continue;
                double snum = sv[k] / (1.0 + sv[k] * P->tau_num_C * delta);
                es[k] = exp(-snum);
                /* e^{-snum} - e^{-s}: by expm1 where the two are close */
                double d = sv[k] - snum;
                double diff = d < 0.5 ? exp(-sv[k]) * expm1(d) : exp(-snum) - exp(-sv[k]);
                wsamp[k] = ora_coef_w(sv[k]) - diff;
                /* the slope coefficient C5 + (dt/2) e^{-dt/tau_num} likewise */
                if (slopes) w5samp[k] = ora_coef_w5_over_dt(sv[k]) + 0.5 * diff;
            }
        }
    }

    /* ---- wave split and sample counts (A1) ---- */
    int64_t total = 0;
    for (size_t k = 0; k < ncg; ++k) {
        rhoh[k] = s->rho[k] - s->rhop[k];
        double e_over_v = es[k] * rhoh[k];
        double E = e_over_v * V;
        int64_t N = 0;
        if (E > 0.0) {
            double q = e_over_v / P->w_ref;
            if (q >= (double)P->n_cap) N = P->n_cap;
            else N = (int64_t)floor(q);
        }
        s->nb[k] = N;
        s->wnew[k] = N >= 1 ? E / (double)N : 0.0;
        sampled[k] = N >= 1;
        total += N;
    }
    /* Boundary-source particles: the ghost cell beyond a Planckian side holds
     * rho^h = phi(T_b) and the interior cell's opacity (the ghost of the wave
     * flux), so its collisionless part e^{-s} phi(T_b) V is sampled like an
     * interior cell's (same count rule and weight E/N).  Its births follow the
     * interior births of the adjacent (cell, group), side by side. */
    int64_t total_ghost = 0;
    if (bpart) {
        for (int i = 0; i < nc; ++i) {
            int ix = i % P->nx, iy = i / P->nx;
            for (int side = 0; side < 4; ++side) {
                if (P->bc[side] != ORA_BC_PLANCK) continue;
                int adj = side == XLO ? ix == 0 : side == XHI ? ix == P->nx - 1
                        : side == YLO ? (P->dim == 2 && iy == 0) : (P->dim == 2 && iy == P->ny - 1);
                if (!adj) continue;
                for (int g = 0; g < G; ++g) {
                    size_t k = (size_t)i * G + g;
                    double e_over_v = exp(-sv[k]) * ghost_phi(s, side, g, 0.0);
                    int64_t N = 0;
                    if (e_over_v * V > 0.0) {
                        double q = e_over_v / P->w_ref;
                        if (q >= (double)P->n_cap) N = P->n_cap;
                        else N = (int64_t)floor(q);
                    }
                    ngh[k * 4 + side] = N;
                    gsamp[k * 4 + side] = N >= 1;
                    s->nb[k] += N;
                    total_ghost += N;
                }
            }
        }
    }
    int64_t n_old = s->np;
    if (n_old + total + total_ghost > P->pool_cap) {
        free(sig); free(sv); free(es); free(wsamp); free(rhoh); free(A); free(wnet); free(sampled);
        free(w5samp); free(Bw); free(sx); free(sy); free(ngh); free(gsamp);
        return ORA_EPOOL;
    }
    dg.n_alive_in = n_old;
    dg.n_births = total + total_ghost;
    dg.n_ghost_births = total_ghost;
    if (slopes) wave_slopes(s, rhoh, sx, sy);

    /* ---- sample the collisionless wave particles (A2) ---- */
    int64_t slot = n_old;
    uint64_t id = s->nbirth;
    int64_t n_all = n_old + total + total_ghost;
    /* ghost side + 1 of every boundary-source particle of this step (0: not one) */
    unsigned char* gside = bpart ? (unsigned char*)calloc((size_t)(n_all > 0 ? n_all : 1), 1) : NULL;
    for (int i = 0; i < nc; ++i) {
        int ix = i % P->nx, iy = i / P->nx;
        double xl = P->x0 + (double)ix * s->dx;
        double yl = P->y0 + (double)iy * s->dy;
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            if (s->nb[k] == 0) continue;
            double nl = s->nu[g], nh = s->nu[g + 1];
            /* the slopes of the wave part, in cell widths per rho^h */
            double bx = 0.0, by = 0.0;
            if (slopes && rhoh[k] > 0.0) {
                bx = sx[k] * s->dx / rhoh[k];
                if (P->dim == 2) by = sy[k] * s->dy / rhoh[k];
            }
            /* the interior births of (i, g), then those of the ghosts beyond
             * its Planckian sides */
            int64_t nint = s->nb[k];
            if (bpart) for (int side = 0; side < 4; ++side) nint -= ngh[k * 4 + side];
            for (int part = -1; part < 4; ++part) {
                int64_t n = part < 0 ? nint : (bpart ? ngh[k * 4 + part] : 0);
                if (n == 0) continue;
                double Tq = part < 0 ? s->T[i] : P->bcT[part];
                double beta = ora_freq_slope(nl, nh, Tq);
                double wq = part < 0 ? s->wnew[k] : exp(-sv[k]) * ghost_phi(s, part, g, 0.0) * V / (double)n;
                /* the cell the particles are placed in: the interior cell, or its
                 * ghost one cell width beyond the side */
                double cxl = xl, cyl = yl;
                if (part == XLO) cxl = xl - s->dx;
                if (part == XHI) cxl = xl + s->dx;
                if (part == YLO) cyl = yl - s->dy;
                if (part == YHI) cyl = yl + s->dy;
                for (int64_t j = 0; j < n; ++j, ++id, ++slot) {
                    uint32_t st = (uint32_t)s->step;
                    double U0 = ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 0);
                    double U1 = ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 1);
                    double px, py = 0.0;
                    if (part < 0 && (bx != 0.0 || by != 0.0)) {
                        place_on_slope(cxl, s->dx, cyl, s->dy, bx, by, U0, U1, P->dim, &px, &py);
                    } else {
                        px = cxl + U0 * s->dx;
                        if (P->dim == 2) py = cyl + U1 * s->dy;
                    }
                    s->px[slot] = px;
                    if (P->dim == 1) {
                        s->pox[slot] = 2.0 * U1 - 1.0;
                        s->py[slot] = 0.0;
                        s->poy[slot] = 0.0;
                        s->pnu[slot] = ora_sample_nu(nl, nh, beta, ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 2));
                    } else {
                        s->py[slot] = py;
                        double oz = 2.0 * ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 2) - 1.0;
                        double psi = 6.283185307179586 * ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 3);
                        double sn = sqrt(1.0 - oz * oz);
                        s->pox[slot] = sn * cos(psi);
                        s->poy[slot] = sn * sin(psi);
                        s->pnu[slot] = ora_sample_nu(nl, nh, beta, ora_uniform(P->seed, id, st, ORA_PURPOSE_BIRTH, 4));
                    }
                    s->pw[slot] = wq;
                    s->pid[slot] = id;
                    s->pcell[slot] = i;
                    s->pg[slot] = g;
                    if (part >= 0) gside[slot] = (unsigned char)(part + 1);
                }
            }
        }
    }

    /* ---- free transport of every particle (A3) ---- */
    size_t nfx = (size_t)(P->nx + 1) * P->ny, nfy = (size_t)P->nx * (P->ny + 1);
    memset(s->ftx, 0, sizeof(double) * nfx * G * 2);
    memset(s->fty, 0, sizeof(double) * nfy * G * 2);
    memset(s->dep, 0, sizeof(double) * ncg);
    memset(s->surv, 0, sizeof(double) * ncg);
    memset(s->start, 0, sizeof(double) * ncg);
    double exit_w = 0.0, in_w = 0.0;
    int64_t ncross = 0, keep = 0;
    for (int64_t k = 0; k < n_all; ++k) {
        particle pp = { s->px[k], s->py[k], s->pox[k], s->poy[k], s->pnu[k], s->pw[k],
                        s->pid[k], s->pcell[k], s->pg[k] };
        const int gk = gside ? gside[k] : 0;
        if (!gk) s->start[(size_t)pp.cell * G + pp.g] += pp.w;
        int out = (P->dim == 1) ? push_1d(s, &pp, k >= n_old, gk, &exit_w, &in_w, &ncross)
                                : push_2d(s, &pp, k >= n_old, gk, &exit_w, &in_w, &ncross);
        if (gk && out != 3) dg.n_ghost_entered++;
        size_t kk = (size_t)pp.cell * G + pp.g;
        if (out == 3) { /* never entered */ }
        else if (out == 1) { s->dep[kk] += pp.w; dg.n_collided++; }
        else if (out == 2) { dg.n_exited++; }
        else {
            s->surv[kk] += pp.w;
            s->px[keep] = pp.x; s->py[keep] = pp.y; s->pox[keep] = pp.ox; s->poy[keep] = pp.oy;
            s->pnu[keep] = pp.nu; s->pw[keep] = pp.w; s->pid[keep] = pp.id;
            s->pcell[keep] = pp.cell; s->pg[keep] = pp.g;
            keep++;
        }
    }
    dg.n_alive_out = keep;
    dg.n_crossings = ncross;
    dg.exit_particles = exit_w / c;
    dg.inflow_particles = in_w / c;

    /* ---- wave free-transport flux and the static source Q (A4) ---- */
    for (size_t k = 0; k < ncg; ++k) A[k] = sampled[k] ? wsamp[k] : ora_coef_c4(sv[k]);
    if (slopes)
        for (size_t k = 0; k < ncg; ++k) Bw[k] = sampled[k] ? w5samp[k] : ora_coef_c5_over_dt(sv[k]);
    for (int i = 0; i < nc; ++i)
        for (int g = 0; g < G; ++g) {
            double in, out;
            cell_particle_flux(s, i, g, &in, &out);
            wnet[(size_t)i * G + g] = in - out;
        }
    dg.inflow_wave = wave_source(s, rhoh, sx, sy, A, Bw, sv, gsamp, wnet, s->Q);
    /* with the wave flux taken from the iterate (Algorithm 2), each sweep forms
     * Q again from rho^{h,k} = rho^k - rho^p (k = 0: the above) */
    double* rhk = wave_iter ? (double*)malloc(sizeof(double) * ncg) : NULL;

    /* ---- source iteration for Eq. macroSysFinal (A5; Appendix B, Algorithm 2) ---- */
    /* With a temperature-dependent opacity every sweep first recomputes sigma,
     * lambda = c sigma dt / eps^2 and the face coefficients from its iterate
     * T^k (the coefficient step of Algorithm 2); otherwise they are the step's. */
    const int tdep = P->T_power != 0.0 || P->opacity_stim || s->tab_lsig != NULL;
    /* Linearized variant: the emission of the new temperature is taken as
     * phi^k + phi'(T^k) (T^{k+1} - T^k), so each cell's energy balance is solved
     * for T^{k+1} as one local Newton step; its fixed point is that of the
     * literal iteration (Eq. macroSysFinal). */
    const int lin = (P->flags & ORA_FLAG_SI_LINEARIZED) != 0;
    double* dph = lin ? (double*)malloc(sizeof(double) * ncg) : NULL;
    double* bk = (double*)malloc(sizeof(double) * G);
    double* sigk = tdep ? (double*)malloc(sizeof(double) * ncg) : sig;
    double* lam = tdep ? (double*)malloc(sizeof(double) * ncg) : sv;    /* c sigma dt / eps^2 */
    double* phi = (double*)malloc(sizeof(double) * ncg);
    double* phin = (double*)malloc(sizeof(double) * ncg);
    double* rk = (double*)malloc(sizeof(double) * ncg);
    double* Tk = (double*)malloc(sizeof(double) * nc);
    double* Tn1 = (double*)malloc(sizeof(double) * nc);
    double* uend = (double*)malloc(sizeof(double) * nc);      /* material energy the last sweep gave */
    double* rn1 = (double*)malloc(sizeof(double) * ncg);
    double* em = (double*)malloc(sizeof(double) * ncg);
    /* face coefficients D for the 2*dim faces of every cell */
    double* Df = (double*)malloc(sizeof(double) * ncg * 4);
    for (int i = 0; i < nc; ++i) {
        nbface f[4];
        int nf = cell_faces(s, i, f);
        for (int g = 0; g < G; ++g) {
            size_t k = (size_t)i * G + g;
            for (int q = 0; q < nf; ++q) {
                double sf = f[q].nb >= 0 ? harmonic(sig[k], sig[(size_t)f[q].nb * G + g]) : sig[k];
                Df[k * 4 + q] = face_D(s, sf, f[q].h);
            }
        }
    }
    for (int i = 0; i < nc; ++i) {
        Tk[i] = s->T[i];
        for (int g = 0; g < G; ++g)
            phi[(size_t)i * G + g] = ora_phi_group(s->T[i], s->nu[g], s->nu[g + 1], P->a, c);
    }
    memcpy(rk, s->rho, sizeof(double) * ncg);
    int converged = 0, sweeps = 0, bad = 0;
    double drho = 0, mrho = 0, dT = 0, mT = 0;
    for (int it = 0; it < P->si_max_iters; ++it) {
        if (wave_iter && it > 0) {
            for (size_t k = 0; k < ncg; ++k) rhk[k] = rk[k] - s->rhop[k];
            if (slopes) wave_slopes(s, rhk, sx, sy);
            dg.inflow_wave = wave_source(s, rhk, sx, sy, A, Bw, sv, gsamp, wnet, s->Q);
        }
        if (tdep) {
            for (int i = 0; i < nc; ++i)
                for (int g = 0; g < G; ++g) {
                    size_t k = (size_t)i * G + g;
                    sigk[k] = group_sigma(s, k, g, Tk[i]);
                    lam[k] = c * sigk[k] * dt / (eps * eps);
                }
            for (int i = 0; i < nc; ++i) {
                nbface f[4];
                int nf = cell_faces(s, i, f);
                for (int g = 0; g < G; ++g) {
                    size_t k = (size_t)i * G + g;
                    for (int q = 0; q < nf; ++q) {
                        double sf = f[q].nb >= 0 ? harmonic(sigk[k], sigk[(size_t)f[q].nb * G + g]) : sigk[k];
                        Df[k * 4 + q] = face_D(s, sf, f[q].h);
                    }
                }
            }
        }
        if (lin)
            for (int i = 0; i < nc; ++i)
                for (int g = 0; g < G; ++g)
                    dph[(size_t)i * G + g] = ora_dphi_group(Tk[i], s->nu[g], s->nu[g + 1], P->a, c);
        drho = mrho = dT = mT = 0.0;
        for (int i = 0; i < nc; ++i) {
            nbface f[4];
            int nf = cell_faces(s, i, f);
            double sum = 0.0, dsum = 0.0;
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                double lap = 0.0;
                for (int q = 0; q < nf; ++q) {
                    double pn = f[q].nb >= 0 ? phi[(size_t)f[q].nb * G + g]
                                             : ghost_phi(s, f[q].side, g, phi[k]);
                    lap += f[q].S * Df[k * 4 + q] * (pn - phi[k]);
                }
                /* rho^{k+1} = (b + lam phi^k)/(1 + lam) with b = Q + (dt/V) lap; the
                 * material exchange sigma (rho^{k+1} - phi^k) is evaluated through the
                 * identical expression sigma (b - phi^k)/(1 + lam), which does not cancel
                 * when lam = c sigma dt / eps^2 is large. */
                double b = s->Q[k] + (dt / V) * lap;
                bk[g] = b;
                sum += sigk[k] * (b - phi[k]) / (1.0 + lam[k]);
                if (lin) dsum += sigk[k] * dph[k] / (1.0 + lam[k]);
            }
            double Tnew;
            if (s->pinned[i]) {
                Tnew = s->T[i];
                uend[i] = ora_material_energy(s, i, Tnew);
            } else if (!olson_cell(s, i)) {
                const double w = dt / (eps * eps * s->cv[i]);
                Tnew = lin ? Tk[i] + (s->T[i] - Tk[i] + w * sum) / (1.0 + w * dsum) : s->T[i] + w * sum;
                uend[i] = s->cv[i] * Tnew;
            } else {
                /* Olson's heat capacity: the energy equation in U, U(T^{n+1}) = U(T^n) +
                 * exchange.  Literal: U(T^{k+1}) = U(T^n) + exchange(phi^k), solved for
                 * T^{k+1}.  Linearized: one Newton step at T^k, U and the emission both
                 * linearized, T^{k+1} = T^k + (U(T^n) - U(T^k) + exchange(phi^k)) /
                 * (C_v(T^k) + (dt/eps^2) sum_g sigma phi'/(1 + lam)); its material
                 * energy is U(T^k) + C_v(T^k)(T^{k+1} - T^k). */
                const double ex = dt / (eps * eps) * sum;
                const double un = ora_material_energy(s, i, s->T[i]);
                if (lin) {
                    const double uk = ora_material_energy(s, i, Tk[i]), ck = ora_heat_capacity(s, i, Tk[i]);
                    Tnew = Tk[i] + (un - uk + ex) / (ck + dt / (eps * eps) * dsum);
                    uend[i] = uk + ck * (Tnew - Tk[i]);
                } else {
                    uend[i] = un + ex;
                    Tnew = olson_temperature(s, i, uend[i], Tk[i]);
                }
            }
            /* the new temperature's emission: phi^k, or its linearization */
            const double dTi = lin && !s->pinned[i] ? Tnew - Tk[i] : 0.0;
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                const double pe = lin ? phi[k] + dph[k] * dTi : phi[k];
                double r = (bk[g] + lam[k] * pe) / (1.0 + lam[k]);
                rn1[k] = r;
                em[k] = (bk[g] - pe) / (1.0 + lam[k]);
                double dr = fabs(r - rk[k]);
                if (dr > drho || dr != dr) drho = dr;
                if (fabs(r) > mrho) mrho = fabs(r);
            }
            if (!(Tnew > 0.0) || !isfinite(Tnew)) bad = 1;
            Tn1[i] = Tnew;
            double dd = fabs(Tnew - Tk[i]);
            if (dd > dT || dd != dd) dT = dd;
            if (Tnew > mT) mT = Tnew;
        }
        sweeps = it + 1;
        if (bad) break;
        /* energy bookkeeping uses the phi^k that produced this sweep */
        if (drho <= P->si_tol * mrho && dT <= P->si_tol * mT) {
            converged = 1;
        }
        if (converged || it + 1 == P->si_max_iters) break;
        for (int i = 0; i < nc; ++i)
            for (int g = 0; g < G; ++g)
                phin[(size_t)i * G + g] = ora_phi_group(Tn1[i], s->nu[g], s->nu[g + 1], P->a, c);
        memcpy(phi, phin, sizeof(double) * ncg);
        memcpy(rk, rn1, sizeof(double) * ncg);
        memcpy(Tk, Tn1, sizeof(double) * nc);
    }
    int status = ORA_OK;
    if (bad) status = ORA_ENONFINITE;
    else if (!converged) status = ORA_ENOCONV;

    if (status == ORA_OK) {
        /* boundary equilibrium inflow and pinned-cell injection with the final phi^k */
        double inflow_eq = 0.0, inj = 0.0;
        for (int i = 0; i < nc; ++i) {
            nbface f[4];
            int nf = cell_faces(s, i, f);
            for (int g = 0; g < G; ++g) {
                size_t k = (size_t)i * G + g;
                for (int q = 0; q < nf; ++q) {
                    if (f[q].nb >= 0) continue;
                    double pn = ghost_phi(s, f[q].side, g, phi[k]);
                    inflow_eq += dt * f[q].S * Df[k * 4 + q] * (pn - phi[k]) / c;
                }
                if (s->pinned[i]) inj -= V * (dt * sigk[k] / (eps * eps)) * em[k];
                if (src_on(s)) inj += V * dt * s->qsrc[k] / c;
            }
        }
        double e0 = 0.0, e1 = 0.0;
        for (int i = 0; i < nc; ++i) {
            double r0 = 0.0, r1 = 0.0;
            for (int g = 0; g < G; ++g) { r0 += s->rho[(size_t)i * G + g]; r1 += rn1[(size_t)i * G + g]; }
            e0 += V * (r0 / c + ora_material_energy(s, i, s->T[i]));
            e1 += V * (r1 / c + uend[i]);
        }
        dg.inflow_eq = inflow_eq;
        dg.injection = inj;
        dg.e_start = e0;
        dg.e_end = e1;
        dg.residual = e1 - e0 - (dg.inflow_wave + inflow_eq + dg.inflow_particles - dg.exit_particles + inj);
        dg.sweeps = sweeps;
        dg.si_drho = drho; dg.si_rho = mrho; dg.si_dT = dT; dg.si_T = mT;

        if (s->recording) rec_push(s, rhoh, wnet, sampled);

        /* ---- commit (absorb collided particles: already dropped from the pool) ---- */
        memcpy(s->rho, rn1, sizeof(double) * ncg);
        memcpy(s->T, Tn1, sizeof(double) * nc);
        for (size_t k = 0; k < ncg; ++k) s->rhop[k] = s->surv[k] / V;
        s->np = keep;
        s->nbirth += (uint64_t)(total + total_ghost);   /* every birth takes an id, entered or not */
        s->step++;
        s->diag = dg;
    }
    free(sig); free(sv); free(es); free(wsamp); free(rhoh); free(A); free(wnet); free(sampled);
    free(phi); free(phin); free(rk); free(Tk); free(Tn1); free(rn1); free(em); free(Df); free(uend);
    free(w5samp); free(Bw); free(sx); free(sy); free(ngh); free(gsamp); free(gside); free(rhk);
    if (tdep) { free(sigk); free(lam); }
    free(dph); free(bk);
    return status;
}

int ora_step(ora_sim* s, int nsteps)
{
    if (!s->have_opacity || !s->have_material) return ORA_EINVAL;
    for (int n = 0; n < nsteps; ++n) {
        int st = step_once(s);
        if (st != ORA_OK) return st;
    }
    return ORA_OK;
}

int ora_get_fields(const ora_sim* s, double* rho, double* T, double* rhop)
{
    size_t ncg = (size_t)s->ncell * s->p.G;
    if (rho) memcpy(rho, s->rho, sizeof(double) * ncg);
    if (T) memcpy(T, s->T, sizeof(double) * s->ncell);
    if (rhop) memcpy(rhop, s->rhop, sizeof(double) * ncg);
    return ORA_OK;
}

int ora_get_tallies(const ora_sim* s, double* fx, double* fy, double* dep, double* surv,
                    int64_t* nbirth, double* wnew, double* Q)
{
    const ora_params* P = &s->p;
    size_t ncg = (size_t)s->ncell * P->G;
    size_t nfx = (size_t)(P->nx + 1) * P->ny, nfy = (size_t)P->nx * (P->ny + 1);
    if (fx) memcpy(fx, s->ftx, sizeof(double) * nfx * P->G * 2);
    if (fy) memcpy(fy, s->fty, sizeof(double) * nfy * P->G * 2);
    if (dep) memcpy(dep, s->dep, sizeof(double) * ncg);
    if (surv) memcpy(surv, s->surv, sizeof(double) * ncg);
    if (nbirth) memcpy(nbirth, s->nb, sizeof(int64_t) * ncg);
    if (wnew) memcpy(wnew, s->wnew, sizeof(double) * ncg);
    if (Q) memcpy(Q, s->Q, sizeof(double) * ncg);
    return ORA_OK;
}

int ora_get_start_weights(const ora_sim* s, double* start)
{
    memcpy(start, s->start, sizeof(double) * (size_t)s->ncell * s->p.G);
    return ORA_OK;
}

int64_t ora_pool_size(const ora_sim* s) { return s->np; }

int ora_get_pool(const ora_sim* s, double* x, double* y, double* ox, double* oy, double* nu,
                 double* w, uint64_t* id, int32_t* cell, int32_t* g)
{
    size_t n = (size_t)s->np;
    if (x) memcpy(x, s->px, sizeof(double) * n);
    if (y) memcpy(y, s->py, sizeof(double) * n);
    if (ox) memcpy(ox, s->pox, sizeof(double) * n);
    if (oy) memcpy(oy, s->poy, sizeof(double) * n);
    if (nu) memcpy(nu, s->pnu, sizeof(double) * n);
    if (w) memcpy(w, s->pw, sizeof(double) * n);
    if (id) memcpy(id, s->pid, sizeof(uint64_t) * n);
    if (cell) memcpy(cell, s->pcell, sizeof(int32_t) * n);
    if (g) memcpy(g, s->pg, sizeof(int32_t) * n);
    return ORA_OK;
}

int ora_set_pool(ora_sim* s, int64_t n, const double* x, const double* y, const double* ox,
                 const double* oy, const double* nu, const double* w, const uint64_t* id,
                 const int32_t* cell, const int32_t* g, uint64_t birth_counter, const double* rhop)
{
    if (n < 0 || n > s->p.pool_cap) return ORA_EPOOL;
    size_t k = (size_t)n;
    memcpy(s->px, x, sizeof(double) * k);
    if (y) memcpy(s->py, y, sizeof(double) * k); else memset(s->py, 0, sizeof(double) * k);
    memcpy(s->pox, ox, sizeof(double) * k);
    if (oy) memcpy(s->poy, oy, sizeof(double) * k); else memset(s->poy, 0, sizeof(double) * k);
    memcpy(s->pnu, nu, sizeof(double) * k);
    memcpy(s->pw, w, sizeof(double) * k);
    memcpy(s->pid, id, sizeof(uint64_t) * k);
    memcpy(s->pcell, cell, sizeof(int32_t) * k);
    memcpy(s->pg, g, sizeof(int32_t) * k);
    s->np = n;
    s->nbirth = birth_counter;
    if (rhop) memcpy(s->rhop, rhop, sizeof(double) * (size_t)s->ncell * s->p.G);
    return ORA_OK;
}

int ora_set_fields(ora_sim* s, const double* rho, const double* T, int step)
{
    if (!rho || !T || step < 0) return ORA_EINVAL;
    size_t ncg = (size_t)s->ncell * s->p.G;
    for (int i = 0; i < s->ncell; ++i)
        if (!(T[i] > 0) || !isfinite(T[i])) return ORA_EINVAL;
    memcpy(s->rho, rho, sizeof(double) * ncg);
    memcpy(s->T, T, sizeof(double) * s->ncell);
    s->step = step;
    return ORA_OK;
}

int ora_get_diag(const ora_sim* s, ora_diag* d) { *d = s->diag; return ORA_OK; }

int ora_get_counters(const ora_sim* s, uint64_t* birth_counter, int* step)
{
    if (birth_counter) *birth_counter = s->nbirth;
    if (step) *step = s->step;
    return ORA_OK;
}

/* Recording hooks used by the adjoint (oracle_adjoint.c). */
int ora_record(ora_sim* s, int on)
{
    /* the frozen-tally map covers neither the joint cells' tau_num (a maximum
     * over T^n) nor a temperature-dependent opacity: not recorded */
    if (on && (s->p.tau_num_C > 0.0 || s->p.T_power != 0.0 || s->p.opacity_stim)) return ORA_EINVAL;
    /* nor the slopes, the iterate's wave flux or boundary-source particles */
    if (on && (s->p.flags & (ORA_FLAG_SLOPES | ORA_FLAG_WAVE_ITER | ORA_FLAG_BOUNDARY_PARTICLES))) return ORA_EINVAL;
    /* nor Olson's heat capacity, a volumetric source or a tabulated opacity */
    if (on && (s->olH || s->qsrc || s->tab_lsig)) return ORA_EINVAL;
    free_rec(s);
    s->recording = on ? 1 : 0;
    if (on) {
        size_t ncg = (size_t)s->ncell * s->p.G;
        s->kappa0 = (double*)malloc(sizeof(double) * ncg);
        memcpy(s->kappa0, s->kappa, sizeof(double) * ncg);
    }
    return ORA_OK;
}

/* Accessors for oracle_adjoint.c (declared in oracle_internal.h). */
int ora__nrec(const ora_sim* s) { return s->nrec; }
const ora_rec_step* ora__rec(const ora_sim* s, int k) { return &s->rec[k]; }
const ora_params* ora__params(const ora_sim* s) { return &s->p; }
const double* ora__simpson(const ora_sim* s) { return s->simpson; }
const double* ora__cv(const ora_sim* s) { return s->cv; }
const unsigned char* ora__pinned(const ora_sim* s) { return s->pinned; }
const double* ora__kappa_rec(const ora_sim* s) { return s->kappa0; }
const double* ora__T(const ora_sim* s) { return s->T; }
const double* ora__rho(const ora_sim* s) { return s->rho; }
double ora__V(const ora_sim* s) { return s->V; }
double ora__dx(const ora_sim* s) { return s->dx; }
double ora__dy(const ora_sim* s) { return s->dy; }
