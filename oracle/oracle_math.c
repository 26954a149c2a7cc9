/*
 * FP64 CPU oracle -- scalar building blocks.  TEST INFRASTRUCTURE ONLY.
 *
 *  - Philox4x32-10 counter-based generator, from its published definition
 *    (Salmon et al., SC'11); the paper only asks for eta ~ U(0,1) (Sec. 2.2,
 *    sampling of t_c; Appendix A, sampling of nu).
 *  - The multigroup Planck integral behind B_g (Sec. 2.1, definition of B_g).
 *  - The UGKS flux coefficients C2 (Eq. C2Formula), C4 (Sec. 2.2, F^{fr,UGKS})
 *    and C4 - e^{-s} (Sec. 2.2, F^{fr,wave}).
 *  - The linear-frequency sampler (Eqs. Blinear, kg and Appendix A).
 */
#include <math.h>
#include <stdint.h>
#include "oracle.h"
#include "bernoulli_coef.h"

/* ------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of
 *   (c0,c1,c2,c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
 * with the key advanced by the Weyl constants between rounds. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double ora_uniform(uint64_t seed, uint64_t id, uint32_t step, uint32_t purpose, uint32_t d)
{
    uint32_t ctr[4], key[2], r[4];
    ctr[0] = (uint32_t)id;
    ctr[1] = (uint32_t)(id >> 32);
    ctr[2] = step;
    ctr[3] = (purpose << 24) | (d >> 1);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    ora_philox4x32_10(ctr, key, r);
    uint32_t a = (d & 1u) ? r[2] : r[0];
    uint32_t b = (d & 1u) ? r[3] : r[1];
    uint64_t k = ((uint64_t)a << 20) | (uint64_t)(b >> 12);   /* 52 random bits */
    return ((double)k + 0.5) * 0x1p-52;
}

/* ------------------------------------------------------------------ */
/* Planck integrals.  int_0^inf t^3/(e^t-1) dt = pi^4/15. */
static const double ORA_PI4_15 = 6.4939394022668291;   /* pi^4 / 15 */

/* L(x) = int_0^x t^3/(e^t-1) dt via the Bernoulli series (converges for
 * |x| < 2 pi; used for x < 2 where 24 terms reach double precision). */
double ora_planck_head(double x)
{
    double sum = 0.0;
    for (int j = 0; j < ORA_NLCOEF; ++j) {
        double term = ORA_LCOEF[j] * pow(x, (double)ORA_LPOW[j]);
        sum += term;
        if (j > 3 && fabs(term) < 1e-18 * fabs(sum)) break;
    }
    return sum;
}

/* Pi(x) = int_x^inf t^3/(e^t-1) dt.  For x >= 2 expand 1/(e^t-1) = sum_n e^{-nt}
 * and integrate term by term:  int_x^inf t^3 e^{-nt} dt =
 * e^{-nx} (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4).  For x < 2 use pi^4/15 - L(x). */
double ora_planck_tail(double x)
{
    if (x < 2.0) return ORA_PI4_15 - ora_planck_head(x);
    double sum = 0.0;
    for (int n = 1; n < 200; ++n) {
        double dn = (double)n;
        double e = exp(-dn * x);
        double term = e * (x * x * x / dn + 3.0 * x * x / (dn * dn)
                           + 6.0 * x / (dn * dn * dn) + 6.0 / (dn * dn * dn * dn));
        sum += term;
        if (term <= 1e-18 * sum) break;
    }
    return sum;
}

/* int_{xl}^{xh} t^3/(e^t-1) dt without cancellation: both edges in the head
 * region -> difference of heads; otherwise difference of tails. */
static double planck_band(double xl, double xh)
{
    if (xh < 2.0) return ora_planck_head(xh) - ora_planck_head(xl);
    return ora_planck_tail(xl) - ora_planck_tail(xh);
}

/* phi_g(T): the group equilibrium value of rho (the angle-integrated group
 * Planck emission, 4 pi B_g in the 3-D notation of Sec. 2.1).  With h = k = 1,
 * int_{nl}^{nh} int_{S^2} B dOmega dnu = a c T^4 (15/pi^4) int_{nl/T}^{nh/T} t^3/(e^t-1) dt. */
double ora_phi_group(double T, double nl, double nh, double a, double c)
{
    double band = planck_band(nl / T, nh / T);
    double T2 = T * T;
    return a * c * T2 * T2 * band / ORA_PI4_15;
}

/* x^4 / (e^x - 1), zero for large x. */
static double planck_edge_weight(double x)
{
    if (x > 700.0) return 0.0;
    double x2 = x * x;
    return x2 * x2 / expm1(x);
}

/* d phi_g/dT = 4 phi_g / T + a c T^3 (15/pi^4) [ xl^4/(e^xl-1) - xh^4/(e^xh-1) ]
 * (differentiate the band integral through its limits nu/T). */
double ora_dphi_group(double T, double nl, double nh, double a, double c)
{
    double phi = ora_phi_group(T, nl, nh, a, c);
    double T3 = T * T * T;
    return 4.0 * phi / T
           + a * c * T3 * (planck_edge_weight(nl / T) - planck_edge_weight(nh / T)) / ORA_PI4_15;
}

/* ------------------------------------------------------------------ */
/* Flux coefficients.  With tau = eps^2/(c sigma) and s = dt/tau:
 *   C4 = (tau/dt)(1 - e^{-s}) = (1 - e^{-s})/s                 (F^{fr,UGKS})
 *   W  = C4 - e^{-s}                                            (F^{fr,wave})
 *   C2 = (2/dt) tau^2 (1 - e^{-s}) - tau - tau e^{-s}           (Eq. C2Formula)
 *      = dt [2(1 - e^{-s})/s - 1 - e^{-s}] / s.
 * Small s cancels catastrophically, so the power series are used there:
 *   W      = sum_{n>=1} (-1)^{n+1} n s^n / (n+1)!
 *   C2/dt  = sum_{n>=2} (-1)^n (1-n) s^{n-1} / (n+1)!                      */
double ora_coef_c4(double s)
{
    if (s == 0.0) return 1.0;
    return -expm1(-s) / s;
}

double ora_coef_w(double s)
{
    if (s < 1.0) {
        double sum = 0.0, pw = 1.0, fact = 1.0;   /* pw = s^n, fact = (n+1)! */
        for (int n = 1; n < 60; ++n) {
            pw *= s;
            fact *= (double)(n + 1);
            double term = (double)n * pw / fact;
            sum += (n & 1) ? term : -term;
            if (term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return ora_coef_c4(s) - exp(-s);
}

double ora_coef_c2_over_dt(double s)
{
    if (s < 2.0) {
        double sum = 0.0, pw = 1.0, fact = 2.0;    /* pw = s^{n-1}, fact = (n+1)! */
        for (int n = 2; n < 80; ++n) {
            pw = (n == 2) ? s : pw * s;
            fact *= (double)(n + 1);
            double term = (double)(n - 1) * pw / fact;
            sum += (n & 1) ? term : -term;            /* (-1)^n (1-n) = (-1)^{n+1}(n-1) */
            if (term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return (2.0 * ora_coef_c4(s) - 1.0 - exp(-s)) / s;
}

/* C5 / dt, the slope coefficient of the UGKS free-transport flux (Sec. 2.2):
 * C5 = tau e^{-s} - (tau^2/dt)(1 - e^{-s}) with tau = dt/s, i.e. the time
 * average of -t e^{-t/tau} over the step:
 *   C5/dt = -int_0^1 u e^{-s u} du = ((1 + s) e^{-s} - 1) / s^2,
 * by its series -sum_{n>=0} (-s)^n / (n! (n+2)) below s = 2. */
double ora_coef_c5_over_dt(double s)
{
    if (s < 2.0) {
        double sum = 0.0, pw = 1.0, fact = 1.0;    /* pw = s^n, fact = n! */
        for (int n = 0; n < 80; ++n) {
            if (n > 0) { pw *= s; fact *= (double)n; }
            double term = pw / (fact * (double)(n + 2));
            sum += (n & 1) ? term : -term;
            if (n > 0 && term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return ((1.0 + s) * exp(-s) - 1.0) / (s * s);
}

/* (C5 + (dt/2) e^{-s}) / dt, the slope coefficient of the wave flux of a cell
 * whose collisionless part was sampled (Sec. 2.2, F^{fr,wave}): the two terms
 * cancel as s -> 0, so below s = 2 it is summed as
 *   sum_{n>=1} (-s)^n n / (2 n! (n+2)). */
double ora_coef_w5_over_dt(double s)
{
    if (s < 2.0) {
        double sum = 0.0, pw = 1.0, fact = 1.0;    /* pw = s^n, fact = n! */
        for (int n = 1; n < 80; ++n) {
            pw *= s;
            fact *= (double)n;
            double term = (double)n * pw / (2.0 * fact * (double)(n + 2));
            sum += (n & 1) ? -term : term;
            if (term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return ora_coef_c5_over_dt(s) + 0.5 * exp(-s);
}

/* Derivatives in s, needed by the adjoint of the macroscopic solve.  From the
 * closed forms above:
 *   dC4/ds      = (e^{-s} - C4)/s = -W/s
 *   dW/ds       = dC4/ds + e^{-s} = e^{-s} - W/s
 *   d(C2/dt)/ds = (2 dC4/ds + e^{-s} - C2/dt)/s
 * W/s comes from W's series below s = 1 (it tends to 1/2 at s = 0); the last
 * form cancels for small s, where the series of C2/dt is differentiated term
 * by term instead:  d(C2/dt)/ds = sum_{n>=2} (-1)^{n+1} (n-1)^2 s^{n-2}/(n+1)!. */
static double w_over_s(double s)
{
    if (s < 1.0) {
        double sum = 0.0, pw = 1.0, fact = 1.0;   /* pw = s^{n-1}, fact = (n+1)! */
        for (int n = 1; n < 60; ++n) {
            if (n > 1) pw *= s;
            fact *= (double)(n + 1);
            double term = (double)n * pw / fact;
            sum += (n & 1) ? term : -term;
            if (term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return ora_coef_w(s) / s;
}

double ora_coef_c4_ds(double s) { return -w_over_s(s); }

double ora_coef_w_ds(double s) { return exp(-s) - w_over_s(s); }

double ora_coef_c2_over_dt_ds(double s)
{
    if (s < 2.0) {
        double sum = 0.0, pw = 1.0, fact = 2.0;    /* pw = s^{n-2}, fact = (n+1)! */
        for (int n = 2; n < 80; ++n) {
            if (n > 2) pw *= s;
            fact *= (double)(n + 1);
            double term = (double)((n - 1) * (n - 1)) * pw / fact;
            sum += (n & 1) ? term : -term;
            if (term < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return (-2.0 * w_over_s(s) + exp(-s) - ora_coef_c2_over_dt(s)) / s;
}

/* ------------------------------------------------------------------ */
/* Linear-frequency sampling (Eqs. Blinear, kg; Appendix A).
 * B_lin(nu) = B(nmid) + k_g (nu - nmid),  k_g = (B(nh) - B(nl)) / (nh - nl).
 * Normalised by B(nmid) and with u' = (nu - nmid)/dnu in [-1/2, 1/2]:
 *   B_lin / B(nmid) = 1 + beta u',   beta = k_g dnu / B(nmid) = r_h - r_l,
 *   r = B(nu)/B(nmid) = (nu/nmid)^3 e^{-(nu - nmid)/T} (1 - e^{-nmid/T}) / (1 - e^{-nu/T}).
 * beta is limited to [-2, 2] so that the linear pdf stays non-negative on the
 * group (reading of the paper: the linear fit can go negative for steep Wien
 * tails; the limiter keeps the group integral B(nmid) dnu). */
double ora_freq_slope(double nl, double nh, double T)
{
    double nm = 0.5 * (nl + nh);
    double em = -expm1(-nm / T);
    double rh = nh / nm, rl = nl / nm;
    double Bh = rh * rh * rh * exp(-(nh - nm) / T) * em / (-expm1(-nh / T));
    double Bl = rl * rl * rl * exp(-(nl - nm) / T) * em / (-expm1(-nl / T));
    double beta = Bh - Bl;
    if (beta > 2.0) beta = 2.0;
    if (beta < -2.0) beta = -2.0;
    return beta;
}

/* Solve G(nu) = U with G the CDF of the linear pdf (Appendix A's quadratic,
 * with its numerator read as B(nmid)(nu - nl) + (k/2)(nu^2 - nl^2) - k nmid (nu - nl),
 * which is what its printed a, b, c coefficients encode).  In u':
 *   (beta/2) u'^2 + u' + q = 0,  q = 1/2 - beta/8 - U,
 * root with non-negative density: u' = -2q / (1 + sqrt(1 - 2 beta q)). */
double ora_linear_offset(double beta, double U)
{
    double q = 0.5 - 0.125 * beta - U;
    double disc = 1.0 - 2.0 * beta * q;
    if (disc < 0.0) disc = 0.0;
    return -2.0 * q / (1.0 + sqrt(disc));
}

double ora_sample_nu(double nl, double nh, double beta, double U)
{
    double nm = 0.5 * (nl + nh);
    double dnu = nh - nl;
    double up = ora_linear_offset(beta, U);
    double nu = nm + up * dnu;
    if (nu < nl) nu = nl;
    if (nu > nh) nu = nh;
    return nu;
}
