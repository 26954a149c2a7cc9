// Device-side scalar building blocks of the UGKWP hot path (gfx950).
//
//  - keyed counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11);
//    the paper only requires eta ~ U(0,1) (Sec. 2.2, collision times;
//    Appendix A, frequencies);
//  - the group Planck integral behind B_g (Sec. 2.1);
//  - the UGKS time-averaged flux coefficients C4, C4 - e^{-s} (Sec. 2.2,
//    F^{fr,UGKS}, F^{fr,wave}) and C2 (Eq. C2Formula);
//  - the linear-frequency sampler (Eqs. Blinear, kg; Appendix A).
//
// Every expression that feeds a discrete decision (a collision test, a face
// crossing, a particle count) is written in a fixed evaluation order; the
// library is compiled with floating-point contraction off so the rounding is
// exactly that of the written order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ugk {

enum : uint32_t { PURPOSE_BIRTH = 1, PURPOSE_FLIGHT = 2 };

// pi^4 / 15 = int_0^inf t^3/(e^t-1) dt
#define UGK_PI4_15 6.49393940226682914909602217

struct Philox4 { uint32_t v[4]; };

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo = (uint64_t)0xD2511F53u * c0;
        const uint64_t hi = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(hi >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(lo >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)hi;
        c3 = (uint32_t)lo;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Two 52-bit uniforms in (0,1) per Philox call: u = (k + 1/2) 2^-52.
__host__ __device__ inline double u52(uint32_t hi, uint32_t lo)
{
    const uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)k + 0.5) * 2.220446049250313080847e-16;   // 2^-52
}

// Draw d of (seed, particle id, step, purpose): counter (id_lo, id_hi, step,
// purpose<<24 | d/2), key (seed_lo, seed_hi); even d takes words 0,1, odd d 2,3.
__host__ __device__ inline double keyed_uniform(uint64_t seed, uint64_t id, uint32_t step,
                                                uint32_t purpose, uint32_t d)
{
    const Philox4 r = philox4x32_10((uint32_t)id, (uint32_t)(id >> 32), step,
                                    (purpose << 24) | (d >> 1), (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
    return (d & 1u) ? u52(r.v[2], r.v[3]) : u52(r.v[0], r.v[1]);
}

// Both draws of one Philox call (d0 even): out0 = draw d0, out1 = draw d0+1.
__host__ __device__ inline void keyed_uniform_pair(uint64_t seed, uint64_t id, uint32_t step,
                                                   uint32_t purpose, uint32_t d0, double& out0,
                                                   double& out1)
{
    const Philox4 r = philox4x32_10((uint32_t)id, (uint32_t)(id >> 32), step,
                                    (purpose << 24) | (d0 >> 1), (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
    out0 = u52(r.v[0], r.v[1]);
    out1 = u52(r.v[2], r.v[3]);
}

// -ln(u) for u in (0, 1), the uniforms above.  u = 2^e m with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.1716,
// summed as 2s (1 + s^2/3 + s^4/5 + ... + s^22/23): the first term left out is
// below 2^-54 of the sum.  ln 2 is split so that e ln2_hi is exact (ln2_hi
// keeps 32 significant bits).  The result is within a few ulp of the correctly
// rounded value; the tests compare it with the host libm.
__host__ __device__ inline double neg_log_unit(double u)
{
    int e;
    double m = frexp(u, &e);                       // u = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);        // m - 1 is exact here
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double t = s + s;
    const double lnm = fma(t, z * p, t);
    const double de = (double)e;
    const double ln2_hi = 0x1.62e42fee00000p-1, ln2_lo = 0x1.a39ef35793c76p-33;
    return -fma(de, ln2_hi, fma(de, ln2_lo, lnm));
}

// ---------------------------------------------------------------------------
// Planck band integrals.  head(x) = int_0^x t^3/(e^t-1) dt by its Taylor series
// in x (x < 2, coefficients in constant memory supplied by the host);
// tail(x) = int_x^inf t^3/(e^t-1) dt = sum_n e^{-nx}(x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4).

constexpr int HEAD_TERMS = 18;  // even-power terms after x^3, x^4: truncation below 4e-20 of head(x) for x < 2

struct HeadSeries {
    int nterm;                 // HEAD_TERMS
    double c[40];              // coefficient of x^(5 + 2j)
    double inv[64];            // inv[n] = 1/n (correctly rounded), n >= 1
};

__device__ inline double planck_head(double x, const HeadSeries& hs)
{
    // x^3/3 - x^4/8 + sum_j c_j x^(5+2j), Horner in x^2 (a fixed number of
    // terms: the coefficients are loaded together)
    const double x2 = x * x;
    double acc = 0.0;
#pragma unroll
    for (int j = HEAD_TERMS - 1; j >= 0; --j) acc = fma(acc, x2, hs.c[j]);
    const double x3 = x2 * x;
    return x3 * (1.0 / 3.0) - x3 * x * 0.125 + acc * x3 * x2;
}

// Four terms per pass (their 1/n loaded together), stopping after the pass
// whose last term is below 1e-18 of the sum: at most 60 terms, 21 at x = 2.
__device__ inline double planck_tail_series(double x, const HeadSeries& hs)
{
    const double e1 = exp(-x);
    if (e1 == 0.0) return 0.0;
    const double x2 = x * x, x3 = x2 * x, x6 = 6.0 * x, x23 = 3.0 * x2;
    double en = e1, sum = 0.0;
    for (int n = 1; n <= 57; n += 4) {
        double last = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double in = hs.inv[n + m];
            const double p = fma(fma(fma(6.0, in, x6), in, x23), in, x3);
            last = en * p * in;
            sum += last;
            en *= e1;
        }
        if (last <= 1e-18 * sum) break;
    }
    return sum;
}

// x^4 / (e^x - 1): the edge term of d phi_g / dT (the band integral of a
// group differentiated through its limits nu / T)
__device__ inline double planck_edge_weight(double x)
{
    if (x > 700.0) return 0.0;
    const double x2 = x * x;
    return x2 * x2 / expm1(x);
}

// Edge value used by group bands: head(x) below 2, tail(x) from 2 on.
__device__ inline double planck_edge_value(double x, const HeadSeries& hs)
{
    return x < 2.0 ? planck_head(x, hs) : planck_tail_series(x, hs);
}

// int_{xl}^{xh} t^3/(e^t-1) from edge values vl = edge_value(xl), vh = edge_value(xh).
__device__ inline double planck_band_from_edges(double xl, double vl, double xh, double vh)
{
    if (xh < 2.0) return vh - vl;                       // both heads
    if (xl < 2.0) return (UGK_PI4_15 - vl) - vh;        // head below, tail above
    return vl - vh;                                     // both tails
}

// phi_g(T) = a c T^4 (15/pi^4) band
__device__ inline double phi_from_band(double a, double c, double T, double band)
{
    const double T2 = T * T;
    return a * c * T2 * T2 * band / UGK_PI4_15;
}

// ---------------------------------------------------------------------------
// Flux coefficients as functions of s = c sigma dt / eps^2.

__host__ __device__ inline double coef_c4(double s)
{
    return s == 0.0 ? 1.0 : -expm1(-s) / s;
}

// The power-series coefficients of the functions below, fixed at compile time
// (each a ratio of integers rounded once), so that a term costs a multiply
// and no division.  Index n is the series' own summation index.
struct SeriesCoefs {
    double w[61];     // n / (n+1)!                       C4 - e^{-s}
    double c2[81];    // (n-1) / (n+1)!                   C2/dt
    double c5[81];    // 1 / (n! (n+2))                   C5/dt
    double w5[81];    // n / (2 n! (n+2))                 (C5 + dt/2 e^{-s})/dt
    double wos[61];   // n / (n+1)!                       (C4 - e^{-s})/s
    double c2ds[81];  // (n-1)^2 / (n+1)!                 d(C2/dt)/ds
};

constexpr SeriesCoefs make_series_coefs()
{
    SeriesCoefs t{};
    double fact = 1.0;                       // n!
    for (int n = 0; n < 81; ++n) {
        if (n > 0) fact *= (double)n;
        const double fact1 = fact * (double)(n + 1);     // (n+1)!
        if (n < 61) {
            t.w[n] = (double)n / fact1;
            t.wos[n] = (double)n / fact1;
        }
        t.c2[n] = (double)(n - 1) / fact1;
        t.c5[n] = 1.0 / (fact * (double)(n + 2));
        t.w5[n] = (double)n / (2.0 * fact * (double)(n + 2));
        t.c2ds[n] = (double)((n - 1) * (n - 1)) / fact1;
    }
    return t;
}

constexpr SeriesCoefs kSeries = make_series_coefs();

// C4 - e^{-s}; alternating series sum_{n>=1} (-1)^{n+1} n s^n/(n+1)! below s = 1 to
// avoid cancellation.
__host__ __device__ inline double coef_w(double s)
{
    if (s < 1.0) {
        double p = 1.0, sum = 0.0;
        for (int n = 1; n < 60; ++n) {
            p *= s;
            const double t = kSeries.w[n] * p;
            sum += (n & 1) ? t : -t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return coef_c4(s) - exp(-s);
}

// C2/dt = [2 C4 - 1 - e^{-s}] / s; series sum_{n>=2} (-1)^{n+1} (n-1) s^{n-1}/(n+1)! below s = 2.
__host__ __device__ inline double coef_c2_over_dt(double s)
{
    if (s < 2.0) {
        double p = 1.0, sum = 0.0;                       // p = s^{n-1}
        for (int n = 2; n < 80; ++n) {
            p *= s;
            const double t = kSeries.c2[n] * p;
            sum += (n & 1) ? t : -t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return (2.0 * coef_c4(s) - 1.0 - exp(-s)) / s;
}

// C5/dt of the slope term of the UGKS free-transport flux (Sec. 2.2):
// -int_0^1 u e^{-s u} du = ((1 + s) e^{-s} - 1) / s^2.  Below s = 2 the
// expansion -1/2 + s/3 - s^2/8 + ... = sum_n (-1)^{n+1} s^n / (n! (n+2)).
__host__ __device__ inline double coef_c5(double s)
{
    if (s < 2.0) {
        double p = 1.0, sum = -0.5;                      // n = 0 term
        for (int n = 1; n < 80; ++n) {
            p *= s;
            const double t = kSeries.c5[n] * p;
            sum += (n & 1) ? t : -t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return ((1.0 + s) * exp(-s) - 1.0) / (s * s);
}

// (C5 + (dt/2) e^{-s}) / dt, the slope coefficient of the wave flux of a
// sampled cell; below s = 2, sum_{n>=1} (-1)^n n s^n / (2 n! (n+2)) (the two
// terms of the closed form cancel as s -> 0).
__host__ __device__ inline double coef_w5(double s)
{
    if (s < 2.0) {
        double p = 1.0, sum = 0.0;
        for (int n = 1; n < 80; ++n) {
            p *= s;
            const double t = kSeries.w5[n] * p;
            sum += (n & 1) ? -t : t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return coef_c5(s) + 0.5 * exp(-s);
}

// Derivatives in s (for the adjoint of the macroscopic solve).  With
// W/s -> 1/2 as s -> 0 taken from W's series below s = 1:
//   C4' = -W/s,   W' = e^{-s} - W/s,   (C2/dt)' = (e^{-s} - 2 W/s - C2/dt) / s,
// the last replaced below s = 2 by its series
//   sum_{n>=2} (-1)^{n+1} (n-1)^2 s^{n-2} / (n+1)!   (it cancels there).
__host__ __device__ inline double coef_w_over_s(double s)
{
    if (s < 1.0) {
        double p = 1.0, sum = 0.5;                      // n = 1 term: 1/2
        for (int n = 2; n < 60; ++n) {
            p *= s;                                     // s^{n-1}
            const double t = kSeries.wos[n] * p;
            sum += (n & 1) ? t : -t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return coef_w(s) / s;
}

__host__ __device__ inline double coef_c4_ds(double s) { return -coef_w_over_s(s); }

__host__ __device__ inline double coef_w_ds(double s) { return exp(-s) - coef_w_over_s(s); }

__host__ __device__ inline double coef_c2_over_dt_ds(double s)
{
    if (s < 2.0) {
        double p = 1.0, sum = -1.0 / 6.0;               // n = 2 term
        for (int n = 3; n < 80; ++n) {
            p *= s;                                     // s^{n-2}
            const double t = kSeries.c2ds[n] * p;
            sum += (n & 1) ? t : -t;
            if (t < 1e-18 * fabs(sum)) break;
        }
        return sum;
    }
    return (exp(-s) - 2.0 * coef_w_over_s(s) - coef_c2_over_dt(s)) / s;
}

// ---------------------------------------------------------------------------
// Linear-frequency sampling.  beta = (B(nh) - B(nl)) / B(nmid) limited to [-2, 2]
// (keeps the linear pdf non-negative on the group); evaluated as ratios of
// Planck functions so that nothing under- or overflows for steep Wien tails.
__host__ __device__ inline double freq_slope(double nl, double nh, double T)
{
    const double nm = 0.5 * (nl + nh);
    const double em = -expm1(-nm / T);
    const double rh = nh / nm, rl = nl / nm;
    const double bh = rh * rh * rh * exp(-(nh - nm) / T) * em / (-expm1(-nh / T));
    const double bl = rl * rl * rl * exp(-(nl - nm) / T) * em / (-expm1(-nl / T));
    double beta = bh - bl;
    beta = beta > 2.0 ? 2.0 : beta;
    beta = beta < -2.0 ? -2.0 : beta;
    return beta;
}

// Inverse CDF of the pdf (1 + beta u')/dnu, u' = (nu - nmid)/dnu in [-1/2, 1/2]:
// (beta/2) u'^2 + u' + q = 0, q = 1/2 - beta/8 - U, stable root -2q/(1 + sqrt(1 - 2 beta q)).
__host__ __device__ inline double sample_nu(double nl, double nh, double beta, double U)
{
    const double nm = 0.5 * (nl + nh);
    const double dnu = nh - nl;
    const double q = 0.5 - 0.125 * beta - U;
    double disc = 1.0 - 2.0 * beta * q;
    disc = disc < 0.0 ? 0.0 : disc;
    const double up = -2.0 * q / (1.0 + sqrt(disc));
    double nu = nm + up * dnu;
    nu = nu < nl ? nl : nu;
    nu = nu > nh ? nh : nu;
    return nu;
}

// Offset u' in [-1/2, 1/2] whose CDF under the density 1 + beta u' is U
// (the same quadratic as sample_nu); places new particles along the slope of
// their cell's wave part.
__host__ __device__ inline double linear_offset(double beta, double U)
{
    const double q = 0.5 - 0.125 * beta - U;
    double disc = 1.0 - 2.0 * beta * q;
    disc = disc < 0.0 ? 0.0 : disc;
    return -2.0 * q / (1.0 + sqrt(disc));
}

// ---------------------------------------------------------------------------
// Olson's material (Sec. 3.4, Eq. cvolson).  The ionisation fraction alpha solves
// alpha^2 = e^{-chi/T} (1 - alpha); with h = e^{-chi/(2T)} and r = sqrt(h^2 + 4) it is
// h (r - h)/2 (no overflow for cold material), and dalpha/dT = (chi/T^2)(alpha - h/r).
__host__ __device__ inline double olson_alpha(double T, double chi, double* dalpha)
{
    const double h = exp(-0.5 * chi / T);
    const double r = sqrt(h * h + 4.0);
    const double al = 0.5 * h * (r - h);
    if (dalpha) *dalpha = (chi / (T * T)) * (al - h / r);
    return al;
}

// Heat capacity H [1 + alpha + (T + chi) alpha'] (the printed a T_keV^3 is the unit
// a (1 keV)^3, folded into H) and the material energy H [T (1 + alpha) + chi alpha]
// whose derivative it is.
__host__ __device__ inline double olson_cv(double H, double chi, double T)
{
    double da;
    const double al = olson_alpha(T, chi, &da);
    return H * (1.0 + al + (T + chi) * da);
}

__host__ __device__ inline double olson_energy(double H, double chi, double T)
{
    const double al = olson_alpha(T, chi, nullptr);
    return H * (T * (1.0 + al) + chi * al);
}

// The temperature whose Olson material energy is u > 0.  The energy rises
// strictly with T: a bracket [lo, hi] with energy(lo) <= u <= energy(hi) is found
// by doubling from T0, then Newton steps from T0 that stay inside the bracket
// (else its midpoint), until a step moves T by at most 1e-15 T.  Returns -1 for
// u <= 0 (no temperature).
__host__ __device__ inline double olson_temperature(double H, double chi, double u, double T0)
{
    if (!(u > 0.0) || !isfinite(u)) return -1.0;
    double lo = 0.0, hi = T0 > 0.0 ? T0 : 1.0;
    for (int n = 0; n < 2100 && olson_energy(H, chi, hi) < u; ++n) {
        lo = hi;
        hi = 2.0 * hi;
    }
    double T = (T0 > lo && T0 < hi) ? T0 : 0.5 * (lo + hi);
    for (int n = 0; n < 200; ++n) {
        const double f = olson_energy(H, chi, T) - u;
        if (f == 0.0) break;
        if (f < 0.0) lo = T; else hi = T;
        double Tn = T - f / olson_cv(H, chi, T);
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        const double d = fabs(Tn - T);
        T = Tn;
        if (d <= 1e-15 * T) break;
    }
    return T;
}

// ---------------------------------------------------------------------------
// Tabulated opacity: the interval [i, i+1] of n ascending nodes holding x and the
// weight of node i+1 (clamped to the end intervals: weight 0 or 1 beyond them).
__host__ __device__ inline int table_locate(const double* nodes, int n, double x, double* frac)
{
    if (x <= nodes[0]) { *frac = 0.0; return 0; }
    if (x >= nodes[n - 1]) { *frac = 1.0; return n - 2; }
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (nodes[mid] <= x) lo = mid; else hi = mid;
    }
    *frac = (x - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
    return lo;
}

// The same interval found from a first guess: for nodes evenly spaced from
// nodes[0] with 1/spacing inv (inv = 0: no guess, plain bisection) the guess is
// the interval of x on that grid, then moved until nodes[i] <= x < nodes[i+1]
// holds as bisection would leave it.  Same result as table_locate.
__host__ __device__ inline int table_locate_guess(const double* nodes, int n, double x, double inv,
                                                  double* frac)
{
    if (!(inv > 0.0)) return table_locate(nodes, n, x, frac);
    if (x <= nodes[0]) { *frac = 0.0; return 0; }
    if (x >= nodes[n - 1]) { *frac = 1.0; return n - 2; }
    double gq = (x - nodes[0]) * inv;
    int i = gq < 0.0 ? 0 : (gq > (double)(n - 2) ? n - 2 : (int)gq);
    while (i > 0 && nodes[i] > x) --i;
    while (i < n - 2 && nodes[i + 1] <= x) ++i;
    *frac = (x - nodes[i]) / (nodes[i + 1] - nodes[i]);
    return i;
}

// nu^-p with the exact cube for the paper's p = 3.
__host__ __device__ inline double nu_pow(double nu, double p)
{
    return p == 3.0 ? 1.0 / (nu * nu * nu) : pow(nu, -p);
}

}  // namespace ugk
