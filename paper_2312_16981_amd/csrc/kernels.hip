// HIP kernels (gfx950) of one UGKWP time step; see the paper's Algorithm 1.
//
//   k_tables       per (cell, group): Simpson group opacity (Sec. 3), s = c sigma dt / eps^2,
//                  e^{-s}, C4 and C4 - e^{-s} (Sec. 2.2)
//   k_face_D       per face and group: harmonic face opacity and
//                  D = -(c/eps)^2 (1/3) C2 / h (Appendix B, K_g and M_g)
//   k_count        wave split rho^h = rho^n - rho^p (Sec. 2.2) and the number of
//                  collisionless particles N = floor(e^{-s} rho^h / w_ref) (Eq. IhpFormula)
//   k_scan_*       exclusive scan of N -> particle slots and birth ids
//   k_sample       new particles: uniform position, isotropic direction,
//                  linear-frequency nu (Appendix A), t_f = dt
//   k_push         free flight with reset at interfaces (Eq. particle tf formula,
//                  Remark 1), gross face tallies (Eq. wfrpFormula), deletion of
//                  collided particles (their slots stay empty until the next sort)
//   k_sort_scatter counting sort of the survivors by (cell, group) slot, which
//                  also compacts the pool
//   k_si_sweep     source iteration (Appendix B, Eq. macroSysAppendixIte, Algorithm 2);
//                  sweep 0 also evaluates the wave free-transport flux (Sec. 2.2,
//                  F^{fr,wave}; Remark 3) and the static part Q of the macroscopic
//                  update (Eq. macroSysFinal)
//   k_si_decide    convergence decision of a sweep (batched contexts)
//   k_finish       commit of the step and energy bookkeeping
//
// Counts that the host does not know without a round trip (births, survivors,
// pool size) stay in device memory; the kernels that need them loop over the
// device count, and every kernel that changes the committed state checks that
// the step neither failed nor left a source iteration unconverged.
#include "common.hpp"
#include "device_math.hpp"
#include "kernels.hpp"
#include "device_common.hpp"
#include "../../include/ugkwp.h"

namespace ugk {

__constant__ HeadSeries c_head;

// What a particle flight reads of its instance, copied into registers once
// (scalar registers when the whole launch serves one instance).
struct Geo {
    double x0, y0, dx, dy;
    uint32_t cg_off, fx_off, fy_off;   // slot indices stay below 2^30 (checked at set-up)
    uint64_t seed;
    int nx, ny, lgGp, cell_off, edge_off;
    int reflect;           // bit q: side q (XLO, XHI, YLO, YHI) is reflective
};

// Column and row of local cell lcell of an nx-wide instance: the quotient from the
// double reciprocal of nx (off by at most one for lcell < 2^29), corrected.
__device__ inline void cell_col_row(int lcell, int nx, double inv_nx, int& ix, int& iy)
{
    int q = (int)((double)lcell * inv_nx);
    int r = lcell - q * nx;
    if (r < 0) {
        q -= 1;
        r += nx;
    } else if (r >= nx) {
        q += 1;
        r -= nx;
    }
    ix = r;
    iy = q;
}

__device__ inline Geo geo_of(const Inst& I)
{
    Geo o;
    o.x0 = I.x0; o.y0 = I.y0; o.dx = I.dx; o.dy = I.dy;
    o.cg_off = (uint32_t)I.cg_off; o.fx_off = (uint32_t)I.fx_off; o.fy_off = (uint32_t)I.fy_off;
    o.seed = I.seed;
    o.nx = I.nx; o.ny = I.ny; o.lgGp = I.lgGp; o.cell_off = I.cell_off; o.edge_off = I.edge_off;
    o.reflect = 0;
    for (int q = 0; q < 4; ++q) o.reflect |= (I.bc[q] == BC_REFLECT ? 1 : 0) << q;
    return o;
}

// sigma(nu, cell) = kappa[cell][g] * f(nu): f = nu^-3 (the paper's opacities),
// nu^-p, or the Simpson group factor S_g with the group-opacity flag.  f is
// fixed for a particle, so the push computes it once.  SIG_STIM: nu^-p times
// the stimulated-emission factor 1 - e^{-nu/T} of the cell the particle is in
// (Sec. 3.3), evaluated at every cell entry.
// SIG_TAB: a tabulated sigma(nu, T) (Sec. 3.4-3.5), from the row of the cell the
// particle is in (ln sigma along the table's nu nodes at the cell's T^n) at the
// particle's own nu interval, evaluated at every cell entry.
enum { SIG_NU3 = 0, SIG_POW = 1, SIG_GROUP = 2, SIG_STIM = 3, SIG_TAB = 4 };

// Stimulated-emission factor 1 - e^{-nu/T} (Sec. 3.3's opacity), or 1 without it.
__device__ inline double stim_factor(const Consts& K, double nu, double T)
{
    return K.stim ? -expm1(-nu / T) : 1.0;
}

// Frequency factor of group g at temperature T: Simpson's mean of nu^-p over
// the group, times the stimulated-emission factor when that is on.
__device__ inline double group_factor(const Dev& D, const Consts& K, int edge_off, int g, double T)
{
    if (!K.stim) return D.simpson[edge_off + g];
    const double nl = D.nu[edge_off + g], nh = D.nu[edge_off + g + 1], nm = 0.5 * (nl + nh);
    return (nu_pow(nl, K.nu_power) * stim_factor(K, nl, T) + 4.0 * nu_pow(nm, K.nu_power) * stim_factor(K, nm, T)
            + nu_pow(nh, K.nu_power) * stim_factor(K, nh, T)) / 6.0;
}

// Group opacity of material m at T from the table (Sec. 3.4-3.5's printed
// opacities, tabulated by the caller): sigma is bilinear in (ln nu, ln T) on
// ln sigma, constant beyond the end nodes, and the group value is Simpson's rule
// over the group (edge index e = edge_off + g).  The nu intervals and weights of the group's
// three Simpson points are fixed by the edges and read from tab_gi / tab_ga
// (k_tab_groups at set-up); only T is located here.
__device__ inline double table_group_sigma(const Dev& D, const Consts& K, int m, int e, double T)
{
    double b;
    const int jt = table_locate_guess(D.tab_lT, K.tab_nT, log(T), K.tab_lT_inv, &b);
    const int n = K.tab_nnu;
    const double* L0 = D.tab_lsig + ((int64_t)m * K.tab_nT + jt) * n;
    double v[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int i = D.tab_gi[3 * e + p];
        const double a = D.tab_ga[3 * e + p];
        const double* L = L0 + i;
        const double lo = (1.0 - a) * L[0] + a * L[1], hi = (1.0 - a) * L[n] + a * L[n + 1];
        v[p] = exp((1.0 - b) * lo + b * hi);
    }
    return (v[0] + 4.0 * v[1] + v[2]) / 6.0;
}

// The volumetric source acts in the steps that start before its switch-off time.
__device__ inline bool source_on(const Consts& K, uint32_t step)
{
    return K.has_src && (double)step * K.dt < K.q_toff;
}

// The flight scale of a particle, tau = eps^2 / (c sigma), with sigma = kappa
// nu^-p (Remark 2; Simpson's group factor S_g instead of nu^-p with
// UGKWP_FLAG_GROUP_SIGMA), is evaluated as the particle's factor eps^2 nu^p
// / c times the cell's 1/kappa: no division per particle or per crossing.
template <int SM>
__device__ inline double tau_factor(const Dev& D, const Consts& K, const Geo& I, double nu, int g)
{
    if (SM == SIG_GROUP) return K.e2c / D.simpson[I.edge_off + g];
    if (SM == SIG_NU3) return K.e2c * (nu * nu * nu);
    if (SM == SIG_STIM && K.nu_power == 3.0) return K.e2c * (nu * nu * nu);
    if (SM == SIG_TAB) return K.e2c;
    return K.e2c * pow(nu, K.nu_power);
}

__device__ inline double phi_group_direct(double T, double nl, double nh, double a, double c)
{
    const double xl = nl / T, xh = nh / T;
    const double band = planck_band_from_edges(xl, planck_edge_value(xl, c_head), xh,
                                               planck_edge_value(xh, c_head));
    return phi_from_band(a, c, T, band);
}

// A step commits only when nothing failed and every instance's source iteration converged.
__device__ inline bool step_committed(const Dev& D, const Consts& K)
{
    return D.counters[CNT_ERR] == 0 && D.counters[CNT_CONV] == (unsigned long long)K.n_inst;
}

// ---------------------------------------------------------------------------
// set-up kernels

// With a temperature-dependent opacity (K.t_power != 0 or K.stim) the tables are those
// of the cells' temperature T^n, and the step launches this kernel again at
// its start (gated like the step's other launches).
__global__ void k_tables(Dev D, Consts K)
{
    if (!gate_open(D, K, 0)) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    if (!s.active) {
        D.sig[j] = 0.0; D.sv[j] = 0.0; D.es[j] = 1.0; D.c4[j] = 1.0; D.wc[j] = 0.0; D.inv_kappa[j] = 0.0;
        return;
    }
    const Inst& I = D.inst[s.inst];
    const double Tc = D.T[I.cell_off + s.lcell];
    const double kap = K.t_power != 0.0 ? D.kappa[j] * pow(Tc, -K.t_power) : D.kappa[j];
    const double sg = K.table ? table_group_sigma(D, K, D.tab_mat[I.cell_off + s.lcell], I.edge_off + s.g, Tc)
                              : kap * group_factor(D, K, I.edge_off, s.g, Tc);
    // flights: tau = (eps^2/c) f(nu)^-1 / kappa; with the stimulated-emission
    // factor or a table and group opacities the group opacity's T dependence goes
    // here (the push divides by S_g), per particle the push applies it itself
    // (a table's per-particle flights read the cell rows instead)
    D.inv_kappa[j] = ((K.stim || K.table) && (K.flags & 1u)) ? D.simpson[I.edge_off + s.g] / sg
                     : K.table ? 1.0 / sg
                               : 1.0 / kap;   // +inf for kappa = 0: no collision
    const double sv = s_of_sigma(K, sg);
    D.sig[j] = sg;
    D.sv[j] = sv;
    D.es[j] = exp(-sv);
    D.c4[j] = coef_c4(sv);
    D.wc[j] = coef_w(sv);
}

// The push's rows of a tabulated opacity: for every cell and nu node, ln sigma of
// the cell's material interpolated to the cell's T^n (launched with the tables at
// the start of each step).
__global__ void k_tab_rows(Dev D, Consts K)
{
    if (!gate_open(D, K, 0)) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)K.ncell * K.tab_nnu) return;
    const int cell = (int)(j / K.tab_nnu), i = (int)(j % K.tab_nnu);
    double b;
    const int jt = table_locate_guess(D.tab_lT, K.tab_nT, log(D.T[cell]), K.tab_lT_inv, &b);
    const double* L = D.tab_lsig + ((int64_t)D.tab_mat[cell] * K.tab_nT + jt) * K.tab_nnu + i;
    D.tab_row[j] = (1.0 - b) * L[0] + b * L[K.tab_nnu];
}

// The nu intervals and upper-node weights of the three Simpson points (lower
// edge, midpoint, upper edge) of the group starting at every edge e < n_edges - 1,
// once at set-up (after the logs of the nodes).
__global__ void k_tab_groups(Dev D, Consts K, int64_t n_edges)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e + 1 >= n_edges) return;
    const double nl = D.nu[e], nh = D.nu[e + 1], nm = 0.5 * (nl + nh);
    const double pts[3] = {nl, nm, nh};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        double a;
        const int i = table_locate(D.tab_lnu, K.tab_nnu, log(pts[p]), &a);
        D.tab_gi[3 * e + p] = i;
        D.tab_ga[3 * e + p] = a;
    }
}

// ln of the table's nodes and values, once at set-up (n entries of each array).
__global__ void k_tab_logs(double* v, int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) v[j] = log(v[j]);
}

// D of a face with face opacity sf and centre distance h (Appendix B, Eq. C2Formula).
__device__ inline double face_coef(const Consts& K, double sf, double h)
{
    const double s = s_of_sigma(K, sf);
    const double c2 = K.dt * coef_c2_over_dt(s);
    return -(K.c * K.c / (3.0 * K.eps * K.eps)) * c2 / h;
}

// One instance, one axis: faces (nx+1)*ny (axis 0) or nx*(ny+1) (axis 1), Gp groups each.
__global__ void k_face_D(Dev D, Consts K, int inst, int axis)
{
    const Inst& I = D.inst[inst];
    const int64_t nface = axis == 0 ? (int64_t)(I.nx + 1) * I.ny : (int64_t)I.nx * (I.ny + 1);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nface * I.Gp) return;
    const int64_t f = j >> I.lgGp;
    const int g = (int)(j & (I.Gp - 1));
    double* Dout = axis == 0 ? D.Dx + I.fx_off : D.Dy + I.fy_off;
    if (g >= I.G) { Dout[j] = 0.0; return; }
    int cl, cr;     // local cells on the low / high side (-1 = outside)
    double h;
    if (axis == 0) {
        const int iy = (int)(f / (I.nx + 1)), fx = (int)(f % (I.nx + 1));
        cl = fx > 0 ? iy * I.nx + fx - 1 : -1;
        cr = fx < I.nx ? iy * I.nx + fx : -1;
        h = I.dx;
    } else {
        const int fy = (int)(f / I.nx), ix = (int)(f % I.nx);
        cl = fy > 0 ? (fy - 1) * I.nx + ix : -1;
        cr = fy < I.ny ? fy * I.nx + ix : -1;
        h = I.dy;
    }
    double sf;
    if (cl >= 0 && cr >= 0) {
        const double a = D.sig[I.cg_off + ((int64_t)cl << I.lgGp) + g];
        const double b = D.sig[I.cg_off + ((int64_t)cr << I.lgGp) + g];
        sf = (a + b > 0.0) ? 2.0 * (a * b) / (a + b) : 0.0;
    } else {
        sf = D.sig[I.cg_off + ((int64_t)(cl >= 0 ? cl : cr) << I.lgGp) + g];
    }
    Dout[j] = face_coef(K, sf, h);
}

// Planckian ghost values phi_g(T_b) per instance and side.
__global__ void k_ghost_phi(Dev D, Consts K, double* phib)
{
    const int inst = blockIdx.x;
    const int side = threadIdx.x / MAX_G, g = threadIdx.x % MAX_G;
    const Inst& I = D.inst[inst];
    double v = 0.0;
    if (g < I.G && I.bc[side] == BC_PLANCK)
        v = phi_group_direct(I.bcT[side], D.nu[I.edge_off + g], D.nu[I.edge_off + g + 1], K.a, K.c);
    phib[((int64_t)inst * 4 + side) * MAX_G + g] = v;
}

// rho^0 = phi(Tr0) per (cell, group), and phi(T^0), the first step's
// source-iteration start (later steps start from the last sweep's phi)
__global__ void k_init_rho(Dev D, Consts K, const double* Tr0)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    double v = 0.0, p = 0.0;
    if (s.active) {
        const Inst& I = D.inst[s.inst];
        const int cell = I.cell_off + s.lcell;
        const double nl = D.nu[I.edge_off + s.g], nh = D.nu[I.edge_off + s.g + 1];
        v = phi_group_direct(Tr0[cell], nl, nh, K.a, K.c);
        p = phi_group_direct(D.T[cell], nl, nh, K.a, K.c);
    }
    D.rho[j] = v;
    D.rhop[j] = 0.0;
    D.phi0[j] = p;
}

// The source Q(x) = B(nu, Ts) f(x) of Sec. 3.4-3.5 on the transport equation's
// right side, as the rate of rho per (cell, group) slot: (c/eps^2) f_cell phi_g(Ts).
__global__ void k_source_planck(Dev D, Consts K, double* q, const double* f, double Ts)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    double v = 0.0;
    if (s.active) {
        const Inst& I = D.inst[s.inst];
        const double nl = D.nu[I.edge_off + s.g], nh = D.nu[I.edge_off + s.g + 1];
        v = K.c / (K.eps * K.eps) * f[I.cell_off + s.lcell] * phi_group_direct(Ts, nl, nh, K.a, K.c);
    }
    q[j] = v;
}

// ---------------------------------------------------------------------------
// A1: wave split and particle counts

// The sampling fraction of a slot when the numerical collision time of
// thin-thick-joint cells is on (Sec. 3.2, second case): a face is joint when
// the group opacity changes across it by a factor >= tau_jump; over the joint
// faces of the cell, delta = max |T^l - T^r| / (T^l + T^r) (T^n), and
// dt/tau_num = s / (1 + s C delta) replaces s = dt/tau in e^{-s}.  The wave
// coefficient of the slot when it samples, C4(s) - e^{-dt/tau_num} =
// W(s) - (e^{-dt/tau_num} - e^{-s}), goes to wsn (W(s) outside joint cells).
__device__ inline double joint_fraction(const Dev& D, const Consts& K, const Inst& I, const Slot& s, int64_t j,
                                        double es, double T, double* diff_out)
{
    const int nx = I.nx, ix = s.lcell % nx, iy = s.lcell / nx, Gp = I.Gp;
    const double sg = D.sig[j];
    double delta = -1.0;
    for (int q = 0; q < 2 * I.dim; ++q) {
        const bool lo = (q & 1) == 0;
        const bool inside = q < 2 ? (lo ? ix > 0 : ix < nx - 1) : (lo ? iy > 0 : iy < I.ny - 1);
        if (!inside) continue;
        const int dc = q < 2 ? (lo ? -1 : 1) : (lo ? -nx : nx);
        const double sn = D.sig[j + (int64_t)dc * Gp];
        const double hi = sg > sn ? sg : sn, lw = sg > sn ? sn : sg;
        if (!(hi > 0.0) || hi < K.tau_jump * lw) continue;
        const double Tn = D.T[I.cell_off + s.lcell + dc];
        const double d = fabs(T - Tn) / (T + Tn);
        if (d > delta) delta = d;
    }
    double frac = es, w = D.wc[j], diff = 0.0;
    if (delta >= 0.0) {
        const double sv = D.sv[j];
        const double snum = sv / (1.0 + sv * K.tau_C * delta);
        frac = exp(-snum);
        const double dd = sv - snum;
        diff = dd < 0.5 ? es * expm1(dd) : frac - es;
        w -= diff;
    }
    D.wsn[j] = w;
    *diff_out = diff;
    return frac;
}

// Boundary-source particles: the ghost cell beyond Planckian side q of the
// slot's cell (if the cell touches that side) holds rho^h = phi(T_b) with the
// interior cell's opacity, and samples e^{-s} phi(T_b) V as an interior cell
// would (the same count rule).  Returns its births (0 elsewhere).
__device__ inline int ghost_births(const Dev& D, const Consts& K, const Inst& I, const Slot& s, int q, double es)
{
    if (I.bc[q] != BC_PLANCK) return 0;
    const int nx = I.nx, ix = s.lcell % nx, iy = s.lcell / nx;
    const bool adj = q == XLO ? ix == 0 : q == XHI ? ix == nx - 1 : q == YLO ? iy == 0 : iy == I.ny - 1;
    if (!adj) return 0;
    const double eov = es * D.phib[((int64_t)s.inst * 4 + q) * MAX_G + s.g];
    if (!(eov * I.V > 0.0)) return 0;
    const double qn = eov / I.w_ref;
    return (qn >= (double)K.n_cap) ? (int)K.n_cap : (int)floor(qn);
}

// Also opens the step's record (block 0: the persistent entries from the
// record before, everything else cleared), clears the tallies the push and
// the commit add to (grid-stride over the flat arrays), and, when part is
// given, writes the per-block sum of N for the scan that follows.
constexpr int COUNT_THREADS = 256;

template <bool SINGLE>
__global__ __launch_bounds__(COUNT_THREADS) void k_count(Dev D, Consts K, ZeroList Z, int64_t* part)
{
    const int64_t j = (int64_t)blockIdx.x * COUNT_THREADS + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * COUNT_THREADS;
    // the step count (the gate), the slot's loads and its wavefront's instance
    // record are requested together, before any store
    const uint32_t now = *D.step;
    const bool in = j < K.n_cg;
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    double rho = 0.0, rhop = 0.0, es = 0.0, nl = 0.0, nh = 0.0, T = 0.0, sv = 0.0;
    if (in && s.active) {
        rho = D.rho[j];
        rhop = D.rhop[j];
        es = D.es[j];
        if (K.flags & UGKWP_FLAG_SLOPES) sv = D.sv[j];    // the slope coefficient's s
        nl = D.nu[I.edge_off + s.g];
        nh = D.nu[I.edge_off + s.g + 1];
        T = D.T[I.cell_off + s.lcell];
    }
    if (!(K.gate == GATE_OFF || now == K.gate)) return;
    if (blockIdx.x == 0) {
        if (threadIdx.x < N_COUNTERS) {
            const int q = threadIdx.x;
            D.counters[q] = (q == CNT_SLOTS || q == CNT_LIVE) ? D.prev_counters[q] : 0ull;
        }
        if (threadIdx.x < 2) D.n_births_total[threadIdx.x] = 0;
        for (int q = threadIdx.x; q < K.n_inst; q += COUNT_THREADS) {
            InstState st;
            st.conv_sweeps = 0;
            st.bad = 0;
            st.births = D.prev_ist[q].births;
            D.ist[q] = st;
        }
        for (int q = threadIdx.x; q < 8 * K.n_inst; q += COUNT_THREADS) D.diag[q] = 0.0;
    }
    // Non-temporal zeros: the cleared tallies are next touched by the push's
    // atomics, so keeping them out of the caches leaves room for the sweep inputs.
    for (int r = 0; r < Z.n; ++r) {
        uint64_t* p = (uint64_t*)Z.ptr[r];
        for (int64_t q = j; q < Z.words[r]; q += stride) __builtin_nontemporal_store(0ull, p + q);
    }
    int N = 0;
    if (in) {
        if (!s.active) {
            D.nb[j] = 0;
            D.nbi[j] = 0;
            D.rhoh[j] = 0.0;
            D.wnew[j] = 0.0;
        } else {
            const double rh = rho - rhop;
            D.rhoh[j] = rh;
            double frac = es, diff = 0.0;
            if (K.tau_C > 0.0) frac = joint_fraction(D, K, I, s, j, es, T, &diff);
            const double eov = frac * rh;
            const double E = eov * I.V;
            if (E > 0.0) {
                const double q = eov / I.w_ref;
                N = (q >= (double)K.n_cap) ? (int)K.n_cap : (int)floor(q);
            }
            D.nbi[j] = N;
            D.wnew[j] = N >= 1 ? E / (double)N : 0.0;
            if (N >= 1) D.beta[j] = freq_slope(nl, nh, T);
            // slope coefficient of the wave flux (over dt): C5 + dt/2 e^{-dt/tau}
            // where the slot samples (tau_num in joint cells), else C5
            if (K.flags & UGKWP_FLAG_SLOPES) D.bcoef[j] = N >= 1 ? coef_w5(sv) + 0.5 * diff : coef_c5(sv);
            // boundary-source particles of the ghosts beyond this cell's Planckian sides
            // (sides unrolled: a side indexed at run time would put the instance
            // record in scratch memory)
            if (K.flags & UGKWP_FLAG_BOUNDARY_PARTICLES) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < 2 * I.dim) N += ghost_births(D, K, I, s, q, es);
            }
            D.nb[j] = N;
        }
    }
    if (part) {
        __shared__ int64_t wsum[COUNT_THREADS / WAVE];
        int64_t v = N;
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
        if ((threadIdx.x & (WAVE - 1)) == 0) wsum[threadIdx.x / WAVE] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < COUNT_THREADS / WAVE; ++w) t += wsum[w];
            part[blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of nb (int32) -> boff (int64); 256 threads x 16 items per block

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int64_t block_excl_scan(int64_t v, int64_t* total)
{
    __shared__ int64_t wsum[SCAN_THREADS / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int64_t o = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += o;
    }
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    int64_t woff = 0, tot = 0;
    for (int w = 0; w < SCAN_THREADS / WAVE; ++w) {
        if (w < wid) woff += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return woff + inc - v;
}

__device__ inline bool scan_open(const ScanGate& q) { return q.expect == GATE_OFF || *q.step == q.expect; }

// A chunk of SCAN_CHUNK items is read in SCAN_ITEMS / 4 passes; in pass r,
// thread t holds the four consecutive items from 4 (t + SCAN_THREADS r), so
// that a wavefront's loads and stores cover contiguous memory.  The last chunk
// (possibly partial) takes the same path with a bounds test per item.
constexpr int SCAN_PASSES = SCAN_ITEMS / 4;

__device__ inline int4 scan_load4(const int32_t* in, int64_t i, int64_t n, bool full)
{
    if (full) return *reinterpret_cast<const int4*>(in + i);
    int4 v;
    v.x = i + 0 < n ? in[i + 0] : 0;
    v.y = i + 1 < n ? in[i + 1] : 0;
    v.z = i + 2 < n ? in[i + 2] : 0;
    v.w = i + 3 < n ? in[i + 3] : 0;
    return v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(ScanGate q, const int32_t* in, int64_t n,
                                                                int64_t* part)
{
    if (!scan_open(q)) return;
    const int64_t c0 = (int64_t)blockIdx.x * SCAN_CHUNK;
    const bool full = c0 + SCAN_CHUNK <= n;
    int4 v[SCAN_PASSES];
#pragma unroll
    for (int r = 0; r < SCAN_PASSES; ++r) v[r] = scan_load4(in, c0 + 4 * ((int64_t)threadIdx.x + SCAN_THREADS * r), n, full);
    int64_t sum = 0;
#pragma unroll
    for (int r = 0; r < SCAN_PASSES; ++r) sum += (int64_t)v[r].x + v[r].y + v[r].z + v[r].w;
    int64_t tot;
    block_excl_scan(sum, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(ScanGate q, int64_t* part, int64_t nblk, int64_t* total)
{
    if (!scan_open(q)) return;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += SCAN_THREADS) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nblk ? part[b] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, &tot);
        if (b < nblk) part[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Exclusive scan of in[0..n) (one item per thread, COUNT_THREADS per block) from
// the per-block sums part[0..nblk) written by k_count: every block sums the
// partials before it itself (nblk is small), block 0 also writes the total.
__global__ __launch_bounds__(COUNT_THREADS) void k_scan_small(ScanGate q, const int32_t* in, int64_t n,
                                                              const int64_t* part, int nblk, int64_t* out,
                                                              int64_t* total)
{
    if (!scan_open(q)) return;
    __shared__ int64_t red[COUNT_THREADS / WAVE][2];
    int64_t before = 0, all = 0;
    for (int b = threadIdx.x; b < nblk; b += COUNT_THREADS) {
        const int64_t v = part[b];
        all += v;
        if (b < (int)blockIdx.x) before += v;
    }
    for (int m = 32; m >= 1; m >>= 1) {
        before += __shfl_xor(before, m, WAVE);
        all += __shfl_xor(all, m, WAVE);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        red[threadIdx.x / WAVE][0] = before;
        red[threadIdx.x / WAVE][1] = all;
    }
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int w = 0; w < COUNT_THREADS / WAVE; ++w) {
        base += red[w][0];
        tot += red[w][1];
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = tot;
    const int64_t i = (int64_t)blockIdx.x * COUNT_THREADS + threadIdx.x;
    const int64_t v = i < n ? in[i] : 0;
    // block-wide exclusive scan of one item per thread
    __shared__ int64_t wsum[COUNT_THREADS / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int64_t o = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += o;
    }
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    int64_t woff = 0;
    for (int w = 0; w < wid; ++w) woff += wsum[w];
    if (i < n) out[i] = base + woff + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_final(ScanGate q, const int32_t* in, int64_t n,
                                                          const int64_t* part, int64_t* out)
{
    if (!scan_open(q)) return;
    const int64_t c0 = (int64_t)blockIdx.x * SCAN_CHUNK;
    const bool full = c0 + SCAN_CHUNK <= n;
    int4 v[SCAN_PASSES];
#pragma unroll
    for (int r = 0; r < SCAN_PASSES; ++r) v[r] = scan_load4(in, c0 + 4 * ((int64_t)threadIdx.x + SCAN_THREADS * r), n, full);
    int64_t carry = part[blockIdx.x];
#pragma unroll
    for (int r = 0; r < SCAN_PASSES; ++r) {
        const int64_t sum = (int64_t)v[r].x + v[r].y + v[r].z + v[r].w;
        int64_t tot;
        const int64_t ex = carry + block_excl_scan(sum, &tot);
        carry += tot;
        const int64_t i = c0 + 4 * ((int64_t)threadIdx.x + SCAN_THREADS * r);
        const int64_t o0 = ex, o1 = o0 + v[r].x, o2 = o1 + v[r].y, o3 = o2 + v[r].z;
        if (full) {
            longlong2* p = reinterpret_cast<longlong2*>(out + i);
            p[0] = make_longlong2(o0, o1);
            p[1] = make_longlong2(o2, o3);
        } else {
            if (i + 0 < n) out[i + 0] = o0;
            if (i + 1 < n) out[i + 1] = o1;
            if (i + 2 < n) out[i + 2] = o2;
            if (i + 3 < n) out[i + 3] = o3;
        }
    }
}

// ---------------------------------------------------------------------------
// A2: sample the collisionless wave particles

template <int DIM>
__global__ void k_sample(Dev D, Consts K, Pool P)
{
    if (!gate_open(D, K, 0)) return;
    const uint32_t step = *D.step;
    const int64_t n_slots = (int64_t)D.counters[CNT_SLOTS];
    const int64_t total = D.n_births_total[0];
    if (n_slots + total > K.pool_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr((unsigned long long*)(D.counters + CNT_ERR), ERR_POOL);
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) D.counters[CNT_PUSHED] = (unsigned long long)(n_slots + total);
    const int64_t base = n_slots;
    // A wavefront takes 64 consecutive births.  Their slots lie between the
    // slot of its first birth and that of its last, both found by a search in
    // which every lane probes one of 64 pivots per round (a few rounds instead
    // of a dependent load per halving); each lane then bisects that range.
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE * WAVE; j0 < total; j0 += nw * WAVE) {
    const int64_t j = j0 + lane;
    const int64_t jl = min(j0 + WAVE - 1, total - 1);
    int64_t lo0 = 0, hi0 = K.n_cg, lo1 = 0, hi1 = K.n_cg;   // boff[lo] <= target, answer < hi
    while (hi0 - lo0 > 1 || hi1 - lo1 > 1) {
        const int64_t st0 = (hi0 - lo0 + WAVE - 1) / WAVE, st1 = (hi1 - lo1 + WAVE - 1) / WAVE;
        const int64_t p0 = lo0 + lane * st0, p1 = lo1 + lane * st1;
        const bool ok0 = p0 < hi0 && D.boff[p0] <= j0;
        const bool ok1 = p1 < hi1 && D.boff[p1] <= jl;
        const int n0 = __popcll(__ballot(ok0)) - 1, n1 = __popcll(__ballot(ok1)) - 1;
        lo0 += n0 * st0;
        hi0 = min(hi0, lo0 + st0);
        lo1 += n1 * st1;
        hi1 = min(hi1, lo1 + st1);
    }
    if (j >= total) continue;
    int64_t lo = lo0, hi = lo1 + 1;        // boff[lo] <= j, slot(j) < hi
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (D.boff[mid] <= j) lo = mid; else hi = mid;
    }
    const int64_t cg = lo;
    const int inst = D.wave_inst[cg >> 6];
    const Inst& I = D.inst[inst];
    const int64_t local = cg - I.cg_off;
    const int lcell = (int)(local >> I.lgGp), g = (int)(local & (I.Gp - 1));
    const uint64_t id = D.ist[inst].births + (uint64_t)(j - D.boff[I.cg_off]);
    const double nl = D.nu[I.edge_off + g], nh = D.nu[I.edge_off + g + 1];
    const int ix = lcell % I.nx, iy = lcell / I.nx;
    double xl = I.x0 + (double)ix * I.dx;
    double yl = I.y0 + (double)iy * I.dy;
    const int64_t o = base + j;
    // the slot's interior births come first, then those of the ghosts beyond
    // its Planckian sides, side by side (boundary-source particles)
    int part = -1;
    double beta, w = D.wnew[cg];
    const int64_t m = j - D.boff[cg];
    if ((K.flags & UGKWP_FLAG_BOUNDARY_PARTICLES) && m >= D.nbi[cg]) {
        int64_t rest = m - D.nbi[cg];
        const double es = D.es[cg];
        const Slot sl = {inst, lcell, g, true, true};
        for (int q = 0; q < 2 * DIM; ++q) {
            const int nq = ghost_births(D, K, I, sl, q, es);
            if (rest < nq) {
                part = q;
                const double pb = D.phib[((int64_t)inst * 4 + q) * MAX_G + g];
                w = es * pb * I.V / (double)nq;
                break;
            }
            rest -= nq;
        }
        beta = freq_slope(nl, nh, I.bcT[part]);
        if (part == XLO) xl = xl - I.dx;
        if (part == XHI) xl = xl + I.dx;
        if (part == YLO) yl = yl - I.dy;
        if (part == YHI) yl = yl + I.dy;
    } else {
        beta = D.beta[cg];
    }
    // slopes of the wave part in cell widths per rho^h: the linear density the
    // interior births are placed along (uniform where both are zero)
    double bx = 0.0, by = 0.0;
    if ((K.flags & UGKWP_FLAG_SLOPES) && part < 0) {
        const double rh = D.rhoh[cg];
        if (rh > 0.0) {
            bx = D.sx[cg] * I.dx / rh;
            if (DIM == 2) by = D.sy[cg] * I.dy / rh;
        }
    }
    double u0, u1, u2, u3;
    keyed_uniform_pair(I.seed, id, step, PURPOSE_BIRTH, 0, u0, u1);
    double px, py = 0.0;
    if (bx == 0.0 && by == 0.0) {
        px = xl + u0 * I.dx;
        if (DIM == 2) py = yl + u1 * I.dy;
    } else {
        // x from the marginal density 1 + bx u, y from its conditional given x
        double ux;
        if (bx == 0.0) {
            px = xl + u0 * I.dx;
            ux = u0 - 0.5;
        } else {
            ux = linear_offset(bx, u0);
            px = (xl + 0.5 * I.dx) + ux * I.dx;
        }
        if (DIM == 2) {
            const double bc = by / (1.0 + bx * ux);
            py = bc == 0.0 ? yl + u1 * I.dy : (yl + 0.5 * I.dy) + linear_offset(bc, u1) * I.dy;
        }
    }
    if (DIM == 1) {
        u2 = keyed_uniform(I.seed, id, step, PURPOSE_BIRTH, 2);
        P.x[o] = px;
        P.ox[o] = 2.0 * u1 - 1.0;
        P.nu[o] = sample_nu(nl, nh, beta, u2);
    } else {
        keyed_uniform_pair(I.seed, id, step, PURPOSE_BIRTH, 2, u2, u3);
        const double u4 = keyed_uniform(I.seed, id, step, PURPOSE_BIRTH, 4);
        P.x[o] = px;
        P.y[o] = py;
        const double oz = 2.0 * u2 - 1.0;
        const double psi = 6.283185307179586 * u3;
        const double sn = sqrt(1.0 - oz * oz);
        P.ox[o] = sn * cos(psi);
        P.oy[o] = sn * sin(psi);
        P.nu[o] = sample_nu(nl, nh, beta, u4);
    }
    P.w[o] = w;
    // the group word above the id; a boundary-source particle carries its ghost
    // side + 1 above the group bits
    const uint32_t gw = part < 0 ? (uint32_t)g : (uint32_t)(g | ((part + 1) << GHOST_SHIFT));
    P.id[o] = id | ((uint64_t)gw << ID_BITS);
    P.cell[o] = I.cell_off + lcell;
    }
}

// ---------------------------------------------------------------------------
// Slopes of the wave part (UGKWP_FLAG_SLOPES): MINMOD of the differences of
// rho^h to the two neighbours along each axis, with the boundary ghost one cell
// width away (Planckian phi(T_b), vacuum 0, reflective the mirror image), then
// scaled so that the linear profile stays non-negative over the cell
// (|s_x| dx + |s_y| dy <= 2 rho^h); zero where rho^h <= 0.  rho^h of a slot is
// src[j], minus rhop[j] when sub_rhop (the iterate's wave part, Algorithm 2).
__device__ inline double minmod_diff(double a, double b)
{
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

template <int DIM>
__global__ void k_slopes(Dev D, Consts K, const double* src, int sub_rhop)
{
    if (!gate_open(D, K, 0)) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    if (!s.active) {
        D.sx[j] = 0.0;
        D.sy[j] = 0.0;
        return;
    }
    const Inst& I = D.inst[s.inst];
    if (sub_rhop && D.ist[s.inst].conv_sweeps != 0) return;     // converged: not used
    const int nx = I.nx, ix = s.lcell % nx, iy = s.lcell / nx, Gp = I.Gp, g = s.g;
    const double* phib = D.phib + (int64_t)s.inst * 4 * MAX_G;
    auto rh = [&](int64_t k) { return sub_rhop ? src[k] - D.rhop[k] : src[k]; };
    auto ghost = [&](int q, double c0) {
        return I.bc[q] == BC_PLANCK ? phib[q * MAX_G + g] : (I.bc[q] == BC_REFLECT ? c0 : 0.0);
    };
    const double c0 = rh(j);
    const double l = ix > 0 ? rh(j - Gp) : ghost(XLO, c0);
    const double r = ix < nx - 1 ? rh(j + Gp) : ghost(XHI, c0);
    double ax = minmod_diff(c0 - l, r - c0) / I.dx, ay = 0.0;
    if (DIM == 2) {
        const int64_t row = (int64_t)nx * Gp;
        const double b = iy > 0 ? rh(j - row) : ghost(YLO, c0);
        const double t = iy < I.ny - 1 ? rh(j + row) : ghost(YHI, c0);
        ay = minmod_diff(c0 - b, t - c0) / I.dy;
    }
    if (!(c0 > 0.0)) {
        ax = 0.0;
        ay = 0.0;
    } else {
        const double tot = fabs(ax) * I.dx + fabs(ay) * I.dy;
        if (tot > 2.0 * c0) {
            const double f = 2.0 * c0 / tot;
            ax = ax * f;
            ay = ay * f;
        }
    }
    D.sx[j] = ax;
    D.sy[j] = ay;
}

// ---------------------------------------------------------------------------
// A3: free flight, reset at interfaces, tallies, deletion, compaction
//
// One thread per particle, ppt particles per thread (a launch parameter chosen
// by the autotuner, 4 by default).  Tallies (survivor
// and deposited weight per (cell, group), gross face crossings per face, group
// and direction, survivor counts per (cell, group)) are accumulated in a
// per-block LDS hash table and flushed with one global atomic per distinct bin:
// the pool is kept sorted by (cell, group) slot, so a block's particles fall
// into a handful of bins.

constexpr int PUSH_THREADS = 256;
constexpr int PUSH_PPT_DEFAULT = 4;
constexpr int HT_BITS = 10;
constexpr int HT_SIZE = 1 << HT_BITS;
constexpr uint32_t HT_EMPTY = 0xFFFFFFFFu;
constexpr int HT_PROBES = 32;

enum : uint32_t { TAL_SURV = 0, TAL_DEP = 1, TAL_FX = 2, TAL_FY = 3 };

struct TallyTable {
    uint32_t key[HT_SIZE];     // (index << 2) | type
    uint32_t cnt[HT_SIZE];     // survivor count (TAL_SURV only)
    double val[HT_SIZE];
};

__device__ inline double* tally_target(const Dev& D, uint32_t type, uint32_t index)
{
    switch (type) {
        case TAL_SURV: return D.surv + index;
        case TAL_DEP: return D.dep + index;
        case TAL_FX: return D.ftx + index;
        default: return D.fty + index;
    }
}

__device__ inline void lds_tally(TallyTable& T, const Dev& D, uint32_t type, uint32_t index, double w)
{
    const uint32_t key = (index << 2) | type;
    uint32_t h = (key * 2654435761u) >> (32 - HT_BITS);
#pragma unroll 1
    for (int probe = 0; probe < HT_PROBES; ++probe) {
        const uint32_t prev = atomicCAS(&T.key[h], HT_EMPTY, key);
        if (prev == HT_EMPTY || prev == key) {
            __hip_atomic_fetch_add(&T.val[h], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (type == TAL_SURV)
                __hip_atomic_fetch_add(&T.cnt[h], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        h = (h + 1) & (HT_SIZE - 1);
    }
    // table crowded: go straight to memory
    unsafeAtomicAdd(tally_target(D, type, index), w);
    if (type == TAL_SURV) atomicAdd(D.scount + index, 1u);
}

// Add a value (and a survivor count) to the bin of `key` in the LDS table;
// with the table crowded, straight to memory.
__device__ inline void lds_add(TallyTable& T, const Dev& D, uint32_t key, double w, uint32_t n)
{
    const uint32_t type = key & 3u;
    uint32_t h = (key * 2654435761u) >> (32 - HT_BITS);
#pragma unroll 1
    for (int probe = 0; probe < HT_PROBES; ++probe) {
        const uint32_t prev = atomicCAS(&T.key[h], HT_EMPTY, key);
        if (prev == HT_EMPTY || prev == key) {
            __hip_atomic_fetch_add(&T.val[h], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (type == TAL_SURV)
                __hip_atomic_fetch_add(&T.cnt[h], n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        h = (h + 1) & (HT_SIZE - 1);
    }
    unsafeAtomicAdd(tally_target(D, type, key >> 2), w);
    if (type == TAL_SURV) atomicAdd(D.scount + (key >> 2), n);
}

struct Flight {
    double x, y, ox, oy;   // position and direction (mu in 1-D)
    double t, t_rem, tau;  // time flown, flight time left, flight scale in this cell
    double u_odd;          // the odd draw of the last Philox block (draws 2m and 2m+1 share one)
    uint32_t d;            // FLIGHT draws used
    int ix, iy;
    int32_t flips;         // FLIP_X / FLIP_Y toggled by each reflection during this step
    bool coll;
    int ti;                // SIG_TAB: the particle's nu interval among the table nodes
    double ta;             // and the weight of its upper node
};

// The flight scale of a particle in local cell lcell of its instance.
template <int SM>
__device__ inline double cell_tau(const Dev& D, const Consts& K, const Geo& I, double tfac, int lcell, int g,
                                  double nu, const Flight& f)
{
    if (SM == SIG_TAB) {
        const double* row = D.tab_row + (int64_t)(I.cell_off + lcell) * K.tab_nnu + f.ti;
        return tfac * exp(-((1.0 - f.ta) * row[0] + f.ta * row[1]));
    }
    double t = tfac * D.inv_kappa[I.cg_off + ((uint32_t)lcell << I.lgGp) + (uint32_t)g];
    if (SM == SIG_STIM) t = t / stim_factor(K, nu, D.T[I.cell_off + lcell]);
    return t;
}

__device__ inline void draw_flight(const Consts& K, const Geo& I, uint64_t id, uint32_t step, Flight& f)
{
    double u;
    if ((f.d & 1u) == 0) keyed_uniform_pair(I.seed, id, step, PURPOSE_FLIGHT, f.d, u, f.u_odd);
    else u = f.u_odd;                  // the first crossing's draw: no second Philox evaluation
    f.d++;
    const double room = K.dt - f.t;
    // -ln u >= 1 - u: when tau (1 - u) clears the time left by far more than the
    // rounding of either side, the flight outlasts the step without the logarithm
    if (f.tau * (1.0 - u) > room * (1.0 + 1e-9)) {
        f.coll = false;
        f.t_rem = room;
        return;
    }
    const double a = f.tau * neg_log_unit(u);
    f.coll = a < room;
    f.t_rem = f.coll ? a : room;
}

// Flight of one particle through the step.  Returns 0 survives, 1 collided, 2 left the domain.
template <int DIM, int SM>
__device__ inline int fly(const Dev& D, const Consts& K, const Geo& I, TallyTable& T, uint64_t id,
                          uint32_t step, double tfac, int g, double nu, double w, Flight& f)
{
    for (;;) {
        // time to the face ahead on each axis: the face is selected first and
        // divided once (a branch per sign would make a wavefront holding both
        // signs evaluate both divisions)
        const double vx = K.cv * f.ox;
        const double xl = I.x0 + (double)f.ix * I.dx, xr = I.x0 + (double)(f.ix + 1) * I.dx;
        const double qx = ((vx > 0 ? xr : xl) - f.x) / vx;
        const double tx = (vx > 0 || vx < 0) ? qx : INFINITY;
        double vy = 0.0, yl = 0.0, yr = 0.0, ty = INFINITY;
        if (DIM == 2) {
            vy = K.cv * f.oy;
            yl = I.y0 + (double)f.iy * I.dy;
            yr = I.y0 + (double)(f.iy + 1) * I.dy;
            const double qy = ((vy > 0 ? yr : yl) - f.y) / vy;
            ty = (vy > 0 || vy < 0) ? qy : INFINITY;
        }
        const bool xaxis = DIM == 1 || tx <= ty;
        const double tf = xaxis ? tx : ty;
        if (!(tf < f.t_rem)) {
            double xn = f.x + vx * f.t_rem;
            xn = xn < xl ? xl : xn;
            xn = xn > xr ? xr : xn;
            f.x = xn;
            if (DIM == 2) {
                double yn = f.y + vy * f.t_rem;
                yn = yn < yl ? yl : yn;
                yn = yn > yr ? yr : yn;
                f.y = yn;
            }
            return f.coll ? 1 : 0;
        }
        f.t = f.t + tf;
        bool pos, boundary;
        int side;
        uint32_t type, index;
        if (xaxis) {
            pos = vx > 0;
            f.x = pos ? xr : xl;
            if (DIM == 2) {
                double yn = f.y + vy * tf;
                yn = yn < yl ? yl : yn;
                yn = yn > yr ? yr : yn;
                f.y = yn;
            }
            boundary = pos ? (f.ix == I.nx - 1) : (f.ix == 0);
            side = pos ? XHI : XLO;
            const uint32_t face = (uint32_t)(f.iy * (I.nx + 1) + (pos ? f.ix + 1 : f.ix));
            type = TAL_FX;
            index = ((I.fx_off + (face << I.lgGp) + (uint32_t)g) << 1) + (pos ? 0u : 1u);
        } else {
            pos = vy > 0;
            f.y = pos ? yr : yl;
            double xn = f.x + vx * tf;
            xn = xn < xl ? xl : xn;
            xn = xn > xr ? xr : xn;
            f.x = xn;
            boundary = pos ? (f.iy == I.ny - 1) : (f.iy == 0);
            side = pos ? YHI : YLO;
            const uint32_t face = (uint32_t)((pos ? f.iy + 1 : f.iy) * I.nx + f.ix);
            type = TAL_FY;
            index = ((I.fy_off + (face << I.lgGp) + (uint32_t)g) << 1) + (pos ? 0u : 1u);
        }
        if (boundary) {
            if ((I.reflect >> side) & 1) {
                if (xaxis) { f.ox = -f.ox; f.flips ^= FLIP_X; } else { f.oy = -f.oy; f.flips ^= FLIP_Y; }
                f.t_rem = f.t_rem - tf;
                continue;
            }
            lds_tally(T, D, type, index, w);
            return 2;
        }
        lds_tally(T, D, type, index, w);
        if (xaxis) f.ix += pos ? 1 : -1; else f.iy += pos ? 1 : -1;
        f.tau = cell_tau<SM>(D, K, I, tfac, f.iy * I.nx + f.ix, g, nu, f);
        draw_flight(K, I, id, step, f);
    }
}

// A boundary-source particle born in the ghost cell beyond `side`: it flies
// straight (a new particle: no collision in the ghost) to the domain face;
// if it meets the face within the step at a point of the domain's extent, the
// crossing is tallied there, it stands in the cell it enters at the time it
// entered, and its flight is drawn in that cell (Remark 1).  Returns false for
// a particle that never enters (dropped without a tally).  The domain's faces
// are computed as the cells' faces are.
template <int DIM, int SM>
__device__ inline bool enter_from_ghost(const Dev& D, const Consts& K, const Geo& I, TallyTable& T, uint64_t id,
                                        uint32_t step, double tfac, int g, double nu, double w, int side,
                                        Flight& f)
{
    const bool xside = side == XLO || side == XHI;
    const bool lo = side == XLO || side == YLO;
    const double vx = K.cv * f.ox, vy = DIM == 2 ? K.cv * f.oy : 0.0;
    const double vn = xside ? vx : vy;
    if (lo ? !(vn > 0) : !(vn < 0)) return false;
    const double xend = I.x0 + (double)I.nx * I.dx;
    const double yend = DIM == 2 ? I.y0 + (double)I.ny * I.dy : 0.0;
    const double pf = xside ? (lo ? I.x0 : xend) : (lo ? I.y0 : yend);
    const double te = (pf - (xside ? f.x : f.y)) / vn;
    if (!(te < K.dt)) return false;
    uint32_t type, index;
    if (xside) {
        if (DIM == 2) {
            const double ye = f.y + vy * te;
            if (ye < I.y0 || ye > yend) return false;
            int iy = (int)floor((ye - I.y0) / I.dy);
            iy = iy > I.ny - 1 ? I.ny - 1 : (iy < 0 ? 0 : iy);
            const double yl = I.y0 + (double)iy * I.dy, yr = I.y0 + (double)(iy + 1) * I.dy;
            f.y = ye < yl ? yl : (ye > yr ? yr : ye);
            f.iy = iy;
        }
        f.x = pf;
        f.ix = lo ? 0 : I.nx - 1;
        const uint32_t face = (uint32_t)(f.iy * (I.nx + 1) + (lo ? 0 : I.nx));
        type = TAL_FX;
        index = ((I.fx_off + (face << I.lgGp) + (uint32_t)g) << 1) + (lo ? 0u : 1u);
    } else {
        const double xe = f.x + vx * te;
        if (xe < I.x0 || xe > xend) return false;
        int ix = (int)floor((xe - I.x0) / I.dx);
        ix = ix > I.nx - 1 ? I.nx - 1 : (ix < 0 ? 0 : ix);
        const double xl = I.x0 + (double)ix * I.dx, xr = I.x0 + (double)(ix + 1) * I.dx;
        f.x = xe < xl ? xl : (xe > xr ? xr : xe);
        f.ix = ix;
        f.y = pf;
        f.iy = lo ? 0 : I.ny - 1;
        const uint32_t face = (uint32_t)((lo ? 0 : I.ny) * I.nx + f.ix);
        type = TAL_FY;
        index = ((I.fy_off + (face << I.lgGp) + (uint32_t)g) << 1) + (lo ? 0u : 1u);
    }
    lds_tally(T, D, type, index, w);
    f.t = te;
    f.tau = cell_tau<SM>(D, K, I, tfac, f.iy * I.nx + f.ix, g, nu, f);
    draw_flight(K, I, id, step, f);
    return true;
}

// One pool record as the push reads it (every field, also for an empty slot:
// all slots below the capacity are allocated, and the values are then unused).
// Element i of a pool array by a 32-bit byte offset from the array's base (the
// capacity is at most 2^29 slots), so that the load can take the base in
// scalar registers and the offset in one vector register.
template <class T>
__device__ inline T& at(T* base, uint32_t i)
{
    return *(T*)((char*)base + (size_t)(i * (uint32_t)sizeof(T)));
}

// The push reads each pool record once and writes the moving fields once:
// those accesses are non-temporal, so that they stream past the caches that
// hold the flights' tables and tallies (lattice push 1216 -> 1174 us; a plain
// streaming kernel of the same accesses ran 4-5% faster so).  The sort keeps
// plain accesses: several blocks write a key's range, and non-temporal stores
// of those partial lines doubled its time.
template <class T>
__device__ inline T ldnt(const T* base, uint32_t i)
{
    return __builtin_nontemporal_load((const T*)((const char*)base + (size_t)(i * (uint32_t)sizeof(T))));
}

template <class T>
__device__ inline void stnt(T* base, uint32_t i, T v)
{
    __builtin_nontemporal_store(v, (T*)((char*)base + (size_t)(i * (uint32_t)sizeof(T))));
}

template <int DIM>
struct PoolRec {
    double x, y, ox, oy, nu, w;
    uint64_t idw;          // id | group word << ID_BITS (split where it is used, so
                           // that a load issued ahead is not waited for here)
    int32_t word;
    __device__ inline void load(const Pool& P, uint32_t i)
    {
        word = ldnt(P.cell, i);
        idw = ldnt(P.id, i);
        x = ldnt(P.x, i);
        ox = ldnt(P.ox, i);
        if (DIM == 2) {
            y = ldnt(P.y, i);
            oy = ldnt(P.oy, i);
        }
        nu = ldnt(P.nu, i);
        w = ldnt(P.w, i);
    }
};

// Each block takes chunks of PUSH_THREADS * ppt consecutive pool slots;
// a thread handles ppt of them.  Stable fields are only read; the new
// position and cell word go to the other moving-field buffer at the same slot,
// so the committed pool stays intact until the step commits.
// The wavefronts per SIMD the single-instance pushes of the nu^-3 and group
// opacities are held to (their registers fit without spilling: 4 in 2-D, 5 in
// 1-D); the other instances are left to the compiler.
template <int DIM, bool SINGLE, int SM>
constexpr int push_min_waves()
{
    return (!SINGLE || (SM != SIG_NU3 && SM != SIG_GROUP)) ? 1 : (DIM == 2 ? 4 : 5);
}
#ifndef UGK_PUSH_ATTR
#define UGK_PUSH_ATTR __attribute__((amdgpu_waves_per_eu(push_min_waves<DIM, SINGLE, SM>())))
#endif
#ifndef UGK_PUSH_PREFETCH_2D
#define UGK_PUSH_PREFETCH_2D 1
#endif
template <int DIM, bool SINGLE, int SM, int BS>
__global__ __launch_bounds__(BS) UGK_PUSH_ATTR void k_push(Dev D, Consts K, Pool In, Pool Out, int ppt)
{
    constexpr bool PUSH_PREFETCH = DIM == 2 && UGK_PUSH_PREFETCH_2D;
    if (!gate_open(D, K, 0)) return;
    const uint32_t step = *D.step;
    __shared__ TallyTable T;
    __shared__ unsigned long long bsurv[BS / WAVE];
    if (D.counters[CNT_ERR] & ERR_POOL) return;
    const int64_t n_slots = (int64_t)D.counters[CNT_SLOTS];
    const int64_t n_total = (int64_t)D.counters[CNT_PUSHED];
    const int64_t chunk = (int64_t)BS * ppt;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    unsigned long long nsurv = 0;
    Geo geo0{};
    double inv_nx0 = 0.0;
    if (SINGLE) {
        geo0 = geo_of(D.inst[0]);
        inv_nx0 = 1.0 / (double)geo0.nx;
    }
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < n_total; c0 += (int64_t)gridDim.x * chunk) {
        for (int h = threadIdx.x; h < HT_SIZE; h += BS) {
            T.key[h] = HT_EMPTY;
            T.cnt[h] = 0u;
            T.val[h] = 0.0;
        }
        __syncthreads();
        // 2-D: the records of the next round are read while this round's flights
        // run (1-D: the registers this takes would cost a wavefront per SIMD)
        PoolRec<DIM> nxt;
        if (PUSH_PREFETCH) {
            const int64_t i0 = c0 + threadIdx.x;
            if (i0 < n_total) nxt.load(In, (uint32_t)i0);
        }
#pragma unroll 1
        for (int r = 0; r < ppt; ++r) {
            const int64_t i = c0 + (int64_t)r * BS + threadIdx.x;
            const uint32_t iu = (uint32_t)i;
            // the outcome tally of this lane's particle (survival or deposition)
            bool has = false;
            uint32_t tkey = 0u;
            double tw = 0.0;
            PoolRec<DIM> cur;
            if (PUSH_PREFETCH) {
                cur = nxt;
                if (r + 1 < ppt && i + BS < n_total) nxt.load(In, iu + BS);
            } else if (i < n_total) {
                cur.word = ldnt(In.cell, iu);      // the rest only for a live slot
            }
            const int32_t word = cur.word;
            const int cell = word & CELL_MASK;
            if (i >= n_total) {
                // past the end of the pool: nothing
            } else if (word < 0) {                 // empty slot stays empty
                stnt(Out.cell, iu, DEAD);
            } else if (cell >= K.ncell) {
                atomicOr((unsigned long long*)(D.counters + CNT_ERR), ERR_RECORD);
                stnt(Out.cell, iu, DEAD);
            } else {
                if (!PUSH_PREFETCH) {
                    cur.idw = ldnt(In.id, iu);
                    cur.x = ldnt(In.x, iu);
                    cur.ox = ldnt(In.ox, iu);
                    if (DIM == 2) {
                        cur.y = ldnt(In.y, iu);
                        cur.oy = ldnt(In.oy, iu);
                    }
                    cur.nu = ldnt(In.nu, iu);
                    cur.w = ldnt(In.w, iu);
                }
                const int32_t gword = (int32_t)(cur.idw >> ID_BITS);
                const int g = gword & GROUP_MASK;
                const int gside = gword >> GHOST_SHIFT;    // boundary-source particle: 1 + ghost side
                const Geo I = SINGLE ? geo0 : geo_of(D.inst[D.cell_inst[cell]]);
                Flight f;
                f.x = cur.x;
                f.ox = (word & FLIP_X) ? -cur.ox : cur.ox;
                if (DIM == 2) {
                    f.y = cur.y;
                    f.oy = (word & FLIP_Y) ? -cur.oy : cur.oy;
                } else {
                    f.y = 0.0;
                    f.oy = 0.0;
                }
                const double nu = cur.nu, w = cur.w;
                const uint64_t id = cur.idw & ID_MASK;
                const int lcell = cell - I.cell_off;
                if (DIM == 1) {
                    f.ix = lcell;
                    f.iy = 0;
                } else if (SINGLE) {
                    cell_col_row(lcell, I.nx, inv_nx0, f.ix, f.iy);
                } else {
                    f.ix = lcell % I.nx;
                    f.iy = lcell / I.nx;
                }
                f.t = 0.0;
                f.d = 0;
                f.flips = 0;
                const double tfac = tau_factor<SM>(D, K, I, nu, g);
                f.ti = 0;
                f.ta = 0.0;
                if (SM == SIG_TAB) f.ti = table_locate(D.tab_lnu, K.tab_nnu, log(nu), &f.ta);
                f.tau = cell_tau<SM>(D, K, I, tfac, lcell, g, nu, f);
                int out;
                if (gside && !enter_from_ghost<DIM, SM>(D, K, I, T, id, step, tfac, g, nu, w, gside - 1, f)) {
                    out = 3;                                        // never entered the domain
                } else {
                    if (gside) {
                        // entered: its flight is drawn; the group word loses the ghost mark
                        at(In.id, iu) = id | ((uint64_t)g << ID_BITS);
                    } else if (i < n_slots) {
                        draw_flight(K, I, id, step, f);             // old particle: t_f = min(-tau ln eta, dt)
                    } else {
                        f.coll = false;                             // new collisionless particle: t_f = dt
                        f.t_rem = K.dt;
                    }
                    out = fly<DIM, SM>(D, K, I, T, id, step, tfac, g, nu, w, f);
                }
                if (out < 2) {
                    const uint32_t cg = I.cg_off + ((uint32_t)(f.iy * I.nx + f.ix) << I.lgGp) + (uint32_t)g;
                    has = true;
                    tkey = (cg << 2) | (out == 0 ? TAL_SURV : TAL_DEP);
                    tw = w;
                }
                if (out == 0) {
                    // pending reversals relative to the stored direction: those
                    // carried in, toggled by this step's reflections
                    const int32_t nw = (I.cell_off + f.iy * I.nx + f.ix) | ((word ^ f.flips) & (FLIP_X | FLIP_Y));
                    stnt(Out.x, iu, f.x);
                    if (DIM == 2) stnt(Out.y, iu, f.y);
                    stnt(Out.cell, iu, nw);
                    nsurv++;
                } else {
                    stnt(Out.cell, iu, DEAD);
                }
            }
            if (has) lds_add(T, D, tkey, tw, 1u);
        }
        __syncthreads();
        // flush the chunk's tallies: one global atomic per distinct bin
        for (int h = threadIdx.x; h < HT_SIZE; h += BS) {
            const uint32_t key = T.key[h];
            if (key == HT_EMPTY) continue;
            const uint32_t type = key & 3u, index = key >> 2;
            unsafeAtomicAdd(tally_target(D, type, index), T.val[h]);
            if (type == TAL_SURV) atomicAdd(D.scount + index, T.cnt[h]);
        }
        __syncthreads();
    }
    // survivors of this block (summed by the commit)
    for (int m = 32; m >= 1; m >>= 1) nsurv += __shfl_xor(nsurv, m, WAVE);
    if (lane == 0) bsurv[wid] = nsurv;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < BS / WAVE; ++k) t += bsurv[k];
        D.blk_surv[blockIdx.x] = t;
    }
}

// Counting-sort scatter of the live particles (In -> Out) by (cell, group)
// slot: compacts the pool, applies pending direction reversals, and leaves the
// pool ordered so that the blocks of the next pushes see few tally bins.  soff
// holds the exclusive scan of the survivor counts and serves as the per-slot
// write cursor.  Each block ranks the particles of a chunk per key in an LDS
// table and reserves every key's range with one global atomic; the input is
// nearly sorted, so a chunk holds few keys.  Blocks of 1024 threads (one per
// CU at the 2-D kernel's register count) sorted the 2-D lattice's pool 8% faster
// than four blocks of 256 per CU; 1024 threads of two particles each did not.
constexpr int SORT_THREADS = 1024;
constexpr int SORT_PPT = 4;
constexpr int ST_BITS = 10;
constexpr int ST_SIZE = 1 << ST_BITS;

struct RankTable {
    uint32_t key[ST_SIZE];
    uint32_t cnt[ST_SIZE];
    unsigned long long base[ST_SIZE];
};

template <int DIM, bool SINGLE>
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(Dev D, Consts K, Pool In, Pool Out)
{
    __shared__ RankTable R;
    if (!gate_open(D, K, 1) || !step_committed(D, K)) return;
    const int64_t n = (int64_t)D.counters[CNT_PUSHED];
    const int64_t nlive = (int64_t)D.counters[CNT_SURV];
    if (blockIdx.x == 0 && threadIdx.x == 0) D.counters[CNT_SLOTS] = (unsigned long long)nlive;
    const int64_t chunk = SORT_THREADS * SORT_PPT;
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < n; c0 += (int64_t)gridDim.x * chunk) {
        for (int h = threadIdx.x; h < ST_SIZE; h += SORT_THREADS) {
            R.key[h] = HT_EMPTY;
            R.cnt[h] = 0u;
        }
        __syncthreads();
        int slot[SORT_PPT];          // table entry (>= 0), -1 empty slot, -2 ranked globally
        int64_t pos[SORT_PPT];       // local rank, or the global position when ranked globally
        // the records, read while the ranks are found (their stores come after the
        // block's ranks, and loads issued after a store could not pass it)
        double rx[SORT_PPT], ry[SORT_PPT], rox[SORT_PPT], roy[SORT_PPT], rnu[SORT_PPT], rw[SORT_PPT];
        uint64_t rid[SORT_PPT];
        int32_t rword[SORT_PPT];
#pragma unroll
        for (int r = 0; r < SORT_PPT; ++r) {
            const int64_t i = c0 + (int64_t)r * SORT_THREADS + threadIdx.x;
            slot[r] = -1;
            pos[r] = 0;
            rword[r] = -1;
            if (i >= n) continue;
            const int32_t word = In.cell[i];
            rword[r] = word;
            if (word < 0) continue;
            const int cell = word & CELL_MASK;
            const uint64_t idw = In.id[i];          // id | group word << ID_BITS
            const int g = (int)(idw >> ID_BITS);
            rid[r] = idw;
            rx[r] = In.x[i];
            rox[r] = In.ox[i];
            if (DIM == 2) {
                ry[r] = In.y[i];
                roy[r] = In.oy[i];
            }
            rnu[r] = In.nu[i];
            rw[r] = In.w[i];
            bool ok = cell < K.ncell;
            int64_t key = 0;
            if (ok) {
                const Inst& I = D.inst[SINGLE ? 0 : D.cell_inst[cell]];
                ok = g >= 0 && g < I.G;
                key = I.cg_off + ((int64_t)(cell - I.cell_off) << I.lgGp) + g;
            }
            if (!ok) {
                atomicOr((unsigned long long*)(D.counters + CNT_ERR), ERR_RECORD);
                continue;
            }
            const uint32_t k32 = (uint32_t)key;
            uint32_t h = (k32 * 2654435761u) >> (32 - ST_BITS);
            bool placed = false;
#pragma unroll 1
            for (int probe = 0; probe < HT_PROBES; ++probe) {
                const uint32_t prev = atomicCAS(&R.key[h], HT_EMPTY, k32);
                if (prev == HT_EMPTY || prev == k32) {
                    slot[r] = (int)h;
                    pos[r] = atomicAdd(&R.cnt[h], 1u);
                    placed = true;
                    break;
                }
                h = (h + 1) & (ST_SIZE - 1);
            }
            if (!placed) {
                slot[r] = -2;
                pos[r] = (int64_t)atomicAdd((unsigned long long*)(D.soff + key), 1ull);
            }
        }
        __syncthreads();
        for (int h = threadIdx.x; h < ST_SIZE; h += SORT_THREADS) {
            const uint32_t k32 = R.key[h];
            if (k32 != HT_EMPTY)
                R.base[h] = atomicAdd((unsigned long long*)(D.soff + k32), (unsigned long long)R.cnt[h]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_PPT; ++r) {
            if (slot[r] == -1) continue;
            const int64_t o = slot[r] >= 0 ? (int64_t)R.base[slot[r]] + pos[r] : pos[r];
            if (o < 0 || o >= nlive) {
                atomicOr((unsigned long long*)(D.counters + CNT_ERR), ERR_COUNT);
                continue;
            }
            const int32_t word = rword[r];
            Out.x[o] = rx[r];
            Out.ox[o] = (word & FLIP_X) ? -rox[r] : rox[r];
            if (DIM == 2) {
                Out.y[o] = ry[r];
                Out.oy[o] = (word & FLIP_Y) ? -roy[r] : roy[r];
            }
            Out.nu[o] = rnu[r];
            Out.w[o] = rw[r];
            Out.id[o] = rid[r];
            Out.cell[o] = word & CELL_MASK;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// A4: wave free-transport flux and the static source Q

// The faces of a slot's cell in the order XLO, XHI, YLO, YHI (the first two in
// 1-D): whether the neighbour across lies in the instance, its slot, the face's
// tally slot and area.  Index arithmetic only, so that a kernel can issue every
// load of the stencil before it waits for the first.
struct CellFaces {
    bool inside[4];
    int64_t nbj[4], fslot[4];
    double S[4];
};

template <int DIM>
__device__ inline CellFaces cell_faces(const Inst& I, int64_t j, int ix, int iy, int g)
{
    CellFaces F;
    const int Gp = I.Gp, nx = I.nx;
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) {
        const bool lo = (q & 1) == 0;
        if (q < 2) {
            F.inside[q] = lo ? ix > 0 : ix < nx - 1;
            F.nbj[q] = j + (lo ? -Gp : Gp);
            F.fslot[q] = I.fx_off + (((int64_t)iy * (nx + 1) + ix + (lo ? 0 : 1)) << I.lgGp) + g;
            F.S[q] = I.dy;
        } else {
            F.inside[q] = lo ? iy > 0 : iy < I.ny - 1;
            F.nbj[q] = j + (lo ? -(int64_t)nx * Gp : (int64_t)nx * Gp);
            F.fslot[q] = I.fy_off + (((int64_t)(iy + (lo ? 0 : 1)) * nx + ix) << I.lgGp) + g;
            F.S[q] = I.dx;
        }
    }
    return F;
}

// Wave flux through the faces of slot j and its static source Q (Remark 3:
// coefficient C4 - e^{-s} where the cell sampled particles, C4 where it did
// not).  *inflow gets the energy the wave flux brings in through the domain
// boundary.
// EXT: compiled with the slope terms and the boundary-source ghosts (which the
// flags then switch); without it the base flux only, at fewer registers.
template <int DIM, bool EXT>
__device__ inline double wave_source(const Dev& D, const Consts& K, const Inst& I, int64_t j, const Slot& s,
                                     const CellFaces& F, double* inflow_out, const double* src, bool sub_rhop)
{
    const int g = s.g, nx = I.nx;
    const int ix = DIM == 1 ? s.lcell : s.lcell % nx, iy = DIM == 1 ? 0 : s.lcell / nx;
    const double cq = K.cq;
    const double* phib = D.phib + (int64_t)s.inst * 4 * MAX_G;
    constexpr int nf = 2 * DIM;
    const bool slopes = EXT && (K.flags & UGKWP_FLAG_SLOPES) != 0;
    const bool bpart = EXT && (K.flags & UGKWP_FLAG_BOUNDARY_PARTICLES) != 0;
    // every load first
    // the wave coefficient of a sampled slot: W(s), or this step's joint-cell value
    const double* wsamp = K.tau_C > 0.0 ? D.wsn : D.wc;
    const int nb_here = D.nbi[j];
    const double wc_here = wsamp[j], c4_here = D.c4[j], rho_here = D.rho[j];
    const double rhoh_here = sub_rhop ? src[j] - D.rhop[j] : src[j];
    double sl_here[2] = {0.0, 0.0}, b_here = 0.0, es_here = 0.0, wphys_here = 0.0;
    if (slopes) {
        sl_here[0] = D.sx[j];
        if (DIM == 2) sl_here[1] = D.sy[j];
        b_here = D.bcoef[j];
    }
    if (bpart) {
        es_here = D.es[j];
        wphys_here = D.wc[j];
    }
    int nb_n[4];
    double wc_n[4], c4_n[4], rhoh_n[4], pb[4], sl_n[4], b_n[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        nb_n[q] = 0;
        wc_n[q] = c4_n[q] = rhoh_n[q] = pb[q] = sl_n[q] = b_n[q] = 0.0;
        if (q >= nf) continue;
        if (F.inside[q]) {
            const int64_t n = F.nbj[q];
            nb_n[q] = D.nbi[n];
            wc_n[q] = wsamp[n];
            c4_n[q] = D.c4[n];
            rhoh_n[q] = sub_rhop ? src[n] - D.rhop[n] : src[n];
            if (slopes) {
                sl_n[q] = q < 2 ? D.sx[n] : D.sy[n];
                b_n[q] = D.bcoef[n];
            }
        } else if (I.bc[q] == BC_PLANCK) {
            pb[q] = phib[q * MAX_G + g];
        }
    }
    // gross particle crossings into / out of the cell
    const int64_t fl = I.fx_off + (((int64_t)iy * (nx + 1) + ix) << I.lgGp) + g;
    const int64_t fr = fl + I.Gp;
    const double tx0 = D.ftx[fl * 2 + 0], tx1 = D.ftx[fr * 2 + 1], tx2 = D.ftx[fl * 2 + 1], tx3 = D.ftx[fr * 2 + 0];
    double ty0 = 0.0, ty1 = 0.0, ty2 = 0.0, ty3 = 0.0;
    if (DIM == 2) {
        const int64_t fb = I.fy_off + (((int64_t)iy * nx + ix) << I.lgGp) + g;
        const int64_t ft = fb + ((int64_t)nx << I.lgGp);
        ty0 = D.fty[fb * 2 + 0]; ty1 = D.fty[ft * 2 + 1];
        ty2 = D.fty[fb * 2 + 1]; ty3 = D.fty[ft * 2 + 0];
    }
    const double Ah = nb_here > 0 ? wc_here : c4_here;
    const double here = Ah * rhoh_here;
    const double cs = K.c * K.c * K.dt / (6.0 * K.eps * K.eps);
    double fsum = 0.0, inflow = 0.0;
    // flux through a face along +axis: cq (A_low rho^h_low - A_high rho^h_high), with
    // slopes the upwind profiles at the face and cs (B_low s_low + B_high s_high)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nf) continue;
        const bool lo = (q & 1) == 0;
        double Fpos;
        double there;
        if (!F.inside[q]) {
            const int bc = I.bc[q];
            if (bc == BC_REFLECT) continue;
            // a Planckian ghost that emitted boundary-source particles keeps C4 - e^{-s}
            double Ag = c4_here;
            if (bpart && bc == BC_PLANCK) {
                const double eov = es_here * pb[q];
                if (eov * I.V > 0.0 && K.n_cap >= 1 && eov / I.w_ref >= 1.0) Ag = wphys_here;
            }
            there = bc == BC_PLANCK ? Ag * pb[q] : 0.0;
        }
        if (!slopes) {
            if (F.inside[q]) {
                const double An = nb_n[q] > 0 ? wc_n[q] : c4_n[q];
                there = An * rhoh_n[q];
            }
            Fpos = lo ? cq * (there - here) : cq * (here - there);
        } else {
            const double slh = sl_here[q >> 1], h = q < 2 ? I.dx : I.dy;
            // this cell is the high cell of a LO face and the low cell of a HI face
            const double hv = Ah * (rhoh_here + (lo ? -0.5 : 0.5) * h * slh);
            const double hs = b_here * slh;
            double ts = 0.0;
            if (F.inside[q]) {
                const double An = nb_n[q] > 0 ? wc_n[q] : c4_n[q];
                there = An * (rhoh_n[q] + (lo ? 0.5 : -0.5) * h * sl_n[q]);
                ts = b_n[q] * sl_n[q];
            }
            Fpos = lo ? cq * (there - hv) + cs * (ts + hs) : cq * (hv - there) + cs * (hs + ts);
        }
        const double Fin = lo ? Fpos : -Fpos;
        fsum += F.S[q] * Fin;
        if (!F.inside[q]) inflow += K.dt * F.S[q] * Fin / K.c;
    }
    double a_in = tx0 + tx1;
    double a_out = tx2 + tx3;
    if (DIM == 2) {
        a_in += ty0 + ty1;
        a_out += ty2 + ty3;
    }
    *inflow_out = inflow;
    const double Q = rho_here + I.dt_V * fsum + (a_in - a_out) / I.V;
    // a volumetric source adds dt q in the steps it is on
    return source_on(K, *D.step) ? Q + K.dt * D.qsrc[j] : Q;
}

// Q of sweep k >= 1 with UGKWP_FLAG_WAVE_ITER: the wave flux from the iterate
// rho^k (src) less rho^p (Algorithm 2), and the boundary wave inflow of the
// sweep into winflow[k & 1] (the commit takes that of the last sweep).
// Instances whose iteration has converged are left alone.
template <int DIM>
__global__ __launch_bounds__(256) void k_wave_q(Dev D, Consts K, int k, const double* src)
{
    if (!gate_open(D, K, 0)) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    if (!s.cell_ok || !s.active) return;
    if (D.ist[s.inst].conv_sweeps != 0) return;
    const Inst& I = D.inst[s.inst];
    const int nx = I.nx;
    const int ix = DIM == 1 ? s.lcell : s.lcell % nx, iy = DIM == 1 ? 0 : s.lcell / nx;
    const CellFaces F = cell_faces<DIM>(I, j, ix, iy, s.g);
    double inflow = 0.0;
    D.Q[j] = wave_source<DIM, true>(D, K, I, j, s, F, &inflow, src, true);
    D.winflow[(int64_t)(k & 1) * K.n_cg + j] = inflow;
}

// ---------------------------------------------------------------------------
// A5: source iteration.  Thread per (cell, group) slot; the Gp slots of a cell
// share one wavefront, so the group sum of the temperature update and the
// group-edge sharing of the Planck integrals are wavefront shuffles.  Sweep 0
// also evaluates the wave flux and Q (A4) for its slot and keeps Q for the
// later sweeps; it starts from rho^0 = rho^n, T^0 = T^n and phi^0 = phi(T^n),
// which phi0 already holds (the previous commit's last sweep output, the same
// expression at the same temperature).

constexpr int SI_THREADS = 256;

// phi^k buffers: sweep 0 reads phi0 = phi(T^n), sweep k writes phi1 (k even)
// or phi2 (k odd) and sweep k + 1 reads it; phi0 is only rewritten by the commit.
__host__ __device__ inline const double* sweep_in(const Dev& D, int k)
{
    return k == 0 ? D.phi0 : (((k - 1) & 1) ? D.phi2 : D.phi1);
}
__host__ __device__ inline double* sweep_out(const Dev& D, int k) { return (k & 1) ? D.phi2 : D.phi1; }

// Residual sub-slots of sweep k for instance inst: [RES_SLOTS][n_inst][RES_SUB],
// so that the slots of sweep 0 form one range cleared at the start of a step.
__device__ inline Resid* res_slot(const Dev& D, const Consts& K, int inst, int k)
{
    return D.res + ((int64_t)(k % RES_SLOTS) * K.n_inst + inst) * RES_SUB;
}

// The stopping test after sweep k for instance inst, taken by one wavefront
// from the instance's 64 residual sub-slots (lane l reads sub-slot l).
__device__ inline bool si_converged(const Dev& D, const Consts& K, int inst, int k, int lane)
{
    const Resid r = res_slot(D, K, inst, k)[lane];
    const double drho = bitsd(wave_max_bits(bitsd(r.drho))), mrho = bitsd(wave_max_bits(bitsd(r.rho)));
    const double dT = bitsd(wave_max_bits(bitsd(r.dT))), mT = bitsd(wave_max_bits(bitsd(r.T)));
    return drho <= K.si_tol * mrho && dT <= K.si_tol * mT;
}

// Sweep k: rho^{k+1}, T^{k+1} and phi^{k+1} from phi^k for every instance whose
// iteration is still running.  The residual maxima of the sweep go to sub-slots
// of the instance (spread over 64 addresses by block); k_si_decide reads them.
// With decide_prev (single-instance contexts), every block first takes the
// convergence decision of sweep k-1 itself, from the same sub-slots, so no
// decide launch sits between sweeps; block 0 records it.
// FIRST: sweep 0 (its own instantiation, so that the wave-flux code does not
// weigh on the registers of the later sweeps); SINGLE: a context of one
// instance; DIM: the dimension of every instance of the context.
// LIN: the linearized iteration. A sweep takes the new temperature's emission
// as phi^k + phi'(T^k) (T^{k+1} - T^k) and solves each cell's energy balance
// for T^{k+1}, a local Newton step with the literal iteration's fixed point
// (Eq. macroSysFinal) that also converges under stiff material coupling.
template <bool FIRST, bool SINGLE, int DIM, bool TDEP, bool LIN, bool EXT>
__global__ __launch_bounds__(SI_THREADS) void k_si_sweep(Dev D, Consts K, int k, const double* phi_in,
                                                          double* phi_out, int decide_prev, const double* rho_in,
                                                          double* rho_out)
{
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int64_t j = (int64_t)blockIdx.x * SI_THREADS + threadIdx.x;
    // The gate (step count), for batches the flags of the block's wavefronts
    // (a block whose four wavefronts all belong to converged instances returns
    // after them) and for one instance the state and residuals of the sweep
    // before (the stopping test) are requested together; the slot's data only
    // once the block is known to run.
    const uint32_t now = *D.step;
    uint32_t flags = 0xFFFFFFFFu;
    if (K.n_inst > 1 && !FIRST) flags = ((const uint32_t*)D.wave_run)[blockIdx.x];
    int cs_prev = 0;
    Resid res_prev = {0ull, 0ull, 0ull, 0ull};
    if (decide_prev) {
        cs_prev = D.ist[0].conv_sweeps;
        if (wid == 0) res_prev = res_slot(D, K, 0, k - 1)[lane];
    }
    if (!(K.gate == GATE_OFF || now == K.gate) || flags == 0) return;
    if (FIRST && j == 0 && K.has_src) *D.src_on = source_on(K, now) ? 1 : 0;   // for the commit's ledger
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    if (decide_prev) {
        // the whole block stops when the iteration has converged (decided now
        // or by an earlier sweep): a speculative sweep past convergence costs
        // little
        __shared__ int stop;
        if (wid == 0) {
            bool conv = false;
            if (cs_prev == 0) {
                const double drho = bitsd(wave_max_bits(bitsd(res_prev.drho)));
                const double mrho = bitsd(wave_max_bits(bitsd(res_prev.rho)));
                const double dTm = bitsd(wave_max_bits(bitsd(res_prev.dT)));
                const double mTm = bitsd(wave_max_bits(bitsd(res_prev.T)));
                conv = drho <= K.si_tol * mrho && dTm <= K.si_tol * mTm;
            }
            if (lane == 0) {
                stop = (conv || cs_prev != 0) ? 1 : 0;
                if (conv && blockIdx.x == 0) {
                    D.ist[0].conv_sweeps = k;
                    atomicAdd((unsigned long long*)(D.counters + CNT_CONV), 1ull);
                }
            }
        }
        __syncthreads();
        if (stop) return;
    }
    const int cs_inst = D.ist[s.inst].conv_sweeps;
    const bool wave_on = ((flags >> (8 * wid)) & 0xFFu) != 0;
    const int g = s.g, Gp = I.Gp, G = I.G;
    const bool load = wave_on && s.cell_ok;       // the slot's cell is updated (every group lane)
    const bool act = load && s.active;            // and the slot is a group of it

    // every load of the sweep is issued here, before the first wait
    const int nx = I.nx;
    const int ix = DIM == 1 ? s.lcell : s.lcell % nx, iy = DIM == 1 ? 0 : s.lcell / nx;
    const int cell = I.cell_off + s.lcell;
    const CellFaces F = cell_faces<DIM>(I, j, ix, iy, g);
    constexpr int nf = 2 * DIM;
    const double* phib = D.phib + (int64_t)s.inst * 4 * MAX_G;
    double phi = 0.0, Qj = 0.0, lam = 0.0, sig = 0.0, rho_prev = 0.0;
    double Df[4] = {0.0, 0.0, 0.0, 0.0}, pn[4] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
        phi = phi_in[j];
        if (!FIRST) Qj = D.Q[j];
        if (!TDEP) {
            // (TDEP sweeps form both from T^k; reading s here costs less than
            // forming it from sigma, a division per slot)
            lam = D.sv[j];
            sig = D.sig[j];
        }
        rho_prev = rho_in[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nf) continue;
            if (!TDEP) Df[q] = q < 2 ? D.Dx[F.fslot[q]] : D.Dy[F.fslot[q]];
            if (F.inside[q]) pn[q] = phi_in[F.nbj[q]];
            else if (I.bc[q] == BC_PLANCK) pn[q] = phib[q * MAX_G + g];
        }
    }
    // temperature-dependent opacity: kappa of the slot and of the neighbours
    // across each face, and the neighbours' iterate T^k
    // (a tabulated opacity: the group sigma of the slot and of the neighbours at the
    // iterate, written by the sweep before; sweep 0 takes the step's tables at T^n)
    double kap_j = 0.0, Sg = 0.0, Sn[4] = {0.0, 0.0, 0.0, 0.0};
    double kap_n[4] = {0.0, 0.0, 0.0, 0.0}, T_nb[4] = {1.0, 1.0, 1.0, 1.0};
    double tsig_j = 0.0, tsig_n[4] = {0.0, 0.0, 0.0, 0.0};
    int mat_j = 0;
    if (TDEP && act) {
        const double* tsig = FIRST ? D.sig : D.tab_sig + (int64_t)(k & 1) * K.n_cg;
        if (K.table) {
            mat_j = D.tab_mat[cell];
            tsig_j = tsig[j];
        } else {
            kap_j = D.kappa[j];
            Sg = group_factor(D, K, I.edge_off, g, FIRST ? D.T[cell] : D.T_new[cell]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nf || !F.inside[q]) continue;
            if (K.table) {
                tsig_n[q] = tsig[F.nbj[q]];
                continue;
            }
            const bool lo = (q & 1) == 0;
            const int nbc = cell + (q < 2 ? (lo ? -1 : 1) : (lo ? -nx : nx));
            T_nb[q] = FIRST ? D.T[nbc] : D.T_new[nbc];
            kap_n[q] = D.kappa[F.nbj[q]];
            Sn[q] = K.stim ? group_factor(D, K, I.edge_off, g, T_nb[q]) : Sg;
        }
    }
    double Tn = 1.0, Tk = 1.0, dtcv = 0.0, olH = 0.0, olchi = 0.0;
    uint8_t pinned = 0;
    double nu_lo = 0.0, nu_top = 0.0;
    if (load) {
        Tn = D.T[cell];
        Tk = FIRST ? Tn : D.T_new[cell];
        pinned = D.pinned[cell];
        dtcv = D.dtcv[cell];
        if (TDEP && K.olson) {
            olH = D.olH[cell];
            olchi = D.olchi[cell];
        }
        if (g <= G) nu_lo = D.nu[I.edge_off + g];
        if (g == G - 1 && G == Gp) nu_top = D.nu[I.edge_off + G];
    }
    double inflow = 0.0;
    if (FIRST && act) Qj = wave_source<DIM, EXT>(D, K, I, j, s, F, &inflow, D.rhoh, false);

    const bool run = wave_on && cs_inst == 0 && j < K.n_cg;
    double dr = 0.0, mr = 0.0, dT = 0.0, mT = 0.0;
    const bool work = run && s.cell_ok;
    // linearized iteration: d phi_g / dT at T^k, its upper-edge term from lane g+1
    double dph = 0.0;
    if (LIN) {
        const bool edge_lane = work && g <= G;
        const double we = edge_lane ? planck_edge_weight(nu_lo / Tk) : 0.0;
        double wh = __shfl_down(we, 1, Gp < 2 ? 2 : Gp);
        if (work && g == G - 1 && G == Gp) wh = planck_edge_weight(nu_top / Tk);
        if (work && s.active) dph = 4.0 * phi / Tk + K.a * K.c * (Tk * Tk * Tk) * (we - wh) / UGK_PI4_15;
    }
    double contrib = 0.0, dcon = 0.0, r = 0.0, b = 0.0;
    if (work && s.active) {
        if (TDEP) {
            // the coefficient step of Algorithm 2: sigma, lambda and the face
            // coefficients of this sweep from the iterate T^k
            const double sk = K.table ? tsig_j : kap_j * pow(Tk, -K.t_power) * Sg;
            sig = sk;
            lam = s_of_sigma(K, sk);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= nf) continue;
                double sf = sk;
                if (F.inside[q]) {
                    const double sn = K.table ? tsig_n[q] : kap_n[q] * pow(T_nb[q], -K.t_power) * Sn[q];
                    sf = (sk + sn > 0.0) ? 2.0 * (sk * sn) / (sk + sn) : 0.0;
                }
                Df[q] = face_coef(K, sf, q < 2 ? I.dx : I.dy);
            }
        }
        double lap = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nf) continue;
            const double p = F.inside[q] ? pn[q] : (I.bc[q] == BC_REFLECT ? phi : pn[q]);
            lap += F.S[q] * Df[q] * (p - phi);
        }
        b = Qj + I.dt_V * lap;
        const double em = (b - phi) / (1.0 + lam);
        contrib = sig * em;
        if (LIN) {
            dcon = sig * dph / (1.0 + lam);
        } else {
            r = (b + lam * phi) / (1.0 + lam);
            dr = fabs(r - rho_prev);
            mr = fabs(r);
        }
    }
    // group sum over the Gp lanes of the cell (every lane gets the same bits)
    contrib = group_sum(contrib, Gp);
    if (LIN) dcon = group_sum(dcon, Gp);

    double Tnew = 1.0, uend = 0.0;
    bool bad = false;
    if (work) {
        if (TDEP && olH > 0.0) {
            // Olson's heat capacity: the energy equation in the material energy U,
            // U(T^{n+1}) = U(T^n) + exchange.  Literal: U(T^{k+1}) = U(T^n) +
            // exchange(phi^k), solved for T^{k+1}; linearized: one Newton step at
            // T^k with U and the emission linearized, whose material energy is
            // U(T^k) + C_v(T^k)(T^{k+1} - T^k).
            const double un = olson_energy(olH, olchi, Tn);
            if (pinned) {
                Tnew = Tn;
                uend = un;
            } else if (LIN) {
                const double uk = olson_energy(olH, olchi, Tk), ck = olson_cv(olH, olchi, Tk);
                Tnew = Tk + (un - uk + K.dt / (K.eps * K.eps) * contrib) / (ck + K.dt / (K.eps * K.eps) * dcon);
                uend = uk + ck * (Tnew - Tk);
            } else {
                uend = un + K.dt / (K.eps * K.eps) * contrib;
                Tnew = olson_temperature(olH, olchi, uend, Tk);
            }
        } else if (LIN) Tnew = pinned ? Tn : Tk + (Tn - Tk + dtcv * contrib) / (1.0 + dtcv * dcon);
        else Tnew = pinned ? Tn : Tn + dtcv * contrib;
        if (LIN && s.active) {
            // rho^{k+1} with the linearized emission of T^{k+1}
            const double pe = pinned ? phi : phi + dph * (Tnew - Tk);
            r = (b + lam * pe) / (1.0 + lam);
            dr = fabs(r - rho_prev);
            mr = fabs(r);
        }
        if (!(Tnew > 0.0) || !isfinite(Tnew)) {
            bad = true;
            Tnew = 1.0;
        }
        if (g == 0) {
            dT = fabs(Tnew - Tk);
            mT = Tnew;
        }
    }
    // phi^{k+1}: lane g evaluates the Planck edge value at its lower edge nu_g / T,
    // takes the upper one from lane g+1 (lane G-1 evaluates it itself when G = Gp)
    double phi_new = 0.0;
    {
        const bool edge_lane = work && g <= G;
        const double xe = edge_lane ? nu_lo / Tnew : 0.0;
        const double ve = edge_lane ? planck_edge_value(xe, c_head) : 0.0;
        double xh = __shfl_down(xe, 1, Gp < 2 ? 2 : Gp);
        double vh = __shfl_down(ve, 1, Gp < 2 ? 2 : Gp);
        if (work && g == G - 1 && (G == Gp)) {
            xh = nu_top / Tnew;
            vh = planck_edge_value(xh, c_head);
        }
        if (work && s.active) phi_new = phi_from_band(K.a, K.c, Tnew, planck_band_from_edges(xe, ve, xh, vh));
    }
    // stores
    if (FIRST && K.n_inst > 1 && lane == 0) D.wave_run[(int64_t)blockIdx.x * (SI_THREADS / WAVE) + wid] = 1;
    const int64_t rel = j - I.cg_off;
    if (run && rel >= 0 && rel < RES_SUB) {
        Resid z = {0ull, 0ull, 0ull, 0ull};
        res_slot(D, K, s.inst, k + 1)[rel] = z;
    }
    if (work && s.active) {
        if (FIRST) D.Q[j] = Qj;
        rho_out[j] = r;
        phi_out[j] = phi_new;
        // a tabulated opacity: the next sweep's group sigma, at this sweep's T^{k+1}
        if (TDEP && K.table)
            D.tab_sig[(int64_t)((k + 1) & 1) * K.n_cg + j] = table_group_sigma(D, K, mat_j, I.edge_off + g, Tnew);
        // the boundary wave inflow: summed here, or with the wave flux of every
        // sweep from its iterate kept per slot for the commit (that of the last sweep)
        if (FIRST && (K.flags & UGKWP_FLAG_WAVE_ITER)) D.winflow[j] = inflow;
        else if (inflow != 0.0)
            atomicAdd(D.diag_sub + ((int64_t)s.inst * DIAG_SUB + (blockIdx.x & (DIAG_SUB - 1))) * 8 + 0, inflow);
    }
    if (work && g == 0) {
        if (bad) {
            atomicOr(&D.ist[s.inst].bad, 1);
            atomicOr((unsigned long long*)(D.counters + CNT_ERR), ERR_TEMP);
        }
        D.T_new[cell] = Tnew;
        if (TDEP && olH > 0.0) D.uend[cell] = uend;
    }
    // residual maxima: wavefront, then runs of wavefronts of one instance in the block
    // the four maxima are non-negative (or NaN): reduced as bit patterns
    const unsigned long long bdr = wave_max_bits(dr), bmr = wave_max_bits(mr);
    const unsigned long long bdT = wave_max_bits(dT), bmT = wave_max_bits(mT);
    __shared__ unsigned long long wres[SI_THREADS / WAVE][4];
    __shared__ int winst[SI_THREADS / WAVE];
    __shared__ int wrun[SI_THREADS / WAVE];
    if (lane == 0) {
        wres[wid][0] = bdr; wres[wid][1] = bmr; wres[wid][2] = bdT; wres[wid][3] = bmT;
        winst[wid] = s.inst;
        wrun[wid] = run ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int w0 = 0;
        const int nw = SI_THREADS / WAVE;
        while (w0 < nw) {
            int w1 = w0, any = 0;
            unsigned long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
            while (w1 < nw && winst[w1] == winst[w0]) {
                if (wrun[w1]) {
                    any = 1;
                    a0 = max(a0, wres[w1][0]); a1 = max(a1, wres[w1][1]);
                    a2 = max(a2, wres[w1][2]); a3 = max(a3, wres[w1][3]);
                }
                ++w1;
            }
            if (any) {
                Resid* r = res_slot(D, K, winst[w0], k) + (blockIdx.x & (RES_SUB - 1));
                atomicMax(&r->drho, a0);
                atomicMax(&r->rho, a1);
                atomicMax(&r->dT, a2);
                atomicMax(&r->T, a3);
            }
            w0 = w1;
        }
    }
}

// Convergence after sweep k, one wavefront per instance still running: lane l
// reads sub-slot l; converged when max|rho^{k+1} - rho^k| <= si_tol max|rho^{k+1}|
// and max|T^{k+1} - T^k| <= si_tol max T^{k+1} (Algorithm 2's stopping test).
__global__ void k_si_decide(Dev D, Consts K, int k)
{
    if (!gate_open(D, K, 0)) return;
    const int inst = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (inst >= K.n_inst || D.ist[inst].conv_sweeps != 0) return;
    const bool conv = si_converged(D, K, inst, k, lane);
    if (conv) {
        // the instance's wavefronts stop running in the following sweeps
        for (int64_t w = D.inst_cg[inst] / WAVE + lane; w < D.inst_cg[inst + 1] / WAVE; w += WAVE) D.wave_run[w] = 0;
        if (lane == 0) {
            D.ist[inst].conv_sweeps = k + 1;
            atomicAdd((unsigned long long*)(D.counters + CNT_CONV), 1ull);
        }
    }
}

// ---------------------------------------------------------------------------
// commit and diagnostics

// Energy bookkeeping of the step per instance: diag[inst*8 + q],
// q = 0 inflow_wave (written by k_wave_source), 1 inflow_eq, 2 exit, 3 injection,
// 4 e_start, 5 e_end.  Uses the final source-iteration input phi^k; the
// commit also keeps the last sweep's phi(T^{n+1}) in phi0 for the next step.  Sums are
// reduced per wavefront and per run of same-instance wavefronts of the block
// before one atomic per quantity.
constexpr int DIAG_THREADS = 256;

// last_sweep >= 0 (single instance): the convergence decision of that sweep
// is taken here rather than by a decide launch; wavefront 0 of every block
// takes it from the same residual sub-slots, and block 0 records it.
// Occupancy floor of the commit, whose loads are all issued before its first
// wait: 8 wavefronts per SIMD for batches (at 64 VGPRs, with some spilling: 3%
// off a step of 512 slabs), 6 in 2-D; single 1-D instances, whose commits are
// small and latency bound, are left to the compiler.
template <bool SINGLE, int DIM>
constexpr int finish_min_waves() { return DIM == 2 ? 6 : (SINGLE ? 1 : 8); }

template <bool SINGLE, int DIM>
__global__ __launch_bounds__(DIAG_THREADS) __attribute__((amdgpu_waves_per_eu(finish_min_waves<SINGLE, DIM>())))
void k_finish(Dev D, Consts K, int last_sweep, int push_blocks)
{
    const int64_t j = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x;
    // the loads come first (nothing is stored before the gate): step count,
    // the stopping state of the last sweep (one instance), the slot's data
    const uint32_t now = *D.step;
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    const int cs0 = last_sweep >= 0 ? D.ist[0].conv_sweeps : 0;
    Resid rl = {0ull, 0ull, 0ull, 0ull};
    if (last_sweep >= 0 && threadIdx.x < WAVE) rl = res_slot(D, K, 0, last_sweep)[threadIdx.x];
    const int cs_inst = D.ist[s.inst].conv_sweeps;
    const bool in = j < K.n_cg;
    const int g = s.g, nx = I.nx;
    const int ix = DIM == 1 ? s.lcell : s.lcell % nx, iy = DIM == 1 ? 0 : s.lcell / nx;
    const int cell = I.cell_off + s.lcell;
    double surv = 0.0, rho = 0.0, rho_new = 0.0, phi = 0.0, phi_next = 0.0, cv = 0.0, T0 = 0.0, T1 = 0.0;
    double olH = 0.0, olchi = 0.0, uend = 0.0, qs = 0.0;
    int src = 0;
    uint8_t pin = 0;
    bool bnd[4] = {false, false, false, false};
    int64_t fs[4] = {0, 0, 0, 0};
    double Df[4] = {0.0, 0.0, 0.0, 0.0}, tal[4] = {0.0, 0.0, 0.0, 0.0}, pb[4] = {0.0, 0.0, 0.0, 0.0};
    double tal_in[4] = {0.0, 0.0, 0.0, 0.0};
    const bool witer = (K.flags & UGKWP_FLAG_WAVE_ITER) != 0;
    if (in && s.active) {
        surv = D.surv[j];
        rho = D.rho[j];
        if (!witer) rho_new = D.rho_new[j];
        pin = D.pinned[cell];
        if (g == 0) {
            cv = D.cvol[cell];
            T0 = D.T[cell];
            T1 = D.T_new[cell];
            if (K.olson) {
                olH = D.olH[cell];
                olchi = D.olchi[cell];
                if (olH > 0.0) uend = D.uend[cell];
            }
        }
        if (K.has_src) {
            src = *D.src_on;
            qs = D.qsrc[j];
        }
        const double* phib = D.phib + (int64_t)s.inst * 4 * MAX_G;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) {
            const int axis = q >> 1;
            const bool lo = (q & 1) == 0;
            bnd[q] = axis == 0 ? (lo ? ix == 0 : ix == nx - 1) : (lo ? iy == 0 : iy == I.ny - 1);
            if (!bnd[q]) continue;
            fs[q] = axis == 0 ? I.fx_off + (((int64_t)iy * (nx + 1) + ix + (lo ? 0 : 1)) << I.lgGp) + g
                              : I.fy_off + (((int64_t)(iy + (lo ? 0 : 1)) * nx + ix) << I.lgGp) + g;
            Df[q] = axis == 0 ? D.Dx[fs[q]] : D.Dy[fs[q]];
            tal[q] = (axis == 0 ? D.ftx : D.fty)[fs[q] * 2 + (lo ? 1 : 0)];
            tal_in[q] = (axis == 0 ? D.ftx : D.fty)[fs[q] * 2 + (lo ? 0 : 1)];
            if (I.bc[q] == BC_PLANCK) pb[q] = phib[q * MAX_G + g];
        }
    }
    // the commit below advances *D.step while other blocks may still start:
    // both the step's own value and the next one open this launch
    if (!(K.gate == GATE_OFF || now == K.gate || now == K.gate + 1)) return;
    // the sweeps the iteration took: a converged single instance has it in its
    // state, or converged at the last sweep (decided below); batches have it
    // per instance
    const int ns_guess = last_sweep >= 0 ? (cs0 != 0 ? cs0 : last_sweep + 1) : cs_inst;
    double winf = 0.0;
    if (in && s.active && ns_guess >= 1) {
        phi = sweep_in(D, ns_guess - 1)[j];          // phi^k of the last sweep
        phi_next = sweep_out(D, ns_guess - 1)[j];    // phi(T^{n+1}): the next step's phi^0
        if (witer) {
            // the last sweep's output and the boundary wave inflow of its wave flux
            rho_new = ((ns_guess & 1) ? D.rho_new : D.rho_alt)[j];
            winf = D.winflow[(int64_t)((ns_guess - 1) & 1) * K.n_cg + j];
        }
    }
    int ns_single = 0;
    if (last_sweep >= 0) {
        __shared__ int sh_ns;
        if (threadIdx.x < WAVE) {
            // a block starting after block 0's record reads that record: the same value
            int ns = cs0;
            if (ns == 0) {
                const double drho = bitsd(wave_max_bits(bitsd(rl.drho))), mrho = bitsd(wave_max_bits(bitsd(rl.rho)));
                const double dTm = bitsd(wave_max_bits(bitsd(rl.dT))), mTm = bitsd(wave_max_bits(bitsd(rl.T)));
                if (drho <= K.si_tol * mrho && dTm <= K.si_tol * mTm) ns = last_sweep + 1;
            }
            if (threadIdx.x == 0) sh_ns = ns;
        }
        __syncthreads();
        ns_single = sh_ns;
        if (blockIdx.x == 0 && threadIdx.x == 0 && ns_single != 0 && cs0 == 0) {
            D.ist[0].conv_sweeps = ns_single;
            atomicAdd((unsigned long long*)(D.counters + CNT_CONV), 1ull);
        }
        if (D.counters[CNT_ERR] != 0 || ns_single == 0) return;
    } else if (!step_committed(D, K)) {
        return;
    }
    if (blockIdx.x == 0) {
        // survivors of the push: sum of its per-block counts
        __shared__ unsigned long long part[DIAG_THREADS / WAVE];
        unsigned long long t = 0;
        for (int b = threadIdx.x; b < push_blocks; b += DIAG_THREADS) t += D.blk_surv[b];
        for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, WAVE);
        if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long sum = 0;
            for (int q = 0; q < DIAG_THREADS / WAVE; ++q) sum += part[q];
            D.counters[CNT_SURV] = sum;
        }
    }
    // commit: survivor density for the next step, birth counters, pool size
    if (in) {
        D.rhop[j] = s.active ? surv / I.V : 0.0;
        if (j == I.cg_off) {
            const int64_t end = s.inst + 1 < K.n_inst ? D.boff[D.inst_cg[s.inst + 1]] : D.n_births_total[0];
            D.ist[s.inst].births += (uint64_t)(end - D.boff[I.cg_off]);
        }
        if (j == 0) {
            D.counters[CNT_SLOTS] = D.counters[CNT_PUSHED];
            D.counters[CNT_LIVE] = D.counters[CNT_SURV];
            const uint32_t n1 = *D.step + 1u;
            *D.step = n1;
            D.counters[CNT_DONE] = n1;
        }
    }
    // the commit's rho^{n+1} lives in rho_new
    if (witer && in && s.active && !(ns_guess & 1)) D.rho_new[j] = rho_new;
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // inflow_eq, exit/c, injection, e0, e1,
                                                         // inflow_wave (WAVE_ITER), inflow_particles
    if (in && s.active && (K.t_power != 0.0 || K.stim || K.table) && (bnd[0] || bnd[1] || bnd[2] || bnd[3])) {
        // temperature-dependent opacity: the boundary faces' coefficients at the
        // step's final temperature (the iteration has converged on it)
        const double Tf = D.T_new[cell];
        const double sk = K.table ? table_group_sigma(D, K, D.tab_mat[cell], I.edge_off + g, Tf)
                                  : D.kappa[j] * pow(Tf, -K.t_power) * group_factor(D, K, I.edge_off, g, Tf);
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q)
            if (bnd[q]) Df[q] = face_coef(K, sk, (q >> 1) == 0 ? I.dx : I.dy);
    }
    if (in && s.active) {
        D.phi0[j] = phi_next;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) {
            if (!bnd[q]) continue;
            const double S = (q >> 1) == 0 ? I.dy : I.dx;
            const int bc = I.bc[q];
            const double pn = bc == BC_PLANCK ? pb[q] : (bc == BC_REFLECT ? phi : 0.0);
            v[0] += K.dt * S * Df[q] * (pn - phi) / K.c;
            v[1] += tal[q] / K.c;
            v[6] += tal_in[q] / K.c;
        }
        v[5] = winf;
        if (pin) v[2] = I.V * (K.dt * D.sig[j] / (K.eps * K.eps)) * (phi - rho_new);
        if (src) v[2] += I.V * K.dt * qs / K.c;
        v[3] = I.V * rho / K.c;
        v[4] = I.V * rho_new / K.c;
        if (g == 0 && olH > 0.0) {
            // Olson's material energy, and the one the last sweep gave
            v[3] += I.V * olson_energy(olH, olchi, T0);
            v[4] += I.V * uend;
        } else if (g == 0) {
            v[3] += I.V * cv * T0;
            v[4] += I.V * cv * T1;
        }
    }
    // the diag entry of each sum: inflow_eq 1, exit 2, injection 3, e_start 4,
    // e_end 5, inflow_wave 0, inflow_particles 6
    constexpr int NV = 7;
    const int dst[NV] = {1, 2, 3, 4, 5, 0, 6};
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    __shared__ double wsum[DIAG_THREADS / WAVE][NV];
    __shared__ int winst[DIAG_THREADS / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    if (lane == 0) {
        for (int q = 0; q < NV; ++q) wsum[wid][q] = v[q];
        winst[wid] = j < K.n_cg ? s.inst : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = DIAG_THREADS / WAVE;
        int w0 = 0;
        while (w0 < nw) {
            int w1 = w0;
            double acc[NV] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            while (w1 < nw && winst[w1] == winst[w0]) {
                for (int q = 0; q < NV; ++q) acc[q] += wsum[w1][q];
                ++w1;
            }
            if (winst[w0] >= 0) {
                double* dg = D.diag_sub + ((int64_t)winst[w0] * DIAG_SUB + (blockIdx.x & (DIAG_SUB - 1))) * 8;
                for (int q = 0; q < NV; ++q)
                    if (acc[q] != 0.0) atomicAdd(dg + dst[q], acc[q]);
            }
            w0 = w1;
        }
    }
}

// Fold the energy-sum sub-slots into diag[inst][8].
__global__ void k_diag_reduce(Dev D, Consts K)
{
    if (!gate_open(D, K, 1)) return;
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= K.n_inst) return;
    for (int q = 0; q < 8; ++q) {
        double acc = 0.0;
        for (int b = 0; b < DIAG_SUB; ++b) acc += D.diag_sub[((int64_t)inst * DIAG_SUB + b) * 8 + q];
        D.diag[(int64_t)inst * 8 + q] = acc;
    }
}

__global__ void k_eval_phi(int n, const double* T, int G, const double* nu, double a, double c, double* out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)n * G) return;
    const int i = (int)(j / G), g = (int)(j % G);
    out[j] = phi_group_direct(T[i], nu[g], nu[g + 1], a, c);
}

__global__ void k_eval_coef(int n, const double* s, double* c4, double* w, double* c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    c4[j] = coef_c4(s[j]);
    w[j] = coef_w(s[j]);
    c2[j] = coef_c2_over_dt(s[j]);
}

__global__ void k_eval_uniform(int n, uint64_t seed, const uint64_t* id, uint32_t step, uint32_t purpose,
                               const uint32_t* d, double* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[j] = keyed_uniform(seed, id[j], step, purpose, d[j]);
}

__global__ void k_eval_neg_log(int n, const double* u, double* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[j] = neg_log_unit(u[j]);
}

__global__ void k_eval_sample_nu(int n, const double* nl, const double* nh, const double* T, const double* U,
                                 double* beta, double* nu)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double b = freq_slope(nl[j], nh[j], T[j]);
    beta[j] = b;
    nu[j] = sample_nu(nl[j], nh[j], b, U[j]);
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t set_head_series(const HeadSeries& hs)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_head), &hs, sizeof(HeadSeries));
}

void launch_tables(const Dev& D, const Consts& K, hipStream_t st)
{
    k_tables<<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K);
    if (K.table) k_tab_rows<<<blocks((int64_t)K.ncell * K.tab_nnu, 256), 256, 0, st>>>(D, K);
}

void launch_tab_logs(double* v, int64_t n, hipStream_t st)
{
    if (n > 0) k_tab_logs<<<blocks(n, 256), 256, 0, st>>>(v, n);
}

void launch_tab_groups(const Dev& D, const Consts& K, int64_t n_edges, hipStream_t st)
{
    if (n_edges > 1) k_tab_groups<<<blocks(n_edges, 256), 256, 0, st>>>(D, K, n_edges);
}

void launch_face_D(const Dev& D, const Consts& K, int inst, int axis, int64_t nslots, hipStream_t st)
{
    if (nslots > 0) k_face_D<<<blocks(nslots, 256), 256, 0, st>>>(D, K, inst, axis);
}

void launch_ghost_phi(const Dev& D, const Consts& K, double* phib, hipStream_t st)
{
    k_ghost_phi<<<K.n_inst, 4 * MAX_G, 0, st>>>(D, K, phib);
}

void launch_init_rho(const Dev& D, const Consts& K, const double* Tr0, hipStream_t st)
{
    k_init_rho<<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, Tr0);
}

void launch_source_planck(const Dev& D, const Consts& K, double* q, const double* f, double Ts, hipStream_t st)
{
    k_source_planck<<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, q, f, Ts);
}

// Tally clears, particle counts and their exclusive scan (births per slot ->
// first birth slot, total births): two launches while the per-block sums of
// the count fit one scan pass, four otherwise.
constexpr unsigned SMALL_SCAN_BLOCKS = 1024;

int64_t count_partials_size() { return SMALL_SCAN_BLOCKS; }

void launch_count_scan(const Dev& D, const Consts& K, const ZeroList& Z, int64_t* part, hipStream_t st)
{
    const unsigned nb = blocks(K.n_cg, COUNT_THREADS);
    const ScanGate q = scan_gate(D, K, 0);
    if (nb <= SMALL_SCAN_BLOCKS) {
        if (K.n_inst == 1) k_count<true><<<nb, COUNT_THREADS, 0, st>>>(D, K, Z, part);
        else k_count<false><<<nb, COUNT_THREADS, 0, st>>>(D, K, Z, part);
        k_scan_small<<<nb, COUNT_THREADS, 0, st>>>(q, D.nb, K.n_cg, part, (int)nb, D.boff, D.n_births_total);
    } else {
        if (K.n_inst == 1) k_count<true><<<nb, COUNT_THREADS, 0, st>>>(D, K, Z, nullptr);
        else k_count<false><<<nb, COUNT_THREADS, 0, st>>>(D, K, Z, nullptr);
        launch_scan(q, D.nb, K.n_cg, part, D.boff, D.n_births_total, st);
    }
}

int64_t scan_partials_size(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK; }

ScanGate scan_gate(const Dev& D, const Consts& K, uint32_t after)
{
    return ScanGate{D.step, K.gate == GATE_OFF ? GATE_OFF : K.gate + after};
}

void launch_scan(const ScanGate& q, const int32_t* in, int64_t n, int64_t* part, int64_t* out, int64_t* total,
                 hipStream_t st)
{
    const int64_t nb = scan_partials_size(n);
    k_scan_partials<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(q, in, n, part);
    k_scan_top<<<1, SCAN_THREADS, 0, st>>>(q, part, nb, total);
    k_scan_final<<<(unsigned)nb, SCAN_THREADS, 0, st>>>(q, in, n, part, out);
}

void launch_slopes(int dim, const Dev& D, const Consts& K, const double* src, bool sub_rhop, hipStream_t st)
{
    if (dim == 1) k_slopes<1><<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, src, sub_rhop ? 1 : 0);
    else k_slopes<2><<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, src, sub_rhop ? 1 : 0);
}

static int num_cus();

// The sampler runs as a grid of the blocks that fit at once (its wavefronts
// take 64 births per round; 512 blocks left the 2-D sampler at half occupancy).
template <int DIM>
static unsigned sample_blocks()
{
    static int per = 0;     // resident blocks per CU (a property of the kernel)
    if (per == 0) {
        int q = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_sample<DIM>, 256, 0) != hipSuccess || q < 1) q = 2;
        per = q;
    }
    return (unsigned)(per * num_cus());
}

void launch_sample(int dim, const Dev& D, const Consts& K, const Pool& P, hipStream_t st)
{
    if (dim == 1) k_sample<1><<<sample_blocks<1>(), 256, 0, st>>>(D, K, P);
    else k_sample<2><<<sample_blocks<2>(), 256, 0, st>>>(D, K, P);
}

// Push block sizes the launch shape may take (threads per block).
constexpr int PUSH_BS[2] = {256, 512};

static int push_bs_index(int threads)
{
    return threads == PUSH_BS[1] ? 1 : 0;
}

static int sig_mode(const Consts& K)
{
    if (K.flags & 1u) return SIG_GROUP;
    if (K.table) return SIG_TAB;
    if (K.stim) return SIG_STIM;
    return K.nu_power == 3.0 ? SIG_NU3 : SIG_POW;
}

template <int DIM, bool SINGLE, int SM, int BS>
static int push_occupancy()
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_push<DIM, SINGLE, SM, BS>, BS, 0) != hipSuccess)
        per = 0;
    return per;
}

template <int DIM, bool SINGLE, int SM>
static int push_occupancy_bs(int threads)
{
    if (threads == 512) return push_occupancy<DIM, SINGLE, SM, 512>();
    return push_occupancy<DIM, SINGLE, SM, 256>();
}

template <int DIM, bool SINGLE>
static int push_occupancy_sm(int sm, int threads)
{
    switch (sm) {
        case SIG_NU3: return push_occupancy_bs<DIM, SINGLE, SIG_NU3>(threads);
        case SIG_POW: return push_occupancy_bs<DIM, SINGLE, SIG_POW>(threads);
        case SIG_GROUP: return push_occupancy_bs<DIM, SINGLE, SIG_GROUP>(threads);
        case SIG_TAB: return push_occupancy_bs<DIM, SINGLE, SIG_TAB>(threads);
        default: return push_occupancy_bs<DIM, SINGLE, SIG_STIM>(threads);
    }
}

// Resident push blocks per CU of the given block size (cached per kernel).
static int g_push_occ[2][2][5][2] = {};

int push_blocks_per_cu(int dim, const Consts& K, int threads)
{
    const bool single = K.n_inst == 1;
    const int sm = sig_mode(K);
    int& per = g_push_occ[dim - 1][single ? 1 : 0][sm][push_bs_index(threads)];
    if (per == 0) {
        if (dim == 1) per = single ? push_occupancy_sm<1, true>(sm, threads) : push_occupancy_sm<1, false>(sm, threads);
        else per = single ? push_occupancy_sm<2, true>(sm, threads) : push_occupancy_sm<2, false>(sm, threads);
        if (per < 1) per = 2;
    }
    return per;
}

static int num_cus()
{
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu < 1 ? 256 : ncu;
}

template <int DIM, bool SINGLE, int SM>
static void push_bs(const PushShape& sh, const Dev& D, const Consts& K, const Pool& In, const Pool& Out,
                    hipStream_t st)
{
    if (sh.threads == 512) k_push<DIM, SINGLE, SM, 512><<<sh.blocks, 512, 0, st>>>(D, K, In, Out, sh.ppt);
    else k_push<DIM, SINGLE, SM, 256><<<sh.blocks, 256, 0, st>>>(D, K, In, Out, sh.ppt);
}

template <int DIM, bool SINGLE>
static void push_mode(int sm, const PushShape& sh, const Dev& D, const Consts& K, const Pool& In, const Pool& Out,
                      hipStream_t st)
{
    if (sm == SIG_NU3) push_bs<DIM, SINGLE, SIG_NU3>(sh, D, K, In, Out, st);
    else if (sm == SIG_POW) push_bs<DIM, SINGLE, SIG_POW>(sh, D, K, In, Out, st);
    else if (sm == SIG_GROUP) push_bs<DIM, SINGLE, SIG_GROUP>(sh, D, K, In, Out, st);
    else if (sm == SIG_TAB) push_bs<DIM, SINGLE, SIG_TAB>(sh, D, K, In, Out, st);
    else push_bs<DIM, SINGLE, SIG_STIM>(sh, D, K, In, Out, st);
}

PushShape push_default_shape(int dim, const Consts& K)
{
    PushShape p;
    p.threads = PUSH_THREADS;
    p.blocks = num_cus() * push_blocks_per_cu(dim, K, PUSH_THREADS);
    p.ppt = PUSH_PPT_DEFAULT;
    return p;
}

int push_num_cus() { return num_cus(); }

void launch_push(int dim, const Dev& D, const Consts& K, const Pool& In, const Pool& Out, const PushShape& sh,
                 hipStream_t st)
{
    const bool single = K.n_inst == 1;
    const int sm = sig_mode(K);
    if (dim == 1) {
        if (single) push_mode<1, true>(sm, sh, D, K, In, Out, st);
        else push_mode<1, false>(sm, sh, D, K, In, Out, st);
    } else {
        if (single) push_mode<2, true>(sm, sh, D, K, In, Out, st);
        else push_mode<2, false>(sm, sh, D, K, In, Out, st);
    }
}

// The scatter runs as a persistent grid of the blocks that fit at once (a
// second round of blocks measured about 3% slower on the 2-D lattice).
template <int DIM, bool SINGLE>
static unsigned sort_blocks()
{
    static int per = 0;     // resident blocks per CU (a property of the kernel)
    if (per == 0) {
        int q = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_sort_scatter<DIM, SINGLE>, SORT_THREADS, 0) !=
                hipSuccess || q < 1)
            q = 4;
        per = q;
    }
    return (unsigned)(per * num_cus());
}

void launch_sort_scatter(int dim, const Dev& D, const Consts& K, const Pool& In, const Pool& Out, hipStream_t st)
{
    const bool single = K.n_inst == 1;
    const unsigned nb = dim == 1 ? (single ? sort_blocks<1, true>() : sort_blocks<1, false>())
                                 : (single ? sort_blocks<2, true>() : sort_blocks<2, false>());
    if (dim == 1) {
        if (single) k_sort_scatter<1, true><<<nb, SORT_THREADS, 0, st>>>(D, K, In, Out);
        else k_sort_scatter<1, false><<<nb, SORT_THREADS, 0, st>>>(D, K, In, Out);
    } else {
        if (single) k_sort_scatter<2, true><<<nb, SORT_THREADS, 0, st>>>(D, K, In, Out);
        else k_sort_scatter<2, false><<<nb, SORT_THREADS, 0, st>>>(D, K, In, Out);
    }
}

template <bool TDEP, bool LIN, bool EXT>
static auto sweep_kernel_ext(const Consts& K, bool fold, int k)
{
    return K.inst0.dim == 1
               ? (fold ? (k == 0 ? k_si_sweep<true, true, 1, TDEP, LIN, EXT> : k_si_sweep<false, true, 1, TDEP, LIN, false>)
                       : (k == 0 ? k_si_sweep<true, false, 1, TDEP, LIN, EXT> : k_si_sweep<false, false, 1, TDEP, LIN, false>))
               : (fold ? (k == 0 ? k_si_sweep<true, true, 2, TDEP, LIN, EXT> : k_si_sweep<false, true, 2, TDEP, LIN, false>)
                       : (k == 0 ? k_si_sweep<true, false, 2, TDEP, LIN, EXT> : k_si_sweep<false, false, 2, TDEP, LIN, false>));
}

// the first sweep evaluates the wave flux: with slope terms or boundary-source
// ghosts, its extended instantiation
template <bool TDEP, bool LIN>
static auto sweep_kernel(const Consts& K, bool fold, int k)
{
    return (K.flags & (UGKWP_FLAG_SLOPES | UGKWP_FLAG_BOUNDARY_PARTICLES)) ? sweep_kernel_ext<TDEP, LIN, true>(K, fold, k)
                                                                           : sweep_kernel_ext<TDEP, LIN, false>(K, fold, k);
}

// rho^m of the source iteration: rho^n for m = 0; from the wave flux of each
// sweep's iterate on (UGKWP_FLAG_WAVE_ITER), whose sweeps read their
// neighbours' rho^k, rho^m alternates between rho_new (m odd) and rho_alt
// (m even); otherwise every sweep keeps its iterate in rho_new.
const double* sweep_rho(const Dev& D, const Consts& K, int m)
{
    if (m == 0) return D.rho;
    if (!(K.flags & UGKWP_FLAG_WAVE_ITER)) return D.rho_new;
    return (m & 1) ? D.rho_new : D.rho_alt;
}

void launch_si_sweeps(const Dev& D, const Consts& K, int k0, int k1, hipStream_t st)
{
    const bool fold = K.n_inst == 1;
    const bool witer = (K.flags & UGKWP_FLAG_WAVE_ITER) != 0;
    const int dim = K.inst0.dim;
    for (int k = k0; k < k1; ++k) {
        if (witer && k > 0) {
            // the wave flux of this sweep from its iterate: slopes, then Q
            if (K.flags & UGKWP_FLAG_SLOPES) launch_slopes(dim, D, K, sweep_rho(D, K, k), true, st);
            if (dim == 1) k_wave_q<1><<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, k, sweep_rho(D, K, k));
            else k_wave_q<2><<<blocks(K.n_cg, 256), 256, 0, st>>>(D, K, k, sweep_rho(D, K, k));
        }
        // every instance of a context has the same dimension
        const bool lin = (K.flags & UGKWP_FLAG_SI_LINEARIZED) != 0;
        // a temperature-dependent or tabulated opacity and Olson's heat capacity take
        // the sweeps that re-evaluate the material from the iterate
        auto kern = (K.t_power != 0.0 || K.stim || K.table || K.olson) ? (lin ? sweep_kernel<true, true>(K, fold, k) : sweep_kernel<true, false>(K, fold, k))
                                     : (lin ? sweep_kernel<false, true>(K, fold, k) : sweep_kernel<false, false>(K, fold, k));
        kern<<<blocks(K.n_cg, SI_THREADS), SI_THREADS, 0, st>>>(D, K, k, sweep_in(D, k), sweep_out(D, k),
                                                                    fold && k > k0 ? 1 : 0, sweep_rho(D, K, k),
                                                                    const_cast<double*>(sweep_rho(D, K, k + 1)));
        if (!fold) k_si_decide<<<blocks((int64_t)K.n_inst * WAVE, 256), 256, 0, st>>>(D, K, k);
    }
}

void launch_finish(const Dev& D, const Consts& K, bool reduce_diag, int last_sweep, int push_blocks, hipStream_t st)
{
    auto fin = K.inst0.dim == 1 ? (K.n_inst == 1 ? k_finish<true, 1> : k_finish<false, 1>)
                                    : (K.n_inst == 1 ? k_finish<true, 2> : k_finish<false, 2>);
    fin<<<blocks(K.n_cg, DIAG_THREADS), DIAG_THREADS, 0, st>>>(D, K, K.n_inst == 1 ? last_sweep : -1,
                                                                   push_blocks);
    if (reduce_diag) k_diag_reduce<<<blocks(K.n_inst, 64), 64, 0, st>>>(D, K);
}

void launch_eval_phi(int n, const double* T, int G, const double* nu, double a, double c, double* out,
                     hipStream_t st)
{
    k_eval_phi<<<blocks((int64_t)n * G, 256), 256, 0, st>>>(n, T, G, nu, a, c, out);
}

void launch_eval_coef(int n, const double* s, double* c4, double* w, double* c2, hipStream_t st)
{
    k_eval_coef<<<blocks(n, 256), 256, 0, st>>>(n, s, c4, w, c2);
}

void launch_eval_uniform(int n, uint64_t seed, const uint64_t* id, uint32_t step, uint32_t purpose,
                         const uint32_t* d, double* out, hipStream_t st)
{
    k_eval_uniform<<<blocks(n, 256), 256, 0, st>>>(n, seed, id, step, purpose, d, out);
}

void launch_eval_neg_log(int n, const double* u, double* out, hipStream_t st)
{
    k_eval_neg_log<<<blocks(n, 256), 256, 0, st>>>(n, u, out);
}

void launch_eval_sample_nu(int n, const double* nl, const double* nh, const double* T, const double* U,
                           double* beta, double* nu, hipStream_t st)
{
    k_eval_sample_nu<<<blocks(n, 256), 256, 0, st>>>(n, nl, nh, T, U, beta, nu);
}

}  // namespace ugk
