// HIP kernels (gfx950) of the recording and the reverse sweep of the adjoint
// of the frozen-tally macroscopic map; see adjoint.hpp for what is stored and
// differentiated.  Same (cell, group) slot layout and wavefront-per-cell
// structure as the forward source iteration (kernels.hip): the Gp group lanes
// of a cell sit in one wavefront, group sums are shuffles, Planck edge values
// are shared by neighbouring lanes.
#include "adjoint.hpp"
#include "device_common.hpp"

namespace ugk {

__constant__ HeadSeries c_head_adj;

hipError_t set_head_series_adj(const HeadSeries& hs)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_head_adj), &hs, sizeof(HeadSeries));
}

constexpr int ADJ_THREADS = 256;

// Heat-capacity weight dt / (eps^2 C_v) of the temperature update; 0 in pinned cells.
__device__ inline double temp_weight(const Dev& D, const Consts& K, int cell)
{
    return D.pinned[cell] ? 0.0 : D.dtcv[cell];
}

__device__ inline bool adj_gate(const Adj& A, uint32_t gate)
{
    return gate == GATE_OFF || A.status[ADJ_DONE] == (unsigned long long)gate;
}

// Convergence of instance inst after sweep k, one wavefront (lane l reads
// sub-slot l): relative max-norm change of mu at most 1e-15, 1e-13 from the
// 61st sweep on.
__device__ inline bool adj_converged(const Adj& A, int inst, int k, int lane)
{
    const AdjResid r = A.res[((int64_t)inst * RES_SLOTS + k % RES_SLOTS) * RES_SUB + lane];
    const double dm = bitsd(wave_max_bits(bitsd(r.dmu))), mm = bitsd(wave_max_bits(bitsd(r.mu)));
    const double tol = k >= 60 ? 1e-13 : 1e-15;
    return dm <= tol * mm;
}

// Record instance inst converged after ns sweeps of reverse step r.
__device__ inline void adj_mark_converged(const Dev& D, const Adj& A, int inst, int ns, int r)
{
    const Inst& I = D.inst[inst];
    A.conv[inst] = ns;
    atomicAdd(A.status + ADJ_CONV, 1ull);
    atomicAdd(A.status + ADJ_CGU, (unsigned long long)ns * (unsigned long long)(I.ncell * I.G));
    atomicMax(A.status + ADJ_MAXK, (unsigned long long)ns);
    atomicMax(A.stepk + r, ns);
}

// ---------------------------------------------------------------------------
// recording, launched behind the step's commit with the step's own buffers:
// D.T_new holds T^{n+1}

__global__ void k_rec_store(Dev D, Consts K, Adj A, int r)
{
    if (!gate_open(D, K, 1)) return;
    const int64_t j = (int64_t)blockIdx.x * ADJ_THREADS + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    const int64_t o = (int64_t)r * K.n_cg + j;
    A.rQ[o] = D.Q[j];
    A.rRhoh[o] = D.rhoh[j];
    A.rSamp[o] = D.nb[j] > 0 ? 1 : 0;
    if (s.cell_ok && s.g == 0) {
        const int cell = D.inst[s.inst].cell_off + s.lcell;
        A.rT[(int64_t)r * K.ncell + cell] = D.T_new[cell];
    }
}

// ---------------------------------------------------------------------------
// kappa-dependent coefficients of the reverse sweep (once per adjoint)

__global__ void k_adj_coef(Dev D, Consts K, Adj A)
{
    const int64_t j = (int64_t)blockIdx.x * ADJ_THREADS + threadIdx.x;
    if (j >= K.n_cg) return;
    const Slot s = decode_slot(D, K, j);
    const double sv = D.sv[j];
    A.c4d[j] = s.active ? coef_c4_ds(sv) : 0.0;
    A.wd[j] = s.active ? coef_w_ds(sv) : 0.0;
}

// dD_f/dsigma of the cells on either side of each face: D_f = -(c^2/3eps^2) C2(s_f)/h
// with s_f = c sf dt/eps^2 and sf the harmonic mean of the two cells' sigma (the
// interior cell's sigma on a domain face).
__global__ void k_adj_face(Dev D, Consts K, Adj A, int inst, int axis)
{
    const Inst& I = D.inst[inst];
    const int64_t nface = axis == 0 ? (int64_t)(I.nx + 1) * I.ny : (int64_t)I.nx * (I.ny + 1);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nface * I.Gp) return;
    const int64_t f = j >> I.lgGp;
    const int g = (int)(j & (I.Gp - 1));
    double* Dl = axis == 0 ? A.Dlx + I.fx_off : A.Dly + I.fy_off;
    double* Dh = axis == 0 ? A.Dhx + I.fx_off : A.Dhy + I.fy_off;
    if (g >= I.G) { Dl[j] = 0.0; Dh[j] = 0.0; return; }
    int cl, cr;
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
    double sf, dl = 0.0, dr = 0.0;
    if (cl >= 0 && cr >= 0) {
        const double a = D.sig[I.cg_off + ((int64_t)cl << I.lgGp) + g];
        const double b = D.sig[I.cg_off + ((int64_t)cr << I.lgGp) + g];
        const double ab = a + b;
        sf = ab > 0.0 ? 2.0 * (a * b) / ab : 0.0;
        if (ab > 0.0) {
            dl = 2.0 * (b * b) / (ab * ab);
            dr = 2.0 * (a * a) / (ab * ab);
        }
    } else {
        sf = D.sig[I.cg_off + ((int64_t)(cl >= 0 ? cl : cr) << I.lgGp) + g];
        if (cl >= 0) dl = 1.0; else dr = 1.0;
    }
    const double ks = K.c * K.dt / (K.eps * K.eps);
    const double dDdsf = -(K.c * K.c / (3.0 * K.eps * K.eps)) * K.dt * ks * coef_c2_over_dt_ds(ks * sf) / h;
    Dl[j] = dDdsf * dl;
    Dh[j] = dDdsf * dr;
}

// ---------------------------------------------------------------------------
// per recorded step, in reverse

// phi and phi' at T^{n+1}; mu^0 = Tbar; convergence state of the step reset.
template <bool SINGLE>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_prep(Dev D, Consts K, Adj A, int r, uint32_t gate)
{
    const int64_t j = (int64_t)blockIdx.x * ADJ_THREADS + threadIdx.x;
    // the loads first (nothing is stored before the gate)
    const unsigned long long done = A.status[ADJ_DONE];
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    const int g = s.g, G = I.G, Gp = I.Gp;
    const bool work = s.cell_ok;
    const int cell = I.cell_off + s.lcell;
    const double T = work ? A.rT[(int64_t)r * K.ncell + cell] : 1.0;
    const bool edge_lane = work && g <= G;
    const double nu_lo = edge_lane ? D.nu[I.edge_off + g] : 0.0;
    const double nu_top = work && g == G - 1 && G == Gp ? D.nu[I.edge_off + G] : 0.0;
    const double tbar = work && g == 0 ? A.Tbar[cell] : 0.0;
    if (!(gate == GATE_OFF || done == (unsigned long long)gate)) return;
    if (j == 0) {
        A.status[ADJ_CONV] = 0;
        A.stepk[r] = 0;
    }
    // lane g: lower edge of group g; the upper edge comes from lane g+1
    const double xe = edge_lane ? nu_lo / T : 0.0;
    const double ve = edge_lane ? planck_edge_value(xe, c_head_adj) : 0.0;
    const double we = edge_lane ? planck_edge_weight(xe) : 0.0;
    double xh = __shfl_down(xe, 1, Gp < 2 ? 2 : Gp);
    double vh = __shfl_down(ve, 1, Gp < 2 ? 2 : Gp);
    double wh = __shfl_down(we, 1, Gp < 2 ? 2 : Gp);
    if (work && g == G - 1 && G == Gp) {
        xh = nu_top / T;
        vh = planck_edge_value(xh, c_head_adj);
        wh = planck_edge_weight(xh);
    }
    if (j < K.n_cg) {
        if (s.active) {
            const double phi = phi_from_band(K.a, K.c, T, planck_band_from_edges(xe, ve, xh, vh));
            const double T3 = T * T * T;
            A.phi[j] = phi;
            A.dphi[j] = 4.0 * phi / T + K.a * K.c * T3 * (we - wh) / UGK_PI4_15;
        } else {
            A.phi[j] = 0.0;
            A.dphi[j] = 0.0;
        }
        if (work && g == 0) A.mu0[cell] = tbar;
        const int64_t rel = j - I.cg_off;
        if (rel >= 0 && rel < RES_SUB) {
            AdjResid z = {0ull, 0ull};
            A.res[((int64_t)s.inst * RES_SLOTS + 0) * RES_SUB + rel] = z;
        }
        if (rel == 0) A.conv[s.inst] = 0;
    }
}

// bbar = w sigma/(1+lambda) mu + rbar/(1+lambda) of slot jj in cell c
__device__ inline double bbar_of(const Dev& D, const Consts& K, const Adj& A, const double* mu, int64_t jj,
                                 int c)
{
    const double sg = D.sig[jj];
    const double lam = s_of_sigma(K, sg);
    return temp_weight(D, K, c) * sg / (1.0 + lam) * mu[c] + A.rbar[jj] / (1.0 + lam);
}

// Face q (XLO, XHI, YLO, YHI) of slot j: neighbour slot and cell, face slot, area.
struct FaceRef {
    bool inside;
    int64_t nbj, fslot;
    int nbcell;
    double S;
};

template <int DIM>
__device__ inline FaceRef face_ref(const Inst& I, int64_t j, int lcell, int g, int q)
{
    FaceRef f;
    const int nx = I.nx, ix = DIM == 1 ? lcell : lcell % nx, iy = DIM == 1 ? 0 : lcell / nx, Gp = I.Gp;
    const bool lo = (q & 1) == 0;
    if ((q >> 1) == 0) {
        f.inside = lo ? ix > 0 : ix < nx - 1;
        f.nbj = j + (lo ? -Gp : Gp);
        f.nbcell = I.cell_off + lcell + (lo ? -1 : 1);
        f.fslot = I.fx_off + (((int64_t)iy * (nx + 1) + ix + (lo ? 0 : 1)) << I.lgGp) + g;
        f.S = I.dy;
    } else {
        f.inside = lo ? iy > 0 : iy < I.ny - 1;
        f.nbj = j + (lo ? -(int64_t)nx * Gp : (int64_t)nx * Gp);
        f.nbcell = I.cell_off + lcell + (lo ? -nx : nx);
        f.fslot = I.fy_off + (((int64_t)(iy + (lo ? 0 : 1)) * nx + ix) << I.lgGp) + g;
        f.S = I.dx;
    }
    return f;
}

// One sweep of the transposed source iteration, preconditioned by its local
// diagonal d = w sum_g sigma phi_g'/(1+lambda) (the transpose of the linearized
// forward sweep; the plain iteration diverges where d > 1, stiff coupling):
//   m        = Tbar + sum_g phi_g' [ -w sigma/(1+lambda) mu^k + lambda/(1+lambda) rbar
//                                    + (dt/V) sum_f S_f D_f (bbar_nb - bbar) ]
//   mu^{k+1} = mu^k + (m - mu^k) / (1 + d).
// Residual maxima go to 64 sub-slots of the instance; k_adj_decide reads them.
// With decide_prev (single instance), every block first takes the decision of
// sweep k-1 from those sub-slots itself; block 0 records it.
template <bool SINGLE, int DIM>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_sweep(Dev D, Consts K, Adj A, int k, const double* mu_in,
                                                           double* mu_out, int r, uint32_t gate, int decide_prev)
{
    const int64_t j = (int64_t)blockIdx.x * ADJ_THREADS + threadIdx.x;
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    // the gate (done count) and, for one instance, the state and residuals of
    // the sweep before (the stopping test) are requested together; the slot's
    // data once the block is known to run
    const unsigned long long done = A.status[ADJ_DONE];
    const int cs_prev = decide_prev ? A.conv[0] : 0;
    AdjResid res_prev = {0ull, 0ull};
    if (decide_prev && wid == 0) res_prev = A.res[((int64_t)0 * RES_SLOTS + (k - 1) % RES_SLOTS) * RES_SUB + lane];
    if (!(gate == GATE_OFF || done == (unsigned long long)gate)) return;
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    if (decide_prev) {
        // the whole block stops when the iteration has converged (now or before)
        __shared__ int stop;
        if (wid == 0) {
            bool conv = false;
            if (cs_prev == 0) {
                const double dm = bitsd(wave_max_bits(bitsd(res_prev.dmu)));
                const double mm = bitsd(wave_max_bits(bitsd(res_prev.mu)));
                conv = dm <= ((k - 1) >= 60 ? 1e-13 : 1e-15) * mm;
            }
            if (lane == 0) {
                stop = (conv || cs_prev != 0) ? 1 : 0;
                if (conv && blockIdx.x == 0) adj_mark_converged(D, A, 0, k, r);
            }
        }
        __syncthreads();
        if (stop) return;
    }
    const int cs_inst = A.conv[s.inst];

    const int g = s.g, Gp = I.Gp;
    const int cell = I.cell_off + s.lcell;
    constexpr int nf = 2 * DIM;
    // every load of the sweep before the first wait
    const bool act = s.cell_ok && s.active;
    double lam = 0.0, mui = 0.0, tw = 0.0, sg = 0.0, rb = 0.0, dphi = 0.0, tbar = 0.0;
    FaceRef fr[4];
    double Df[4], nlam[4], ntw[4], nsig[4], nmu[4], nrb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < nf) fr[q] = face_ref<DIM>(I, j, s.lcell, g, q);
        Df[q] = nlam[q] = ntw[q] = nsig[q] = nmu[q] = nrb[q] = 0.0;
    }
    if (act) {
        mui = mu_in[cell];
        tw = temp_weight(D, K, cell);
        sg = D.sig[j];
        lam = s_of_sigma(K, sg);
        rb = A.rbar[j];
        dphi = A.dphi[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nf) continue;
            Df[q] = (q >> 1) == 0 ? D.Dx[fr[q].fslot] : D.Dy[fr[q].fslot];
            if (fr[q].inside) {
                ntw[q] = temp_weight(D, K, fr[q].nbcell);
                nsig[q] = D.sig[fr[q].nbj];
                nlam[q] = s_of_sigma(K, nsig[q]);
                nmu[q] = mu_in[fr[q].nbcell];
                nrb[q] = A.rbar[fr[q].nbj];
            }
        }
    }
    if (s.cell_ok && g == 0) {
        tbar = A.Tbar[cell];
        if (!act) mui = mu_in[cell];
    }

    const bool run = cs_inst == 0 && j < K.n_cg;
    const bool work = run && s.cell_ok;

    const int64_t rel = j - I.cg_off;
    if (run && rel >= 0 && rel < RES_SUB) {
        AdjResid z = {0ull, 0ull};
        A.res[((int64_t)s.inst * RES_SLOTS + (k + 1) % RES_SLOTS) * RES_SUB + rel] = z;
    }

    double contrib = 0.0, diag = 0.0;
    if (work && s.active) {
        const double fac = tw * sg / (1.0 + lam);
        diag = fac * dphi;
        const double bb = fac * mui + rb / (1.0 + lam);
        double lt = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= nf) continue;
            if (fr[q].inside) {
                const double bn = ntw[q] * nsig[q] / (1.0 + nlam[q]) * nmu[q] + nrb[q] / (1.0 + nlam[q]);
                lt += fr[q].S * Df[q] * (bn - bb);
            } else if (I.bc[q] != BC_REFLECT) {
                lt -= fr[q].S * Df[q] * bb;
            }
        }
        const double phibar = -fac * mui + lam / (1.0 + lam) * rb + I.dt_V * lt;
        contrib = dphi * phibar;
    }
    contrib = group_sum(contrib, Gp);
    diag = group_sum(diag, Gp);

    double dm = 0.0, mm = 0.0;
    if (work && g == 0) {
        const double mun = mui + (tbar + contrib - mui) / (1.0 + diag);
        if (!isfinite(mun)) atomicOr(A.status + ADJ_ERR, 1ull);
        mu_out[cell] = mun;
        dm = fabs(mun - mui);
        mm = fabs(mun);
    }
    // both maxima are non-negative (or NaN): reduced as bit patterns
    const unsigned long long bdm = wave_max_bits(dm), bmm = wave_max_bits(mm);
    __shared__ unsigned long long wres[ADJ_THREADS / WAVE][2];
    __shared__ int winst[ADJ_THREADS / WAVE];
    __shared__ int wrun[ADJ_THREADS / WAVE];
    if (lane == 0) {
        wres[wid][0] = bdm; wres[wid][1] = bmm;
        winst[wid] = s.inst;
        wrun[wid] = run ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = ADJ_THREADS / WAVE;
        int w0 = 0;
        while (w0 < nw) {
            int w1 = w0, any = 0;
            unsigned long long a0 = 0, a1 = 0;
            while (w1 < nw && winst[w1] == winst[w0]) {
                if (wrun[w1]) {
                    any = 1;
                    a0 = max(a0, wres[w1][0]);
                    a1 = max(a1, wres[w1][1]);
                }
                ++w1;
            }
            if (any) {
                AdjResid* rr = A.res + ((int64_t)winst[w0] * RES_SLOTS + k % RES_SLOTS) * RES_SUB +
                               (blockIdx.x & (RES_SUB - 1));
                atomicMax(&rr->dmu, a0);
                atomicMax(&rr->mu, a1);
            }
            w0 = w1;
        }
    }
}

// Convergence after sweep k, one wavefront per instance still running.
__global__ void k_adj_decide(Dev D, Consts K, Adj A, int k, int r, uint32_t gate)
{
    if (!adj_gate(A, gate)) return;
    const int inst = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (inst >= K.n_inst || A.conv[inst] != 0) return;
    if (adj_converged(A, inst, k, lane) && lane == 0) adj_mark_converged(D, A, inst, k + 1, r);
}

// With the converged mu: cotangents of lambda (= s), sigma, Q, A rho^h and D_f;
// dJ/dkappa += S_g dJ/dsigma; rbar^n = bbar + A ubar; Tbar^n = mu.
// last_sweep >= 0 (single instance): the convergence after that sweep is
// decided here (wavefront 0 of every block, the same answer; block 0 records
// it).  The step's cotangents are formed only when every instance converged
// and nothing non-finite was seen; block 0 then counts the step done.
template <bool SINGLE, int DIM>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_grad(Dev D, Consts K, Adj A, int r, uint32_t gate,
                                                          int last_sweep)
{
    const int64_t j = (int64_t)blockIdx.x * ADJ_THREADS + threadIdx.x;
    // every load that does not need the sweep count goes out before the first
    // wait (nothing is stored before the gate): the done count, the stopping
    // state of the last sweep (one instance), the slot's and its neighbours' data
    const unsigned long long done = A.status[ADJ_DONE];
    const int cs0 = last_sweep >= 0 ? A.conv[0] : 0;
    AdjResid rl = {0ull, 0ull};
    if (last_sweep >= 0 && threadIdx.x < WAVE)
        rl = A.res[((int64_t)0 * RES_SLOTS + last_sweep % RES_SLOTS) * RES_SUB + threadIdx.x];
    Inst I;
    const Slot s = decode_slot_rec<SINGLE>(D, K, j, I);
    const int cs_inst = A.conv[s.inst];
    const bool act = s.active;                    // implies j < n_cg
    const int g = s.g;
    const int cell = I.cell_off + s.lcell;
    const int64_t o = (int64_t)r * K.n_cg + j;
    constexpr int nf = 2 * DIM;
    double wi = 0.0, lam = 0.0, sig = 0.0, rb = 0.0, phik = 0.0, rQ = 0.0, rRhoh = 0.0, c4d = 0.0, Af = 0.0,
           dA = 0.0, simp = 0.0;
    uint8_t samp = 0;
    FaceRef fr[4];
    double Df[4], dDds[4], phin[4], ghost[4], nw[4], nsig[4], nlam[4], nrb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Df[q] = dDds[q] = phin[q] = ghost[q] = nw[q] = nsig[q] = nlam[q] = nrb[q] = 0.0;
        if (q < nf) fr[q] = face_ref<DIM>(I, j, s.lcell, g, q);
    }
    if (act) {
        wi = temp_weight(D, K, cell);
        sig = D.sig[j];
        lam = s_of_sigma(K, sig);
        rb = A.rbar[j];
        phik = A.phi[j];
        rQ = A.rQ[o];
        samp = A.rSamp[o];
        rRhoh = A.rRhoh[o];
        c4d = A.c4d[j];
        Af = samp ? D.wc[j] : D.c4[j];
        dA = samp ? A.wd[j] : c4d;
        simp = D.simpson[I.edge_off + g];
        const double* phib = D.phib + (int64_t)s.inst * 4 * MAX_G;
#pragma unroll
        for (int q = 0; q < nf; ++q) {
            const bool xax = (q >> 1) == 0, lo = (q & 1) == 0;
            const int64_t fs = fr[q].fslot;
            Df[q] = xax ? D.Dx[fs] : D.Dy[fs];
            // this cell is the high side of its low face and the low side of its high face
            dDds[q] = xax ? (lo ? A.Dhx[fs] : A.Dlx[fs]) : (lo ? A.Dhy[fs] : A.Dly[fs]);
            if (fr[q].inside) {
                phin[q] = A.phi[fr[q].nbj];
                nw[q] = temp_weight(D, K, fr[q].nbcell);
                nsig[q] = D.sig[fr[q].nbj];
                nlam[q] = s_of_sigma(K, nsig[q]);
                nrb[q] = A.rbar[fr[q].nbj];
            } else if (I.bc[q] == BC_PLANCK) {
                ghost[q] = phib[q * MAX_G + g];
            }
        }
    }
    // the done count below advances while other blocks may still start
    if (!(gate == GATE_OFF || done == (unsigned long long)gate || done == (unsigned long long)gate + 1)) return;
    int ns_single = 0;
    if (last_sweep >= 0) {
        __shared__ int sh_ns;
        if (threadIdx.x < WAVE) {
            int ns = cs0;
            if (ns == 0) {
                const double dm = bitsd(wave_max_bits(bitsd(rl.dmu))), mm = bitsd(wave_max_bits(bitsd(rl.mu)));
                if (dm <= (last_sweep >= 60 ? 1e-13 : 1e-15) * mm) ns = last_sweep + 1;
            }
            if (threadIdx.x == 0) sh_ns = ns;
        }
        __syncthreads();
        ns_single = sh_ns;
        if (blockIdx.x == 0 && threadIdx.x == 0 && ns_single != 0 && cs0 == 0)
            adj_mark_converged(D, A, 0, ns_single, r);
        if (ns_single == 0 || A.status[ADJ_ERR] != 0) return;
    } else if (A.status[ADJ_CONV] != (unsigned long long)K.n_inst || A.status[ADJ_ERR] != 0) {
        return;
    }
    if (j == 0 && gate != GATE_OFF) A.status[ADJ_DONE] = (unsigned long long)gate + 1;
    if (j >= K.n_cg) return;
    if (!act) {
        A.rbar_next[j] = 0.0;
        return;
    }
    // the converged mu of the step: the buffer the last sweep wrote
    const int ns = last_sweep >= 0 ? ns_single : cs_inst;
    const double* mu = (ns & 1) ? A.mu1 : A.mu0;
    const double mui = mu[cell];
    double nmu[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < nf; ++q)
        if (fr[q].inside) nmu[q] = mu[fr[q].nbcell];
    const double bb = wi * sig / (1.0 + lam) * mui + rb / (1.0 + lam);
    const double dtV = I.dt_V;
    const double cq = K.cq;
    double lap = 0.0, accu = 0.0, sig_face = 0.0, s_planck = 0.0;
#pragma unroll
    for (int q = 0; q < nf; ++q) {
        if (fr[q].inside) {
            const double bbn = nw[q] * nsig[q] / (1.0 + nlam[q]) * nmu[q] + nrb[q] / (1.0 + nlam[q]);
            lap += fr[q].S * Df[q] * (phin[q] - phik);
            accu += fr[q].S * (bbn - bb);
            sig_face += dtV * fr[q].S * (bb - bbn) * (phin[q] - phik) * dDds[q];
        } else {
            const int bc = I.bc[q];
            if (bc == BC_REFLECT) continue;
            lap += fr[q].S * Df[q] * (ghost[q] - phik);
            accu -= fr[q].S * bb;
            sig_face += dtV * fr[q].S * bb * (ghost[q] - phik) * dDds[q];
            if (bc == BC_PLANCK) s_planck += dtV * fr[q].S * cq * bb * ghost[q] * c4d;
        }
    }
    const double b = rQ + dtV * lap;
    const double em = (b - phik) / (1.0 + lam);
    const double ubar = dtV * cq * accu;
    double sbar = -em / (1.0 + lam) * (wi * sig * mui + rb);
    sbar += ubar * rRhoh * dA;
    sbar += s_planck;
    const double sigbar = wi * em * mui;
    const double ks = K.c * K.dt / (K.eps * K.eps);
    A.grad[j] += simp * (sigbar + ks * sbar + sig_face);
    A.rbar_next[j] = bb + Af * ubar;
    if (g == 0) A.Tbar[cell] = mui;
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned ablocks(int64_t n) { return (unsigned)((n + ADJ_THREADS - 1) / ADJ_THREADS); }

void launch_rec_store(const Dev& D, const Consts& K, const Adj& A, int r, hipStream_t st)
{
    k_rec_store<<<ablocks(K.n_cg), ADJ_THREADS, 0, st>>>(D, K, A, r);
}

void launch_adj_coef(const Dev& D, const Consts& K, const Adj& A, hipStream_t st)
{
    k_adj_coef<<<ablocks(K.n_cg), ADJ_THREADS, 0, st>>>(D, K, A);
}

void launch_adj_face(const Dev& D, const Consts& K, const Adj& A, int inst, int axis, int64_t nslots,
                     hipStream_t st)
{
    if (nslots > 0) k_adj_face<<<ablocks(nslots), ADJ_THREADS, 0, st>>>(D, K, A, inst, axis);
}

void launch_adj_prep(const Dev& D, const Consts& K, const Adj& A, int r, uint32_t gate, hipStream_t st)
{
    (K.n_inst == 1 ? k_adj_prep<true> : k_adj_prep<false>)<<<ablocks(K.n_cg), ADJ_THREADS, 0, st>>>(D, K, A, r, gate);
}

void launch_adj_decide(const Dev& D, const Consts& K, const Adj& A, int k, int r, uint32_t gate, hipStream_t st)
{
    k_adj_decide<<<ablocks((int64_t)K.n_inst * WAVE), ADJ_THREADS, 0, st>>>(D, K, A, k, r, gate);
}

void launch_adj_sweeps(const Dev& D, const Consts& K, const Adj& A, int k0, int k1, int r, uint32_t gate,
                       hipStream_t st)
{
    const bool fold = K.n_inst == 1;
    for (int k = k0; k < k1; ++k) {
        const double* in = (k & 1) ? A.mu1 : A.mu0;
        double* out = (k & 1) ? A.mu0 : A.mu1;
        auto sw = K.inst0.dim == 1 ? (fold ? k_adj_sweep<true, 1> : k_adj_sweep<false, 1>)
                                   : (fold ? k_adj_sweep<true, 2> : k_adj_sweep<false, 2>);
        sw<<<ablocks(K.n_cg), ADJ_THREADS, 0, st>>>(D, K, A, k, in, out, r,
                                                                                    gate, fold && k > k0 ? 1 : 0);
        if (!fold) launch_adj_decide(D, K, A, k, r, gate, st);
    }
}

void launch_adj_grad(const Dev& D, const Consts& K, const Adj& A, int r, uint32_t gate, int last_sweep,
                     hipStream_t st)
{
    const bool single = K.n_inst == 1;
    auto gr = K.inst0.dim == 1 ? (single ? k_adj_grad<true, 1> : k_adj_grad<false, 1>)
                               : (single ? k_adj_grad<true, 2> : k_adj_grad<false, 2>);
    gr<<<ablocks(K.n_cg), ADJ_THREADS, 0, st>>>(D, K, A, r, gate, single ? last_sweep : -1);
}

}  // namespace ugk
