// Host runtime of the UGKWP library: validation, device memory, the per-step
// launch sequence of Algorithm 1, and the C ABI declared in include/ugkwp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ugkwp.h"
#include "common.hpp"
#include "device_math.hpp"
#include "adjoint.hpp"
#include "kernels.hpp"

using namespace ugk;

namespace {

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(x)                                          \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) throw HipError{e_, #x};      \
    } while (0)

struct ApiError {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw ApiError{code, buf};
}

// Taylor coefficients of int_0^x t^3/(e^t-1) dt beyond x^3/3 - x^4/8:
// c_j multiplies x^(5+2j) and equals B_{2k} / ((2k)! (2k+3)), k = j+1, with
// B_{2k}/(2k)! = (-1)^{k+1} 2 zeta(2k) / (2 pi)^{2k}.  zeta(2k) is summed directly
// (closed forms for k = 1, 2) in long double.
HeadSeries make_head_series()
{
    HeadSeries hs;
    hs.nterm = HEAD_TERMS;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < hs.nterm; ++j) {
        const int k = j + 1;
        long double zeta;
        if (k == 1) zeta = pi * pi / 6.0L;
        else if (k == 2) zeta = pi * pi * pi * pi / 90.0L;
        else {
            zeta = 0.0L;
            const int N = 4000;
            for (int n = N; n >= 1; --n) zeta += powl((long double)n, -2.0L * k);
            zeta += powl((long double)N, 1.0L - 2.0L * k) / (2.0L * k - 1.0L) - 0.5L * powl((long double)N, -2.0L * k);
        }
        long double v = 2.0L * zeta / powl(2.0L * pi, 2.0L * k) / (2.0L * k + 3.0L);
        if (!(k & 1)) v = -v;
        hs.c[j] = (double)v;
    }
    hs.inv[0] = 0.0;
    for (int n = 1; n < 64; ++n) hs.inv[n] = 1.0 / (double)n;
    return hs;
}

bool g_head_ready = false;

void ensure_head_series()
{
    if (!g_head_ready) {
        const HeadSeries hs = make_head_series();
        HIPCHK(set_head_series(hs));
        HIPCHK(set_head_series_adj(hs));
        g_head_ready = true;
    }
}

struct HostInst {
    int dim = 1, nx = 0, ny = 1;
    double x0 = 0, x1 = 1, y0 = 0, y1 = 1;
    int bc[4] = {0, 0, 0, 0};
    double bcT[4] = {0, 0, 0, 0};
    int G = 0;
    std::vector<double> edges;
    uint64_t seed = 0;
    double w_ref = 0;
};

int next_pow2(int g)
{
    int p = 1;
    while (p < g) p <<= 1;
    return p;
}

int ilog2(int p)
{
    int l = 0;
    while ((1 << l) < p) ++l;
    return l;
}

constexpr int MAX_PUSH_BLOCKS = 8192;     // per-block survivor counts kept by the push
constexpr int RUN_AHEAD = 16;             // steps enqueued per host synchronisation
constexpr int N_RECORDS = RUN_AHEAD + 1;  // step records: a batch's steps and the state it starts from
constexpr int PUSH_TIME_EVERY = 8;        // default: without phase timing, the push of one step in 8 is timed

template <class T>
T* dalloc(std::vector<void*>& owned, size_t n)
{
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) fail(UGKWP_ENOMEM, "hipMalloc of %zu bytes failed", n * sizeof(T));
    owned.push_back(p);
    return (T*)p;
}

// rows x width bytes from src (row pitch spitch) to dst (row pitch dpitch).  A
// pitched copy into pageable host memory would go row by row, so it is staged
// in one contiguous transfer and unpacked on the host (synchronously).
void copy_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t rows,
               hipMemcpyKind kind, hipStream_t st)
{
    if (rows == 0 || width == 0) return;
    if (dpitch == width && spitch == width) {
        HIPCHK(hipMemcpyAsync(dst, src, width * rows, kind, st));
        return;
    }
    if (kind == hipMemcpyDeviceToHost) {
        std::vector<char> tmp(spitch * (rows - 1) + width);
        HIPCHK(hipMemcpyAsync(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t r = 0; r < rows; ++r) memcpy((char*)dst + r * dpitch, tmp.data() + r * spitch, width);
        return;
    }
    HIPCHK(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, kind, st));
}

}  // namespace

struct ugkwp_ctx {
    ugkwp_params P{};
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;                    // the GPU current at ugkwp_create: the context's memory lives there
    std::string err;

    // geometry
    int dim = 0, n_inst = 0;
    std::vector<HostInst> hi;
    std::vector<Inst> inst;
    std::vector<int64_t> inst_cg;
    Consts K{};
    int ncell = 0;
    int64_t n_fx = 0, n_fy = 0, n_edges = 0;

    // device state
    std::vector<void*> owned;
    Dev D{};
    Pool mv[2]{};          // moving fields (x, y, cell word), alternate every step
    Pool stb[2]{};         // stable fields (direction, nu, w, id, g), switch on sorts
    int cur_mv = 0, cur_st = 0;
    int64_t n_alive = 0;   // live particles
    int64_t n_slots = 0;   // pool slots incl. holes
    uint32_t step_idx = 0;
    bool have_opacity = false, have_material = false;
    int64_t* part = nullptr;
    int64_t n_part = 0;
    double* d_phib = nullptr;
    // Olson's material models (allocated on first use)
    double* olH_buf = nullptr;
    double* olchi_buf = nullptr;
    double* uend_buf = nullptr;
    double* qsrc_buf = nullptr;
    int* src_on_buf = nullptr;
    int32_t* tab_mat_buf = nullptr;
    double* tab_sig_buf = nullptr;

    // step records: counters | birth totals | per-instance state | per-instance
    // energy sums [| their sub-slots], N_RECORDS of them on the device (every
    // step of a batch writes its own), read back together after the batch into
    // pinned h_ring, or one of them into h_status when a step is taken up alone.
    // cur_rec holds the committed state; D points at it between steps.
    char* d_ring = nullptr;
    char* h_ring = nullptr;
    void* h_status = nullptr;
    size_t status_bytes = 0, ring_stride = 0;
    size_t off_tot = 0, off_ist = 0, off_diag = 0, off_sub = 0;
    int cur_rec = 0;
    bool host_diag = false;            // the host folds the energy sums' sub-slots
    double* diag_sub_dev = nullptr;    // the sub-slots when the device folds them
    hipEvent_t ev[7]{};                // autotuner and adjoint timing
    hipEvent_t sev[RUN_AHEAD][7]{};    // per step of a batch: phase boundaries, push
    int cur_slot = 0;                  // event set of the step being enqueued or read
    int last_sweeps = 4;
    int64_t last_births = 0;
    int sort_interval = 0;             // 0: 32 steps in 1-D, 16 in 2-D (measured on the benchmark media)
    ugkwp_diag diag{};
    ugkwp_totals tot{};                // running sums since the last reset

    // launch shape of the push (default: occupancy-filled persistent grid, 4
    // particles per thread; ugkwp_autotune may change it)
    PushShape push_shape{0, 4, 256};
    uint64_t ids_used = 0;             // the largest birth counter of an instance (particle ids below it)

    // each step's launch sequence captured as a HIP graph, one per launch
    // configuration (pool buffer parities, rho/T parity, sort, speculative sweeps)
    bool use_graph = false;
    bool phase_times = false;          // time every phase of a step (else the push only)
    int push_time_every = PUSH_TIME_EVERY;   // the push of steps with index a multiple of this is timed
    hipStream_t cap_st = nullptr;
    std::map<uint32_t, hipGraphExec_t> graphs;
    const double* rho_buf0 = nullptr;
    int graphs_built = 0;

    void drop_graphs()
    {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }

    // adjoint: record of the forward run and reverse-sweep buffers
    std::vector<void*> rec_owned;
    Adj A{};
    int rec_cap = 0, nrec = 0;
    std::vector<int> rec_sweeps;      // forward source-iteration sweeps per recorded step
    unsigned long long* h_adj = nullptr;   // pinned copy of A.status

    ~ugkwp_ctx() { release(); }

    void free_record()
    {
        for (void* p : rec_owned) (void)hipFree(p);
        rec_owned.clear();
        A = Adj{};
        rec_cap = nrec = 0;
        rec_sweeps.clear();
    }

    void release()
    {
        drop_graphs();
        if (cap_st) (void)hipStreamDestroy(cap_st);
        cap_st = nullptr;
        free_record();
        if (h_adj) (void)hipHostFree(h_adj);
        h_adj = nullptr;
        for (void* p : owned) (void)hipFree(p);
        owned.clear();
        if (h_status) (void)hipHostFree(h_status);
        h_status = nullptr;
        if (h_ring) (void)hipHostFree(h_ring);
        h_ring = nullptr;
        for (auto& e : ev)
            if (e) { (void)hipEventDestroy(e); e = nullptr; }
        for (auto& row : sev)
            for (auto& e : row)
                if (e) { (void)hipEventDestroy(e); e = nullptr; }
        if (own_stream && st) (void)hipStreamDestroy(st);
        st = nullptr;
        own_stream = false;
    }

    void free_device()
    {
        drop_graphs();
        free_record();
        for (void* p : owned) (void)hipFree(p);
        owned.clear();
        D = Dev{};
        mv[0] = mv[1] = stb[0] = stb[1] = Pool{};
        have_opacity = have_material = false;
        olH_buf = olchi_buf = uend_buf = qsrc_buf = nullptr;
        src_on_buf = nullptr;
        tab_mat_buf = nullptr;
        tab_sig_buf = nullptr;
        K.olson = K.table = K.has_src = 0;
    }

    // ---------------------------------------------------------------- set-up
    void setup(const std::vector<HostInst>& in)
    {
        ensure_head_series();
        if (in.empty()) fail(UGKWP_EINVAL, "no instances");
        const int d0 = in[0].dim;
        for (const auto& h : in) {
            if (h.dim != 1 && h.dim != 2) fail(UGKWP_EINVAL, "dim must be 1 or 2");
            if (h.dim != d0) fail(UGKWP_EINVAL, "all instances of a context share one dimension");
            if (h.nx < 1 || h.ny < 1 || (h.dim == 1 && h.ny != 1)) fail(UGKWP_EINVAL, "bad cell counts");
            if (!(h.x1 > h.x0) || (h.dim == 2 && !(h.y1 > h.y0))) fail(UGKWP_EINVAL, "empty domain");
            if (h.G < 1 || h.G > MAX_G) fail(UGKWP_EINVAL, "G must be in 1..%d", MAX_G);
            for (int g = 0; g < h.G; ++g)
                if (!(h.edges[g] > 0) || !(h.edges[g + 1] > h.edges[g]) || !std::isfinite(h.edges[g + 1]))
                    fail(UGKWP_EINVAL, "group edges must be positive, finite and ascending");
            for (int q = 0; q < 2 * h.dim; ++q) {
                if (h.bc[q] < 0 || h.bc[q] > 2) fail(UGKWP_EINVAL, "bad boundary type");
                if (h.bc[q] == UGKWP_BC_PLANCK && !(h.bcT[q] > 0 && std::isfinite(h.bcT[q])))
                    fail(UGKWP_EINVAL, "Planckian boundary temperature must be positive");
            }
            if (!(h.w_ref > 0)) fail(UGKWP_EINVAL, "w_ref must be positive");
            if ((int64_t)h.nx * h.ny > (1 << 28)) fail(UGKWP_EINVAL, "too many cells");
        }
        {
            // tally bins are addressed with 30-bit indices in the push's LDS table
            int64_t cg = 0, fx = 0, fy = 0;
            for (const auto& h : in) {
                const int64_t gp = next_pow2(h.G);
                cg += (int64_t)h.nx * h.ny * gp + WAVE;
                fx += (int64_t)(h.nx + 1) * h.ny * gp;
                if (h.dim == 2) fy += (int64_t)h.nx * (h.ny + 1) * gp;
            }
            if (cg >= (1ll << 30) || 2 * fx >= (1ll << 30) || 2 * fy >= (1ll << 30))
                fail(UGKWP_EINVAL, "mesh too large for one context (more than 2^30 cell-group or face slots)");
        }
        free_device();
        dim = d0;
        n_inst = (int)in.size();
        hi = in;
        inst.assign(n_inst, Inst{});
        inst_cg.assign(n_inst + 1, 0);
        int64_t cg = 0, fx = 0, fy = 0, ed = 0;
        int cells = 0;
        for (int k = 0; k < n_inst; ++k) {
            const HostInst& h = in[k];
            Inst& I = inst[k];
            I.dim = h.dim; I.nx = h.nx; I.ny = h.ny; I.ncell = h.nx * h.ny;
            I.G = h.G; I.Gp = next_pow2(h.G); I.lgGp = ilog2(I.Gp);
            I.cell_off = cells;
            I.edge_off = (int)ed;
            for (int q = 0; q < 4; ++q) { I.bc[q] = h.bc[q]; I.bcT[q] = h.bcT[q]; }
            cg = (cg + WAVE - 1) / WAVE * WAVE;
            I.cg_off = cg;
            inst_cg[k] = cg;
            cg += (int64_t)I.ncell * I.Gp;
            I.fx_off = fx;
            fx += (int64_t)(h.nx + 1) * h.ny * I.Gp;
            I.fy_off = fy;
            if (h.dim == 2) fy += (int64_t)h.nx * (h.ny + 1) * I.Gp;
            I.x0 = h.x0; I.y0 = h.dim == 2 ? h.y0 : 0.0;
            I.dx = (h.x1 - h.x0) / h.nx;
            I.dy = h.dim == 2 ? (h.y1 - h.y0) / h.ny : 1.0;
            I.V = I.dx * I.dy;
            I.dt_V = P.dt / I.V;
            I.w_ref = h.w_ref;
            I.seed = h.seed;
            cells += I.ncell;
            ed += h.G + 1;
        }
        const int64_t n_cg = (cg + WAVE - 1) / WAVE * WAVE;
        inst_cg[n_inst] = n_cg;
        ncell = cells;
        n_fx = fx; n_fy = fy; n_edges = ed;

        K.c = P.c; K.a = P.a; K.eps = P.eps; K.dt = P.dt;
        K.e2c = P.eps * P.eps / P.c;
        K.cv = P.c / P.eps;
        K.lam_scale = P.c * P.dt / (P.eps * P.eps);
        K.cq = P.c / (4.0 * P.eps);
        K.tau_C = P.tau_num_C;
        K.tau_jump = P.tau_num_jump;
        K.t_power = P.opacity_T_power;
        K.stim = P.opacity_stim;
        K.nu_power = P.nu_power;
        K.si_tol = P.si_tol;
        K.n_cap = P.n_cap;
        K.pool_cap = P.pool_capacity;
        K.flags = P.flags;
        K.gate = GATE_OFF;
        K.n_inst = n_inst;
        K.n_cg = n_cg;
        K.n_fx2 = 2 * fx;
        K.ncell = ncell;
        K.inst0 = inst[0];

        // device memory
        std::vector<double> edges, simpson;
        for (const auto& h : in) {
            for (int g = 0; g <= h.G; ++g) edges.push_back(h.edges[g]);
            for (int g = 0; g < h.G; ++g) {
                const double nl = h.edges[g], nh = h.edges[g + 1], nm = 0.5 * (nl + nh);
                simpson.push_back((nu_pow(nl, P.nu_power) + 4.0 * nu_pow(nm, P.nu_power) + nu_pow(nh, P.nu_power)) / 6.0);
            }
            simpson.push_back(0.0);
        }
        std::vector<int32_t> wave_inst((size_t)(n_cg / WAVE));
        for (int k = 0, w = 0; w < (int)wave_inst.size(); ++w) {
            while (k + 1 < n_inst && inst_cg[k + 1] <= (int64_t)w * WAVE) ++k;
            wave_inst[w] = k;
        }
        std::vector<int32_t> cell_inst(ncell);
        for (int k = 0; k < n_inst; ++k)
            for (int c = 0; c < inst[k].ncell; ++c) cell_inst[inst[k].cell_off + c] = k;

        Inst* d_inst = dalloc<Inst>(owned, n_inst);
        int64_t* d_inst_cg = dalloc<int64_t>(owned, n_inst + 1);
        int32_t* d_cell_inst = dalloc<int32_t>(owned, ncell);
        int32_t* d_wave_inst = dalloc<int32_t>(owned, wave_inst.size());
        double* d_nu = dalloc<double>(owned, edges.size());
        double* d_simp = dalloc<double>(owned, simpson.size());
        d_phib = dalloc<double>(owned, (size_t)n_inst * 4 * MAX_G);
        HIPCHK(hipMemcpy(d_inst, inst.data(), sizeof(Inst) * n_inst, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_inst_cg, inst_cg.data(), sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_cell_inst, cell_inst.data(), sizeof(int32_t) * ncell, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_wave_inst, wave_inst.data(), sizeof(int32_t) * wave_inst.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_nu, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_simp, simpson.data(), sizeof(double) * simpson.size(), hipMemcpyHostToDevice));

        Dev& d = D;
        d = Dev{};
        d.inst = d_inst;
        d.inst_cg = d_inst_cg;
        d.wave_inst = d_wave_inst;
        d.cell_inst = d_cell_inst;
        d.nu = d_nu;
        d.simpson = d_simp;
        d.phib = d_phib;
        const size_t ncg = (size_t)n_cg;
        d.kappa = dalloc<double>(owned, ncg);
        d.sig = dalloc<double>(owned, ncg);
        d.inv_kappa = dalloc<double>(owned, ncg);
        d.sv = dalloc<double>(owned, ncg);
        d.es = dalloc<double>(owned, ncg);
        d.c4 = dalloc<double>(owned, ncg);
        d.wc = dalloc<double>(owned, ncg);
        d.rho = dalloc<double>(owned, ncg);
        rho_buf0 = d.rho;
        d.rho_new = dalloc<double>(owned, ncg);
        d.rhop = dalloc<double>(owned, ncg);
        d.rhoh = dalloc<double>(owned, ncg);
        d.Q = dalloc<double>(owned, ncg);
        d.phi0 = dalloc<double>(owned, ncg);
        d.phi1 = dalloc<double>(owned, ncg);
        d.phi2 = dalloc<double>(owned, ncg);
        // slots the sweeps never write (padding groups and cells) stay zero
        for (double* q : {d.phi0, d.phi1, d.phi2, d.rho, d.rho_new})
            HIPCHK(hipMemsetAsync(q, 0, sizeof(double) * ncg, st));
        d.nb = dalloc<int32_t>(owned, ncg);
        d.boff = dalloc<int64_t>(owned, ncg + 1);
        d.wnew = dalloc<double>(owned, ncg);
        d.wsn = dalloc<double>(owned, ncg);
        d.sx = dalloc<double>(owned, ncg);
        d.sy = dalloc<double>(owned, ncg);
        d.bcoef = dalloc<double>(owned, ncg);
        d.rho_alt = dalloc<double>(owned, ncg);
        d.winflow = dalloc<double>(owned, 2 * ncg);
        d.nbi = dalloc<int32_t>(owned, ncg);
        d.beta = dalloc<double>(owned, ncg);
        d.dep = dalloc<double>(owned, ncg);
        d.surv = dalloc<double>(owned, ncg);
        d.scount = dalloc<uint32_t>(owned, ncg);
        d.soff = dalloc<int64_t>(owned, ncg + 1);
        d.ftx = dalloc<double>(owned, (size_t)n_fx * 2);
        d.fty = dalloc<double>(owned, (size_t)std::max<int64_t>(n_fy, 1) * 2);
        d.Dx = dalloc<double>(owned, (size_t)n_fx);
        d.Dy = dalloc<double>(owned, (size_t)std::max<int64_t>(n_fy, 1));
        d.cvol = dalloc<double>(owned, ncell);
        d.dtcv = dalloc<double>(owned, ncell);
        d.T = dalloc<double>(owned, ncell);
        d.T_new = dalloc<double>(owned, ncell);
        d.pinned = dalloc<uint8_t>(owned, ncell);
        // step records (see the member comment); offsets are multiples of 16 bytes
        off_tot = sizeof(unsigned long long) * N_COUNTERS;
        off_ist = off_tot + 16;
        off_diag = off_ist + (sizeof(InstState) * (size_t)n_inst + 15) / 16 * 16;
        off_sub = off_diag + sizeof(double) * 8 * (size_t)n_inst;
        // few instances: the energy sums' sub-slots travel with the record and
        // the host folds them (no reduction launch)
        host_diag = n_inst <= 16;
        status_bytes = off_sub + (host_diag ? sizeof(double) * DIAG_SUB * 8 * (size_t)n_inst : 0);
        ring_stride = (status_bytes + 255) / 256 * 256;
        d_ring = dalloc<char>(owned, ring_stride * N_RECORDS);
        HIPCHK(hipMemsetAsync(d_ring, 0, ring_stride * N_RECORDS, st));
        if (h_status) (void)hipHostFree(h_status);
        h_status = nullptr;
        HIPCHK(hipHostMalloc(&h_status, status_bytes, hipHostMallocDefault));
        if (h_ring) (void)hipHostFree(h_ring);
        h_ring = nullptr;
        HIPCHK(hipHostMalloc((void**)&h_ring, ring_stride * N_RECORDS, hipHostMallocDefault));
        d.step = dalloc<uint32_t>(owned, 1);
        HIPCHK(hipMemsetAsync(d.step, 0, sizeof(uint32_t), st));
        d.res = dalloc<Resid>(owned, (size_t)n_inst * RES_SLOTS * RES_SUB);
        {
            // one flag per wavefront of slots, read four at a time by the sweeps' blocks
            const size_t nflag = ((size_t)(n_cg / WAVE) + 3) / 4 * 4;
            d.wave_run = dalloc<uint8_t>(owned, nflag);
            HIPCHK(hipMemsetAsync(d.wave_run, 0, nflag, st));
        }
        diag_sub_dev = host_diag ? nullptr : dalloc<double>(owned, (size_t)n_inst * DIAG_SUB * 8);
        cur_rec = 0;
        point_record(d, 0, 0);
        n_part = std::max<int64_t>(scan_partials_size(n_cg), count_partials_size());
        part = dalloc<int64_t>(owned, (size_t)n_part + 1);
        HIPCHK(hipMemsetAsync(d.ist, 0, sizeof(InstState) * n_inst, st));
        HIPCHK(hipMemsetAsync((void*)d.boff, 0, sizeof(int64_t) * (ncg + 1), st));
        HIPCHK(hipMemsetAsync(d.ftx, 0, sizeof(double) * n_fx * 2, st));
        HIPCHK(hipMemsetAsync(d.fty, 0, sizeof(double) * std::max<int64_t>(n_fy, 1) * 2, st));
        HIPCHK(hipMemsetAsync(d.dep, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.surv, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.nb, 0, sizeof(int32_t) * ncg, st));
        HIPCHK(hipMemsetAsync(d.nbi, 0, sizeof(int32_t) * ncg, st));
        HIPCHK(hipMemsetAsync(d.sx, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.sy, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.bcoef, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.winflow, 0, sizeof(double) * 2 * ncg, st));
        HIPCHK(hipMemsetAsync(d.wnew, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.Q, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(d.rhoh, 0, sizeof(double) * ncg, st));
        launch_ghost_phi(D, K, d_phib, st);

        const int64_t cap = std::max<int64_t>(P.pool_capacity, 1);
        for (int b = 0; b < 2; ++b) {
            mv[b].x = dalloc<double>(owned, cap);
            mv[b].cell = dalloc<int32_t>(owned, cap);
            stb[b].ox = dalloc<double>(owned, cap);
            if (dim == 2) {
                mv[b].y = dalloc<double>(owned, cap);
                stb[b].oy = dalloc<double>(owned, cap);
            }
            stb[b].nu = dalloc<double>(owned, cap);
            stb[b].w = dalloc<double>(owned, cap);
            stb[b].id = dalloc<uint64_t>(owned, cap);
        }
        d.blk_surv = dalloc<unsigned long long>(owned, MAX_PUSH_BLOCKS);
        push_shape = push_default_shape(dim, K);
        push_shape.blocks = std::min(push_shape.blocks, MAX_PUSH_BLOCKS);
        cur_mv = cur_st = 0;
        n_alive = n_slots = 0;
        step_idx = 0;
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
    }

    // point D's record entries at record `slot`, the record before it at `prev`
    void point_record(Dev& d, int slot, int prev) const
    {
        char* r = d_ring + (size_t)slot * ring_stride;
        const char* q = d_ring + (size_t)prev * ring_stride;
        d.counters = (unsigned long long*)r;
        d.n_births_total = (int64_t*)(r + off_tot);
        d.ist = (InstState*)(r + off_ist);
        d.diag = (double*)(r + off_diag);
        d.diag_sub = host_diag ? (double*)(r + off_sub) : diag_sub_dev;
        d.prev_counters = (const unsigned long long*)q;
        d.prev_ist = (const InstState*)(q + off_ist);
    }

    // pack a host [ncell][G] array of instance k into the padded device layout
    void pack_cg(std::vector<double>& dst, int k, const double* src) const
    {
        const Inst& I = inst[k];
        for (int c = 0; c < I.ncell; ++c)
            for (int g = 0; g < I.G; ++g) dst[I.cg_off + ((int64_t)c << I.lgGp) + g] = src[(int64_t)c * I.G + g];
    }

    void set_opacity(const std::vector<const double*>& kap)
    {
        if (rec_cap > 0) fail(UGKWP_EINVAL, "the opacity cannot change while a record is kept (ugkwp_record(ctx, 0) first)");
        std::vector<double> h((size_t)K.n_cg, 0.0);
        for (int k = 0; k < n_inst; ++k) {
            const Inst& I = inst[k];
            for (int64_t q = 0; q < (int64_t)I.ncell * I.G; ++q)
                if (!(kap[k][q] >= 0.0) || !std::isfinite(kap[k][q])) fail(UGKWP_EINVAL, "kappa must be finite and >= 0");
            pack_cg(h, k, kap[k]);
        }
        HIPCHK(hipMemcpyAsync((void*)D.kappa, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
        launch_tables(D, K, st);
        for (int k = 0; k < n_inst; ++k) {
            const Inst& I = inst[k];
            launch_face_D(D, K, k, 0, (int64_t)(I.nx + 1) * I.ny * I.Gp, st);
            if (dim == 2) launch_face_D(D, K, k, 1, (int64_t)I.nx * (I.ny + 1) * I.Gp, st);
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        have_opacity = true;
    }

    // staging: device room for ncell doubles that receives Tr0 (nullptr: allocated
    // here and freed after the call)
    void set_material(const std::vector<const double*>& cv, const std::vector<const double*>& T0,
                      const std::vector<const double*>& Tr0, const std::vector<const uint8_t*>& pinned,
                      double* staging = nullptr)
    {
        std::vector<double> hcv(ncell), hT(ncell), hTr(ncell), hw(ncell);
        std::vector<uint8_t> hp(ncell, 0);
        for (int k = 0; k < n_inst; ++k) {
            const Inst& I = inst[k];
            for (int c = 0; c < I.ncell; ++c) {
                const double a = cv[k][c], b = T0[k][c], r = Tr0[k][c];
                if (!(a > 0) || !(b > 0) || !(r > 0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(r))
                    fail(UGKWP_EINVAL, "cv, T0 and Tr0 must be positive and finite");
                hcv[I.cell_off + c] = a;
                hw[I.cell_off + c] = P.dt / (P.eps * P.eps * a);
                hT[I.cell_off + c] = b;
                hTr[I.cell_off + c] = r;
                hp[I.cell_off + c] = pinned[k] ? (pinned[k][c] ? 1 : 0) : 0;
            }
        }
        double* d_tr = staging;
        if (!staging) HIPCHK(hipMalloc(&d_tr, sizeof(double) * ncell));
        HIPCHK(hipMemcpyAsync((void*)D.cvol, hcv.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync((void*)D.dtcv, hw.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(D.T, hT.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync((void*)D.pinned, hp.data(), ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d_tr, hTr.data(), sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        launch_init_rho(D, K, d_tr, st);
        HIPCHK(hipMemsetAsync(D.ist, 0, sizeof(InstState) * n_inst, st));
        HIPCHK(hipMemsetAsync(D.counters, 0, sizeof(unsigned long long) * N_COUNTERS, st));
        HIPCHK(hipMemsetAsync(D.step, 0, sizeof(uint32_t), st));
        HIPCHK(hipStreamSynchronize(st));
        if (!staging) (void)hipFree(d_tr);
        HIPCHK(hipGetLastError());
        n_alive = n_slots = 0;
        step_idx = 0;
        last_births = 0;
        cur_mv = cur_st = 0;
        have_material = true;
        nrec = 0;
        rec_sweeps.clear();
    }

    // ---------------------------------------------------------------- Olson's material models
    // The device arrays of a model, allocated on its first set-up call and kept.
    template <class T>
    T* model_array(T*& p, size_t n)
    {
        if (!p) p = dalloc<T>(owned, n);
        return p;
    }

    // H and chi per cell (all instances); NULL H: off
    void set_heat_capacity(const double* H, const double* chi)
    {
        if (rec_cap > 0) fail(UGKWP_EINVAL, "the material cannot change while a record is kept (ugkwp_record(ctx, 0) first)");
        drop_graphs();
        if (!H) {
            K.olson = 0;
            return;
        }
        if (!chi) fail(UGKWP_EINVAL, "null chi");
        for (int c = 0; c < ncell; ++c)
            if (!(H[c] >= 0.0) || !std::isfinite(H[c]) || !(chi[c] >= 0.0) || !std::isfinite(chi[c]))
                fail(UGKWP_EINVAL, "H and chi must be finite and >= 0");
        double* dH = model_array(olH_buf, (size_t)ncell);
        double* dchi = model_array(olchi_buf, (size_t)ncell);
        model_array(uend_buf, (size_t)ncell);
        HIPCHK(hipMemcpyAsync(dH, H, sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dchi, chi, sizeof(double) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(uend_buf, 0, sizeof(double) * ncell, st));
        HIPCHK(hipStreamSynchronize(st));
        D.olH = dH;
        D.olchi = dchi;
        D.uend = uend_buf;
        K.olson = 1;
    }

    // q [cell][G] of every instance, or (f != nullptr) the Planckian source
    // (c/eps^2) f phi_g(Ts); both null: off
    void set_source(const double* q, const double* f, double Ts, double t_off)
    {
        if (rec_cap > 0) fail(UGKWP_EINVAL, "the source cannot change while a record is kept (ugkwp_record(ctx, 0) first)");
        drop_graphs();
        if (!q && !f) {
            K.has_src = 0;
            return;
        }
        if (!(t_off >= 0.0)) fail(UGKWP_EINVAL, "t_off must be >= 0");
        double* dq = model_array(qsrc_buf, (size_t)K.n_cg);
        model_array(src_on_buf, 1);
        if (q) {
            std::vector<double> h((size_t)K.n_cg, 0.0);
            int64_t off = 0;
            for (int k = 0; k < n_inst; ++k) {
                const Inst& I = inst[k];
                for (int64_t e = 0; e < (int64_t)I.ncell * I.G; ++e)
                    if (!(q[off + e] >= 0.0) || !std::isfinite(q[off + e])) fail(UGKWP_EINVAL, "q must be finite and >= 0");
                pack_cg(h, k, q + off);
                off += (int64_t)I.ncell * I.G;
            }
            HIPCHK(hipMemcpyAsync(dq, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        } else {
            if (!(Ts > 0.0) || !std::isfinite(Ts)) fail(UGKWP_EINVAL, "the source temperature must be positive and finite");
            for (int c = 0; c < ncell; ++c)
                if (!(f[c] >= 0.0) || !std::isfinite(f[c])) fail(UGKWP_EINVAL, "f must be finite and >= 0");
            double* df = nullptr;
            HIPCHK(hipMalloc(&df, sizeof(double) * ncell));
            hipError_t e = hipMemcpyAsync(df, f, sizeof(double) * ncell, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) {
                launch_source_planck(D, K, dq, df, Ts, st);
                e = hipStreamSynchronize(st);
            }
            (void)hipFree(df);
            if (e != hipSuccess) fail(UGKWP_EHIP, "set_source_planck: %s", hipGetErrorString(e));
        }
        HIPCHK(hipMemsetAsync(src_on_buf, 0, sizeof(int), st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        D.qsrc = dq;
        D.src_on = src_on_buf;
        K.has_src = 1;
        K.q_toff = t_off;
    }

    void set_opacity_table(int nmat, const int32_t* mat, int nnu, const double* nu, int nT, const double* T,
                           const double* sig)
    {
        if (rec_cap > 0) fail(UGKWP_EINVAL, "the opacity cannot change while a record is kept (ugkwp_record(ctx, 0) first)");
        if (nmat < 1 || nnu < 2 || nT < 2 || !mat || !nu || !T || !sig) fail(UGKWP_EINVAL, "bad table sizes or null arrays");
        for (int c = 0; c < ncell; ++c)
            if (mat[c] < 0 || mat[c] >= nmat) fail(UGKWP_EINVAL, "material index out of range");
        for (int k = 0; k < nnu; ++k)
            if (!(nu[k] > 0) || !std::isfinite(nu[k]) || (k > 0 && !(nu[k] > nu[k - 1])))
                fail(UGKWP_EINVAL, "nu nodes must be positive, finite and ascending");
        for (int k = 0; k < nT; ++k)
            if (!(T[k] > 0) || !std::isfinite(T[k]) || (k > 0 && !(T[k] > T[k - 1])))
                fail(UGKWP_EINVAL, "T nodes must be positive, finite and ascending");
        const size_t nt = (size_t)nmat * nT * nnu;
        for (size_t k = 0; k < nt; ++k)
            if (!(sig[k] > 0) || !std::isfinite(sig[k])) fail(UGKWP_EINVAL, "table values must be positive and finite");
        drop_graphs();
        // the arrays of an earlier table are kept in `owned` until the context ends
        int32_t* dmat = model_array(tab_mat_buf, (size_t)ncell);
        double* dnu = dalloc<double>(owned, (size_t)nnu);
        double* dT = dalloc<double>(owned, (size_t)nT);
        double* dsig = dalloc<double>(owned, nt);
        double* drow = dalloc<double>(owned, (size_t)ncell * nnu);
        int32_t* dgi = dalloc<int32_t>(owned, (size_t)n_edges * 3);
        double* dga = dalloc<double>(owned, (size_t)n_edges * 3);
        double* dtsig = model_array(tab_sig_buf, (size_t)K.n_cg * 2);
        HIPCHK(hipMemcpyAsync(dmat, mat, sizeof(int32_t) * ncell, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dnu, nu, sizeof(double) * nnu, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dT, T, sizeof(double) * nT, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dsig, sig, sizeof(double) * nt, hipMemcpyHostToDevice, st));
        launch_tab_logs(dnu, nnu, st);
        launch_tab_logs(dT, nT, st);
        launch_tab_logs(dsig, (int64_t)nt, st);
        D.tab_mat = dmat;
        D.tab_lnu = dnu;
        D.tab_lT = dT;
        D.tab_lsig = dsig;
        D.tab_row = drow;
        D.tab_gi = dgi;
        D.tab_ga = dga;
        D.tab_sig = dtsig;
        K.table = 1;
        K.tab_nnu = nnu;
        K.tab_nT = nT;
        {
            // evenly spaced in ln T: the locate may start from the grid's guess
            const double d0 = (std::log(T[nT - 1]) - std::log(T[0])) / (nT - 1);
            bool even = d0 > 0;
            for (int k = 0; k + 1 < nT && even; ++k)
                even = std::fabs((std::log(T[k + 1]) - std::log(T[k])) - d0) <= 1e-9 * d0;
            K.tab_lT_inv = even ? 1.0 / d0 : 0.0;
        }
        launch_tab_groups(D, K, n_edges, st);
        HIPCHK(hipMemsetAsync(dtsig, 0, sizeof(double) * 2 * (size_t)K.n_cg, st));
        // the push now runs the table's flights: its default launch shape follows
        push_shape = push_default_shape(dim, K);
        push_shape.blocks = std::min(push_shape.blocks, MAX_PUSH_BLOCKS);
        if (have_material) {
            launch_tables(D, K, st);
            for (int k = 0; k < n_inst; ++k) {
                const Inst& I = inst[k];
                launch_face_D(D, K, k, 0, (int64_t)(I.nx + 1) * I.ny * I.Gp, st);
                if (dim == 2) launch_face_D(D, K, k, 1, (int64_t)I.nx * (I.ny + 1) * I.Gp, st);
            }
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        have_opacity = true;
    }

    Pool view(int m, int t) const
    {
        Pool p = stb[t];
        p.x = mv[m].x;
        p.y = mv[m].y;
        p.cell = mv[m].cell;
        return p;
    }
    Pool moving(int m) const
    {
        Pool p{};
        p.x = mv[m].x;
        p.y = mv[m].y;
        p.cell = mv[m].cell;
        return p;
    }

    // ---------------------------------------------------------------- stepping
    // Algorithm 1 per step, and steps run ahead of the host.  A batch of up to
    // RUN_AHEAD steps is enqueued without waiting: every launch of step n
    // carries n as its gate (gate_open), and every step writes its own record
    // of counters and sums.  One copy and one synchronisation per batch bring
    // the records back.  The host plans the batch as if every step commits;
    // the first step that does not commit has made every later launch of the
    // batch return at once, so it is taken up alone (more sweeps, or the error
    // it raised) and planning resumes after it.  Source-iteration sweeps are
    // launched speculatively (the most the last batch needed, plus one;
    // converged sweeps return at once).
    // Host view of the state a step's launches depend on.
    struct Plan {
        double* rho;
        double* rho_new;
        double* T;
        double* T_new;
        int cur_mv, cur_st;
        uint32_t step;
        int64_t n_slots;       // known after processing; an estimate while planned
        int nrec;
        int rec;               // record holding the state the step starts from
        int slot;              // record the step writes
        bool do_sort;
        bool push_timed;       // events around the push (a few microseconds each)
        int sweeps;            // sweeps launched
    };

    Plan state_now() const
    {
        Plan p{};
        p.rho = D.rho; p.rho_new = D.rho_new; p.T = D.T; p.T_new = D.T_new;
        p.cur_mv = cur_mv; p.cur_st = cur_st;
        p.step = step_idx;
        p.n_slots = n_slots;
        p.nrec = nrec;
        p.rec = cur_rec;
        p.slot = -1;
        return p;
    }

    void set_state(const Plan& p)
    {
        D.rho = p.rho; D.rho_new = p.rho_new; D.T = p.T; D.T_new = p.T_new;
        cur_mv = p.cur_mv; cur_st = p.cur_st;
        step_idx = p.step;
        n_slots = p.n_slots;
        nrec = p.nrec;
        cur_rec = p.rec;
        point_record(D, p.rec, p.rec);
    }

    // the record after `r` (with graphs, two alternate: their addresses are
    // part of the captured launches)
    int next_record(int r) const { return use_graph ? (r ^ 1) : (r + 1) % N_RECORDS; }

    // the state after step p commits (n_slots_after from its status, or estimated)
    Plan after(const Plan& p, int64_t n_slots_after) const
    {
        Plan q = p;
        std::swap(q.rho, q.rho_new);
        std::swap(q.T, q.T_new);
        if (p.do_sort) q.cur_st = 1 - p.cur_st;    // sorted, compact pool: moving fields in mv[cur_mv]
        else q.cur_mv = 1 - p.cur_mv;              // positions of this step in the other moving buffer
        q.n_slots = n_slots_after;
        q.step = p.step + 1;
        q.rec = p.slot;
        q.slot = -1;
        if (rec_cap > 0) q.nrec = p.nrec + 1;
        q.do_sort = false;
        q.sweeps = 0;
        return q;
    }

    bool sort_due(uint32_t step, int64_t slots) const
    {
        // sort periodically, and whenever holes have filled half the pool
        const int si = sort_interval > 0 ? sort_interval : (dim == 1 ? 32 : 16);
        return si <= 1 || (step % (uint32_t)si) == (uint32_t)(si - 1) ||
               slots > P.pool_capacity / 2;
    }

    // A step record read back to the host.
    struct StatusView {
        const unsigned long long* counters;
        const int64_t* total;
        const InstState* ist;
        const double* diag;
        const double* sub;
    };
    StatusView status_at(const char* base) const
    {
        StatusView v;
        v.counters = (const unsigned long long*)base;
        v.total = (const int64_t*)(base + off_tot);
        v.ist = (const InstState*)(base + off_ist);
        v.diag = (const double*)(base + off_diag);
        v.sub = host_diag ? (const double*)(base + off_sub) : nullptr;
        return v;
    }

    // RAII: the launches enqueued while it lives carry `step` as their gate.
    struct GateScope {
        Consts& k;
        GateScope(Consts& kk, uint32_t step) : k(kk) { k.gate = step; }
        ~GateScope() { k.gate = GATE_OFF; }
    };

    void enqueue_finish(bool do_sort, int rec, int last_sweep)
    {
        launch_finish(D, K, !host_diag, last_sweep, push_shape.blocks, st);
        if (do_sort) {
            if (phase_times) HIPCHK(hipEventRecord(sev[cur_slot][5], st));
            launch_scan(scan_gate(D, K, 1), (const int32_t*)D.scount, K.n_cg, part, D.soff, D.n_births_total + 1, st);
            launch_sort_scatter(dim, D, K, view(1 - cur_mv, cur_st), view(cur_mv, 1 - cur_st), st);
            if (phase_times) HIPCHK(hipEventRecord(sev[cur_slot][6], st));
        }
        if (rec >= 0) launch_rec_store(D, K, A, rec, st);
    }

    // The launches before the push: tally clears, counts, scan, sampling.
    void enqueue_pre_push()
    {
        ZeroList z{};
        auto add = [&](void* p, int64_t words) {
            if (words > 0) { z.ptr[z.n] = p; z.words[z.n] = words; z.n++; }
        };
        add(D.ftx, n_fx * 2);
        if (dim == 2) add(D.fty, n_fy * 2);
        add(D.dep, K.n_cg);
        add(D.surv, K.n_cg);
        add(D.scount, K.n_cg / 2);
        add(D.diag_sub, (int64_t)DIAG_SUB * 8 * n_inst);
        add(D.res, (int64_t)n_inst * RES_SUB * (int64_t)(sizeof(Resid) / 8));   // sweep 0's residual slots
        // a temperature-dependent opacity: the step's tables at its T^n
        if (K.t_power != 0.0 || K.stim || K.table) launch_tables(D, K, st);
        launch_count_scan(D, K, z, part, st);
        if (K.flags & UGKWP_FLAG_SLOPES) launch_slopes(dim, D, K, D.rhoh, false, st);
        launch_sample(dim, D, K, view(cur_mv, cur_st), st);
    }

    void enqueue_sweeps(int k0, int k1) { launch_si_sweeps(D, K, k0, k1, st); }

    // Run `enq` on the context stream: replayed from the HIP graph captured for
    // `key` (captured on first use), or launched directly without graphs.
    template <class F>
    void launch_group(uint32_t key, F&& enq)
    {
        if (!use_graph) {
            enq();
            return;
        }
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            if (!cap_st) HIPCHK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            std::swap(st, cap_st);
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                try {
                    enq();
                } catch (...) {
                    (void)hipStreamEndCapture(st, &g);
                    if (g) (void)hipGraphDestroy(g);
                    std::swap(st, cap_st);
                    throw;
                }
                e = hipStreamEndCapture(st, &g);
            }
            std::swap(st, cap_st);
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                // this runtime cannot capture these launches: launch directly from now on
                (void)hipGetLastError();
                use_graph = false;
                enq();
                return;
            }
            it = graphs.emplace(key, ex).first;
            graphs_built++;
        }
        HIPCHK(hipGraphLaunch(it->second, st));
    }

    // Graph keys: what the captured kernel arguments depend on.
    uint32_t parity() const { return D.rho == rho_buf0 ? 1u : 0u; }

    // Enqueue the launches of step p (the host state is p's).  Graph replays
    // carry no gate: with graphs, steps run one at a time.
    void enqueue_step(Plan& p)
    {
        GateScope gs(K, use_graph ? GATE_OFF : p.step);
        point_record(D, p.slot, p.rec);
        hipEvent_t* e = sev[cur_slot];
        if (phase_times) HIPCHK(hipEventRecord(e[0], st));
        launch_group(0x100000u | (uint32_t)cur_mv | ((uint32_t)cur_st << 1) | (parity() << 2) |
                         ((uint32_t)p.slot << 3),
                     [&] { enqueue_pre_push(); });
        if (p.push_timed) HIPCHK(hipEventRecord(e[1], st));
        launch_push(dim, D, K, view(cur_mv, cur_st), moving(1 - cur_mv), push_shape, st);
        if (p.push_timed) HIPCHK(hipEventRecord(e[2], st));
        // the wave flux and Q are evaluated by the first sweep: no launch of their own
        if (phase_times) HIPCHK(hipEventRecord(e[3], st));
        const int first = p.sweeps;
        launch_group(0x200000u | (uint32_t)first | (parity() << 16) | ((uint32_t)p.slot << 17),
                     [&] { enqueue_sweeps(0, first); });
        if (phase_times) HIPCHK(hipEventRecord(e[4], st));
        enqueue_finish(p.do_sort, rec_cap > 0 ? p.nrec : -1, first - 1);
    }

    // Step p did not commit: raise its error, or add sweeps until it converges.
    // Returns the record of the committed step (in h_status).
    StatusView take_up(Plan& p, StatusView s)
    {
        const int kmax = P.si_max_iters;
        point_record(D, p.slot, p.rec);
        for (;;) {
            const unsigned long long err = s.counters[CNT_ERR];
            if (err & ERR_POOL)
                fail(UGKWP_EPOOL, "particle pool capacity %lld exceeded (%lld alive + %lld births)",
                     (long long)P.pool_capacity, (long long)s.counters[CNT_SLOTS], (long long)s.total[0]);
            if (err & ERR_TEMP) fail(UGKWP_ENONFINITE, "source iteration produced a non-positive or non-finite temperature");
            if (err) fail(UGKWP_EHIP, "internal error %llu: particle records or survivor counts inconsistent", err);
            if (s.counters[CNT_DONE] == (unsigned long long)p.step + 1) return s;
            if (s.counters[CNT_DONE] != 0)
                fail(UGKWP_EHIP, "internal error: step %u recorded as step %llu", p.step, s.counters[CNT_DONE]);
            if (s.counters[CNT_CONV] == (unsigned long long)n_inst)
                fail(UGKWP_EHIP, "internal error: converged step %u not committed", p.step);
            if (p.sweeps >= kmax) fail(UGKWP_ENOCONV, "source iteration did not converge in %d sweeps", kmax);
            const int kend = std::min(p.sweeps + 4, kmax);
            {
                GateScope gs(K, use_graph ? GATE_OFF : p.step);
                enqueue_sweeps(p.sweeps, kend);
                p.sweeps = kend;
                if (phase_times) HIPCHK(hipEventRecord(sev[cur_slot][4], st));
                enqueue_finish(p.do_sort, rec_cap > 0 ? p.nrec : -1, kend - 1);
            }
            HIPCHK(hipMemcpyAsync(h_status, D.counters, status_bytes, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            s = status_at((const char*)h_status);
        }
    }

    // bookkeeping of committed step p from its status block
    void account(const Plan& p, const StatusView& s)
    {
        ugkwp_diag dg{};
        dg.n_alive_in = n_alive;
        dg.n_births = s.total[0];
        dg.n_pushed = n_alive + s.total[0];
        dg.n_alive_out = (int64_t)s.counters[CNT_SURV];
        int smax = 0, ssum = 0;
        int64_t cgu = 0;
        for (int q = 0; q < n_inst; ++q) {
            ids_used = std::max(ids_used, (uint64_t)s.ist[q].births);
            smax = std::max(smax, s.ist[q].conv_sweeps);
            ssum += s.ist[q].conv_sweeps;
            cgu += (int64_t)s.ist[q].conv_sweeps * inst[q].ncell * inst[q].G;
            double fold[8];
            const double* g = s.diag + 8 * q;
            if (host_diag) {
                // the same order as the device reduction: sub-slot 0, 1, ...
                for (int c = 0; c < 8; ++c) {
                    double acc = 0.0;
                    for (int b = 0; b < DIAG_SUB; ++b) acc += s.sub[((size_t)q * DIAG_SUB + b) * 8 + c];
                    fold[c] = acc;
                }
                g = fold;
            }
            dg.inflow_wave += g[0];
            dg.inflow_eq += g[1];
            dg.exit_particles += g[2];
            dg.injection += g[3];
            dg.e_start += g[4];
            dg.e_end += g[5];
            dg.inflow_particles += g[6];
        }
        dg.sweeps_max = smax;
        dg.sweeps_sum = ssum;
        dg.residual = dg.e_end - dg.e_start -
                      (dg.inflow_wave + dg.inflow_eq + dg.inflow_particles - dg.exit_particles + dg.injection);
        hipEvent_t* e = sev[cur_slot];
        float ms = 0;
        dg.push_timed = p.push_timed ? 1 : 0;
        if (p.push_timed) { HIPCHK(hipEventElapsedTime(&ms, e[1], e[2])); dg.ms_push = ms; }
        if (phase_times) {
            HIPCHK(hipEventElapsedTime(&ms, e[0], e[1])); dg.ms_sample = ms;
            HIPCHK(hipEventElapsedTime(&ms, e[2], e[3])); dg.ms_macro = ms;
            HIPCHK(hipEventElapsedTime(&ms, e[3], e[4])); dg.ms_si = ms;
        }
        dg.ms_sort = 0.0;
        if (p.do_sort && phase_times) { HIPCHK(hipEventElapsedTime(&ms, e[5], e[6])); dg.ms_sort = ms; }
        diag = dg;
        tot.steps += 1;
        tot.n_pushed += dg.n_pushed;
        tot.n_survived += dg.n_alive_out;
        tot.sweeps_max += dg.sweeps_max;
        tot.sweeps_sum += dg.sweeps_sum;
        tot.cg_updates += cgu;
        tot.ms_sample += dg.ms_sample;
        tot.ms_push += dg.ms_push;
        if (p.push_timed) {
            tot.push_timed += 1;
            tot.n_pushed_timed += dg.n_pushed;
            tot.n_survived_timed += dg.n_alive_out;
        }
        tot.ms_macro += dg.ms_macro;
        tot.ms_si += dg.ms_si;
        tot.ms_sort += dg.ms_sort;
        if (rec_cap > 0) rec_sweeps.push_back(smax);
        n_alive = dg.n_alive_out;
        last_births = dg.n_births;
        // slots after the step: compacted to the survivors by a sort, else
        // every slot the push covered
        set_state(after(p, p.do_sort ? dg.n_alive_out : (int64_t)s.counters[CNT_PUSHED]));
    }

    void run(int nsteps)
    {
        int done = 0;
        while (done < nsteps) {
            if (rec_cap > 0 && nrec >= rec_cap)
                fail(UGKWP_EINVAL, "the record holds its maximum of %d steps", rec_cap);
            int m = std::min(nsteps - done, use_graph ? 1 : RUN_AHEAD);
            if (rec_cap > 0) m = std::min(m, rec_cap - nrec);
            // particle ids share their word with the group: a batch may not
            // number births past 2^ID_BITS (each step births fewer than the capacity)
            if (ids_used + (uint64_t)m * (uint64_t)P.pool_capacity > ID_MASK)
                fail(UGKWP_EPOOL, "particle ids would pass 2^%d", ID_BITS);
            const int kmax = P.si_max_iters;
            const int spec = std::min(kmax, last_sweeps + 1);
            // plan and enqueue
            const Plan start = state_now();
            std::vector<Plan> plan;
            plan.reserve(m);
            Plan p = start;
            try {
                for (int i = 0; i < m; ++i) {
                    p.do_sort = sort_due(p.step, p.n_slots);
                    p.push_timed = phase_times || p.step % push_time_every == 0;
                    p.sweeps = spec;
                    p.slot = next_record(p.rec);
                    set_state(p);
                    cur_slot = i;
                    enqueue_step(p);
                    plan.push_back(p);
                    p = after(p, p.do_sort ? n_alive : p.n_slots + last_births);
                }
                HIPCHK(hipMemcpyAsync(h_ring, d_ring, ring_stride * N_RECORDS, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
            } catch (...) {
                (void)hipStreamSynchronize(st);
                set_state(start);
                throw;
            }
            // read the records in order
            set_state(start);
            int batch_max = 0;
            for (int i = 0; i < m; ++i) {
                Plan& q = plan[i];
                cur_slot = i;
                StatusView s = status_at(h_ring + (size_t)q.slot * ring_stride);
                const bool committed =
                    s.counters[CNT_DONE] == (unsigned long long)q.step + 1 && s.counters[CNT_ERR] == 0;
                if (!committed) {
                    const Plan before = state_now();
                    try {
                        s = take_up(q, s);
                    } catch (...) {
                        set_state(before);
                        throw;
                    }
                }
                account(q, s);
                batch_max = std::max(batch_max, diag.sweeps_max);
                done++;
                if (!committed) break;      // later steps of the batch did not run: plan again
            }
            last_sweeps = batch_max;
        }
    }

    // ---------------------------------------------------------------- autotuner
    static constexpr double TUNE_MARGIN = 0.97;
    // Times the push on the committed pool for a grid of launch shapes and keeps
    // the fastest.  The tallies and counters the trial pushes touch are saved
    // and restored; only the launch shape (hence speed) changes.
    void autotune(ugkwp_tune_result* res)
    {
        if (n_slots == 0) fail(UGKWP_EINVAL, "the particle pool is empty: step the context before tuning");
        std::vector<unsigned long long> cnt(N_COUNTERS);
        HIPCHK(hipMemcpyAsync(cnt.data(), D.counters, sizeof(unsigned long long) * N_COUNTERS,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<unsigned long long> trial = cnt;
        trial[CNT_PUSHED] = trial[CNT_SLOTS];
        trial[CNT_ERR] = 0;
        // save what the trial pushes add to
        struct Saved { void* dev; void* copy; size_t bytes; };
        std::vector<Saved> saved;
        auto keep = [&](void* p, size_t bytes) {
            if (!p || bytes == 0) return;
            void* c = nullptr;
            if (hipMalloc(&c, bytes) != hipSuccess) fail(UGKWP_ENOMEM, "autotune: no room to save the tallies");
            saved.push_back({p, c, bytes});
            HIPCHK(hipMemcpyAsync(c, p, bytes, hipMemcpyDeviceToDevice, st));
        };
        struct Release {
            std::vector<Saved>& v;
            ~Release() { for (auto& q : v) (void)hipFree(q.copy); }
        } release{saved};
        keep(D.dep, sizeof(double) * K.n_cg);
        keep(D.surv, sizeof(double) * K.n_cg);
        keep(D.scount, sizeof(uint32_t) * K.n_cg);
        keep(D.ftx, sizeof(double) * 2 * n_fx);
        if (dim == 2) keep(D.fty, sizeof(double) * 2 * n_fy);
        HIPCHK(hipMemcpyAsync(D.counters, trial.data(), sizeof(unsigned long long) * N_COUNTERS,
                              hipMemcpyHostToDevice, st));
        const int ncu = push_num_cus();
        std::vector<PushShape> cand;
        // 256 and 512 threads per block: blocks of 128 tuned well on one pool but
        // ran ~10% slower than their tuning time over the following steps
        for (int threads : {256, 512}) {
            const int occ = std::max(1, push_blocks_per_cu(dim, K, threads));
            for (int ppt : {1, 2, 4, 8})
                for (int bpc : {std::max(1, occ / 2), occ, 2 * occ}) {
                    const PushShape c{std::min(bpc * ncu, MAX_PUSH_BLOCKS), ppt, threads};
                    bool dup = false;
                    for (const auto& q : cand)
                        dup = dup || (q.blocks == c.blocks && q.ppt == c.ppt && q.threads == c.threads);
                    if (!dup) cand.push_back(c);
                }
        }
        PushShape def = push_default_shape(dim, K);
        def.blocks = std::min(def.blocks, MAX_PUSH_BLOCKS);
        auto time_push = [&](const PushShape& sh) {
            const Pool In = view(cur_mv, cur_st), Out = moving(1 - cur_mv);
            launch_push(dim, D, K, In, Out, sh, st);           // warm-up
            float best = 1e30f;
            for (int r = 0; r < 3; ++r) {
                HIPCHK(hipEventRecord(ev[0], st));
                launch_push(dim, D, K, In, Out, sh, st);
                HIPCHK(hipEventRecord(ev[1], st));
                HIPCHK(hipEventSynchronize(ev[1]));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
                best = std::min(best, ms);
            }
            return 1e3 * (double)best;
        };
        double us_def = time_push(def);
        PushShape best = def;
        double us_best = 1e300;
        for (const auto& c : cand) {
            const double us = time_push(c);
            if (us < us_best) { us_best = us; best = c; }
        }
        // The default is timed again after the candidates (its first timing runs
        // on colder caches: the same shape among the candidates came out up to 5%
        // faster), and a candidate replaces it only when at least 3% faster: smaller
        // leads on the tuning pool did not hold over the steps that followed.
        us_def = std::min(us_def, time_push(def));
        if (!(us_best < TUNE_MARGIN * us_def)) {
            best = def;
            us_best = us_def;
        }
        // restore
        for (auto& q : saved) HIPCHK(hipMemcpyAsync(q.dev, q.copy, q.bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(D.counters, cnt.data(), sizeof(unsigned long long) * N_COUNTERS,
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        push_shape = best;
        drop_graphs();
        if (res) {
            res->ppt = best.ppt;
            res->threads = best.threads;
            res->blocks = best.blocks;
            res->candidates = (int)cand.size();
            res->us_best = us_best;
            res->us_default = us_def;
        }
    }

    // ---------------------------------------------------------------- adjoint
    template <class T>
    T* ralloc(size_t n)
    {
        void* p = nullptr;
        if (n == 0) n = 1;
        if (hipMalloc(&p, n * sizeof(T)) != hipSuccess)
            fail(UGKWP_ENOMEM, "hipMalloc of %zu bytes for the record failed", n * sizeof(T));
        rec_owned.push_back(p);
        return (T*)p;
    }

    void record_start(int max_steps)
    {
        free_record();
        if (max_steps <= 0) return;
        const size_t ncg = (size_t)K.n_cg, nc = (size_t)ncell;
        const size_t nfx = (size_t)std::max<int64_t>(n_fx, 1), nfy = (size_t)std::max<int64_t>(n_fy, 1);
        A.rQ = ralloc<double>(ncg * max_steps);
        A.rRhoh = ralloc<double>(ncg * max_steps);
        A.rSamp = ralloc<uint8_t>(ncg * max_steps);
        A.rT = ralloc<double>(nc * max_steps);
        A.phi = ralloc<double>(ncg);
        A.dphi = ralloc<double>(ncg);
        A.rbar = ralloc<double>(ncg);
        A.rbar_next = ralloc<double>(ncg);
        A.mu0 = ralloc<double>(nc);
        A.mu1 = ralloc<double>(nc);
        A.Tbar = ralloc<double>(nc);
        A.grad = ralloc<double>(ncg);
        A.c4d = ralloc<double>(ncg);
        A.wd = ralloc<double>(ncg);
        A.Dlx = ralloc<double>(nfx);
        A.Dhx = ralloc<double>(nfx);
        A.Dly = ralloc<double>(nfy);
        A.Dhy = ralloc<double>(nfy);
        A.res = ralloc<AdjResid>((size_t)n_inst * RES_SLOTS * RES_SUB);
        A.conv = ralloc<int>((size_t)n_inst);
        A.stepk = ralloc<int>((size_t)max_steps);
        A.status = ralloc<unsigned long long>(ADJ_N_STATUS);
        if (!h_adj) HIPCHK(hipHostMalloc((void**)&h_adj, sizeof(unsigned long long) * ADJ_N_STATUS, hipHostMallocDefault));
        rec_cap = max_steps;
        nrec = 0;
        rec_sweeps.clear();
    }

    void adjoint(const double* dJdT, double* grad, bool dev, ugkwp_adjoint_stats* stats)
    {
        if (rec_cap == 0 || nrec == 0) fail(UGKWP_EINVAL, "no recorded steps (ugkwp_record before ugkwp_step)");
        if (!dJdT || !grad) fail(UGKWP_EINVAL, "null array");
        if (!dev)
            for (int c = 0; c < ncell; ++c)
                if (!std::isfinite(dJdT[c])) fail(UGKWP_EINVAL, "dJdT must be finite");
        HIPCHK(hipEventRecord(ev[0], st));
        HIPCHK(hipMemcpyAsync(A.Tbar, dJdT, sizeof(double) * ncell,
                              dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
        HIPCHK(hipMemsetAsync(A.rbar, 0, sizeof(double) * K.n_cg, st));
        HIPCHK(hipMemsetAsync(A.grad, 0, sizeof(double) * K.n_cg, st));
        HIPCHK(hipMemsetAsync(A.conv, 0, sizeof(int) * n_inst, st));
        launch_adj_coef(D, K, A, st);
        for (int q = 0; q < n_inst; ++q) {
            const Inst& I = inst[q];
            launch_adj_face(D, K, A, q, 0, (int64_t)(I.nx + 1) * I.ny * I.Gp, st);
            if (dim == 2) launch_adj_face(D, K, A, q, 1, (int64_t)I.nx * (I.ny + 1) * I.Gp, st);
        }
        // Reverse steps q = 0, 1, ... (recorded step r = nrec - 1 - q) are enqueued
        // RUN_AHEAD at a time with q as their gate; each launches the sweeps the
        // most demanding step so far needed plus one.  One synchronisation per
        // batch reads how many completed; a step that did not converge is taken
        // up alone (more sweeps) and the next batch starts after it.
        const int kmax = 1000;
        HIPCHK(hipMemsetAsync(A.status, 0, sizeof(unsigned long long) * ADJ_N_STATUS, st));
        int sweeps_sum = 0, sweeps_max = 0;
        double ms_sweeps = 0.0;
        int last = rec_sweeps[nrec - 1];    // first guess: the forward's last step
        std::vector<int> hk(RUN_AHEAD);
        auto sweep_ms = [&](hipEvent_t a, hipEvent_t b) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, a, b));
            return (double)ms;
        };
        int done = 0;
        while (done < nrec) {
            const int m = std::min(RUN_AHEAD, nrec - done);
            const int spec = std::min(kmax, last + 1);
            double* const rbar0 = A.rbar;
            double* const rbar1 = A.rbar_next;
            for (int i = 0; i < m; ++i) {
                const uint32_t q = (uint32_t)(done + i);
                const int r = nrec - 1 - (int)q;
                launch_adj_prep(D, K, A, r, q, st);
                HIPCHK(hipEventRecord(sev[i][0], st));
                launch_adj_sweeps(D, K, A, 0, spec, r, q, st);
                HIPCHK(hipEventRecord(sev[i][1], st));
                launch_adj_grad(D, K, A, r, q, spec - 1, st);
                std::swap(A.rbar, A.rbar_next);
            }
            const int r_lo = nrec - done - m;    // recorded steps r_lo .. nrec-1-done
            HIPCHK(hipMemcpyAsync(h_adj, A.status, sizeof(unsigned long long) * ADJ_N_STATUS,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(hk.data(), A.stepk + r_lo, sizeof(int) * m, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int committed = (int)h_adj[ADJ_DONE] - done;
            int batch_max = 0;
            for (int i = 0; i < committed; ++i) {
                const int kneed = hk[m - 1 - i];
                ms_sweeps += sweep_ms(sev[i][0], sev[i][1]);
                sweeps_sum += spec;
                sweeps_max = std::max(sweeps_max, kneed);
                batch_max = std::max(batch_max, kneed);
            }
            done += committed;
            if (committed < m) {
                // reverse step q = done did not complete: its rbar parity, then more sweeps
                const uint32_t q = (uint32_t)done;
                const int r = nrec - 1 - done;
                if (committed & 1) { A.rbar = rbar1; A.rbar_next = rbar0; }
                else { A.rbar = rbar0; A.rbar_next = rbar1; }
                double ms = sweep_ms(sev[committed][0], sev[committed][1]);
                int k = spec;
                for (;;) {
                    if (h_adj[ADJ_ERR]) fail(UGKWP_ENONFINITE, "adjoint of step %d produced a non-finite value", r);
                    if (h_adj[ADJ_CONV] == (unsigned long long)n_inst) break;
                    if (k >= kmax) fail(UGKWP_ENOCONV, "transposed source iteration of step %d did not converge", r);
                    const int kend = std::min(k + 4, kmax);
                    HIPCHK(hipEventRecord(ev[2], st));
                    launch_adj_sweeps(D, K, A, k, kend, r, q, st);
                    launch_adj_decide(D, K, A, kend - 1, r, q, st);
                    HIPCHK(hipEventRecord(ev[3], st));
                    k = kend;
                    HIPCHK(hipMemcpyAsync(h_adj, A.status, sizeof(unsigned long long) * ADJ_N_STATUS,
                                          hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    ms += sweep_ms(ev[2], ev[3]);
                }
                launch_adj_grad(D, K, A, r, q, -1, st);
                std::swap(A.rbar, A.rbar_next);
                int kneed = 0;
                HIPCHK(hipMemcpyAsync(h_adj, A.status, sizeof(unsigned long long) * ADJ_N_STATUS,
                                      hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(&kneed, A.stepk + r, sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                if (h_adj[ADJ_DONE] != (unsigned long long)done + 1)
                    fail(UGKWP_EHIP, "internal error: reverse step %d not completed", r);
                ms_sweeps += ms;
                sweeps_sum += k;
                sweeps_max = std::max(sweeps_max, kneed);
                batch_max = std::max(batch_max, kneed);
                done += 1;
            }
            last = batch_max;
        }
        const long long cg_updates = (long long)h_adj[ADJ_CGU];
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        int64_t out = 0;
        for (int q = 0; q < n_inst; ++q) {
            const Inst& I = inst[q];
            copy_rows(grad + out, sizeof(double) * I.G, A.grad + I.cg_off, sizeof(double) * I.Gp,
                      sizeof(double) * I.G, I.ncell, kind, st);
            out += (int64_t)I.ncell * I.G;
        }
        HIPCHK(hipEventRecord(ev[1], st));
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipGetLastError());
        if (stats) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
            stats->steps = nrec;
            stats->sweeps_launched = sweeps_sum;
            stats->sweeps_max = sweeps_max;
            stats->ms = ms;
            stats->ms_sweeps = ms_sweeps;
            stats->cell_group_updates = cg_updates;
        }
    }

};

// ---------------------------------------------------------------------------
// C ABI

namespace {

template <class F>
int guarded(ugkwp_ctx* c, F&& f)
{
    try {
        f();
        if (c) c->err.clear();
        return UGKWP_OK;
    } catch (const ApiError& e) {
        if (c) c->err = e.msg;
        return e.code;
    } catch (const HipError& e) {
        if (c) c->err = std::string(e.what) + ": " + hipGetErrorString(e.e);
        return UGKWP_EHIP;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return UGKWP_ENOMEM;
    }
}

void require_ready(const ugkwp_ctx* c)
{
    if (c->n_inst == 0) fail(UGKWP_EINVAL, "mesh not initialised");
    if (!c->have_opacity) fail(UGKWP_EINVAL, "opacity not set");
    if (!c->have_material) fail(UGKWP_EINVAL, "material not set");
}

void check_inst(const ugkwp_ctx* c, int k)
{
    if (c->n_inst == 0) fail(UGKWP_EINVAL, "mesh not initialised");
    if (k < 0 || k >= c->n_inst) fail(UGKWP_EINVAL, "instance %d out of range", k);
}

}  // namespace

namespace {
struct Tmp {
    std::vector<void*> p;
    ~Tmp() { for (void* q : p) (void)hipFree(q); }
    template <class T>
    T* up(const T* h, size_t n)
    {
        void* d = nullptr;
        HIPCHK(hipMalloc(&d, std::max<size_t>(n, 1) * sizeof(T)));
        p.push_back(d);
        if (h && n) HIPCHK(hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice));
        return (T*)d;
    }
};
}  // namespace

// ---- checkpoint ----
//
// A saved state is one host buffer: a header, then in the device's padded
// layout rho^n, the survivor density, phi(T^n) and T^n, the per-instance birth
// counters, and the pool's slots as they sit in the device buffers (holes and
// pending reflections included), so that the restored context continues with
// the same particles in the same order.  Every section starts on an 8-byte
// boundary.

namespace {

constexpr char STATE_MAGIC[8] = {'U', 'G', 'K', 'W', 'P', 'S', 'T', '1'};
constexpr uint32_t STATE_VERSION = 2;     // 2: the group word travels in the id word

struct StateHeader {
    char magic[8];
    uint64_t layout;       // fingerprint of mesh, groups, instances and constants
    int32_t dim, n_inst, ncell;
    uint32_t step;
    int64_t n_cg, n_slots, n_alive, bytes;
    uint32_t version, pad;
};

// FNV-1a over the values that fix the meaning of every saved array
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    template <class T>
    void add(const T& v)
    {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
        for (size_t i = 0; i < sizeof(T); ++i) h = (h ^ b[i]) * 1099511628211ull;
    }
};

uint64_t state_layout(const ugkwp_ctx* c)
{
    Fnv f;
    f.add(c->dim);
    f.add(c->n_inst);
    f.add(c->K.c); f.add(c->K.a); f.add(c->K.eps); f.add(c->K.dt); f.add(c->K.nu_power);
    f.add(c->K.flags);
    f.add(c->K.tau_C); f.add(c->K.tau_jump); f.add(c->K.t_power); f.add(c->K.stim);
    f.add(c->K.olson); f.add(c->K.table); f.add(c->K.has_src);
    for (const HostInst& h : c->hi) {
        f.add(h.nx); f.add(h.ny); f.add(h.G);
        f.add(h.x0); f.add(h.x1); f.add(h.y0); f.add(h.y1);
        for (int q = 0; q < 4; ++q) { f.add(h.bc[q]); f.add(h.bcT[q]); }
        for (double e : h.edges) f.add(e);
        f.add(h.seed); f.add(h.w_ref);
    }
    return f.h;
}

// byte offsets of the sections of a saved state
struct StateLayout {
    size_t rho, rhop, phi0, T, births, x, y, ox, oy, nu, w, id, cell, end;
};

size_t up8(size_t b) { return (b + 7) / 8 * 8; }

StateLayout state_sections(const ugkwp_ctx* c, int64_t n_slots)
{
    StateLayout L{};
    const size_t ncg = (size_t)c->K.n_cg, ns = (size_t)n_slots, d2 = c->dim == 2 ? 1 : 0;
    size_t o = up8(sizeof(StateHeader));
    L.rho = o;    o += 8 * ncg;
    L.rhop = o;   o += 8 * ncg;
    L.phi0 = o;   o += 8 * ncg;
    L.T = o;      o += 8 * (size_t)c->ncell;
    L.births = o; o += 8 * (size_t)c->n_inst;
    L.x = o;      o += 8 * ns;
    L.y = o;      o += 8 * ns * d2;
    L.ox = o;     o += 8 * ns;
    L.oy = o;     o += 8 * ns * d2;
    L.nu = o;     o += 8 * ns;
    L.w = o;      o += 8 * ns;
    L.id = o;     o += 8 * ns;
    L.cell = o;   o += up8(4 * ns);
    L.end = o;
    return L;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Scratch of the allocation-free set-up call (ugkwp_set_material_noalloc): the
// device staging of Tr0, which ugkwp_set_material allocates per call.  One
// array per GPU, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not a device address: its device address on each GPU is
// taken once with hipGetSymbolAddress (with that GPU current) and only that
// address is used.
namespace {
constexpr size_t NOALLOC_MAX_CELLS = size_t(1) << 21;     // 16 MiB of doubles
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_MAX_CELLS];
std::mutex scratch_mu;
double* scratch_dev[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on GPU `dev`, which must be current.
double* scratch_address(int dev)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(UGKWP_EINVAL, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(UGKWP_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        scratch_dev[dev] = (double*)ptr;
    }
    return scratch_dev[dev];
}

// Makes the context's GPU current for the enclosing scope.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        HIPCHK(hipGetDevice(&prev));
        if (prev != dev) HIPCHK(hipSetDevice(dev));
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

int ugkwp_set_material_noalloc(ugkwp_ctx* ctx, const double* cv, const double* T0, const double* Tr0,
                               const uint8_t* pinned)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (ctx->n_inst != 1) fail(UGKWP_EINVAL, "set_material_noalloc needs a single-instance context");
        if (!cv || !T0 || !Tr0) fail(UGKWP_EINVAL, "null argument");
        if ((size_t)ctx->ncell > NOALLOC_MAX_CELLS)
            fail(UGKWP_EINVAL, "set_material_noalloc: %d cells exceed its scratch of %zu cells", ctx->ncell,
                 NOALLOC_MAX_CELLS);
        DeviceScope on(ctx->device);
        ctx->set_material({cv}, {T0}, {Tr0}, {pinned}, scratch_address(ctx->device));
    });
}

int ugkwp_create(ugkwp_ctx** out, const ugkwp_params* p, void* hip_stream)
{
    if (!out || !p) return UGKWP_EINVAL;
    *out = nullptr;
    if (!(p->c > 0) || !(p->a > 0) || !(p->eps > 0) || !(p->dt > 0) || !std::isfinite(p->dt) ||
        !(p->si_tol >= 0) || p->si_max_iters < 1 || p->pool_capacity < 0 || p->pool_capacity > (1ll << 29) ||
        p->n_cap < 0 ||
        p->n_cap > (1 << 30) || !(p->nu_power >= 0) || p->sort_interval < 0 ||
        !(p->tau_num_C >= 0) || !std::isfinite(p->tau_num_C) || !(p->tau_num_jump >= 0) ||
        !std::isfinite(p->opacity_T_power) || (p->opacity_stim != 0 && p->opacity_stim != 1))
        return UGKWP_EINVAL;
    ugkwp_ctx* c = new (std::nothrow) ugkwp_ctx();
    if (!c) return UGKWP_ENOMEM;
    c->P = *p;
    int rc = guarded(c, [&] {
        HIPCHK(hipGetDevice(&c->device));
        // the allocation-free set-up call's scratch address on this GPU, taken once
        (void)scratch_address(c->device);
        if (hip_stream) c->st = (hipStream_t)hip_stream;
        else {
            HIPCHK(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking));
            c->own_stream = true;
        }
        c->sort_interval = p->sort_interval;
        c->use_graph = (p->flags & UGKWP_FLAG_GRAPH) != 0;
        c->phase_times = (p->flags & UGKWP_FLAG_PHASE_TIMES) != 0;
        // timing-only events: no system-scope fence (cache write-back) when recorded
        for (auto& e : c->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        for (auto& row : c->sev)
            for (auto& e : row) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    });
    if (rc) { delete c; return rc; }
    *out = c;
    return UGKWP_OK;
}

void ugkwp_destroy(ugkwp_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->st) (void)hipStreamSynchronize(ctx->st);
    delete ctx;
}

const char* ugkwp_last_error(const ugkwp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ugkwp_init_mesh(ugkwp_ctx* ctx, int dim, int nx, int ny, const double lo[2], const double hi[2],
                    const int bc[4], const double bcT[4], int G, const double* nu_edges, uint64_t seed,
                    double w_ref)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (!lo || !hi || !bc || !bcT || !nu_edges) fail(UGKWP_EINVAL, "null argument");
        if (G < 1 || G > MAX_G) fail(UGKWP_EINVAL, "G must be in 1..%d", MAX_G);
        HostInst h;
        h.dim = dim; h.nx = nx; h.ny = dim == 1 ? 1 : ny;
        if (dim == 1 && ny != 1) fail(UGKWP_EINVAL, "ny must be 1 in 1-D");
        h.x0 = lo[0]; h.x1 = hi[0]; h.y0 = lo[1]; h.y1 = hi[1];
        for (int q = 0; q < 4; ++q) { h.bc[q] = bc[q]; h.bcT[q] = bcT[q]; }
        h.G = G;
        h.edges.assign(nu_edges, nu_edges + G + 1);
        h.seed = seed;
        h.w_ref = w_ref;
        ctx->setup({h});
    });
}

int ugkwp_set_opacity(ugkwp_ctx* ctx, const double* kappa)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (ctx->n_inst != 1) fail(UGKWP_EINVAL, "set_opacity needs a single-instance context");
        if (!kappa) fail(UGKWP_EINVAL, "null kappa");
        ctx->set_opacity({kappa});
    });
}

int ugkwp_set_material(ugkwp_ctx* ctx, const double* cv, const double* T0, const double* Tr0,
                       const uint8_t* pinned)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (ctx->n_inst != 1) fail(UGKWP_EINVAL, "set_material needs a single-instance context");
        if (!cv || !T0 || !Tr0) fail(UGKWP_EINVAL, "null argument");
        ctx->set_material({cv}, {T0}, {Tr0}, {pinned});
    });
}

int ugkwp_set_heat_capacity(ugkwp_ctx* ctx, const double* H, const double* chi)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->have_material) fail(UGKWP_EINVAL, "set_heat_capacity needs the mesh and material first");
        ctx->set_heat_capacity(H, chi);
    });
}

int ugkwp_set_source(ugkwp_ctx* ctx, const double* q, double t_off)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->have_material) fail(UGKWP_EINVAL, "set_source needs the mesh and material first");
        ctx->set_source(q, nullptr, 0.0, t_off);
    });
}

int ugkwp_set_source_planck(ugkwp_ctx* ctx, const double* f, double Ts, double t_off)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->have_material) fail(UGKWP_EINVAL, "set_source_planck needs the mesh and material first");
        ctx->set_source(nullptr, f, Ts, t_off);
    });
}

int ugkwp_set_opacity_table(ugkwp_ctx* ctx, int nmat, const int32_t* mat, int nnu, const double* nu, int nT,
                            const double* T, const double* sig)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->have_material) fail(UGKWP_EINVAL, "set_opacity_table needs the mesh and material first");
        ctx->set_opacity_table(nmat, mat, nnu, nu, nT, T, sig);
    });
}

int ugkwp_init_batch(ugkwp_ctx* ctx, int n_inst, const ugkwp_instance* d)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (n_inst < 1 || !d) fail(UGKWP_EINVAL, "need at least one instance");
        std::vector<HostInst> hs(n_inst);
        std::vector<const double*> kap(n_inst), cv(n_inst), T0(n_inst), Tr0(n_inst);
        std::vector<const uint8_t*> pin(n_inst);
        for (int k = 0; k < n_inst; ++k) {
            const ugkwp_instance& s = d[k];
            if (!s.nu_edges || !s.kappa || !s.cv || !s.T0 || !s.Tr0) fail(UGKWP_EINVAL, "instance %d: null array", k);
            if (s.G < 1 || s.G > MAX_G) fail(UGKWP_EINVAL, "instance %d: G must be in 1..%d", k, MAX_G);
            HostInst& h = hs[k];
            h.dim = s.dim; h.nx = s.nx; h.ny = s.dim == 1 ? 1 : s.ny;
            if (s.dim == 1 && s.ny != 1) fail(UGKWP_EINVAL, "instance %d: ny must be 1 in 1-D", k);
            h.x0 = s.x0; h.x1 = s.x1; h.y0 = s.y0; h.y1 = s.y1;
            for (int q = 0; q < 4; ++q) { h.bc[q] = s.bc[q]; h.bcT[q] = s.bcT[q]; }
            h.G = s.G;
            h.edges.assign(s.nu_edges, s.nu_edges + s.G + 1);
            h.seed = s.seed;
            h.w_ref = s.w_ref;
            kap[k] = s.kappa; cv[k] = s.cv; T0[k] = s.T0; Tr0[k] = s.Tr0; pin[k] = s.pinned;
        }
        ctx->setup(hs);
        ctx->set_opacity(kap);
        ctx->set_material(cv, T0, Tr0, pin);
    });
}

int ugkwp_step(ugkwp_ctx* ctx, int nsteps)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        if (nsteps < 0) fail(UGKWP_EINVAL, "negative step count");
        ctx->run(nsteps);
    });
}

int ugkwp_record(ugkwp_ctx* ctx, int max_steps)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (max_steps < 0) fail(UGKWP_EINVAL, "negative record size");
        if (max_steps > 0) require_ready(ctx);
        if (max_steps > 0 && ctx->P.tau_num_C > 0)
            fail(UGKWP_EINVAL, "the adjoint does not cover the numerical collision time of joint cells (tau_num_C > 0)");
        if (max_steps > 0 && (ctx->P.opacity_T_power != 0 || ctx->P.opacity_stim))
            fail(UGKWP_EINVAL, "the adjoint does not cover a temperature-dependent opacity");
        if (max_steps > 0 && (ctx->P.flags & (UGKWP_FLAG_SLOPES | UGKWP_FLAG_WAVE_ITER | UGKWP_FLAG_BOUNDARY_PARTICLES)))
            fail(UGKWP_EINVAL, "the adjoint covers neither the slopes of the wave part, its flux from the iterate, "
                               "nor boundary-source particles");
        if (max_steps > 0 && (ctx->K.olson || ctx->K.table || ctx->K.has_src))
            fail(UGKWP_EINVAL, "the adjoint covers neither Olson's heat capacity, a tabulated opacity nor a volumetric source");
        ctx->record_start(max_steps);
    });
}

int ugkwp_recorded_steps(const ugkwp_ctx* ctx) { return ctx ? ctx->nrec : 0; }

int ugkwp_autotune(ugkwp_ctx* ctx, ugkwp_tune_result* res)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        ctx->autotune(res);
    });
}

int ugkwp_adjoint(ugkwp_ctx* ctx, const double* dJdT, double* grad_kappa, int ptrs_are_device,
                  ugkwp_adjoint_stats* stats)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        ctx->adjoint(dJdT, grad_kappa, ptrs_are_device != 0, stats);
    });
}

int ugkwp_num_instances(const ugkwp_ctx* ctx) { return ctx ? ctx->n_inst : 0; }

int ugkwp_get_fields(ugkwp_ctx* ctx, int inst, double* rho, double* T, double* rhop, int dst_is_device)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (ctx->n_inst == 0) fail(UGKWP_EINVAL, "mesh not initialised");
        const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        const int k0 = inst < 0 ? 0 : inst, k1 = inst < 0 ? ctx->n_inst : inst + 1;
        if (inst >= ctx->n_inst) fail(UGKWP_EINVAL, "instance %d out of range", inst);
        int64_t cg_out = 0, cell_out = 0;
        for (int k = k0; k < k1; ++k) {
            const Inst& I = ctx->inst[k];
            if (rho)
                copy_rows(rho + cg_out, sizeof(double) * I.G, ctx->D.rho + I.cg_off, sizeof(double) * I.Gp,
                          sizeof(double) * I.G, I.ncell, kind, ctx->st);
            if (rhop)
                copy_rows(rhop + cg_out, sizeof(double) * I.G, ctx->D.rhop + I.cg_off, sizeof(double) * I.Gp,
                          sizeof(double) * I.G, I.ncell, kind, ctx->st);
            if (T)
                HIPCHK(hipMemcpyAsync(T + cell_out, ctx->D.T + I.cell_off, sizeof(double) * I.ncell, kind, ctx->st));
            cg_out += (int64_t)I.ncell * I.G;
            cell_out += I.ncell;
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
    });
}

int ugkwp_get_tallies(ugkwp_ctx* ctx, int inst, double* fx, double* fy, double* dep, double* surv,
                      int64_t* nbirth, double* wnew, double* Q)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        check_inst(ctx, inst);
        const Inst& I = ctx->inst[inst];
        const hipMemcpyKind kind = hipMemcpyDeviceToHost;
        hipStream_t st = ctx->st;
        const size_t G = I.G, Gp = I.Gp;
        if (fx)
            copy_rows(fx, sizeof(double) * 2 * G, ctx->D.ftx + 2 * I.fx_off, sizeof(double) * 2 * Gp,
                      sizeof(double) * 2 * G, (size_t)(I.nx + 1) * I.ny, kind, st);
        if (fy && I.dim == 2)
            copy_rows(fy, sizeof(double) * 2 * G, ctx->D.fty + 2 * I.fy_off, sizeof(double) * 2 * Gp,
                      sizeof(double) * 2 * G, (size_t)I.nx * (I.ny + 1), kind, st);
        if (dep) copy_rows(dep, sizeof(double) * G, ctx->D.dep + I.cg_off, sizeof(double) * Gp, sizeof(double) * G, I.ncell, kind, st);
        if (surv) copy_rows(surv, sizeof(double) * G, ctx->D.surv + I.cg_off, sizeof(double) * Gp, sizeof(double) * G, I.ncell, kind, st);
        if (wnew) copy_rows(wnew, sizeof(double) * G, ctx->D.wnew + I.cg_off, sizeof(double) * Gp, sizeof(double) * G, I.ncell, kind, st);
        if (Q) copy_rows(Q, sizeof(double) * G, ctx->D.Q + I.cg_off, sizeof(double) * Gp, sizeof(double) * G, I.ncell, kind, st);
        std::vector<int32_t> nb;
        if (nbirth) {
            nb.resize((size_t)I.ncell * G);
            copy_rows(nb.data(), sizeof(int32_t) * G, ctx->D.nb + I.cg_off, sizeof(int32_t) * Gp, sizeof(int32_t) * G,
                      I.ncell, kind, st);
        }
        HIPCHK(hipStreamSynchronize(st));
        if (nbirth)
            for (size_t q = 0; q < nb.size(); ++q) nbirth[q] = nb[q];
    });
}

int ugkwp_get_diag(ugkwp_ctx* ctx, ugkwp_diag* d)
{
    if (!ctx || !d) return UGKWP_EINVAL;
    *d = ctx->diag;
    return UGKWP_OK;
}

int ugkwp_set_phase_times(ugkwp_ctx* ctx, int on)
{
    if (!ctx) return UGKWP_EINVAL;
    ctx->phase_times = on != 0;
    return UGKWP_OK;
}

int ugkwp_set_push_timing(ugkwp_ctx* ctx, int every)
{
    if (!ctx) return UGKWP_EINVAL;
    if (every < 1) return UGKWP_EINVAL;
    ctx->push_time_every = every;
    return UGKWP_OK;
}

int ugkwp_get_totals(ugkwp_ctx* ctx, ugkwp_totals* t, int reset)
{
    if (!ctx) return UGKWP_EINVAL;
    if (t) *t = ctx->tot;
    if (reset) ctx->tot = ugkwp_totals{};
    return UGKWP_OK;
}

int ugkwp_get_counters(ugkwp_ctx* ctx, int inst, uint64_t* birth_counter, int* step)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        check_inst(ctx, inst);
        InstState s;
        HIPCHK(hipMemcpyAsync(&s, ctx->D.ist + inst, sizeof(InstState), hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        if (birth_counter) *birth_counter = s.births;
        if (step) *step = (int)ctx->step_idx;
    });
}

int64_t ugkwp_pool_size(ugkwp_ctx* ctx) { return ctx ? ctx->n_alive : -1; }

int ugkwp_get_pool(ugkwp_ctx* ctx, double* x, double* y, double* ox, double* oy, double* nu, double* w,
                   uint64_t* id, int32_t* cell, int32_t* g)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        if (ctx->n_inst == 0) fail(UGKWP_EINVAL, "mesh not initialised");
        const Pool p = ctx->view(ctx->cur_mv, ctx->cur_st);
        const size_t ns = (size_t)ctx->n_slots;
        hipStream_t st = ctx->st;
        std::vector<double> hx(ns), hy, hox(ns), hoy, hnu(ns), hw(ns);
        std::vector<uint64_t> hid(ns);
        std::vector<int32_t> hcell(ns);
        if (ctx->dim == 2) { hy.resize(ns); hoy.resize(ns); }
        auto cp = [&](void* dst, const void* src, size_t bytes) {
            if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        };
        cp(hx.data(), p.x, ns * 8);
        cp(hox.data(), p.ox, ns * 8);
        if (ctx->dim == 2) { cp(hy.data(), p.y, ns * 8); cp(hoy.data(), p.oy, ns * 8); }
        cp(hnu.data(), p.nu, ns * 8);
        cp(hw.data(), p.w, ns * 8);
        cp(hid.data(), p.id, ns * 8);
        cp(hcell.data(), p.cell, ns * 4);
        HIPCHK(hipStreamSynchronize(st));
        size_t o = 0;
        for (size_t q = 0; q < ns; ++q) {
            const int32_t word = hcell[q];
            if (word < 0) continue;
            if (x) x[o] = hx[q];
            if (y) y[o] = ctx->dim == 2 ? hy[q] : 0.0;
            if (ox) ox[o] = (word & FLIP_X) ? -hox[q] : hox[q];
            if (oy) oy[o] = ctx->dim == 2 ? ((word & FLIP_Y) ? -hoy[q] : hoy[q]) : 0.0;
            if (nu) nu[o] = hnu[q];
            if (w) w[o] = hw[q];
            if (id) id[o] = hid[q] & ID_MASK;
            if (cell) cell[o] = word & CELL_MASK;
            if (g) g[o] = (int32_t)(hid[q] >> ID_BITS);
            ++o;
        }
        if ((int64_t)o != ctx->n_alive) fail(UGKWP_EHIP, "pool holds %zu live particles, expected %lld", o,
                                              (long long)ctx->n_alive);
    });
}

int ugkwp_set_pool(ugkwp_ctx* ctx, int64_t n, const double* x, const double* y, const double* ox,
                   const double* oy, const double* nu, const double* w, const uint64_t* id,
                   const int32_t* cell, const int32_t* g, uint64_t birth_counter, const double* rhop)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        if (ctx->n_inst != 1) fail(UGKWP_EINVAL, "set_pool needs a single-instance context");
        if (n < 0 || n > ctx->P.pool_capacity) fail(UGKWP_EPOOL, "pool of %lld particles exceeds capacity", (long long)n);
        if (n > 0 && (!x || !ox || !nu || !w || !id || !cell || !g)) fail(UGKWP_EINVAL, "null pool array");
        if (ctx->dim == 2 && n > 0 && (!y || !oy)) fail(UGKWP_EINVAL, "2-D pool needs y and oy");
        const Inst& I = ctx->inst[0];
        for (int64_t q = 0; q < n; ++q)
            if (cell[q] < 0 || cell[q] >= I.ncell || g[q] < 0 || g[q] >= I.G || !(w[q] >= 0) || !(nu[q] > 0) ||
                id[q] > ID_MASK)
                fail(UGKWP_EINVAL, "particle %lld: cell, group, weight, frequency or id out of range", (long long)q);
        if (birth_counter > ID_MASK) fail(UGKWP_EINVAL, "birth counter beyond the id range");
        const Pool p = ctx->view(ctx->cur_mv, ctx->cur_st);
        hipStream_t st = ctx->st;
        auto cp = [&](void* dst, const void* src, size_t bytes) {
            if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        };
        const size_t nn = (size_t)n;
        cp(p.x, x, nn * 8);
        cp(p.ox, ox, nn * 8);
        if (ctx->dim == 2) { cp(p.y, y, nn * 8); cp(p.oy, oy, nn * 8); }
        cp(p.nu, nu, nn * 8);
        cp(p.w, w, nn * 8);
        std::vector<uint64_t> idw(nn);     // id | group word << ID_BITS
        for (size_t q = 0; q < nn; ++q) idw[q] = id[q] | ((uint64_t)(uint32_t)g[q] << ID_BITS);
        cp(p.id, idw.data(), nn * 8);
        cp(p.cell, cell, nn * 4);
        std::vector<double> hp;
        if (rhop) {
            hp.assign((size_t)ctx->K.n_cg, 0.0);
            ctx->pack_cg(hp, 0, rhop);
            cp(ctx->D.rhop, hp.data(), hp.size() * 8);
        }
        InstState s{};
        HIPCHK(hipMemcpyAsync(&s, ctx->D.ist, sizeof(InstState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        s.births = birth_counter;
        ctx->ids_used = birth_counter;
        HIPCHK(hipMemcpyAsync(ctx->D.ist, &s, sizeof(InstState), hipMemcpyHostToDevice, st));
        const unsigned long long na[3] = {(unsigned long long)n, (unsigned long long)n, (unsigned long long)n};
        HIPCHK(hipMemcpyAsync(ctx->D.counters + CNT_SLOTS, na, sizeof(na), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->n_alive = n;
        ctx->n_slots = n;
    });
}

// ---- checkpoint (saved layout: StateHeader and state_sections) ----

int64_t ugkwp_state_bytes(ugkwp_ctx* ctx)
{
    if (!ctx || ctx->n_inst == 0) return UGKWP_EINVAL;
    return (int64_t)state_sections(ctx, ctx->n_slots).end;
}

int ugkwp_get_state(ugkwp_ctx* ctx, void* buf, int64_t bytes)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        const StateLayout L = state_sections(ctx, ctx->n_slots);
        if (!buf || bytes < (int64_t)L.end)
            fail(UGKWP_EINVAL, "state buffer of %lld bytes, %zu needed", (long long)bytes, L.end);
        char* b = static_cast<char*>(buf);
        StateHeader h{};
        std::memcpy(h.magic, STATE_MAGIC, sizeof(h.magic));
        h.layout = state_layout(ctx);
        h.dim = ctx->dim;
        h.n_inst = ctx->n_inst;
        h.ncell = ctx->ncell;
        h.step = ctx->step_idx;
        h.n_cg = ctx->K.n_cg;
        h.n_slots = ctx->n_slots;
        h.n_alive = ctx->n_alive;
        h.bytes = (int64_t)L.end;
        h.version = STATE_VERSION;
        std::memcpy(b, &h, sizeof(h));
        hipStream_t st = ctx->st;
        auto cp = [&](size_t off, const void* src, size_t n) {
            if (n) HIPCHK(hipMemcpyAsync(b + off, src, n, hipMemcpyDeviceToHost, st));
        };
        const size_t ncg = (size_t)ctx->K.n_cg, ns = (size_t)ctx->n_slots;
        cp(L.rho, ctx->D.rho, 8 * ncg);
        cp(L.rhop, ctx->D.rhop, 8 * ncg);
        cp(L.phi0, ctx->D.phi0, 8 * ncg);
        cp(L.T, ctx->D.T, 8 * (size_t)ctx->ncell);
        std::vector<InstState> is((size_t)ctx->n_inst);
        HIPCHK(hipMemcpyAsync(is.data(), ctx->D.ist, sizeof(InstState) * is.size(), hipMemcpyDeviceToHost, st));
        const Pool p = ctx->view(ctx->cur_mv, ctx->cur_st);
        cp(L.x, p.x, 8 * ns);
        cp(L.ox, p.ox, 8 * ns);
        if (ctx->dim == 2) { cp(L.y, p.y, 8 * ns); cp(L.oy, p.oy, 8 * ns); }
        cp(L.nu, p.nu, 8 * ns);
        cp(L.w, p.w, 8 * ns);
        cp(L.id, p.id, 8 * ns);
        cp(L.cell, p.cell, 4 * ns);
        HIPCHK(hipStreamSynchronize(st));
        for (int k = 0; k < ctx->n_inst; ++k) std::memcpy(b + L.births + 8 * (size_t)k, &is[k].births, 8);
    });
}

int ugkwp_set_state(ugkwp_ctx* ctx, const void* buf, int64_t bytes)
{
    if (!ctx) return UGKWP_EINVAL;
    return guarded(ctx, [&] {
        require_ready(ctx);
        if (ctx->rec_cap > 0) fail(UGKWP_EINVAL, "a state cannot be restored while a record is kept (ugkwp_record(ctx, 0) first)");
        if (!buf || bytes < (int64_t)sizeof(StateHeader)) fail(UGKWP_EINVAL, "state buffer too short");
        const char* b = static_cast<const char*>(buf);
        StateHeader h;
        std::memcpy(&h, b, sizeof(h));
        if (std::memcmp(h.magic, STATE_MAGIC, sizeof(h.magic)) != 0 || h.version != STATE_VERSION)
            fail(UGKWP_EINVAL, "not a saved state of this library version");
        if (h.layout != state_layout(ctx) || h.dim != ctx->dim || h.n_inst != ctx->n_inst ||
            h.ncell != ctx->ncell || h.n_cg != ctx->K.n_cg)
            fail(UGKWP_EINVAL, "the state was saved from a context with another mesh, groups or constants");
        if (h.n_slots < 0 || h.n_slots > ctx->P.pool_capacity || h.n_alive < 0 || h.n_alive > h.n_slots)
            fail(UGKWP_EPOOL, "the saved pool of %lld slots does not fit a capacity of %lld",
                 (long long)h.n_slots, (long long)ctx->P.pool_capacity);
        const StateLayout L = state_sections(ctx, h.n_slots);
        if (h.bytes != (int64_t)L.end || bytes < (int64_t)L.end) fail(UGKWP_EINVAL, "state buffer truncated");
        // the pool: every live slot names a cell and a group of its instance
        const size_t ns = (size_t)h.n_slots;
        const int32_t* cw = reinterpret_cast<const int32_t*>(b + L.cell);
        const uint64_t* iw = reinterpret_cast<const uint64_t*>(b + L.id);     // id | group word << ID_BITS
        std::vector<int> first(ctx->n_inst);
        for (int k = 0; k < ctx->n_inst; ++k) first[k] = ctx->inst[k].cell_off;
        int64_t live = 0;
        for (size_t q = 0; q < ns; ++q) {
            if (cw[q] < 0) continue;
            const int cell = cw[q] & CELL_MASK;
            if (cell >= ctx->ncell) fail(UGKWP_EINVAL, "saved particle %zu: cell out of range", q);
            const int k = (int)(std::upper_bound(first.begin(), first.end(), cell) - first.begin()) - 1;
            if ((int64_t)(iw[q] >> ID_BITS) >= ctx->inst[k].G) fail(UGKWP_EINVAL, "saved particle %zu: group out of range", q);
            ++live;
        }
        if (live != h.n_alive) fail(UGKWP_EINVAL, "saved pool holds %lld live particles, header says %lld",
                                    (long long)live, (long long)h.n_alive);
        const double* T = reinterpret_cast<const double*>(b + L.T);
        for (int i = 0; i < ctx->ncell; ++i)
            if (!(T[i] > 0) || !std::isfinite(T[i])) fail(UGKWP_EINVAL, "saved temperature not positive and finite");
        for (int k = 0; k < ctx->n_inst; ++k) {
            uint64_t nb = 0;
            std::memcpy(&nb, b + L.births + 8 * (size_t)k, 8);
            if (nb > ID_MASK) fail(UGKWP_EINVAL, "saved birth counter beyond the id range");
        }

        hipStream_t st = ctx->st;
        auto cp = [&](void* dst, size_t off, size_t n) {
            if (n) HIPCHK(hipMemcpyAsync(dst, b + off, n, hipMemcpyHostToDevice, st));
        };
        const size_t ncg = (size_t)ctx->K.n_cg;
        cp(ctx->D.rho, L.rho, 8 * ncg);
        cp(ctx->D.rhop, L.rhop, 8 * ncg);
        cp(ctx->D.phi0, L.phi0, 8 * ncg);
        cp(ctx->D.T, L.T, 8 * (size_t)ctx->ncell);
        const Pool p = ctx->view(ctx->cur_mv, ctx->cur_st);
        cp(p.x, L.x, 8 * ns);
        cp(p.ox, L.ox, 8 * ns);
        if (ctx->dim == 2) { cp(p.y, L.y, 8 * ns); cp(p.oy, L.oy, 8 * ns); }
        cp(p.nu, L.nu, 8 * ns);
        cp(p.w, L.w, 8 * ns);
        cp(p.id, L.id, 8 * ns);
        cp(p.cell, L.cell, 4 * ns);
        // the committed record: birth counters, pool size, step count
        std::vector<InstState> is((size_t)ctx->n_inst);
        ctx->ids_used = 0;
        for (int k = 0; k < ctx->n_inst; ++k) {
            std::memcpy(&is[k].births, b + L.births + 8 * (size_t)k, 8);
            ctx->ids_used = std::max(ctx->ids_used, (uint64_t)is[k].births);
        }
        HIPCHK(hipMemcpyAsync(ctx->D.ist, is.data(), sizeof(InstState) * is.size(), hipMemcpyHostToDevice, st));
        std::vector<unsigned long long> cnt(N_COUNTERS, 0ull);
        cnt[CNT_SLOTS] = (unsigned long long)h.n_slots;
        cnt[CNT_LIVE] = (unsigned long long)h.n_alive;
        cnt[CNT_DONE] = h.step;
        HIPCHK(hipMemcpyAsync(ctx->D.counters, cnt.data(), sizeof(unsigned long long) * N_COUNTERS,
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->D.step, &h.step, sizeof(uint32_t), hipMemcpyHostToDevice, st));
        // the last step's tallies belong to the run the state came from
        HIPCHK(hipMemsetAsync(ctx->D.ftx, 0, sizeof(double) * ctx->n_fx * 2, st));
        HIPCHK(hipMemsetAsync(ctx->D.fty, 0, sizeof(double) * std::max<int64_t>(ctx->n_fy, 1) * 2, st));
        for (double* q : {ctx->D.dep, ctx->D.surv, ctx->D.wnew, ctx->D.Q})
            HIPCHK(hipMemsetAsync(q, 0, sizeof(double) * ncg, st));
        HIPCHK(hipMemsetAsync(ctx->D.nb, 0, sizeof(int32_t) * ncg, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->step_idx = h.step;
        ctx->n_alive = h.n_alive;
        ctx->n_slots = h.n_slots;
        ctx->last_births = 0;
        ctx->diag = ugkwp_diag{};
    });
}

// ---- element-wise entry points ----


int ugkwp_eval_phi(int n, const double* T, int G, const double* nu_edges, double a, double c, double* out)
{
    if (n < 0 || G < 1 || !T || !nu_edges || !out) return UGKWP_EINVAL;
    return guarded(nullptr, [&] {
        ensure_head_series();
        Tmp t;
        double* dT = t.up(T, n);
        double* dnu = t.up(nu_edges, G + 1);
        double* dout = t.up<double>(nullptr, (size_t)n * G);
        launch_eval_phi(n, dT, G, dnu, a, c, dout, nullptr);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(out, dout, sizeof(double) * n * G, hipMemcpyDeviceToHost));
    });
}

int ugkwp_eval_coef(int n, const double* s, double* c4, double* w, double* c2_over_dt)
{
    if (n < 0 || !s || !c4 || !w || !c2_over_dt) return UGKWP_EINVAL;
    return guarded(nullptr, [&] {
        Tmp t;
        double* ds = t.up(s, n);
        double* a = t.up<double>(nullptr, n);
        double* b = t.up<double>(nullptr, n);
        double* cc = t.up<double>(nullptr, n);
        launch_eval_coef(n, ds, a, b, cc, nullptr);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(c4, a, sizeof(double) * n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(w, b, sizeof(double) * n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(c2_over_dt, cc, sizeof(double) * n, hipMemcpyDeviceToHost));
    });
}

int ugkwp_eval_uniform(int n, uint64_t seed, const uint64_t* id, uint32_t step, uint32_t purpose,
                       const uint32_t* d, double* out)
{
    if (n < 0 || !id || !d || !out) return UGKWP_EINVAL;
    return guarded(nullptr, [&] {
        Tmp t;
        uint64_t* di = t.up(id, n);
        uint32_t* dd = t.up(d, n);
        double* o = t.up<double>(nullptr, n);
        launch_eval_uniform(n, seed, di, step, purpose, dd, o, nullptr);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(out, o, sizeof(double) * n, hipMemcpyDeviceToHost));
    });
}

int ugkwp_eval_neg_log(int n, const double* u, double* out)
{
    if (n < 0 || !u || !out) return UGKWP_EINVAL;
    return guarded(nullptr, [&] {
        Tmp t;
        double* du = t.up(u, n);
        double* o = t.up<double>(nullptr, n);
        launch_eval_neg_log(n, du, o, nullptr);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(out, o, sizeof(double) * n, hipMemcpyDeviceToHost));
    });
}

int ugkwp_eval_sample_nu(int n, const double* nl, const double* nh, const double* T, const double* U,
                         double* beta, double* nu)
{
    if (n < 0 || !nl || !nh || !T || !U || !beta || !nu) return UGKWP_EINVAL;
    return guarded(nullptr, [&] {
        Tmp t;
        double* a = t.up(nl, n);
        double* b = t.up(nh, n);
        double* c = t.up(T, n);
        double* u = t.up(U, n);
        double* ob = t.up<double>(nullptr, n);
        double* on = t.up<double>(nullptr, n);
        launch_eval_sample_nu(n, a, b, c, u, ob, on, nullptr);
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(beta, ob, sizeof(double) * n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(nu, on, sizeof(double) * n, hipMemcpyDeviceToHost));
    });
}

}  // extern "C"
