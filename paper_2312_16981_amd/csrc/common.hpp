// Shared layout of the device state of a UGKWP context.
//
// A context holds n_inst independent instances of one dimension.  Per-cell
// fields are stored instance after instance; per-(cell, group) fields use a
// padded group stride Gp (the power of two >= G, at most 64) so that the Gp
// lanes of one cell sit in one 64-wide wavefront, and each instance's block
// of (cell, group) slots starts on a multiple of 64 so that no wavefront spans
// two instances.  Face quantities use the same Gp stride per face.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ugk {

constexpr int WAVE = 64;
constexpr int MAX_G = 64;
constexpr int RES_SLOTS = 3;     // rotating residual slots of the source iteration
constexpr int RES_SUB = 64;      // sub-slots per residual slot (spread the atomics of many blocks)
constexpr int DIAG_SUB = 16;     // sub-slots of the per-instance energy sums

enum { BC_VACUUM = 0, BC_PLANCK = 1, BC_REFLECT = 2 };
enum { XLO = 0, XHI = 1, YLO = 2, YHI = 3 };

struct Inst {
    int dim, nx, ny, ncell;
    int G, Gp, lgGp;
    int cell_off;          // first global cell index
    int edge_off;          // group edges at nu[edge_off .. edge_off + G]
    int bc[4];
    int64_t cg_off;        // first (cell, group) slot, multiple of 64
    int64_t fx_off;        // first x-face slot ((nx+1)*ny faces, stride Gp)
    int64_t fy_off;        // first y-face slot (nx*(ny+1) faces, stride Gp)
    double x0, y0, dx, dy, V;
    double dt_V;           // dt / V
    double bcT[4];
    double w_ref;
    uint64_t seed;
};

// Context-wide constants.
struct Consts {
    double c, a, eps, dt;
    double e2c;            // eps^2 / c   (tau = e2c / sigma)
    double cv;             // c / eps     (particle speed)
    double lam_scale;      // c dt / eps^2
    double cq;             // c / (4 eps)   (wave flux factor)
    double tau_C;          // numerical collision time of joint cells: C (0 = off)
    double tau_jump;       // opacity ratio across a face that makes its cells joint
    double t_power;        // q of sigma(nu, T) = kappa nu^-p T^-q (0: no T dependence)
    int stim;              // 1: sigma also carries 1 - e^{-nu/T}
    double nu_power;
    // material models of Olson's problems (Sec. 3.4-3.5), all off when 0
    int olson;             // 1: per-cell Olson heat capacity (D.olH, D.olchi) in some cells
    int table;             // 1: tabulated sigma(nu, T) per material replaces kappa nu^-p T^-q
    int tab_nnu, tab_nT;   // table nodes in nu and T
    double tab_lT_inv;     // 1 / spacing of ln T when the T nodes are evenly spaced in ln T (else 0):
                           // a first guess of the interval, bisection's result kept
    int has_src;           // 1: a volumetric source D.qsrc
    double q_toff;         // the source acts in steps that start before this time
    double si_tol;
    int64_t n_cap;
    int64_t pool_cap;
    uint32_t flags;
    uint32_t gate;         // step index a launch belongs to (GATE_OFF: none), see gate_open
    int n_inst;
    int64_t n_cg;          // total (cell, group) slots incl. padding
    int64_t n_fx2;         // x-face tally entries (2 per x-face slot)
    int ncell;             // total cells
    Inst inst0;            // instance 0's record (read from here when it is the only one)
};

constexpr uint32_t GATE_OFF = 0xFFFFFFFFu;

// Residual accumulators of one source-iteration sweep (non-negative doubles as
// their IEEE bit patterns, so that integer atomicMax orders them; NaN wins).
struct Resid {
    unsigned long long drho, rho, dT, T;
};

// Per-instance step state.
struct InstState {
    int conv_sweeps;       // sweeps used by the converged source iteration, 0 = running
    int bad;               // non-finite / non-positive temperature seen
    uint64_t births;       // birth counter B_n (carried from step to step)
};

// Context counters (device, unsigned 64-bit).  They sit in a step record
// together with the birth totals, the per-instance states and energy sums:
// every step of a batch writes its own record, and its first launch carries
// the persistent entries (CNT_SLOTS, CNT_LIVE, the birth counters) over
// from the record of the step before.
enum {
    CNT_SURV = 0,      // particles alive after this step's push
    CNT_DONE = 1,      // the step count after this step's commit, 0 while not committed
    CNT_ERR = 2,       // ERR_* bits raised in this step
    CNT_CONV = 3,      // instances whose source iteration has converged
    CNT_SLOTS = 4,     // pool slots at the start of the step (live particles and holes)
    CNT_PUSHED = 5,    // slots covered by this step's push (CNT_SLOTS + births)
    CNT_LIVE = 6,      // live particles at the start of the step
    N_COUNTERS = 8
};
enum : unsigned long long {
    ERR_POOL = 1,      // pool capacity would be exceeded: nothing sampled, step not committed
    ERR_RECORD = 2,    // a particle record with an out-of-range cell or group
    ERR_COUNT = 4,     // survivor counts disagree with the pool
    ERR_TEMP = 8       // non-positive or non-finite temperature in the source iteration
};

// The cell word of a particle: bits 0..28 the context-global cell, bit 29 a
// pending reversal of the y direction, bit 30 of the x direction (specular
// reflections; the stored direction is rewritten only when the pool is
// sorted), and a negative word marks an empty slot.
constexpr int32_t CELL_MASK = (1 << 29) - 1;
constexpr int32_t FLIP_Y = 1 << 29;
constexpr int32_t FLIP_X = 1 << 30;
constexpr int32_t DEAD = -1;

// The group word of a particle: the group in the low bits; a boundary-source
// particle of this step (UGKWP_FLAG_BOUNDARY_PARTICLES) carries 1 + the side
// of the ghost it was born in from bit GHOST_SHIFT until the push clears it.
constexpr int GHOST_SHIFT = 8;
constexpr int32_t GROUP_MASK = (1 << GHOST_SHIFT) - 1;

// The pool's id word carries the particle id in its low ID_BITS bits and the
// group word above them, so that a record is one word shorter: the push and
// the sort read 4 bytes less per particle.  Ids stay below 2^ID_BITS (the
// runtime refuses a birth count that would reach it).
constexpr int ID_BITS = 48;
constexpr uint64_t ID_MASK = (1ull << ID_BITS) - 1ull;

// A particle pool viewed as structure of arrays.  The moving fields (x, y and
// the cell word) live in one of two buffers that alternate between steps; the
// stable fields (direction, frequency, weight, id, group) are only appended
// to, and move to the other buffer set when the pool is sorted.
struct Pool {
    double* x;
    double* y;
    int32_t* cell;
    double* ox;            // mu in 1-D
    double* oy;
    double* nu;
    double* w;
    uint64_t* id;          // id | group word << ID_BITS
};

struct Dev {
    const Inst* inst;
    const int64_t* inst_cg;     // [n_inst+1] padded starts
    const int32_t* wave_inst;   // [n_cg/64] instance of each aligned run of 64 slots
    const int32_t* cell_inst;   // [ncell]
    const double* nu;           // edges
    const double* simpson;      // [edge_off + g]
    const double* phib;         // [inst][4][MAX_G] Planckian ghost phi
    // per (cell, group) slot
    const double* kappa;
    double* inv_kappa;          // 1/kappa (+inf where kappa = 0), for the particle flights
    double* sig;
    double* sv;                 // s = c sigma dt / eps^2 (= lambda of the source iteration)
    double* es;                 // e^{-s}
    double* c4;
    double* wc;                 // C4 - e^{-s}
    double* rho;                // rho^n
    double* rho_new;            // rho^k during the source iteration, rho^{n+1} after
    double* rhop;               // survivor density from the previous step
    double* rhoh;               // rho^h = rho^n - rhop (start of step)
    double* Q;
    double* phi0;               // phi(T^n): the source iteration's phi^0
    double* phi1;               // phi^{k+1} of the even sweeps
    double* phi2;               // phi^{k+1} of the odd sweeps
    int32_t* nb;                // births per slot
    int64_t* boff;              // exclusive scan of nb
    double* wnew;
    double* wsn;                // wave coefficient of a sampled slot this step (joint cells' tau_num)
    double* sx;                 // slopes of rho^h along x and y (UGKWP_FLAG_SLOPES)
    double* sy;
    double* bcoef;              // slope coefficient of the wave flux: C5 or C5 + dt/2 e^{-s}, over dt
    double* rho_alt;            // rho^k of the even sweeps with UGKWP_FLAG_WAVE_ITER
    double* winflow;            // [2][slot] boundary wave inflow of the last even / odd sweep (WAVE_ITER)
    int32_t* nbi;               // interior births per slot (nb adds the boundary-source births)
    double* beta;
    double* dep;
    double* surv;
    uint32_t* scount;           // survivors per slot (counting sort of the pool)
    int64_t* soff;              // exclusive scan of scount, then write cursor
    // per face slot
    double* ftx;                // [slot*2 + dir]
    double* fty;
    double* Dx;
    double* Dy;
    // per cell
    const double* cvol;         // heat capacity
    const double* dtcv;         // dt / (eps^2 C_v): the temperature update's weight
    double* T;
    double* T_new;
    const uint8_t* pinned;
    // Olson's heat capacity H [1 + alpha + (T + chi) alpha'] where olH > 0 (else the
    // constant cvol), and the material energy the last sweep gave those cells
    const double* olH;
    const double* olchi;
    double* uend;
    // volumetric source: rate per (cell, group) slot, and whether the step's source is on
    const double* qsrc;
    int* src_on;
    // tabulated opacity: material per cell, ln of the nodes and of sigma [mat][T][nu],
    // and per cell the ln sigma along the nu nodes at the cell's T^n (the push's rows)
    const int32_t* tab_mat;
    double* tab_lnu;
    double* tab_lT;
    double* tab_lsig;
    double* tab_row;
    int32_t* tab_gi;            // [edge][3] nu interval of each group's Simpson points
    double* tab_ga;             // [edge][3] and the weight of its upper node
    double* tab_sig;            // [2][slot] group sigma at the iterate written by sweep k for sweep k+1
    // per instance
    InstState* ist;
    Resid* res;                 // [RES_SLOTS][n_inst][RES_SUB]
    uint8_t* wave_run;          // [n_cg/64 rounded up to 4] 1 while the wavefront's instance iterates (batches)
    double* diag;               // [n_inst][8] (folded from diag_sub each step)
    double* diag_sub;           // [n_inst][DIAG_SUB][8]
    // context-wide counters
    uint32_t* step;                 // step index n (keys the random numbers), advanced on commit
    unsigned long long* counters;   // CNT_*
    int64_t* n_births_total;        // [0] births of the step, [1] survivors (sort scan)
    unsigned long long* blk_surv;   // survivors counted by each push block
    // the record of the step before (counters and instance states), read
    // once at the start of a step for the persistent entries
    const unsigned long long* prev_counters;
    const InstState* prev_ist;
};

__host__ __device__ inline int find_inst(const int64_t* starts, int n, int64_t j)
{
    int lo = 0, hi = n;         // starts[lo] <= j < starts[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace ugk
