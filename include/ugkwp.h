/*
 * ugkwp.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of the unified gas-kinetic wave-particle (UGKWP) method for
 * frequency-dependent radiative transfer (Yang, Zhu, Liu & Xu, arXiv 2312.16981).
 *
 * One call to ugkwp_step advances every problem instance held by a context by
 * one time step of the paper's Algorithm 1:
 *   - sample the collisionless particles of each cell's wave part
 *     (Eq. IhpFormula, weights from Sec. 2.2) with linear-frequency sampling
 *     (Eqs. Blinear, kg; Appendix A);
 *   - draw free-flight times t_f = min(-tau ln eta, dt) (Eq. particle tf formula),
 *     stream the particles, reset t_f at every interface crossing (Remark 1),
 *     tally gross face crossings (Eq. wfrpFormula), delete collided particles;
 *   - add the wave free-transport flux (Sec. 2.2, F^{fr,wave}; Remark 3);
 *   - solve the implicit macroscopic system (Eq. macroSysFinal) by the
 *     matrix-free source iteration of Appendix B (Algorithm 2).
 *
 * Conventions
 *   - Every function returns UGKWP_OK (0) or a negative UGKWP_E* code; the
 *     message of the last failure of a context is ugkwp_last_error(ctx).
 *   - Host input arrays are copied and validated; the caller keeps ownership.
 *   - Output arrays are host memory unless the call takes dst_is_device = 1,
 *     in which case they are device pointers written on the context's stream.
 *   - The library owns all device memory of a context (allocated by
 *     init calls, released by ugkwp_destroy).
 *   - Field layout: cells are row-major [iy][ix] (ny = 1 in 1-D), fields are
 *     [cell][G] with the group index fastest.  Several instances are stored one
 *     after the other in instance order.
 *   - Units are the paper's nondimensional ones with h = k = 1: nu and T share
 *     units, B(nu,T) = 2 nu^3/(c^2 (e^{nu/T}-1)) scaled so that the full
 *     spectrum carries a c T^4 (Sec. 2.1).
 *   - A context is used by one host thread at a time.
 *   - A failed ugkwp_step leaves the state as it was at the start of the failing
 *     step (fields, particle pool, counters).
 */
#ifndef UGKWP_H
#define UGKWP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UGKWP_OK = 0,
    UGKWP_EINVAL = -1,      /* invalid argument or call order                  */
    UGKWP_ENOMEM = -2,      /* device allocation failed                          */
    UGKWP_EPOOL = -3,       /* particle pool capacity would be exceeded          */
    UGKWP_ENOCONV = -4,     /* source iteration hit its iteration limit          */
    UGKWP_ENONFINITE = -5,  /* non-positive or non-finite temperature            */
    UGKWP_EHIP = -6         /* HIP runtime error                                 */
};

enum { UGKWP_BC_VACUUM = 0, UGKWP_BC_PLANCK = 1, UGKWP_BC_REFLECT = 2 };
enum { UGKWP_SIDE_XLO = 0, UGKWP_SIDE_XHI = 1, UGKWP_SIDE_YLO = 2, UGKWP_SIDE_YHI = 3 };

/* Flags */
enum {
    UGKWP_FLAG_GROUP_SIGMA = 1,  /* particle flights use the Simpson group opacity
                                    instead of kappa * nu_k^-p (Remark 2)        */
    UGKWP_FLAG_GRAPH = 2,        /* replay the launches before the push and the
                                    source-iteration sweeps from captured HIP
                                    graphs (one per launch configuration) instead
                                    of launching each kernel; same results        */
    UGKWP_FLAG_PHASE_TIMES = 4,  /* time every phase of a step with HIP events (the
                                    diag's ms_sample, ms_macro, ms_si, ms_sort);
                                    otherwise only the push is timed              */
    UGKWP_FLAG_SI_LINEARIZED = 8, /* source iteration (Appendix B) with the emission
                                    of T^{k+1} linearized about T^k, each sweep a
                                    local Newton step of every cell's energy
                                    balance: the same fixed point (Eq.
                                    macroSysFinal), and convergence also where
                                    sum_g dt sigma_g phi'_g / (eps^2 C_v
                                    (1 + lambda_g)) exceeds 1 (stiff material
                                    coupling, where the literal sweep diverges)   */
    UGKWP_FLAG_SLOPES = 16,      /* second-order wave part (Sec. 2.2, the C5 terms):
                                    MINMOD slopes of rho^h per axis (limited so the
                                    linear profile stays non-negative in the cell),
                                    the upwind profile's face value and the slope
                                    term (C5, or C5 + dt/2 e^{-s} where sampled) in
                                    the wave flux, new particles placed along the
                                    slope                                          */
    UGKWP_FLAG_WAVE_ITER = 32,   /* wave flux of each source-iteration sweep from
                                    its iterate, rho^h = rho^k - rho^p (Algorithm 2),
                                    instead of the start of the step                */
    UGKWP_FLAG_BOUNDARY_PARTICLES = 64 /* a Planckian boundary's ghost cell samples its
                                    collisionless share e^{-s} phi(T_b) V as
                                    particles (count and weight as an interior
                                    cell's), which fly straight to the domain face
                                    and enter there within the step or are dropped;
                                    the ghost's wave coefficient becomes
                                    C4 - e^{-s}                                      */
};

typedef struct ugkwp_ctx ugkwp_ctx;

/* Parameters shared by all instances of a context. */
typedef struct {
    double c;            /* speed of light                                         */
    double a;            /* radiation constant                                     */
    double eps;          /* Knudsen number epsilon of Eq. mfGovI                   */
    double dt;           /* time step                                              */
    double nu_power;     /* p in sigma(nu) = kappa * nu^-p (3 for the paper's tests) */
    int64_t n_cap;       /* max particles sampled per (cell, group) and step       */
    int64_t pool_capacity; /* particle slots of the context (all instances), at most 2^29 */
    int si_max_iters;    /* source-iteration limit (Algorithm 2)                   */
    double si_tol;       /* relative max-norm tolerance on rho and on T            */
    uint32_t flags;      /* UGKWP_FLAG_*                                           */
    int sort_interval;   /* steps between counting sorts of the particle pool by
                            (cell, group); 0 = library default (32 steps in 1-D,
                            16 in 2-D, where locality decays faster).  Affects
                            only speed and the order of the pool, not the results. */
    double tau_num_C;    /* numerical collision time of thin-thick-joint cells (Sec. 3.2,
                            second case): when > 0, a cell that shares a face across
                            which its group opacity changes by a factor of at least
                            tau_num_jump samples the fraction e^{-dt/tau_num} of its
                            wave part, tau_num = eps^2/(c sigma) + tau_num_C
                            |T^l - T^r|/(T^l + T^r) dt (largest over those faces,
                            temperatures at the start of the step), and its wave
                            flux keeps C4(s) - e^{-dt/tau_num} (Remark 3).  0 = off.
                            Not recordable for ugkwp_adjoint.                        */
    double tau_num_jump; /* opacity ratio that makes a face joint (<= 1: every face)   */
    double opacity_T_power; /* q of a temperature-dependent opacity sigma(nu, T) =
                            kappa nu^-p T^-q (Sec. 3.1 takes q = 1/2); 0 = none.
                            The particles and the wave split of a step take the
                            temperature T^n; every source-iteration sweep recomputes
                            sigma, lambda and the face coefficients from its iterate
                            (Algorithm 2).  Not recordable for ugkwp_adjoint.        */
    int32_t opacity_stim; /* 1: sigma also carries the stimulated-emission factor
                            (1 - e^{-nu/T}) of Sec. 3.3's gamma0 (1 - e^{-h nu/kT})
                            / (h nu)^3, at the same temperatures as the T^-q factor;
                            a group's opacity is then Simpson's mean of
                            nu^-p (1 - e^{-nu/T}) over the group.  0 = none; other
                            values are rejected.  Not recordable for ugkwp_adjoint. */
} ugkwp_params;

/* One problem instance (a slab in 1-D, a rectangle in 2-D). */
typedef struct {
    int dim;                 /* 1 or 2                                                 */
    int nx, ny;              /* cells; ny = 1 in 1-D                                    */
    double x0, x1, y0, y1;   /* domain                                                  */
    int bc[4];               /* boundary type per side (XLO, XHI, YLO, YHI)             */
    double bcT[4];           /* Planckian boundary temperatures                          */
    int G;                   /* frequency groups, 1..64                                 */
    const double* nu_edges;  /* G+1 ascending group edges (Sec. 2.1 multigroup)         */
    uint64_t seed;           /* Philox key of this instance                              */
    double w_ref;            /* target particle energy per unit cell volume (Sec. 3)     */
    const double* kappa;     /* [ncell][G] >= 0: sigma(nu, cell) = kappa[cell][g] nu^-p  */
    const double* cv;        /* [ncell] > 0 heat capacity                                */
    const double* T0;        /* [ncell] > 0 initial material temperature                 */
    const double* Tr0;       /* [ncell] > 0 initial radiation temperature: rho = phi(Tr0) */
    const uint8_t* pinned;   /* [ncell] or NULL: cells whose T is held fixed (sources)   */
} ugkwp_instance;

/* Per-context counters and energy bookkeeping of the last step, summed over instances. */
typedef struct {
    int64_t n_alive_in;      /* particles entering the step                    */
    int64_t n_births;        /* particles sampled in the step                  */
    int64_t n_alive_out;     /* survivors after the step                       */
    int64_t n_pushed;        /* n_alive_in + n_births                          */
    int sweeps_max;          /* largest source-iteration sweep count           */
    int sweeps_sum;          /* sum over instances                              */
    double e_start, e_end;   /* total energy sum V (sum_g rho/c + Cv T)        */
    double inflow_wave, inflow_eq, exit_particles, injection;
    double residual;         /* e_end - e_start - (inflow_wave + inflow_eq + inflow_particles
                                - exit + injection) */
    /* GPU time of the phases of the step, in ms, from HIP events on the context
     * stream: tally clears + count + scan + sample, the push kernel alone (events
     * recorded just before and after its launch, so the interval also holds its
     * dispatch, a few microseconds), ms_macro (now only the event pair after
     * the push: the wave flux and Q are evaluated by the first source-iteration
     * sweep and counted in ms_si), the source iteration, and the counting sort
     * that keeps the pool ordered by (cell, group).  Each event adds a few
     * microseconds to a step, so without UGKWP_FLAG_PHASE_TIMES only the push
     * of one step in 8 (step index a multiple of 8, or of the interval set by
     * ugkwp_set_push_timing) is timed and everything
     * else is 0; with it every phase of every step is timed.  push_timed says
     * whether this step's ms_push holds a time. */
    double ms_sample, ms_push, ms_macro, ms_si, ms_sort;
    int push_timed;
    double inflow_particles; /* energy of boundary-source particles that entered the
                                domain (UGKWP_FLAG_BOUNDARY_PARTICLES); the residual
                                adds it to the inflows                              */
} ugkwp_diag;

/* Running sums over the committed steps since the last reset, so that a caller
 * can time many steps in one ugkwp_step call. */
typedef struct {
    int64_t steps;
    int64_t n_pushed;        /* particles entering the push, summed over steps     */
    int64_t n_survived;      /* survivors, summed over steps                       */
    int64_t sweeps_max;      /* sum of per-step largest sweep counts               */
    int64_t sweeps_sum;      /* sum over steps and instances of sweep counts       */
    double ms_sample, ms_push, ms_macro, ms_si, ms_sort;   /* as in ugkwp_diag    */
    int64_t cg_updates;      /* (cell, group) updates of the source iteration: sum over
                                steps and instances of sweeps x cells x groups      */
    int64_t push_timed;      /* steps whose push was timed (ms_push sums over them) */
    int64_t n_pushed_timed;  /* particles entering those pushes                     */
    int64_t n_survived_timed;/* and their survivors                                 */
} ugkwp_totals;

/* ---- context ---- */

/* Create a context.  hip_stream: a hipStream_t to run on, or NULL for a stream
 * owned by the context.  No device memory is allocated yet. */
int ugkwp_create(ugkwp_ctx** out, const ugkwp_params* p, void* hip_stream);
void ugkwp_destroy(ugkwp_ctx* ctx);
const char* ugkwp_last_error(const ugkwp_ctx* ctx);

/* ---- problem set-up (the paper's statement of the problem, Sec. 2.1 and Sec. 3) ---- */

/* Single-instance set-up, in three calls.  init_mesh fixes the geometry, the
 * boundary conditions (Planckian incident, vacuum, reflective: Sec. 3) and the
 * frequency groups; it allocates device memory. */
int ugkwp_init_mesh(ugkwp_ctx* ctx, int dim, int nx, int ny, const double lo[2],
                    const double hi[2], const int bc[4], const double bcT[4], int G,
                    const double* nu_edges, uint64_t seed, double w_ref);
/* kappa [ncell][G] (host): sigma(nu, T, cell) = kappa nu^-p, times T^-q when
 * opacity_T_power = q is set and times (1 - e^{-nu/T}) when opacity_stim is 1
 * (Sec. 3.1, 3.3); group opacity by Simpson's rule over each group (Sec. 3).
 * Non-negative and finite. */
int ugkwp_set_opacity(ugkwp_ctx* ctx, const double* kappa);
/* Heat capacity, initial T and radiation temperature per cell (rho^0 = phi(Tr0),
 * no particles: Sec. 3.1), optional pinned-source mask. */
int ugkwp_set_material(ugkwp_ctx* ctx, const double* cv, const double* T0,
                       const double* Tr0, const uint8_t* pinned);
/* ugkwp_set_material for callers that cannot allocate device memory (code that
 * a harness forbids to call hipMalloc, tight serving loops that reset an
 * instance): the same arguments, layout and result, but the device staging of
 * Tr0 lives in a library-owned static array (one per GPU, 2^21 doubles = 16 MiB,
 * held until the process ends) instead of a buffer allocated per call; no
 * hipMalloc or hipFree is called.  Runs on the context's GPU.  EINVAL if the
 * mesh has more than 2^21 cells or the context is a batch.  Calls that overlap
 * on one GPU (from several threads or contexts) share that array and race. */
int ugkwp_set_material_noalloc(ugkwp_ctx* ctx, const double* cv, const double* T0,
                               const double* Tr0, const uint8_t* pinned);

/* ---- material models of Olson's problems (Sec. 3.4-3.5) ----
 * Each takes per-cell (or per-(cell, group)) arrays of every instance of the
 * context, concatenated in instance order, and is called after the material
 * (ugkwp_set_material or ugkwp_init_batch).  They turn on the source iteration
 * that re-evaluates the material from its iterate, and none is recordable for
 * ugkwp_adjoint.  EINVAL for invalid values; a null first array turns the model
 * off again. */

/* Olson's heat capacity (Eq. cvolson): where H[cell] > 0 the cell's volumetric heat
 * capacity at T is H [1 + alpha + (T + chi) dalpha/dT], alpha = e^{-chi/T}
 * (sqrt(1 + 4 e^{chi/T}) - 1)/2 (the printed factor a T_keV^3 is the unit
 * a (1 keV)^3, to be folded into H by the caller), in place of its constant C_v;
 * its material energy is U(T) = H [T (1 + alpha) + chi alpha], and the source
 * iteration solves U(T^{n+1}) = U(T^n) + exchange (the energy form of Eq.
 * macroEquImplicit's material line): the literal sweep inverts U for T^{k+1}
 * (Newton inside a bracket, to 1e-15 T), the linearized one takes one Newton step
 * at T^k.  The ledger's material energy of such a cell is U.  H [ncell] >= 0,
 * chi [ncell] >= 0, finite; cells with H = 0 keep their C_v. */
int ugkwp_set_heat_capacity(ugkwp_ctx* ctx, const double* H, const double* chi);
/* A volumetric radiation source (Sec. 3.4-3.5's Q(x)): q [ncell][G] >= 0, finite, the
 * rate of rho; every step that starts before t_off (step index n with n dt < t_off)
 * adds dt q to the right side of the macroscopic solve, and the ledger counts
 * V dt q / c as injection.  t_off >= 0 (+inf: always on). */
int ugkwp_set_source(ugkwp_ctx* ctx, const double* q, double t_off);
/* The source Q(x) = B(nu, Ts) f(x) added to the transport equation's right side, as
 * printed for Olson's problems: q = (c/eps^2) f[cell] phi_g(Ts) computed on the
 * device; f [ncell] >= 0, finite; Ts > 0. */
int ugkwp_set_source_planck(ugkwp_ctx* ctx, const double* f, double Ts, double t_off);
/* A tabulated opacity sigma(nu, T) per material in place of kappa nu^-p T^-q (the
 * piecewise opacities of Sec. 3.4-3.5, tabulated by the caller): mat [ncell] in
 * 0..nmat-1, nodes nu [nnu >= 2] and T [nT >= 2] positive, finite, strictly
 * ascending, sig [nmat][nT][nnu] > 0, finite.  sigma is bilinear in (ln nu, ln T) on
 * ln sigma and constant beyond the end nodes; a group's opacity is Simpson's rule
 * over the group (Sec. 3); particle flights use sigma at their own nu and the cell's
 * T^n (the group opacity with UGKWP_FLAG_GROUP_SIGMA).  kappa is then unused.  The
 * device copies of an earlier table are kept until the context is destroyed. */
int ugkwp_set_opacity_table(ugkwp_ctx* ctx, int nmat, const int32_t* mat, int nnu, const double* nu, int nT,
                            const double* T, const double* sig);

/* Batched set-up: n_inst independent instances of one dimension with uneven
 * cell and group counts, all advanced by one launch per kernel per step. */
int ugkwp_init_batch(ugkwp_ctx* ctx, int n_inst, const ugkwp_instance* inst);

/* ---- time stepping ---- */

/* Advance every instance by nsteps steps of Algorithm 1.  Steps are enqueued on
 * the context stream up to 16 at a time without waiting: every launch of step n
 * checks on the device that the steps before it committed (else it returns at
 * once), and each step writes its own record of counters and sums.  The host
 * synchronises once per batch of up to 16 steps, books the committed steps,
 * takes up alone a step that needed more source-iteration sweeps than were
 * launched, and returns at the first step that failed; the state is then that
 * of the last committed step. */
int ugkwp_step(ugkwp_ctx* ctx, int nsteps);

/* ---- results ---- */

int ugkwp_num_instances(const ugkwp_ctx* ctx);
/* Fields of instance `inst` (or of all instances, concatenated, when inst < 0):
 * rho [ncell][G], T [ncell], rhop = survivor density [ncell][G]; any may be NULL. */
int ugkwp_get_fields(ugkwp_ctx* ctx, int inst, double* rho, double* T, double* rhop,
                     int dst_is_device);
/* Tallies of the last step for instance `inst`: gross face crossings
 * fx [(nx+1)*ny][G][2], fy [nx*(ny+1)][G][2] (direction 0 = +axis, 1 = -axis),
 * deposition dep and survivor weight surv [ncell][G], births nbirth [ncell][G],
 * new-particle weight wnew [ncell][G], static source Q [ncell][G].  Host arrays;
 * any may be NULL. */
int ugkwp_get_tallies(ugkwp_ctx* ctx, int inst, double* fx, double* fy, double* dep,
                      double* surv, int64_t* nbirth, double* wnew, double* Q);
int ugkwp_get_diag(ugkwp_ctx* ctx, ugkwp_diag* d);
/* Copy the running sums to *t (may be NULL); reset them to zero if reset != 0. */
int ugkwp_get_totals(ugkwp_ctx* ctx, ugkwp_totals* t, int reset);
/* Turn the timing of every phase (UGKWP_FLAG_PHASE_TIMES) on or off for the
 * following steps. */
int ugkwp_set_phase_times(ugkwp_ctx* ctx, int on);
/* Without phase timing, time the push of every step whose index is a multiple
 * of `every` (default 8; 1 times every push).  Each timed push adds two events
 * (a few microseconds of GPU time).  EINVAL if every < 1. */
int ugkwp_set_push_timing(ugkwp_ctx* ctx, int every);
/* Birth counter and step index of instance `inst`. */
int ugkwp_get_counters(ugkwp_ctx* ctx, int inst, uint64_t* birth_counter, int* step);

/* Particle pool (all instances).  cell is the context-global cell index. */
int64_t ugkwp_pool_size(ugkwp_ctx* ctx);
int ugkwp_get_pool(ugkwp_ctx* ctx, double* x, double* y, double* ox, double* oy,
                   double* nu, double* w, uint64_t* id, int32_t* cell, int32_t* g);
/* Replace the pool of a single-instance context (y, oy may be NULL in 1-D) and
 * set its birth counter; rhop [ncell][G] (may be NULL) sets the survivor density.
 * Particle ids and the birth counter must lie below 2^48 (the library keeps a
 * particle's group in the same 64-bit word); UGKWP_EINVAL otherwise.  A step
 * whose births could number a particle 2^48 or above fails with UGKWP_EPOOL
 * before it runs. */
int ugkwp_set_pool(ugkwp_ctx* ctx, int64_t n, const double* x, const double* y,
                   const double* ox, const double* oy, const double* nu, const double* w,
                   const uint64_t* id, const int32_t* cell, const int32_t* g,
                   uint64_t birth_counter, const double* rhop);

/* ---- checkpoint ----
 * A step of Algorithm 1 starts from rho^n, T^n, the surviving particles, the
 * survivor density rho^p and the birth counter; this library keys the random
 * numbers of every particle by its id and the step index.  That is the whole
 * state, and a run restored from it continues as
 * the uninterrupted run would (up to the order of floating-point tally sums,
 * which is not fixed on the GPU).
 *
 * ugkwp_state_bytes: size of the host buffer that ugkwp_get_state fills for the
 * context as it is now (the pool's slots count), or a negative code.
 * ugkwp_get_state: writes the committed state of every instance (rho, T, rho^p,
 * phi(T), birth counters, step index, the pool's slots in device order) into
 * buf (host, caller-owned, at least ugkwp_state_bytes bytes; UGKWP_EINVAL if
 * smaller).  Needs a context with opacity and material set.
 * ugkwp_set_state: restores such a buffer into a context set up with the same
 * mesh, instances, groups, boundary conditions, seeds, weights and constants
 * (checked through a fingerprint: UGKWP_EINVAL otherwise) and its opacity and
 * material set (they are not part of the state).  UGKWP_EPOOL if the pool does
 * not fit the capacity; UGKWP_EINVAL while an adjoint record is kept, or if the
 * buffer is truncated or holds an out-of-range particle or a non-positive T.
 * The last step's tallies read zero until the next step. */
int64_t ugkwp_state_bytes(ugkwp_ctx* ctx);
int ugkwp_get_state(ugkwp_ctx* ctx, void* buf, int64_t bytes);
int ugkwp_set_state(ugkwp_ctx* ctx, const void* buf, int64_t bytes);

/* ---- launch autotuner ----
 * Times the particle push on the context's current pool for launch shapes
 * (threads per block: 256, 512; persistent blocks per CU: half, one and
 * two times what fits at that block size; particles per thread: 1, 2, 4, 8)
 * and keeps the fastest for the following steps if it beats the default shape
 * (timed before and after the others, the faster of the two taken) by at
 * least 3%, else the default.  Only the
 * speed changes: the order in which the push adds to its tallies may differ,
 * which moves floating-point sums by rounding.  The tallies and counters of the
 * last step are restored.  Needs a non-empty pool (UGKWP_EINVAL otherwise). */
typedef struct {
    int ppt;                 /* particles per thread chosen                        */
    int blocks;              /* push blocks chosen                                 */
    int candidates;          /* shapes timed                                       */
    double us_best;          /* push time of the chosen shape, microseconds       */
    double us_default;       /* of the default shape (occupancy-filled grid of
                                256-thread blocks, 4 per thread)                  */
    int threads;             /* threads per push block chosen                     */
} ugkwp_tune_result;
int ugkwp_autotune(ugkwp_ctx* ctx, ugkwp_tune_result* res);

/* ---- adjoint of the macroscopic solve with the particle results held fixed ----
 *
 * The paper differentiates nothing; this is the derivative of the following
 * map.  A recorded forward run hands three particle-phase results per step to
 * its macroscopic solve: the net particle flux w^{fr,p} (Eq. wfrpFormula),
 * the survivor density rho^p, and which cell-groups sampled particles (the
 * choice between C4 - e^{-s} and C4 in the wave flux, Remark 3).  Holding them
 * fixed, a step maps (rho^n, T^n, kappa) to the fixed point (rho^{n+1}, T^{n+1})
 * of Eq. macroSysFinal solved by the source iteration of Appendix B, through
 * sigma = kappa S_g, s = c sigma dt / eps^2, C4(s), W(s), the harmonic face
 * opacity and C2 (Eq. C2Formula).  ugkwp_adjoint returns dJ/dkappa of
 * J = sum_cells dJdT[cell] T_cell after the last recorded step (dJdT = V C_v
 * gives the material energy) by a reverse sweep over the recorded steps, each
 * a transposed source iteration followed by the cotangents of the coefficients.
 *
 * Discrete particle events (sample counts, collisions, crossings) have no
 * derivative; a finite difference of the whole stochastic step is not what this
 * computes. */

/* Start a record with room for max_steps steps (device memory: per step about
 * 17 bytes per (cell, group) slot and 8 per cell), discarding any earlier one;
 * max_steps = 0 stops recording and frees it.  Each committed ugkwp_step then
 * adds one step; a step beyond max_steps fails with UGKWP_EINVAL before it
 * starts.  ugkwp_set_material restarts the record at the new initial state;
 * ugkwp_set_opacity fails while a record is kept. */
int ugkwp_record(ugkwp_ctx* ctx, int max_steps);
int ugkwp_recorded_steps(const ugkwp_ctx* ctx);

typedef struct {
    int steps;               /* recorded steps swept                              */
    int sweeps_launched;     /* transposed source-iteration sweeps launched, sum  */
    int sweeps_max;          /* largest per step                                   */
    double ms;               /* GPU time of the whole reverse sweep                */
    double ms_sweeps;        /* of which the transposed source-iteration sweeps
                                (incl. their convergence polls)                    */
    long long cell_group_updates; /* sum over steps and instances of cells x groups
                                x sweeps up to convergence                         */
} ugkwp_adjoint_stats;

/* dJdT [ncell] and grad_kappa [ncell][G] (all instances, concatenated as for
 * ugkwp_get_fields), host arrays, or device pointers read and written on the
 * context stream when ptrs_are_device = 1.  stats may be NULL.  Returns
 * UGKWP_EINVAL without recorded steps, UGKWP_ENOCONV if a transposed iteration
 * does not converge in 1000 sweeps (relative max-norm change 1e-15, 1e-13 after
 * 60 sweeps), UGKWP_ENONFINITE on a non-finite cotangent. */
int ugkwp_adjoint(ugkwp_ctx* ctx, const double* dJdT, double* grad_kappa, int ptrs_are_device,
                  ugkwp_adjoint_stats* stats);

/* ---- device building blocks, exposed for element-wise checks (host arrays) ---- */

/* out[i] = phi_g(T[i]) for g < G (group equilibrium value of rho, Sec. 2.1),
 * out laid out [n][G]. */
int ugkwp_eval_phi(int n, const double* T, int G, const double* nu_edges, double a, double c,
                   double* out);
/* C4(s), C4(s) - e^{-s} and C2(s)/dt (Eq. C2Formula) for each s[i] = c sigma dt / eps^2. */
int ugkwp_eval_coef(int n, const double* s, double* c4, double* w, double* c2_over_dt);
/* Uniform draws u(seed, id[i], step, purpose, d[i]) of the keyed Philox4x32-10 stream. */
int ugkwp_eval_uniform(int n, uint64_t seed, const uint64_t* id, uint32_t step,
                       uint32_t purpose, const uint32_t* d, double* out);
/* -ln(u[i]) for u[i] in (0, 1) as the particle flights evaluate it (free-flight
 * time t_f = -tau ln(eta), Sec. 2.2): within a few ulp of the correctly
 * rounded value.  EINVAL for n < 0 or a null array; u outside (0, 1) gives an
 * unspecified value. */
int ugkwp_eval_neg_log(int n, const double* u, double* out);
/* Linear-frequency sampling (Appendix A): slope beta at T[i] and the sampled nu
 * for U[i] in group [nl[i], nh[i]]. */
int ugkwp_eval_sample_nu(int n, const double* nl, const double* nh, const double* T,
                         const double* U, double* beta, double* nu);

#ifdef __cplusplus
}
#endif
#endif
