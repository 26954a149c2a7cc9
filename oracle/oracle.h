/*
 * FP64 CPU oracle for the UGKWP particle phase and source iteration
 * (Yang, Zhu, Liu & Xu, "Unified gas-kinetic wave-particle method for
 * frequency-dependent radiation transport", arXiv 2312.16981).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header or table with the GPU library.
 *
 * Every function follows one passage of the paper; the comment above each
 * names it.  Readings of passages that are silent or ambiguous are listed in
 * the design notes of the repository and restated at the point of use here.
 *
 * Parity status: the whole-step result has no printed value in the paper
 * ("parity unpinned" beyond the invariants the tests check: free streaming,
 * diffusion limit, equilibrium, 0-D relaxation, energy conservation, per-cell
 * particle ledger, symmetry, the particle/wave flux correspondence, collision
 * and reset laws, implicit 0-D steps with each material model).  The scalar
 * pieces (Philox, Planck integral, flux and slope coefficients, frequency
 * sampler and slope offset, Olson's ionisation fraction, heat capacity and
 * material energy, the opacity table) are pinned against independent
 * implementations, closed forms, quadrature or brute force.
 */
#ifndef UGKWP_ORACLE_H
#define UGKWP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- scalar building blocks ---------------- */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): out[4] = bijection of
 * the 128-bit counter ctr[4] under the 64-bit key key[2]. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform draw in (0,1) keyed by (seed, particle id, step, purpose, draw d).
 * Counter = (id_lo, id_hi, step, purpose<<24 | d/2), key = (seed_lo, seed_hi);
 * draw d uses words (r0,r1) if d is even, (r2,r3) if odd; u = (k + 1/2) 2^-52
 * with k = r_a<<20 | r_b>>12. */
double ora_uniform(uint64_t seed, uint64_t id, uint32_t step, uint32_t purpose, uint32_t d);
enum { ORA_PURPOSE_BIRTH = 1, ORA_PURPOSE_FLIGHT = 2 };

/* Incomplete Planck integral Pi(x) = int_x^inf t^3/(e^t - 1) dt. */
double ora_planck_tail(double x);
/* L(x) = int_0^x t^3/(e^t-1) dt  (small-argument Bernoulli series, x < 2). */
double ora_planck_head(double x);
/* Group equilibrium value of rho: phi_g(T) = a c T^4 (15/pi^4) int_{nl/T}^{nh/T} t^3/(e^t-1) dt. */
double ora_phi_group(double T, double nl, double nh, double a, double c);
/* d phi_g / dT. */
double ora_dphi_group(double T, double nl, double nh, double a, double c);

/* Flux coefficients of the UGKS free-transport / equilibrium fluxes as
 * functions of s = dt / tau = c sigma dt / eps^2. */
double ora_coef_c4(double s);          /* C4 = (1 - e^{-s}) / s           */
double ora_coef_w(double s);           /* W  = C4 - e^{-s}                 */
double ora_coef_c2_over_dt(double s);  /* C2 / dt  (C2 of the F^eq flux)   */
double ora_coef_c5_over_dt(double s); /* C5/dt (slope term of F^{fr,UGKS})     */
double ora_coef_w5_over_dt(double s); /* (C5 + (dt/2) e^{-s})/dt (F^{fr,wave})  */
/* Their derivatives in s (adjoint of the macroscopic solve). */
double ora_coef_c4_ds(double s);
double ora_coef_w_ds(double s);
double ora_coef_c2_over_dt_ds(double s);

/* Linear-frequency sampling: slope beta = (B(nh) - B(nl)) / B(nmid), limited
 * to [-2, 2], at temperature T. */
double ora_freq_slope(double nl, double nh, double T);
/* Offset u' in [-1/2, 1/2] with CDF of the density 1 + beta u' (|beta| <= 2)
 * equal to U. */
double ora_linear_offset(double beta, double U);
/* Inverse of the linear CDF on [nl, nh] with slope beta for a uniform U. */
double ora_sample_nu(double nl, double nh, double beta, double U);

/* ---------------- simulation ---------------- */

enum { ORA_BC_VACUUM = 0, ORA_BC_PLANCK = 1, ORA_BC_REFLECT = 2 };
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_EPOOL = -3,
       ORA_ENOCONV = -4, ORA_ENONFINITE = -5 };
enum { ORA_FLAG_GROUP_SIGMA = 1,    /* flights use the group (Simpson) sigma */
       ORA_FLAG_SI_LINEARIZED = 8,  /* source iteration with the emission linearized
                                       about T^k (a local Newton step) */
       ORA_FLAG_SLOPES = 16,        /* MINMOD slopes of the wave part: the C5 terms of the
                                       wave flux, new particles placed along the slope */
       ORA_FLAG_WAVE_ITER = 32,     /* wave flux from each sweep's iterate rho^k
                                       (Algorithm 2) instead of the start of the step */
       ORA_FLAG_BOUNDARY_PARTICLES = 64 /* Planckian boundaries also emit collisionless
                                       particles from their ghost cells */ };

typedef struct {
    int dim;              /* 1 or 2 */
    int nx, ny;           /* ny = 1 for dim 1 */
    double x0, x1, y0, y1;
    int bc[4];            /* XLO, XHI, YLO, YHI */
    double bcT[4];        /* Planckian boundary temperatures */
    int G;
    const double* nu;     /* G+1 ascending edges */
    double nu_power;      /* sigma(nu) = kappa * nu^-p */
    double c, a, eps, dt;
    double w_ref;         /* particle energy per unit volume: target weight w_ref * V */
    int64_t n_cap;        /* max births per (cell, group) per step */
    uint64_t seed;
    int64_t pool_cap;
    int si_max_iters;
    double si_tol;
    int flags;
    /* numerical collision time of thin-thick-joint cells (Sec. 3.2, second
     * case): tau_num = eps^2/(c sigma) + C |T^l - T^r|/(T^l + T^r) dt replaces
     * tau in the sampling fraction e^{-dt/tau} when C > 0, in the cells that
     * share a face across which sigma changes by a factor >= jump. */
    double tau_num_C;
    double tau_num_jump;
    /* temperature-dependent opacity sigma(nu, T) = kappa nu^-p T^-q (Sec. 3.1):
     * q = T_power.  The particles and the wave split of a step take T^n; the
     * source iteration re-evaluates sigma, lambda and the face coefficients
     * from its own iterate T^k in every sweep (Algorithm 2). */
    double T_power;
    /* 1: the stimulated-emission factor (1 - e^{-nu/T}) multiplies sigma, as in
     * Sec. 3.3's gamma0 (1 - e^{-h nu / kT}) / (h nu)^3; the group opacity is
     * then Simpson's mean of nu^-p (1 - e^{-nu/T}) over the group.  0: none. */
    int opacity_stim;
} ora_params;

typedef struct ora_sim ora_sim;

typedef struct {
    int64_t n_alive_in, n_births, n_alive_out, n_collided, n_exited;
    int64_t n_crossings;
    int sweeps;
    double e_start, e_end;      /* total energy (radiation rho/c + material) */
    double inflow_wave, inflow_eq, exit_particles, injection;
    double residual;            /* e_end - e_start - (inflow_wave + inflow_eq + inflow_particles
                                   - exit + injection) */
    double si_drho, si_rho, si_dT, si_T;
    double inflow_particles;    /* boundary-source particles that entered the domain */
    int64_t n_ghost_births, n_ghost_entered;
} ora_diag;

ora_sim* ora_create(const ora_params* p);
void ora_destroy(ora_sim* s);
int ora_set_opacity(ora_sim* s, const double* kappa);            /* [ncell][G] */
int ora_set_material(ora_sim* s, const double* cv, const double* T0,
                     const double* Tr0, const unsigned char* pinned);
/* A volumetric radiation source (Sec. 3.4: Q(x), switched off at a time):
 * q [cell][G] adds dt q to rho of every step that starts before t_off. */
int ora_set_source(ora_sim* s, const double* q, double t_off);
/* The source Q(x) = B(nu, Ts) f(x) of Sec. 3.4-3.5 added to the transport
 * equation's right side: its rate in rho is q = (c/eps^2) f_i phi_g(Ts). */
int ora_set_source_planck(ora_sim* s, const double* f, double Ts, double t_off);
/* A tabulated opacity sigma(nu, T) per material (Sec. 3.4-3.5), in place of
 * kappa nu^-p T^-q: mat [cell] in 0..nmat-1, nodes nu[nnu], T[nT] ascending,
 * sig [nmat][nT][nnu] > 0, interpolated bilinearly in (ln nu, ln T) on ln sigma
 * and held constant beyond the end nodes. */
int ora_set_opacity_table(ora_sim* s, int nmat, const int32_t* mat, int nnu, const double* nu,
                          int nT, const double* T, const double* sig);
/* Olson's heat capacity (Sec. 3.4, Eq. cvolson) in the cells with H[i] > 0: the
 * volumetric heat capacity of cell i at T becomes H_i [1 + alpha + (T + chi_i)
 * dalpha/dT] in place of its constant C_v (the printed a T_keV^3 is the unit
 * a (1 keV)^3, folded into H), and the material energy U(T) = H_i [T (1 + alpha)
 * + chi_i alpha], whose derivative that is.  The source iteration then solves
 * U(T^{n+1}) = U(T^n) + exchange, the energy form of Eq. macroEquImplicit's
 * material line: the literal iteration inverts U for T^{k+1}, the linearized one
 * takes one Newton step at T^k.  NULL H: off. */
int ora_set_heat_capacity(ora_sim* s, const double* H, const double* chi);
/* The table's sigma of material m at (nu, T), and Olson's alpha and its derivative. */
double ora_table_sigma(const ora_sim* s, int m, double nu, double T);
double ora_olson_alpha(double T, double chi, double* dalpha);
double ora_heat_capacity(const ora_sim* s, int cell, double T);
double ora_material_energy(const ora_sim* s, int cell, double T);
int ora_step(ora_sim* s, int nsteps);
int ora_get_fields(const ora_sim* s, double* rho, double* T, double* rhop);
/* Tallies of the last step: face gross crossings [face][G][2] (x-faces, then
 * y-faces), deposition and survivor weights [cell][G], births per (cell, g),
 * new-particle weight per (cell, g), static source Q [cell][G]. */
int ora_get_tallies(const ora_sim* s, double* fx, double* fy, double* dep,
                    double* surv, int64_t* nbirth, double* wnew, double* Q);
int64_t ora_pool_size(const ora_sim* s);
int ora_get_pool(const ora_sim* s, double* x, double* y, double* ox, double* oy,
                 double* nu, double* w, uint64_t* id, int32_t* cell, int32_t* g);
int ora_set_pool(ora_sim* s, int64_t n, const double* x, const double* y,
                 const double* ox, const double* oy, const double* nu,
                 const double* w, const uint64_t* id, const int32_t* cell,
                 const int32_t* g, uint64_t birth_counter, const double* rhop);
/* Restore a saved state's radiation density rho [cell][G], temperature T [cell]
 * and step index (the pool, birth counter and survivor density go through
 * ora_set_pool).  Together they are the whole state a step starts from. */
int ora_set_fields(ora_sim* s, const double* rho, const double* T, int step);
int ora_get_diag(const ora_sim* s, ora_diag* d);
int ora_get_counters(const ora_sim* s, uint64_t* birth_counter, int* step);
/* Per-(cell, g) particle ledger of the last step: weight present at the
 * start (survivors + births) of every (cell, g). */
int ora_get_start_weights(const ora_sim* s, double* start);

/* ---------------- adjoint of the frozen-tally macroscopic map ----------------
 * With recording on, every step stores what the particle phase handed to the
 * macroscopic solve (net particle flux, survivor density, sampled flags) plus
 * the start-of-step state.  ora_adjoint returns dJ/dkappa for
 * J = sum_i V_i sum_k dJdT[i] * T_i(final) (dJdT = C_v gives the material energy),
 * holding the recorded particle outputs fixed.  ora_replay_frozen reruns the
 * recorded steps from the recorded initial state with a new kappa and the same
 * frozen particle outputs (used for finite differences). */
int ora_record(ora_sim* s, int on);
int ora_adjoint(ora_sim* s, const double* dJdT, double* grad_kappa);
int ora_replay_frozen(ora_sim* s, const double* kappa, double* T_final);
/* (cell, group) updates done by the transposed iterations of the last ora_adjoint. */
long long ora_adjoint_updates(void);

#ifdef __cplusplus
}
#endif
#endif
