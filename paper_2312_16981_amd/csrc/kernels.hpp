// Launchers of the UGKWP kernels (kernels.hip), called by the host runtime.
#pragma once
#include "common.hpp"
#include "device_math.hpp"

namespace ugk {

// Up to 8 device ranges of 64-bit words cleared at the start of a step.
struct ZeroList {
    int n;
    void* ptr[8];
    int64_t words[8];
};

hipError_t set_head_series(const HeadSeries& hs);

void launch_tables(const Dev& D, const Consts& K, hipStream_t st);
// ln of n doubles in place (the opacity table's nodes and values at set-up).
void launch_tab_logs(double* v, int64_t n, hipStream_t st);
// the nu positions of every group's Simpson points in the table (after the logs)
void launch_tab_groups(const Dev& D, const Consts& K, int64_t n_edges, hipStream_t st);
void launch_face_D(const Dev& D, const Consts& K, int inst, int axis, int64_t nslots, hipStream_t st);
void launch_ghost_phi(const Dev& D, const Consts& K, double* phib, hipStream_t st);
void launch_init_rho(const Dev& D, const Consts& K, const double* Tr0, hipStream_t st);
// q[slot] = (c/eps^2) f[cell] phi_g(Ts): a Planckian volumetric source's rate
void launch_source_planck(const Dev& D, const Consts& K, double* q, const double* f, double Ts, hipStream_t st);
// clears Z, counts particles per slot and scans the counts into birth offsets
void launch_count_scan(const Dev& D, const Consts& K, const ZeroList& Z, int64_t* part, hipStream_t st);
int64_t count_partials_size();    // entries of `part` the small-context path needs
int64_t scan_partials_size(int64_t n);
// Scans of a step's launch sequence return at once when their step's gate is
// shut (see gate_open); expect = GATE_OFF runs them unconditionally.
struct ScanGate {
    const uint32_t* step;
    uint32_t expect;
};
ScanGate scan_gate(const Dev& D, const Consts& K, uint32_t after);
void launch_scan(const ScanGate& q, const int32_t* in, int64_t n, int64_t* part, int64_t* out, int64_t* total,
                 hipStream_t st);
void launch_sample(int dim, const Dev& D, const Consts& K, const Pool& P, hipStream_t st);
// slopes of the wave part (UGKWP_FLAG_SLOPES) from rho^h = src (minus rhop when sub_rhop)
void launch_slopes(int dim, const Dev& D, const Consts& K, const double* src, bool sub_rhop, hipStream_t st);
// Launch shape of the push: persistent blocks, threads per block (256 or 512)
// and particles per thread.
struct PushShape {
    int blocks;
    int ppt;
    int threads;
};
PushShape push_default_shape(int dim, const Consts& K);   // occupancy-filled grid of 256-thread blocks, 4 per thread
int push_blocks_per_cu(int dim, const Consts& K, int threads);   // resident blocks per CU (occupancy)
int push_num_cus();
void launch_push(int dim, const Dev& D, const Consts& K, const Pool& A, const Pool& B, const PushShape& sh,
                 hipStream_t st);
void launch_sort_scatter(int dim, const Dev& D, const Consts& K, const Pool& B, const Pool& A, hipStream_t st);
// sweeps k0..k1-1 of the source iteration, each sweep's convergence decided
// before the next: for a single instance in the next sweep (the last one's in
// launch_finish), else by a decide launch after every sweep
void launch_si_sweeps(const Dev& D, const Consts& K, int k0, int k1, hipStream_t st);
// commit and energy sums; reduce_diag folds the sums' sub-slots on the device;
// last_sweep is the last sweep launched (a single instance's convergence
// after it is decided by the commit launch); the commit also sums the
// survivor counts of the push's push_blocks blocks
void launch_finish(const Dev& D, const Consts& K, bool reduce_diag, int last_sweep, int push_blocks,
                   hipStream_t st);

void launch_eval_phi(int n, const double* T, int G, const double* nu, double a, double c, double* out,
                     hipStream_t st);
void launch_eval_coef(int n, const double* s, double* c4, double* w, double* c2, hipStream_t st);
void launch_eval_uniform(int n, uint64_t seed, const uint64_t* id, uint32_t step, uint32_t purpose,
                         const uint32_t* d, double* out, hipStream_t st);
void launch_eval_neg_log(int n, const double* u, double* out, hipStream_t st);
void launch_eval_sample_nu(int n, const double* nl, const double* nh, const double* T, const double* U,
                           double* beta, double* nu, hipStream_t st);

}  // namespace ugk
