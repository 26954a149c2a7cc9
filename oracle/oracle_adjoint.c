/* placeholder, replaced below */
#include "oracle.h"
int ora_adjoint(ora_sim* s, const double* dJdT, double* grad_kappa) { (void)s; (void)dJdT; (void)grad_kappa; return ORA_EINVAL; }
int ora_replay_frozen(ora_sim* s, const double* kappa, double* T_final) { (void)s; (void)kappa; (void)T_final; return ORA_EINVAL; }
