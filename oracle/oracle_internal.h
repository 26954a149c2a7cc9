/*
 * Internal interface between the oracle's forward step (oracle_sim.c) and its
 * adjoint (oracle_adjoint.c).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#ifndef UGKWP_ORACLE_INTERNAL_H
#define UGKWP_ORACLE_INTERNAL_H
#include "oracle.h"

/* What one recorded step handed from its particle phase to its macroscopic
 * solve, plus the state it started from. */
typedef struct {
    double* rho;            /* rho^n at the start of the step [ncell][G]         */
    double* T;              /* T^n [ncell]                                        */
    double* rhop;           /* survivor density rho^p entering the step           */
    double* rhoh;           /* rho^h = rho^n - rho^p                              */
    double* wnet;           /* net particle flux w^{fr,p} = in - out [ncell][G]   */
    unsigned char* sampled; /* 1 where the cell-group sampled particles (N >= 1)  */
} ora_rec_step;

int ora__nrec(const ora_sim* s);
const ora_rec_step* ora__rec(const ora_sim* s, int k);
const ora_params* ora__params(const ora_sim* s);
const double* ora__simpson(const ora_sim* s);
const double* ora__cv(const ora_sim* s);
const unsigned char* ora__pinned(const ora_sim* s);
const double* ora__kappa_rec(const ora_sim* s);   /* kappa of the recorded run */
const double* ora__T(const ora_sim* s);           /* current (final) temperature */
const double* ora__rho(const ora_sim* s);         /* current (final) rho */
double ora__V(const ora_sim* s);
double ora__dx(const ora_sim* s);
double ora__dy(const ora_sim* s);

#endif
