/*
 * Oracle (test infrastructure only): the parameter block and the pieces of
 * the D2Q9 oracle (lb_oracle.c) that the D2Q17 oracle (d2q17_oracle.c) also
 * calls: the pressure term and the stencils, which do not depend on the
 * velocity set. Neither file is part of, or shared with, the product library.
 */
#ifndef LB_ORACLE_H
#define LB_ORACLE_H

#include <stdint.h>

typedef struct {
  int32_t Lx, Ly;
  int32_t y_periodic; /* 1: periodic in y; 0: moving walls at rows 0, Ly-1 */
  int32_t collision;  /* 0: BGK, Eq.(evoleq); 1: regularised (lbo_regularize) */
  double T;     /* reduced temperature */
  double tau;   /* relaxation time, paper units */
  double kappa; /* surface-tension parameter, paper units */
  double N, Q;  /* stencil parameters; M = (1-2N)/4, R = (1-Q)/2 */
  double U;     /* wall speed (lattice units): lower wall -U, upper +U */
} lbo_params;

/* p^i - p^w of Eq.(force2) with Eq.(eqstate), paper units. */
double lbo_pressure_term(double n, double T);

/* d/dx, d/dy (Eq.(xstencil)) and the Laplacian (Eq.(laplstencil)) of a
 * [Ly][Lx] field, with the lattice's boundary handling; any output may be
 * NULL. */
void lbo_apply_stencils(const lbo_params *p, const double *phi, double par,
                        double *gx, double *gy, double *lap);

#endif
