/*
 * Oracle: plain, slow, FP64 CPU reference of the D2Q17 variant of the van der
 * Waals lattice Boltzmann step of Coclite, Gonnella and Lamura,
 * arXiv:1307.6703. The paper (the remark after Eq.(nav)) names a third-order
 * model with seventeen velocities as the way to remove the spurious term of
 * order u*^3 from its Navier-Stokes equation; it gives no formulas for it.
 * This file writes that model out: the same force (Eq.(force2) with
 * Eq.(eqstate) and Eq.(periodicforce)), the same stencils (Eq.(xstencil),
 * Eq.(laplstencil)) and the same step (pull streaming and BGK collision with a
 * forcing term, Eq.(evoleq), velocity u* of Eq.(newvel)), with the equilibrium
 * and the forcing term expanded to third order in Hermite polynomials.
 * Periodic in x and y only: the paper's wall rule is written for D2Q9.
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the tests, by the smoke check and
 * by the CPU-baseline leg of the benchmark; the product library never links,
 * loads or calls it, and it includes no header of the product.
 *
 * Velocity set. Integer vectors c_i: the rest vector, (+-1, 0) and (0, +-1),
 * (+-1, +-1), (+-2, +-2), (+-3, 0) and (0, +-3). With a scale r, xi_i = r c_i
 * are the abscissas of a quadrature of the unit Gaussian. Its weights w_i
 * (one per shell) and r^2 = s follow from asking that the lattice sums of
 * xi_x^a xi_y^b equal the Gaussian's moments for every a + b <= 7 (odd ones
 * vanish by symmetry): six equations, sum w = 1, <x^2> = 1, <x^4> = 3,
 * <x^2 y^2> = 1, <x^6> = 15, <x^4 y^2> = 3. With v = 1/s the four shell
 * equations of order 4 and 6 give
 *   w(1,0) = 9v^2/8 - 3v^3/4,   w(1,1) = v^2/3 - v^3/4,
 *   w(2,2) = (3v^3 - v^2)/192,  w(3,0) = (6v^3 - v^2)/648,
 * the second-order equation then reads 75 v^2 - 125 v + 36 = 0, whose root
 * with positive weights is s = (125 + 5 sqrt(193))/72 = 2.70086..., and
 * w(0,0) = 1 - 4 (w(1,0) + w(1,1) + w(2,2) + w(3,0)).
 *
 * Units. Lattice units, dx = dt = 1, c_i integer. The reference temperature
 * of the lattice (its sound speed squared) is theta0 = 1/s; the paper's
 * reduced temperature T (T/T_c with T_c the reference) is theta = T theta0.
 * In the paper's units (reference temperature 1, dx = 1) the speeds are
 * e_i = r c_i, so dt = 1/r; converting: tau_l = r tau, force density
 * F_l = F_p / s, pressure p_l = p_p / s.
 *
 * Equilibrium (third-order Hermite expansion of the Maxwellian at temperature
 * theta, with dth = theta - theta0, H2 = c c - theta0 I,
 * H3 = c c c - theta0 (c I + I c + ...)):
 *   f_eq_i = w_i n [1 + c.u/theta0
 *                     + ((c.u)^2 - theta0 u^2 + dth (c^2 - 2 theta0)) / (2 theta0^2)
 *                     + c.u ((c.u)^2 - 3 theta0 u^2 + 3 dth (c^2 - 4 theta0)) / (6 theta0^3)].
 * Its moments up to the third are exact: n, n u, n (u u + theta I),
 * n (u u u + theta (u I + I u + ...)). The third is the one D2Q9 cannot
 * carry; the (1 - T) terms of Eq.(coeff) compensate part of that defect in
 * D2Q9 and have no counterpart here.
 *
 * Forcing term (Eq.(forceterm) carried to third order: the Hermite
 * coefficients of -g.grad_xi f_eq with g = F/n, times 1 - 1/(2 tau_l) as in
 * Eq.(coeff), at u = u*):
 *   F_i = w_i (1 - 1/(2 tau_l)) [c.F/theta0
 *          + (c.u c.F - theta0 u.F)/theta0^2
 *          + (c.F ((c.u)^2 - theta0 u^2) - 2 theta0 u.F c.u + dth c.F (c^2 - 4 theta0))
 *            / (2 theta0^3)].
 * Its moments: 0, (1 - 1/(2 tau_l)) times F, u F + F u, and
 * (F u u + u F u + u u F) + theta (F I + I F + ...).
 *
 * Consequences the tests pin: the shear viscosity is theta (tau_l - 1/2)
 * (lattice units), i.e. eta = n T (tau - dt/2) in the paper's units, and it
 * does not change when the fluid moves as a whole (D2Q9's does, by the u*^3
 * term).
 *
 * Rounding: built with -O2 -ffp-contract=off (no FMA contraction).
 *
 * Layout: populations S[i][y][x], x fastest, i = 0..16 in the order of
 * lbo17_lattice: 0 rest; 1-4 (1,0), (0,1), (-1,0), (0,-1); 5-8 (1,1),
 * (-1,1), (-1,-1), (1,-1); 9-12 the same diagonals times 2; 13-16 the axis
 * vectors times 3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "lb_oracle.h"

static const int CX17[17] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, -2, -2, 2, 3, 0, -3, 0};
static const int CY17[17] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 2, 2, -2, -2, 0, 3, 0, -3};

/* Lattice: velocity components, weights and the scale s = r^2 (see the
 * file header for the derivation). Any output may be NULL. */
void lbo17_lattice(int cx[17], int cy[17], double w[17], double *s_out) {
  double s = (125.0 + 5.0 * sqrt(193.0)) / 72.0;
  double v = 1.0 / s, v2 = v * v, v3 = v2 * v;
  double w10 = 9.0 * v2 / 8.0 - 0.75 * v3;
  double w11 = v2 / 3.0 - 0.25 * v3;
  double w22 = (3.0 * v3 - v2) / 192.0;
  double w30 = (6.0 * v3 - v2) / 648.0;
  double w00 = 1.0 - 4.0 * (w10 + w11 + w22 + w30);
  for (int i = 0; i < 17; i++) {
    if (cx) cx[i] = CX17[i];
    if (cy) cy[i] = CY17[i];
    if (w) {
      int a = abs(CX17[i]), b = abs(CY17[i]);
      if (a == 0 && b == 0) w[i] = w00;
      else if (a + b == 1) w[i] = w10;
      else if (a == 1 && b == 1) w[i] = w11;
      else if (a == 2) w[i] = w22;
      else w[i] = w30;
    }
  }
  if (s_out) *s_out = s;
}

/* The equilibrium of the file header; u in lattice units. */
void lbo17_feq(double n, double ux, double uy, double T, double out[17]) {
  double w[17], s;
  lbo17_lattice(NULL, NULL, w, &s);
  double th0 = 1.0 / s, dth = (T - 1.0) * th0;
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 17; i++) {
    double cu = CX17[i] * ux + CY17[i] * uy;
    double cc = (double)(CX17[i] * CX17[i] + CY17[i] * CY17[i]);
    double e1 = cu / th0;
    double e2 = (cu * cu - th0 * uu + dth * (cc - 2.0 * th0)) / (2.0 * th0 * th0);
    double e3 = cu * (cu * cu - 3.0 * th0 * uu + 3.0 * dth * (cc - 4.0 * th0)) /
                (6.0 * th0 * th0 * th0);
    out[i] = w[i] * n * (1.0 + e1 + e2 + e3);
  }
}

/* The forcing term of the file header (per step, lattice units), at the
 * velocity u = u* and the force density F (lattice units). */
void lbo17_forcing(double ux, double uy, double Fx, double Fy, double T, double tau_l,
                   double out[17]) {
  double w[17], s;
  lbo17_lattice(NULL, NULL, w, &s);
  double th0 = 1.0 / s, dth = (T - 1.0) * th0;
  double pre = 1.0 - 0.5 / tau_l;
  double uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
  for (int i = 0; i < 17; i++) {
    double cu = CX17[i] * ux + CY17[i] * uy;
    double cF = CX17[i] * Fx + CY17[i] * Fy;
    double cc = (double)(CX17[i] * CX17[i] + CY17[i] * CY17[i]);
    double b1 = cF / th0;
    double b2 = (cu * cF - th0 * uF) / (th0 * th0);
    double b3 = (cF * (cu * cu - th0 * uu) - 2.0 * th0 * uF * cu + dth * cF * (cc - 4.0 * th0)) /
                (2.0 * th0 * th0 * th0);
    out[i] = w[i] * pre * (b1 + b2 + b3);
  }
}

static int wrap(int v, int L) {
  int r = v % L;
  return r < 0 ? r + L : r;
}

static int check_params(const lbo_params *p) {
  return p->Lx >= 1 && p->Ly >= 1 && p->y_periodic == 1 && p->collision == 0;
}

/* S(0) = f_eq(n0, u0; T). u0 may be NULL (fluid at rest). */
int lbo17_init(const lbo_params *p, const double *n0, const double *ux0, const double *uy0,
               double *S) {
  if (!check_params(p)) return -1;
  size_t nn = (size_t)p->Lx * p->Ly;
  for (size_t k = 0; k < nn; k++) {
    double fe[17];
    lbo17_feq(n0[k], ux0 ? ux0[k] : 0.0, uy0 ? uy0[k] : 0.0, p->T, fe);
    for (int i = 0; i < 17; i++) S[i * nn + k] = fe[i];
  }
  return 0;
}

/*
 * One step: S_in = post-collision populations after k-1 steps, S_out those
 * after k steps. n_out, ux_out, uy_out (may be NULL) receive the density and
 * the velocity u* computed inside the step (after streaming, before
 * collision). fext: per-column F_ext,x in paper units (force density), may be
 * NULL. Returns 0, or -1 on bad parameters (walls, regularised collision) or
 * allocation failure.
 */
int lbo17_step(const lbo_params *p, const double *fext, const double *S_in, double *S_out,
               double *n_out, double *ux_out, double *uy_out) {
  if (!check_params(p)) return -1;
  const int Lx = p->Lx, Ly = p->Ly;
  const size_t nn = (size_t)Lx * Ly;
  double w[17], s;
  lbo17_lattice(NULL, NULL, w, &s);
  const double tau_l = sqrt(s) * p->tau;
  const double omega = 1.0 / tau_l;
  const double T = p->T;

  double *f = malloc(17 * nn * sizeof(double));
  double *n = malloc(nn * sizeof(double));
  double *P = malloc(nn * sizeof(double));
  double *L = malloc(nn * sizeof(double));
  double *gPx = malloc(nn * sizeof(double));
  double *gPy = malloc(nn * sizeof(double));
  double *gLx = malloc(nn * sizeof(double));
  double *gLy = malloc(nn * sizeof(double));
  if (!f || !n || !P || !L || !gPx || !gPy || !gLx || !gLy) {
    free(f); free(n); free(P); free(L); free(gPx); free(gPy); free(gLx); free(gLy);
    return -1;
  }

  /* 1. Pull streaming (left side of Eq.(evoleq)): f_i(x) = S_i(x - c_i),
   *    periodic in both directions. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++)
      for (int i = 0; i < 17; i++)
        f[i * nn + (size_t)y * Lx + x] =
            S_in[i * nn + (size_t)wrap(y - CY17[i], Ly) * Lx + wrap(x - CX17[i], Lx)];

  /* 2. Density and the pressure term p^i - p^w (Eq.(force2), Eq.(eqstate)). */
#pragma omp parallel for schedule(static)
  for (size_t k = 0; k < nn; k++) {
    double m = 0.0;
    for (int i = 0; i < 17; i++) m += f[i * nn + k];
    n[k] = m;
    P[k] = lbo_pressure_term(m, T);
  }

  /* 3. Laplacian of n, then the gradients of P and of the Laplacian. */
  lbo_apply_stencils(p, n, 1.0, NULL, NULL, L);
  lbo_apply_stencils(p, P, 1.0, gPx, gPy, NULL);
  lbo_apply_stencils(p, L, 1.0, gLx, gLy, NULL);

  /* 4-6. Per node: force (paper units, then / s), u* of Eq.(newvel),
   *      equilibrium, forcing and BGK collision (Eq.(evoleq)). */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
      double nk = n[k];
      double Fx = (gPx[k] + p->kappa * nk * gLx[k] + (fext ? fext[x] : 0.0)) / s;
      double Fy = (gPy[k] + p->kappa * nk * gLy[k]) / s;
      double jx = 0.5 * Fx, jy = 0.5 * Fy;
      for (int i = 0; i < 17; i++) {
        jx += f[i * nn + k] * CX17[i];
        jy += f[i * nn + k] * CY17[i];
      }
      double ux = jx / nk, uy = jy / nk;
      double fe[17], fo[17];
      lbo17_feq(nk, ux, uy, T, fe);
      lbo17_forcing(ux, uy, Fx, Fy, T, tau_l, fo);
      for (int i = 0; i < 17; i++) {
        double fi = f[i * nn + k];
        S_out[i * nn + k] = fi - omega * (fi - fe[i]) + fo[i];
      }
      if (n_out) n_out[k] = nk;
      if (ux_out) ux_out[k] = ux;
      if (uy_out) uy_out[k] = uy;
    }

  free(f); free(n); free(P); free(L); free(gPx); free(gPy); free(gLx); free(gLy);
  return 0;
}

/* Run `steps` steps in place on S. nthreads <= 0 keeps the OpenMP default.
 * Returns the threads used, or -1. */
int lbo17_run(const lbo_params *p, const double *fext, double *S, int64_t steps, double *n_out,
              double *ux_out, double *uy_out, int nthreads) {
  if (!check_params(p)) return -1;
  size_t nn = (size_t)p->Lx * p->Ly;
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  used = omp_get_max_threads();
#else
  (void)nthreads;
#endif
  double *tmp = malloc(17 * nn * sizeof(double));
  if (!tmp) return -1;
  for (int64_t k = 0; k < steps; k++) {
    int last = (k == steps - 1);
    if (lbo17_step(p, fext, S, tmp, last ? n_out : NULL, last ? ux_out : NULL,
                   last ? uy_out : NULL) != 0) {
      free(tmp);
      return -1;
    }
    memcpy(S, tmp, 17 * nn * sizeof(double));
  }
  free(tmp);
  return used;
}
