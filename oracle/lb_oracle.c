/*
 * Oracle: plain, slow, FP64 CPU reference of the isothermal D2Q9 lattice
 * Boltzmann step for a van der Waals liquid-vapor fluid of Coclite, Gonnella
 * and Lamura, "Pattern Formation in Liquid-Vapor Systems under Periodic
 * Potential and Shear" (arXiv:1307.6703).
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the tests, by the smoke check and
 * by the CPU-baseline leg of the benchmark; the product library never links,
 * loads or calls it, and it includes no header of the product.
 *
 * Units. Everything here is in lattice units: dx = dt = 1 and the D2Q9
 * velocities c_i have components in {0, +1, -1}. The paper (Sec. III) works
 * with dx = 1, dt = sqrt(3)/3 and speeds e_i = sqrt(3) c_i. Converting its
 * equations gives:
 *   omega = dt/tau = 1/tau_l with tau_l = sqrt(3) tau (tau in paper units);
 *   force density F_l = F_p / 3; pressure p_l = p_p / 3;
 *   f_eq_i = w_i n [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2 + (T-1)(3|c|^2-2)/2].
 * The paper's temperature T is T/T_c; T_c equals the reference temperature.
 *
 * Rounding: built with -O2 -ffp-contract=off (no FMA contraction).
 *
 * Layout: populations S[i][y][x], x fastest, i = 0..8 in the order
 * 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE (Sec. II).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "lb_oracle.h"

/* D2Q9 abscissas and weights (Sec. II, the Gauss-Hermite velocity set). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* ---------------------------------------------------------------------- */
/* Pointwise pieces, exported so tests can pin each one on its own.        */
/* ---------------------------------------------------------------------- */

/* Eq.(eqfunc) in lattice units. */
void lbo_feq(double n, double ux, double uy, double T, double out[9]) {
  for (int i = 0; i < 9; i++) {
    double cu = CX[i] * ux + CY[i] * uy;
    double cc = (double)(CX[i] * CX[i] + CY[i] * CY[i]);
    out[i] = W[i] * n *
             (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy) +
              0.5 * (T - 1.0) * (3.0 * cc - 2.0));
  }
}

/* Eq.(forceterm) with the coefficients of Eq.(coeff) (A = 0), converted to
 * lattice units and multiplied by dt:
 *   dt F_i = w_i s [3 c.F + X:(3 c c - I)/2],  s = 1 - 1/(2 tau_l),
 *   X = 3(u F + F u) + (1-T)(u grad n + grad n u + D I),  D = div(n u). */
void lbo_forcing(double ux, double uy, double Fx, double Fy, double dnx,
                 double dny, double D, double T, double tau_l,
                 double out[9]) {
  double s = 1.0 - 0.5 / tau_l;
  double Xxx = 3.0 * (ux * Fx + Fx * ux) + (1.0 - T) * (ux * dnx + dnx * ux + D);
  double Xyy = 3.0 * (uy * Fy + Fy * uy) + (1.0 - T) * (uy * dny + dny * uy + D);
  double Xxy = 3.0 * (ux * Fy + Fx * uy) + (1.0 - T) * (ux * dny + dnx * uy);
  double Xyx = 3.0 * (uy * Fx + Fy * ux) + (1.0 - T) * (uy * dnx + dny * ux);
  for (int i = 0; i < 9; i++) {
    double cx = CX[i], cy = CY[i];
    double cF = cx * Fx + cy * Fy;
    /* X : (3 c c - I) */
    double XQ = Xxx * (3.0 * cx * cx - 1.0) + Xyy * (3.0 * cy * cy - 1.0) +
                Xxy * (3.0 * cx * cy) + Xyx * (3.0 * cy * cx);
    out[i] = W[i] * s * (3.0 * cF + 0.5 * XQ);
  }
}

/* Regularisation (Sec. II: the step that re-projects the post-collision
 * populations onto the Hermite space, which the paper names and leaves out
 * at its Knudsen numbers). The equilibrium of Eq.(eqfunc) and the forcing of
 * Eq.(forceterm) are expansions in the Hermite polynomials of order <= 2,
 * H0 = 1, H1 = c, H2 = c c - I/3 (lattice units, c_s^2 = 1/3); the
 * projection keeps the part of a population vector in that space:
 *   a0 = sum_i h_i,  a1 = sum_i h_i c_i,  a2 = sum_i h_i (c_i c_i - I/3),
 *   P[h]_i = w_i [a0 + 3 a1.c_i + (9/2) a2 : (c_i c_i - I/3)].
 * The D2Q9 weights integrate products of these polynomials exactly, so P
 * keeps the moments of order 0, 1, 2 and removes the rest (the terms of
 * order 3 and 4 that D2Q9 can also carry). */
void lbo_regularize(const double h[9], double out[9]) {
  double a0 = 0.0, a1x = 0.0, a1y = 0.0, pxx = 0.0, pyy = 0.0, pxy = 0.0;
  for (int i = 0; i < 9; i++) {
    a0 += h[i];
    a1x += h[i] * CX[i];
    a1y += h[i] * CY[i];
    pxx += h[i] * CX[i] * CX[i];
    pyy += h[i] * CY[i] * CY[i];
    pxy += h[i] * CX[i] * CY[i];
  }
  double a2xx = pxx - a0 / 3.0, a2yy = pyy - a0 / 3.0, a2xy = pxy;
  for (int i = 0; i < 9; i++) {
    double hxx = CX[i] * CX[i] - 1.0 / 3.0, hyy = CY[i] * CY[i] - 1.0 / 3.0;
    double hxy = (double)(CX[i] * CY[i]);
    out[i] = W[i] * (a0 + 3.0 * (a1x * CX[i] + a1y * CY[i]) +
                     4.5 * (a2xx * hxx + a2yy * hyy + 2.0 * a2xy * hxy));
  }
}

/* p^i - p^w of Eq.(force2) with Eq.(eqstate), paper units. */
double lbo_pressure_term(double n, double T) {
  return n * T - (3.0 * n * T / (3.0 - n) - 9.0 / 8.0 * n * n);
}

/* ---------------------------------------------------------------------- */
/* Fields with ghost rows.                                                 */
/* ---------------------------------------------------------------------- */

static int wrapx(int x, int Lx) {
  int r = x % Lx;
  return r < 0 ? r + Lx : r;
}

/* Value of a node field phi[y][x] at any row y. Periodic mode wraps y.
 * Walls mode mirrors about the wall nodes (rows 0 and Ly-1):
 * phi(-j) = par * phi(j), phi(Ly-1+j) = par * phi(Ly-1-j), par = +1 for
 * scalars and x-components, -1 for y-components. This is the neutral wetting
 * condition (normal derivative of n zero at the walls, Sec. II) carried to
 * every field the stencils read. */
static double field_at(const double *phi, const lbo_params *p, int x, int y,
                       double par) {
  int Lx = p->Lx, Ly = p->Ly;
  x = wrapx(x, Lx);
  if (p->y_periodic) {
    int r = y % Ly;
    if (r < 0) r += Ly;
    return phi[(size_t)r * Lx + x];
  }
  double sgn = 1.0;
  while (y < 0 || y > Ly - 1) {
    if (y < 0) y = -y;
    else y = 2 * (Ly - 1) - y;
    sgn *= par;
  }
  return sgn * phi[(size_t)y * Lx + x];
}

/* Eq.(xstencil): d/dx = N (E - W) + M (NE - NW + SE - SW). */
static double grad_x(const double *phi, const lbo_params *p, int x, int y,
                     double par) {
  double N = p->N, M = (1.0 - 2.0 * p->N) / 4.0;
  return N * (field_at(phi, p, x + 1, y, par) - field_at(phi, p, x - 1, y, par)) +
         M * (field_at(phi, p, x + 1, y + 1, par) - field_at(phi, p, x - 1, y + 1, par) +
              field_at(phi, p, x + 1, y - 1, par) - field_at(phi, p, x - 1, y - 1, par));
}

/* d/dy: the x stencil turned to point along +y. */
static double grad_y(const double *phi, const lbo_params *p, int x, int y,
                     double par) {
  double N = p->N, M = (1.0 - 2.0 * p->N) / 4.0;
  return N * (field_at(phi, p, x, y + 1, par) - field_at(phi, p, x, y - 1, par)) +
         M * (field_at(phi, p, x + 1, y + 1, par) - field_at(phi, p, x + 1, y - 1, par) +
              field_at(phi, p, x - 1, y + 1, par) - field_at(phi, p, x - 1, y - 1, par));
}

/* Eq.(laplstencil): Q (E + N + W + S) + R (corners) - 4 (Q + R) centre. */
static double laplacian(const double *phi, const lbo_params *p, int x, int y) {
  double Q = p->Q, R = (1.0 - p->Q) / 2.0;
  double edges = field_at(phi, p, x + 1, y, 1) + field_at(phi, p, x - 1, y, 1) +
                 field_at(phi, p, x, y + 1, 1) + field_at(phi, p, x, y - 1, 1);
  double corners = field_at(phi, p, x + 1, y + 1, 1) + field_at(phi, p, x - 1, y + 1, 1) +
                   field_at(phi, p, x + 1, y - 1, 1) + field_at(phi, p, x - 1, y - 1, 1);
  return Q * edges + R * corners - 4.0 * (Q + R) * field_at(phi, p, x, y, 1);
}

/* Exported stencils over a whole field (tests pin them on polynomials). */
void lbo_apply_stencils(const lbo_params *p, const double *phi, double par,
                        double *gx, double *gy, double *lap) {
  for (int y = 0; y < p->Ly; y++)
    for (int x = 0; x < p->Lx; x++) {
      size_t k = (size_t)y * p->Lx + x;
      if (gx) gx[k] = grad_x(phi, p, x, y, par);
      if (gy) gy[k] = grad_y(phi, p, x, y, par);
      if (lap) lap[k] = laplacian(phi, p, x, y);
    }
}

/* D = div(n u*) of Eq.(coeff) with the gradient stencil, as the step uses
 * it: the ghost of j*_x is even and that of j*_y odd at the walls (reading of
 * the neutral-wetting mirror for a y-component). */
void lbo_divergence(const lbo_params *p, const double *jx, const double *jy,
                    double *D) {
  for (int y = 0; y < p->Ly; y++)
    for (int x = 0; x < p->Lx; x++)
      D[(size_t)y * p->Lx + x] = grad_x(jx, p, x, y, 1) + grad_y(jy, p, x, y, -1);
}

/* ---------------------------------------------------------------------- */
/* Initial state and one time step.                                        */
/* ---------------------------------------------------------------------- */

/* S(0) = f_eq(n0, u0; T). u0 may be NULL (fluid at rest). */
void lbo_init(const lbo_params *p, const double *n0, const double *ux0,
              const double *uy0, double *S) {
  size_t nn = (size_t)p->Lx * p->Ly;
  for (size_t k = 0; k < nn; k++) {
    double fe[9];
    lbo_feq(n0[k], ux0 ? ux0[k] : 0.0, uy0 ? uy0[k] : 0.0, p->T, fe);
    for (int i = 0; i < 9; i++) S[i * nn + k] = fe[i];
  }
}

/*
 * One step: S_in = post-collision populations after k-1 steps; S_out those
 * after k steps. n_out, ux_out, uy_out (may be NULL) receive the moments
 * computed inside this step (after streaming and boundary conditions, before
 * collision): density n and physical velocity u* of Eq.(newvel).
 * fext: per-column external force density F_ext,x (paper units), may be NULL.
 * Returns 0, or -1 on bad parameters / allocation failure.
 */
int lbo_step(const lbo_params *p, const double *fext, const double *S_in,
             double *S_out, double *n_out, double *ux_out, double *uy_out) {
  const int Lx = p->Lx, Ly = p->Ly;
  if (Lx < 1 || Ly < 4 || p->collision < 0 || p->collision > 1) return -1;
  const size_t nn = (size_t)Lx * Ly;
  const double tau_l = sqrt(3.0) * p->tau;
  const double omega = 1.0 / tau_l;
  const double T = p->T;
  const int walls = !p->y_periodic;

  double *f = malloc(9 * nn * sizeof(double));
  double *n = malloc(nn * sizeof(double));
  double *L = malloc(nn * sizeof(double));
  double *P = malloc(nn * sizeof(double));
  double *Fx = malloc(nn * sizeof(double));
  double *Fy = malloc(nn * sizeof(double));
  double *jx = malloc(nn * sizeof(double));
  double *jy = malloc(nn * sizeof(double));
  double *Dv = malloc(nn * sizeof(double));
  if (!f || !n || !L || !P || !Fx || !Fy || !jx || !jy || !Dv) {
    free(f); free(n); free(L); free(P); free(Fx); free(Fy); free(jx); free(jy); free(Dv);
    return -1;
  }

  /* 1. Streaming, pull form of the left side of Eq.(evoleq):
   *    f_i(x, y) = S_i(x - cx_i, y - cy_i). With walls, sources outside the
   *    rows 0..Ly-1 do not exist; those f_i are set by the wall rule below. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++)
      for (int i = 0; i < 9; i++) {
        int sy = y - CY[i];
        int sx = wrapx(x - CX[i], Lx);
        size_t k = (size_t)y * Lx + x;
        if (p->y_periodic) {
          sy = ((sy % Ly) + Ly) % Ly;
        } else if (sy < 0 || sy > Ly - 1) {
          f[i * nn + k] = NAN; /* unknown until the wall rule */
          continue;
        }
        f[i * nn + k] = S_in[i * nn + (size_t)sy * Lx + sx];
      }

  /* 2. Density. Bulk: n = sum_i f_i. Wall nodes: n-hat of the wall rule
   *    (Sec. II): the wall node's own post-collision populations that would
   *    leave the lattice (previous step, not streamed) plus the known
   *    streamed ones. Lower wall: S0 + S4 + S7 + S8 + f1 + f3 + f4 + f7 + f8;
   *    upper wall by the mirror y -> -y: S0 + S2 + S5 + S6 + f1 + f3 + f2 +
   *    f5 + f6. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
#define Fv(i) f[(i) * nn + k]
#define Sv(i) S_in[(i) * nn + k]
      if (walls && y == 0)
        n[k] = Sv(0) + Sv(4) + Sv(7) + Sv(8) + Fv(1) + Fv(3) + Fv(4) + Fv(7) + Fv(8);
      else if (walls && y == Ly - 1)
        n[k] = Sv(0) + Sv(2) + Sv(5) + Sv(6) + Fv(1) + Fv(3) + Fv(2) + Fv(5) + Fv(6);
      else {
        double s = 0.0;
        for (int i = 0; i < 9; i++) s += Fv(i);
        n[k] = s;
      }
#undef Sv
    }

  /* 3-5. Laplacian of n (Eq.(laplstencil)) and the pressure term
   *      p^i - p^w (Eq.(force2), Eq.(eqstate)), on every node. Ghost rows at
   *      walls come from field_at's mirror. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
      L[k] = laplacian(n, p, x, y);
      P[k] = lbo_pressure_term(n[k], T);
    }

  /* 6. Force, Eq.(force2) plus Eq.(periodicforce), paper units, then /3:
   *    F_p = grad(p^i - p^w) + kappa n grad(lap n) + (F_ext,x(x), 0). */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
      double fpx = grad_x(P, p, x, y, 1) + p->kappa * n[k] * grad_x(L, p, x, y, 1) +
                   (fext ? fext[x] : 0.0);
      double fpy = grad_y(P, p, x, y, 1) + p->kappa * n[k] * grad_y(L, p, x, y, 1);
      Fx[k] = fpx / 3.0;
      Fy[k] = fpy / 3.0;
    }

  /* 7. Moving walls (Sec. II), lattice units, wall speed Ub = -U (lower),
   *    Ut = +U (upper). The paper writes the lower wall; the upper one is its
   *    mirror image y -> -y (swap 2<->4, 5<->8, 6<->7, flip Fy). */
  if (walls) {
    const double Ub = -p->U, Ut = p->U;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < Lx; x++) {
      size_t k = x; /* lower wall, y = 0 */
      double fx = Fx[k], fy = Fy[k], nh = n[k];
      Fv(2) = Fv(4);
      Fv(5) = Fv(7) - 0.5 * (Fv(1) - Fv(3)) - 0.25 * (fx + fy) + 0.5 * nh * Ub;
      Fv(6) = Fv(8) + 0.5 * (Fv(1) - Fv(3)) + 0.25 * (fx - fy) - 0.5 * nh * Ub;
      Fv(0) = nh - (Fv(1) + Fv(3)) - 2.0 * (Fv(4) + Fv(7) + Fv(8)) + 0.5 * fy;
      k = (size_t)(Ly - 1) * Lx + x; /* upper wall */
      fx = Fx[k]; fy = Fy[k]; nh = n[k];
      Fv(4) = Fv(2);
      Fv(7) = Fv(5) + 0.5 * (Fv(1) - Fv(3)) + 0.25 * (fx + fy) - 0.5 * nh * Ut;
      Fv(8) = Fv(6) - 0.5 * (Fv(1) - Fv(3)) - 0.25 * (fx - fy) + 0.5 * nh * Ut;
      Fv(0) = nh - (Fv(1) + Fv(3)) - 2.0 * (Fv(2) + Fv(5) + Fv(6)) - 0.5 * fy;
    }
  }

  /* 8. Momentum, Eq.(newvel): n u* = sum_i f_i c_i + F/2 (lattice units).
   *    At wall nodes this equals (n Uwall, 0) by construction of step 7. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
      double sx = 0.0, sy = 0.0;
      for (int i = 0; i < 9; i++) {
        sx += Fv(i) * CX[i];
        sy += Fv(i) * CY[i];
      }
      jx[k] = sx + 0.5 * Fx[k];
      jy[k] = sy + 0.5 * Fy[k];
    }

  lbo_divergence(p, jx, jy, Dv);

  /* 9-12. Per node: grad n and D = div(n u*) with the same stencil (ghosts:
   *       n and jx even, jy odd), equilibrium, forcing, BGK collision
   *       (Eq.(evoleq)) on all nodes including the walls; with collision = 1
   *       the non-equilibrium part f - f_eq is replaced by its projection
   *       (lbo_regularize) before it relaxes:
   *       S = f_eq + (1 - omega) P[f - f_eq] + dt F. */
#pragma omp parallel for schedule(static)
  for (int y = 0; y < Ly; y++)
    for (int x = 0; x < Lx; x++) {
      size_t k = (size_t)y * Lx + x;
      double nk = n[k];
      double ux = jx[k] / nk, uy = jy[k] / nk;
      double dnx = grad_x(n, p, x, y, 1), dny = grad_y(n, p, x, y, 1);
      double D = Dv[k];
      double fe[9], fo[9];
      lbo_feq(nk, ux, uy, T, fe);
      lbo_forcing(ux, uy, Fx[k], Fy[k], dnx, dny, D, T, tau_l, fo);
      if (p->collision == 1) {
        double neq[9], pr[9];
        for (int i = 0; i < 9; i++) neq[i] = Fv(i) - fe[i];
        lbo_regularize(neq, pr);
        for (int i = 0; i < 9; i++)
          S_out[i * nn + k] = fe[i] + (1.0 - omega) * pr[i] + fo[i];
      } else {
        for (int i = 0; i < 9; i++)
          S_out[i * nn + k] = Fv(i) - omega * (Fv(i) - fe[i]) + fo[i];
      }
      if (n_out) n_out[k] = nk;
      if (ux_out) ux_out[k] = ux;
      if (uy_out) uy_out[k] = uy;
    }
#undef Fv

  free(f); free(n); free(L); free(P); free(Fx); free(Fy); free(jx); free(jy); free(Dv);
  return 0;
}

/* Run `steps` steps in place on S (ping-pong through a scratch copy).
 * nthreads <= 0 keeps the OpenMP default. Returns the threads used, or -1. */
int lbo_run(const lbo_params *p, const double *fext, double *S, int64_t steps,
            double *n_out, double *ux_out, double *uy_out, int nthreads) {
  size_t nn = (size_t)p->Lx * p->Ly;
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  used = omp_get_max_threads();
#else
  (void)nthreads;
#endif
  double *tmp = malloc(9 * nn * sizeof(double));
  if (!tmp) return -1;
  for (int64_t s = 0; s < steps; s++) {
    int last = (s == steps - 1);
    if (lbo_step(p, fext, S, tmp, last ? n_out : NULL, last ? ux_out : NULL,
                 last ? uy_out : NULL) != 0) {
      free(tmp);
      return -1;
    }
    memcpy(S, tmp, 9 * nn * sizeof(double));
  }
  free(tmp);
  return used;
}
