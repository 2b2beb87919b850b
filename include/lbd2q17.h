/*
 * lbd2q17.h: C ABI of the D2Q17 variant of the MI355X (gfx950) lattice
 * Boltzmann step for a van der Waals fluid.
 *
 * Method: Coclite, Gonnella, Lamura, arXiv:1307.6703. The remark after
 * Eq.(nav) names a third-order model with seventeen velocities as the way to
 * remove the spurious term of order u*^3 from the Navier-Stokes equation of
 * the D2Q9 scheme (lbvdw.h); the paper gives no formulas for it. This library
 * builds it from the paper's step with the equilibrium (Eq.(eqfunc)) and the
 * forcing term (Eq.(forceterm), Eq.(coeff)) carried to third order in Hermite
 * polynomials on the degree-7 quadrature of seventeen velocities:
 *   pull streaming                      Eq.(evoleq), left side (reach 3)
 *   density                             Sec. II (moments)
 *   Laplacian and gradient stencils     Eq.(laplstencil), Eq.(xstencil)
 *   force F = grad(p^i - p^w)
 *     + kappa n grad(lap n) + F_ext     Eq.(force2), Eq.(eqstate), Eq.(periodicforce)
 *   physical velocity u*                Eq.(newvel)
 *   equilibrium, forcing, BGK collision third order; Eq.(evoleq)
 * The third-order equilibrium has the exact third moment, so the (1 - T)
 * terms of Eq.(coeff), which compensate D2Q9's defect there, have no
 * counterpart. Consequences: the shear viscosity is eta = n T (tau - dt/2) in
 * the paper's units (D2Q9: n (tau - dt/2)), and it does not change when the
 * fluid moves as a whole (D2Q9's drops by the u*^3 term).
 *
 * Velocity set (lb17_lattice): integer vectors c_i in the order 0 rest;
 * 1-4 (1,0), (0,1), (-1,0), (0,-1); 5-8 (1,1), (-1,1), (-1,-1), (1,-1);
 * 9-12 twice those diagonals; 13-16 three times the axis vectors. With
 * s = (125 + 5 sqrt(193))/72 the lattice's sound speed squared is 1/s.
 *
 * Boundaries: periodic in x and y only. The paper's wall rule and n-hat are
 * written for D2Q9; lb_params.y_periodic must be 1 and U must be 0.
 *
 * Units: lattice units (dx = dt = 1, c_i integer). tau and kappa are taken in
 * the paper's units (reference temperature T_c = 1, dx = 1, speeds
 * e_i = sqrt(s) c_i, so dt = 1/sqrt(s)) and converted inside:
 * tau_l = sqrt(s) tau, force density F_l = F_p / s. Densities are n / n_c,
 * T is T / T_c; velocities are in dx/dt.
 *
 * Layout: population arrays exchanged with the caller are planes P[i][y][x]
 * (x fastest), i in the order above; on the device the library keeps the 17
 * planes of each row adjacent, [y][i][x]. Host field arrays are row-major
 * [Ly][Lx] FP64.
 *
 * Precision: lb_params.fp32 = 0 stores and computes in FP64; fp32 = 1 stores
 * g_i = f_i - w^_i nbar in FP32 (w^_i the rest-state weights at T, nbar the
 * mean density) and computes in FP32; fp32 = 2 stores the same FP32
 * deviations but computes in FP64 and rounds each stored value
 * stochastically (as in lbvdw.h: the draws come from a counter-based hash of
 * column, row and step, so runs are deterministic and independent of the
 * launch shape, and a restart with lb17_set_populations continues with the
 * draws of its step). Mass and momentum checks are FP64.
 *
 * Parameters: lb_params of lbvdw.h with y_periodic = 1, U = 0, collision = 0,
 * fp32 in {0, 1, 2}, Ly >= 4, 17 Lx Ly (4 or 8) bytes < 2 GiB, sqrt(s) tau > 1/2,
 * the other fields as documented there (check_every and drift_correct
 * included).
 *
 * Ownership, streams, errors, threading: as in lbvdw.h. The caller owns the
 * device workspace (at least lb17_workspace_bytes() bytes, 256-byte aligned,
 * alive until lb17_destroy); the library calls no hipMalloc; every device
 * operation goes to the caller's stream; calls returning host data
 * synchronise it; negative lb_status values are errors with a message in
 * lb_last_error(); a failed stability check (non-finite or n outside (0, 3))
 * is reported as LB_EUNSTABLE by the next synchronising call, and
 * lb17_step_n then returns LB_ESTATE until the state is replaced.
 */
#ifndef LBD2Q17_H
#define LBD2Q17_H

#include "lbvdw.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb17_handle lb17_handle;

/* The velocity set (integer components), the weights w_i and the scale s;
 * any pointer may be NULL. */
lb_status lb17_lattice(int32_t cx[17], int32_t cy[17], double w[17], double* s);

/* Device workspace size for these parameters. */
lb_status lb17_workspace_bytes(const lb_params* p, size_t* bytes);

/* Create a lattice on the current HIP device (see lb_create). */
lb_status lb17_create(const lb_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      lb17_handle** out);

/* Initial state S(0) = f_eq(n0, u0; T), the third-order equilibrium. Host
 * arrays [Ly][Lx]; ux0, uy0 may be NULL (fluid at rest); every n0 in (0, 3).
 * Resets the step counter, the stability flag and the reference mass. */
lb_status lb17_init_lattice(lb17_handle* h, const double* n0, const double* ux0,
                            const double* uy0);

/* Same, with the initial fields already in device memory (FP64, [Ly][Lx]);
 * synchronises (the fields are checked on the host). */
lb_status lb17_init_lattice_device(lb17_handle* h, const double* d_n0, const double* d_ux0,
                                   const double* d_uy0);

/* Enqueue nsteps >= 0 time steps (asynchronous). The moments of the last
 * step are kept for lb17_get_moments. */
lb_status lb17_step_n(lb17_handle* h, int64_t nsteps);

/* Density and velocity u* (Eq.(newvel)) computed inside the last step (after
 * streaming, before collision); after lb17_init_lattice, the initial fields.
 * Host FP64 [Ly][Lx]; any may be NULL. Synchronises. */
lb_status lb17_get_moments(lb17_handle* h, double* n, double* ux, double* uy);

/* Same into device FP64 arrays (no synchronisation). */
lb_status lb17_get_moments_device(lb17_handle* h, double* d_n, double* d_ux, double* d_uy);

/* FP64 sums over the stored populations: out[0] mass, out[1..2] momentum,
 * out[3..4] min and max node density, out[5] non-finite nodes. Synchronises. */
lb_status lb17_reduce(lb17_handle* h, double out[6]);

/* Full populations as host FP64 [17][Ly][Lx]. Synchronises. */
lb_status lb17_get_populations(lb17_handle* h, double* f);

/* Replace the state by host FP64 populations [17][Ly][Lx] and set the step
 * counter; resets the stability flag and the reference mass. */
lb_status lb17_set_populations(lb17_handle* h, const double* f, int64_t step);

/* Launch shape of the step kernel: threads per workgroup (64, 128, 256 or
 * 512; strips of threads - 4 columns) and rows per workgroup (>= 1); 0 keeps the
 * default. blocks: workgroups per step. */
lb_status lb17_set_launch(lb17_handle* h, int32_t threads, int32_t rows);
lb_status lb17_get_launch(lb17_handle* h, int32_t* threads, int32_t* rows, int32_t* blocks);

/* Time nsteps steps of each candidate launch shape, pick the fastest and
 * apply it; return it (ms_per_step may be NULL). The timed steps are real
 * steps: the lattice advances by nsteps plus one warm-up step per candidate,
 * with the periodic checks that fall in them. The launch shape never changes
 * results. Synchronises. */
lb_status lb17_autotune(lb17_handle* h, int32_t nsteps, int32_t* threads, int32_t* rows,
                        double* ms_per_step);

/* Steps taken since the last init / set_populations plus the restored count. */
lb_status lb17_get_step(lb17_handle* h, int64_t* step);

lb_status lb17_destroy(lb17_handle* h);

#ifdef __cplusplus
}
#endif

#endif
