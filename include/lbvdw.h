/*
 * lbvdw.h: C ABI of the MI355X (gfx950) lattice Boltzmann library for a van der
 * Waals liquid-vapor fluid under a periodic force and wall shear.
 *
 * Method: Coclite, Gonnella, Lamura, "Pattern Formation in Liquid-Vapor
 * Systems under Periodic Potential and Shear", arXiv:1307.6703, Sec. II.
 * One time step (lb_step_n) performs, for every node:
 *   pull streaming                      Eq.(evoleq), left side
 *   density, wall density n-hat         Sec. II (moments; wall rule)
 *   Laplacian and gradient stencils     Eq.(laplstencil), Eq.(xstencil)
 *   force F = grad(p^i - p^w)
 *     + kappa n grad(lap n) + F_ext     Eq.(force2), Eq.(eqstate), Eq.(periodicforce)
 *   moving-wall populations             Sec. II (lower wall; upper by mirror)
 *   physical velocity u*                Eq.(newvel)
 *   equilibrium, forcing, BGK collision Eq.(eqfunc), Eq.(forceterm), Eq.(coeff), Eq.(evoleq)
 *
 * Units: lattice units (dx = dt = 1, D2Q9 speeds c_i in {0,+-1}^2). The paper
 * uses dt = sqrt(3)/3 and e_i = sqrt(3) c_i (Sec. III); tau and kappa are taken
 * in the paper's units and converted inside (tau_l = sqrt(3) tau; force
 * density F_l = F_p / 3). Densities are the reduced density n / n_c, T is
 * T / T_c. Velocities are in dx/dt.
 *
 * Layout: population arrays exchanged with the caller are planes P[i][y][x]
 * (x fastest), i = 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE (on the
 * device the library keeps the nine planes of each row adjacent,
 * [y][i][x]). Host field arrays are row-major [Ly][Lx] FP64. x is periodic. With walls, rows 0 and Ly-1 are the wall nodes: the
 * lower wall moves at -U, the upper at +U (shear rate 2U/(Ly-1)).
 *
 * Precision: fp32 = 0 stores and computes populations in FP64. fp32 = 1 stores
 * g_i = f_i - w^_i nbar in FP32 (w^_i the rest-state weights at T, nbar the
 * mean density) and computes the step in FP32. fp32 = 2 stores the same FP32
 * deviations but computes the step in FP64 and rounds each stored value
 * stochastically: to one of the two neighbouring floats, with the
 * probabilities that make the expected stored value the exact one. The
 * draws come from a counter-based hash of (column, row, step), so runs are
 * deterministic and do not depend on the launch shape. Rounding to nearest
 * repeats the same error at every node of a uniform phase and the lattice
 * integrates that bias; with unbiased rounding FP32 storage stays within 1e-4
 * of FP64 over long runs. Mass and momentum checks are always FP64. The
 * paper fixes no precision (Sec. III gives no arithmetic); these modes are
 * the library's.
 *
 * Ownership: the caller owns all device memory. It passes one device
 * workspace of at least lb_workspace_bytes() bytes (e.g. a torch uint8 tensor)
 * which must stay alive and untouched until lb_destroy. The library calls no
 * hipMalloc. Host arrays passed in are read during the call only. Handles are
 * owned by the library from create to destroy.
 *
 * Streams: every device operation is enqueued on the caller's HIP stream
 * (hipStream_t passed as void*; NULL is the null stream). Calls that return
 * host data synchronise that stream.
 *
 * Errors: every call returns an lb_status; a negative value is an error and
 * lb_last_error() gives a message (thread-local, valid until the next call on
 * the same thread). Parameters are checked before any device work (LB_EINVAL);
 * HIP failures give LB_EDEVICE. A failed stability check (non-finite or
 * n outside (0, 3), the excluded-volume pole of Eq.(eqstate)) is reported as
 * LB_EUNSTABLE by the next synchronising call; after it lb_step_n returns
 * LB_ESTATE until lb_init_lattice or lb_set_populations restarts the lattice.
 *
 * Threading: a handle must not be used by two threads at once. Different
 * handles are independent.
 */
#ifndef LBVDW_H
#define LBVDW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LB_OK = 0,
  LB_EINVAL = -1,    /* invalid argument or parameter set */
  LB_ENOMEM = -2,    /* workspace too small */
  LB_EDEVICE = -3,   /* a HIP call failed */
  LB_EUNSTABLE = -4, /* a stability check found a bad state */
  LB_ESTATE = -5     /* call not valid in the current state */
} lb_status;

typedef struct {
  int32_t Lx, Ly;         /* nodes; Lx >= 1, Ly >= 4; 9*Lx*Ly*(4 or 8 bytes)
                             < 2 GiB (FP32 < 59.6M nodes, FP64 < 29.8M)       */
  int32_t y_periodic;     /* 1: periodic in y; 0: moving walls at rows 0, Ly-1 */
  int32_t fp32;           /* 0: FP64 populations; 1: FP32 deviations, FP32
                             arithmetic; 2: FP32 deviations, FP64 arithmetic,
                             stochastic rounding of the stored values         */
  double T;               /* reduced temperature, 0 < T <= 1.5                */
  double tau;             /* relaxation time, paper units; sqrt(3) tau > 1/2 */
  double kappa;           /* square-gradient coefficient, paper units, >= 0  */
  double N, Q;            /* stencil parameters; M = (1-2N)/4, R = (1-Q)/2    */
  double U;               /* wall speed (lattice units), |U| < 0.3            */
  const double* fext_x;   /* host, Lx values: F_ext,x per column in paper
                             units (force density); NULL means zero. Copied
                             at create.                                       */
  int32_t check_every;    /* run the FP64 check every this many steps; 0 = never */
  int32_t drift_correct;  /* 1: after each check, add the uniform shift that
                             restores the initial mass (FP32 storage)        */
  int32_t collision;      /* 0: BGK of Eq.(evoleq); 1: regularised: the
                             non-equilibrium part f - f_eq is replaced by its
                             projection onto the Hermite polynomials of order
                             <= 2 (the space of Eq.(eqfunc) and
                             Eq.(forceterm)) before it relaxes, the step Sec. II
                             names for tau != 1                               */
} lb_params;

typedef struct lb_handle lb_handle;
typedef struct lb_batch lb_batch;

/* Message of the last failed call on this thread ("" if none). */
const char* lb_last_error(void);

/* Device workspace size for these parameters. */
lb_status lb_workspace_bytes(const lb_params* p, size_t* bytes);

/* Create a lattice on the current HIP device. dev_ws: device pointer to
 * ws_bytes >= lb_workspace_bytes() bytes, 256-byte aligned. hip_stream: the
 * stream all work of this handle goes to. The lattice holds no state until
 * lb_init_lattice or lb_set_populations. */
lb_status lb_create(const lb_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                    lb_handle** out);

/* Initial state S(0) = f_eq(n0, u0; T) (Eq.(eqfunc)). Host arrays [Ly][Lx];
 * ux0, uy0 may be NULL (fluid at rest). Every n0 must lie in (0, 3). Resets
 * the step counter, the stability flag and the reference mass. */
lb_status lb_init_lattice(lb_handle* h, const double* n0, const double* ux0, const double* uy0);

/* Same, with the initial fields already in device memory (FP64, [Ly][Lx]). */
lb_status lb_init_lattice_device(lb_handle* h, const double* d_n0, const double* d_ux0,
                                 const double* d_uy0);

/* Enqueue nsteps >= 0 time steps. Asynchronous: returns before they run. The
 * moments (n, u*) of the last step are kept for lb_get_moments. */
lb_status lb_step_n(lb_handle* h, int64_t nsteps);

/* Density and physical velocity u* (Eq.(newvel)) computed inside the last
 * step (after streaming and the wall rule, before collision); after
 * lb_init_lattice, the initial fields. Host FP64 arrays [Ly][Lx]; any may be
 * NULL. Synchronises the stream. */
lb_status lb_get_moments(lb_handle* h, double* n, double* ux, double* uy);

/* Same into device FP64 arrays (no synchronisation). */
lb_status lb_get_moments_device(lb_handle* h, double* d_n, double* d_ux, double* d_uy);

/* FP64 sums over the stored post-collision populations: out[0] total mass,
 * out[1..2] total momentum (x, y), out[3..4] min and max of the node density,
 * out[5] number of non-finite nodes. Synchronises the stream. */
lb_status lb_reduce(lb_handle* h, double out[6]);

/* Full populations f (deviations added back) as host FP64 [9][Ly][Lx]. */
lb_status lb_get_populations(lb_handle* h, double* f);

/* Replace the state by host FP64 populations [9][Ly][Lx] and set the step
 * counter (checkpoint restore; with fp32 = 2 the stochastic rounding
 * continues with the draws of that step). Resets the stability flag and the
 * reference mass to the mass of f. */
lb_status lb_set_populations(lb_handle* h, const double* f, int64_t step);

/* Change the check cadence and drift correction of lb_params (applies to
 * the following steps). */
lb_status lb_set_checks(lb_handle* h, int32_t check_every, int32_t drift_correct);

/* Steps taken since the last init / set_populations plus the restored count. */
lb_status lb_get_step(lb_handle* h, int64_t* step);

lb_status lb_destroy(lb_handle* h);

/* ---- batched lattices: many independent instances of uneven size ---------
 * All instances share the precision (fp32 field of p[0]). Every time step of
 * the batch advances every instance once, in one kernel launch over all of
 * their tiles; lb_batch_step_n records chunks of steps in a HIP graph and
 * replays it. Per-instance parameters follow lb_params. */

lb_status lb_batch_workspace_bytes(int32_t count, const lb_params* p, size_t* bytes);
lb_status lb_batch_create(int32_t count, const lb_params* p, void* dev_ws, size_t ws_bytes,
                          void* hip_stream, lb_batch** out);
lb_status lb_batch_init(lb_batch* b, int32_t idx, const double* n0, const double* ux0,
                        const double* uy0);
lb_status lb_batch_step_n(lb_batch* b, int64_t nsteps);
lb_status lb_batch_get_moments(lb_batch* b, int32_t idx, double* n, double* ux, double* uy);
lb_status lb_batch_reduce(lb_batch* b, int32_t idx, double out[6]);
/* Per-instance status of the checks so far (LB_OK or LB_EUNSTABLE); syncs. */
lb_status lb_batch_status(lb_batch* b, int32_t* per_instance);
/* Take every instance that failed a check out of the batch so that the
 * others can keep stepping (lb_batch_step_n otherwise returns LB_ESTATE once
 * any instance is unstable). Dropped instances keep their last state and
 * report LB_EUNSTABLE. *dropped (may be NULL) receives the number of
 * instances dropped so far. LB_ESTATE if every instance is unstable. Syncs. */
lb_status lb_batch_drop_unstable(lb_batch* b, int32_t* dropped);
lb_status lb_batch_destroy(lb_batch* b);

/* ---- batch calls for a learned surrogate (all instances the same size) ----
 * These let a caller replace the time stepping of some instances by a
 * prediction of the fields and audit it against the lattice itself. They
 * return LB_EINVAL when the instances differ in size. */

/* The moments of every instance (as lb_get_moments: from the last step, the
 * last init or the last re-entry) into a device FP64 block
 * [count][3][Ly][Lx] (n, u*_x, u*_y). Asynchronous on the batch's stream. */
lb_status lb_batch_get_moments_device(lb_batch* b, double* d_out);

/* Re-entry: for each instance with mask[i] != 0 (host int32 array of count
 * entries), replace the stored populations by the equilibrium of
 * Eq.(eqfunc) at the fields of d_fields (device FP64 [count][3][Ly][Lx]:
 * n, u*_x, u*_y) and make those fields the instance's moments. The step
 * counter does not change; a pending drift shift of these instances is
 * dropped. Synchronises the stream. */
lb_status lb_batch_set_equilibrium_device(lb_batch* b, const double* d_fields,
                                          const int32_t* mask);

/* Re-entry that keeps the non-equilibrium part: for each instance with
 * mask[i] != 0, add f_eq(d_fields) - f_eq(d_from) of Eq.(eqfunc) to the
 * stored populations (d_from, d_fields: device FP64 [count][3][Ly][Lx] as
 * above; d_from is normally the instance's current moments, so that only
 * the equilibrium part moves; with equal fields the populations stay the
 * same bits) and make d_fields the instance's moments. The step counter and
 * a pending drift shift do not change. Synchronises the stream. */
lb_status lb_batch_shift_equilibrium_device(lb_batch* b, const double* d_from,
                                            const double* d_fields, const int32_t* mask);

/* Advance only the instances with mask[i] != 0 by nsteps (even, so that
 * their buffer parity stays that of the batch), with the batch's launch
 * shape (two steps per launch: pairs, with two single steps in place of one
 * pair when the number of pairs is odd; same bits either way), no graph and
 * no drift shift; the last step writes their moments; one FP64 check per
 * instance at the end (flags instabilities as the periodic checks do). The
 * batch step counter does not change. Launches are asynchronous; each tile
 * upload synchronises the stream first. */
lb_status lb_batch_step_subset(lb_batch* b, int64_t nsteps, const int32_t* mask);

/* ---- launch shape ----------------------------------------------------------
 * The step kernel marches strips of columns along y. threads: columns a
 * workgroup loads (64, 128, 256, 320, or 512 with fp32 = 1; it
 * updates threads - 6 of them); rows:
 * rows per y-chunk (>= 1). 0 keeps the default. Applies to the next step.
 * lb_create picks two steps per launch (below) for FP32 lattices of at least
 * 2^20 nodes and 256 columns (256-thread strips when their columns exceed
 * Lx by at most 3%, else 128), one step per launch otherwise. */
lb_status lb_set_launch(lb_handle* h, int32_t threads, int32_t rows);
lb_status lb_get_launch(lb_handle* h, int32_t* threads, int32_t* rows, int32_t* blocks);
lb_status lb_batch_set_launch(lb_batch* b, int32_t threads, int32_t rows);

/* Two time steps per launch (fp32 = 1 only; LB_EINVAL otherwise).
 * A workgroup of threads (64, 128, 192 or 256; 0: 128) runs the step of
 * Eq.(evoleq), with either collision (lb_params.collision), twice over a
 * strip of threads - 14 columns and a y-chunk of
 * rows (0: a default height), keeping the first step's populations in LDS,
 * so the populations cross HBM once per two steps. Every node runs the same
 * arithmetic as with one step per launch, so results are the same bits.
 * Pairs of steps never straddle a check (check_every): a step before a
 * check, and the last of an odd count, runs alone in the default one-step
 * shape. lb_set_launch returns to one step per launch. Applies to the next
 * step. lb_get_steps_per_launch reports 1 or 2 for the current shape. */
lb_status lb_set_launch_fused(lb_handle* h, int32_t threads, int32_t rows);
lb_status lb_get_steps_per_launch(lb_handle* h, int32_t* steps);
/* The same for a batch (all instances share the shape; rows 0: 64). Subset
 * steps (lb_batch_step_subset) run in pairs too (see there). */
lb_status lb_batch_set_launch_fused(lb_batch* b, int32_t threads, int32_t rows);
lb_status lb_batch_get_steps_per_launch(lb_batch* b, int32_t* steps);

/* Time nsteps steps of each candidate launch shape (one step per launch
 * and, with fp32 = 1, two), pick the fastest and apply it; return
 * it (ms_per_step may be NULL; lb_get_steps_per_launch tells which kernel
 * won). The timed steps are real steps: the lattice advances by nsteps plus
 * one or two warm-up steps per candidate. The timed steps include the
 * periodic checks that fall in them (and the single steps before a check
 * that splits a pair), so nsteps a multiple of check_every gives every
 * candidate the same share of them. The launch shape never changes
 * results (every node runs the same arithmetic on the same inputs whatever
 * the tiling). Synchronises. */
lb_status lb_autotune(lb_handle* h, int32_t nsteps, int32_t* threads, int32_t* rows,
                      double* ms_per_step);

/* lb_autotune for a batch: candidate shapes (one and, with fp32 = 1, two steps
 * per launch) are shared by all instances. */
lb_status lb_batch_autotune(lb_batch* b, int32_t nsteps, int32_t* threads, int32_t* rows,
                            double* ms_per_step);

#ifdef __cplusplus
}
#endif

#endif /* LBVDW_H */
