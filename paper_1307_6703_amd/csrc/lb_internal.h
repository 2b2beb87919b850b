// Internal interface between the host-side C ABI (lb_api.hip) and the device
// code (lb_device.hip). Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbk {

// One lattice as the kernels see it. Lives in device memory (an array of
// these for a batch, one for a single lattice).
struct Desc {
  void* S[2];            // populations [Ly][9][Lx] (planes of a row adjacent), buffers 0 and 1
  const void* fext3;     // per-column F_ext,x / 3 (lattice units), Lx values
  double* mom;           // n, ux, uy planes (FP64) of the last step, or null
  const double* shift;   // pending uniform density shift, or null
  uint32_t* rng;         // step counters of the stochastic rounding (two words,
                         // indexed by buffer parity), or null
  int32_t Lx, Ly, periodic, reg;  // reg: regularised collision
  double nbar;           // reference density subtracted in storage (0 in FP64)
  double T, omega, kappa3, N, M, Q, R, U;
};

// A tile: instance (sign bit set: march downwards), first column, first and
// one-past-last row.
struct Tile {
  int32_t inst, x0, y0, y1;
};

// kYWalls / kYPeriodic: every listed lattice has walls / is periodic in y
// (the two-step kernel then compiles the other case out); neither: per lattice.
enum StepFlags : int { kWriteMoments = 1, kApplyShift = 2, kYWalls = 4, kYPeriodic = 8 };

// Reduction results per lattice (FP64), laid out in device memory.
struct ReduceOut {
  double mass, jx, jy, nmin, nmax, nonfinite;
  double mass_ref;   // reference mass (set at init / restore)
  double shift;      // shift to apply at the next step (drift correction)
  uint32_t status;   // sticky: bit 0 set once a check failed
  uint32_t has_ref;  // mass_ref valid
  uint32_t rng_step[2];  // stochastic-rounding step counter, by buffer parity
};

// Precision of a lattice (lb_params.fp32): FP64 storage and arithmetic; FP32
// deviations with FP32 arithmetic; FP32 deviations with FP64 arithmetic and
// stochastic rounding of the stored values.
enum Prec : int { kFP64 = 0, kFP32 = 1, kFP32SR = 2 };

// Launchers (all asynchronous on `stream`). fp32 selects the storage type,
// prec the kernel; reg the regularised collision (every listed lattice).
hipError_t launch_step(int prec, bool reg, int threads, const Desc* d_descs, const Tile* d_tiles,
                       int ntiles, int parity, int flags, hipStream_t stream);
// Two steps per launch (FP32 only; threads 64, 128, 192 or 256; reg the
// regularised collision): tiles of threads-14 columns, reads S[parity],
// writes S[parity ^ 1].
hipError_t launch_step2(int threads, bool reg, const Desc* d_descs, const Tile* d_tiles,
                        int ntiles, int parity, int flags, hipStream_t stream);
hipError_t launch_init(bool fp32, const Desc* d_desc, int parity, const double* d_n0,
                       const double* d_ux, const double* d_uy, int64_t nn, hipStream_t stream);
// Per-block partial sums over S[parity] (nb = reduce_blocks(nn) blocks).
int reduce_blocks(int64_t nn);
hipError_t launch_reduce(bool fp32, const Desc* d_desc, int parity, int64_t nn, double* d_part,
                         int add_shift, hipStream_t stream);
// Fixed-order final reduction of `nb` partials; mode: 0 check (sticky status,
// drift shift), 1 set the reference mass, 2 report only.
// The periodic check (mode 0) of the lattices d_list[0 .. n) of a batch in two
// launches; partials of lattice i at d_part + 6 d_part_off[i]; max_blocks =
// the largest reduce_blocks of the listed lattices. Same bits as checking
// them one by one.
hipError_t launch_check_batch(bool fp32, const Desc* d_descs, int parity, const int32_t* d_list,
                              int n, int max_blocks, const int64_t* d_part_off, double* d_part,
                              ReduceOut* d_reds, int drift, hipStream_t st);
hipError_t launch_reduce_final(const double* d_part, int nb, int64_t nn, ReduceOut* d_out,
                               int mode, int drift, hipStream_t stream);
// Full FP64 populations planes [p0, p1) of S[parity] into d_f (plane-major),
// adding the pending shift when add_shift != 0.
hipError_t launch_get_pops(bool fp32, const Desc* d_desc, int parity, int p0, int p1,
                           int64_t nn, double* d_f, int add_shift, hipStream_t stream);
// Also sets the stochastic-rounding step counter of S[parity] to `step`.
hipError_t launch_set_pops(bool fp32, const Desc* d_desc, int parity, int p0, int p1,
                           int64_t nn, const double* d_f, int64_t step, hipStream_t stream);
// Batch helpers (all instances of the same size nn): gather the moment blocks
// into out[count][3][nn]; write equilibrium populations from fields
// [count][3][nn] for instances with d_mask[i] != 0 (device array), or, with
// from != null, add f_eq(fields) - f_eq(from) to their populations.
hipError_t launch_gather_moments(const Desc* d_descs, int count, int64_t nn, double* out,
                                 hipStream_t st);
hipError_t launch_scatter_eq(bool fp32, const Desc* d_descs, ReduceOut* d_red, int count,
                             int parity, int64_t nn, const double* fields, const double* from,
                             const int32_t* d_mask, hipStream_t st);
// Rest-state weight w^_i at temperature T.
double rest_weight(int i, double T);

}  // namespace lbk
