// Internal interface between the D2Q17 C ABI (d17_api.hip) and its device
// code (d17_device.hip). Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace d17k {

// One periodic D2Q17 lattice as the kernels see it (passed by value).
struct Desc17 {
  void* S[2];            // populations [Ly][17][Lx] (planes of a row adjacent)
  const double* fext;    // per-column F_ext,x / s (lattice units), Lx values
  const double* shift;   // pending uniform density shift (device), or null
  int32_t Lx, Ly;
  double nbar;           // reference density subtracted in storage (0 in FP64)
  double T, omega, kappa_l, N, M, Q, R;
  double ps;             // 1/s: the pressure term in lattice units
  // per shell (rest, (1,0), (1,1), (2,2), (3,0)): weight w, rest-state weight
  // w^ at T, omega w^, and the coefficient a1 = s [1 + (T-1)(s |c|^2 - 4)/2]
  // of the first-order terms of equilibrium and forcing
  double w[5], wr[5], owr[5], a1[5];
  double h1, h2, h3;     // s/2, s^2/2, s^3/6
};

enum Flags17 : int { kWriteMoments = 1, kApplyShift = 2 };

// FP64 reduction results of one lattice, in device memory.
struct Reduce17 {
  double mass, jx, jy, nmin, nmax, nonfinite;
  double mass_ref;   // reference mass (set at init / restore)
  double shift;      // shift to apply at the next step (drift correction)
  uint32_t status;   // sticky: bit 0 set once a check failed
  uint32_t has_ref;
};

// Lattice constants (the velocity set, weights and scale s = r^2).
void lattice17(int cx[17], int cy[17], double w[17], double* s);
// Rest-state weight w^_i = w_i [1 + (T - 1)(s |c_i|^2 - 2)/2].
double rest_weight17(int i, double T);

// One time step over the whole lattice: strips of threads - 4 columns,
// chunks of `rows` rows (one workgroup each, in XCD-aware order); reads
// S[parity], writes S[parity ^ 1]; with kWriteMoments also n, ux, uy (FP64
// planes) into mom. threads: 64, 128, 256 or 512. prec (lb_params.fp32): 0
// FP64; 1 FP32 storage and arithmetic; 2 FP32 storage, FP64 arithmetic and
// stochastic rounding of the stored values with the draws of step rstep.
hipError_t launch_step17(int prec, int threads, int rows, const Desc17& d, int parity, int flags,
                         double* mom, uint32_t rstep, hipStream_t st);
hipError_t launch_init17(bool fp32, const Desc17& d, int parity, const double* n0,
                         const double* ux, const double* uy, hipStream_t st);
int reduce17_blocks(int64_t nn);
hipError_t launch_reduce17(bool fp32, const Desc17& d, int parity, double* part, int add_shift,
                           hipStream_t st);
// mode: 0 check (sticky status; drift shift when drift != 0), 1 set the
// reference mass, 2 report only.
hipError_t launch_reduce17_final(const double* part, int nb, int64_t nn, Reduce17* out, int mode,
                                 int drift, hipStream_t st);
hipError_t launch_get_pops17(bool fp32, const Desc17& d, int parity, int plane, double* f,
                             int add_shift, hipStream_t st);
hipError_t launch_set_pops17(bool fp32, const Desc17& d, int parity, int plane, const double* f,
                             hipStream_t st);

}  // namespace d17k
