// Internal interface of the surrogate kernels (sg_device.hip) and their C ABI
// (sg_api.hip). Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sg {

typedef __bf16 bf16;

enum Mode { FWD_FIRST = 0, FWD_RES = 1, FWD_OUT = 2, BWD = 3 };

// Output tile of the convolution kernel: TR rows (one per wave) x TW columns.
constexpr int TW = 64;
constexpr int TR = 8;
// Work unit of the weight-gradient kernel: WG_RC rows of a WG_SEG-pixel
// column segment of one image.
constexpr int WG_SEG = 64;
constexpr int WG_RC = 16;

struct ConvArgs {
  const bf16* x;       // [B,H,W,CI]: layer input (forward) or dL/dz of the layer above (BWD)
  const bf16* w;       // packed weights [CO][kpad(CI)]
  const float* bias;   // [CO] or null
  const bf16* res;     // FWD_RES: residual input [B,H,W,CO]; BWD: dL/dh of the layer above or null
  const bf16* zprev;   // BWD: pre-activation of the layer below [B,H,W,CO]
  bf16* y;             // FWD_FIRST / FWD_RES: output h; BWD: dL/dz of the layer below
  bf16* z;             // FWD_FIRST / FWD_RES: pre-activation (optional); BWD: dL/dh (optional)
  float* yf;           // FWD_OUT: FP32 output [B,H,W,nout]
  int nout;
  int B, H, W;
};

// The four residual layers in one pass (stack_kernel): strips of SK_ST
// columns, W a multiple of SK_ST.
constexpr int SK_ST = 64;

struct StackArgs {
  const bf16* x;         // h0 [B,H,W,48]
  const bf16* w[4];      // packed weights of residual layers 1..4, each [48][kpad(48)]
  const float* bias[4];  // [48] each, or null
  bf16* y;               // h4 [B,H,W,48]
  int B, H, W;
};

struct WgradArgs {
  const bf16* x;       // layer input [B,H,W,CI]
  const bf16* gz;      // dL/dz [B,H,W,CO]
  float* part;         // per-workgroup partial sums [grid][9 CI CO + CO]
  int B, H, W;
};

// Field scalings of the network tensors.
struct Scales {
  float n, u, v, t;
};

hipError_t launch_conv(int ci, int co, int mode, const ConvArgs& a, int grid, hipStream_t st);
hipError_t launch_wgrad(int ci, int co, const WgradArgs& a, int grid, hipStream_t st);
hipError_t launch_stack(const StackArgs& a, hipStream_t st);
// Per-workgroup partial sums of the weight gradient: [grid][9 CI CO + CO]
// (the last CO entries: bias partials). tmp: 16 (9 cir cor + cor) doubles.
hipError_t launch_wgrad_reduce(const float* part, int nblk, int CI, int CO, int cir, int cor,
                               float scale, double* tmp, float* dw, float* db, hipStream_t st);
hipError_t launch_bias_grad(const bf16* gz, int64_t npix, int C, int nreal, float scale,
                            float* part, float* db, hipStream_t st);
hipError_t launch_mse(const float* pred, const float* target, int64_t npix, int nout, int CO,
                      bf16* gout, double* part, double* loss, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st);
hipError_t launch_pack(const float* w, int cir, int cor, int CI, int CO, int transposed, bf16* wp,
                       hipStream_t st);
hipError_t launch_fields_to_input(const double* mom, int B, int H, int W, const float* vx,
                                  const float* cond, int walls, Scales s, bf16* x, hipStream_t st);
hipError_t launch_make_target(const double* m0, const double* m1, int B, int64_t nn, Scales s,
                              float* target, hipStream_t st);
hipError_t launch_apply_output(const double* m0, const float* out, int B, int64_t nn, Scales s,
                               double* m1, hipStream_t st);
hipError_t launch_compare(const double* a, const double* b, int B, int64_t nn, double* out,
                          hipStream_t st);
hipError_t launch_project_mass(double* a, const double* ref, int B, int64_t nn,
                               const int32_t* mask, hipStream_t st);

}  // namespace sg
