// Host side of the surrogate C ABI (include/lbsurrogate.h): argument checks,
// the network's workspace layout, and the launch sequences of its forward
// pass and training step.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "lb_host.h"
#include "lbsurrogate.h"
#include "sg_internal.h"

using namespace lbh;

namespace {

constexpr int kLayers = LBS_BLOCKS + 2;
constexpr int kWgradBlocks = 512;
constexpr int kMsePart = 512;      // matches the loss kernel
constexpr int kConvGridMax = 1 << 20;  // the launcher caps the grid at the resident workgroups

int kpad(int kin) { return (9 * kin + 31) / 32 * 32; }

// Channel counts of layer l: padded (CI, CO) as the kernels see them, and
// the real counts of the parameter vector.
struct LayerShape {
  int CI, CO, cir, cor;
};

LayerShape layer_shape(int l) {
  if (l == 0) return {LBS_IN_CHANNELS, LBS_WIDTH, LBS_IN_REAL, LBS_WIDTH};
  if (l <= LBS_BLOCKS) return {LBS_WIDTH, LBS_WIDTH, LBS_WIDTH, LBS_WIDTH};
  return {LBS_WIDTH, LBS_OUT_CHANNELS, LBS_WIDTH, LBS_OUT};
}

// offsets (in floats) of layer l's weights and biases in the parameter vector
int64_t param_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) {
    const LayerShape s = layer_shape(i);
    o += 9 * s.cir * s.cor + s.cor;
  }
  return o;
}

int64_t param_count() { return param_offset(kLayers); }

// packed-weight sizes (bf16 elements): forward [CO][kpad(CI)], transposed
// [CI][kpad(CO)]
int64_t pack_fwd_elems(int l) {
  const LayerShape s = layer_shape(l);
  return (int64_t)s.CO * kpad(s.CI);
}
int64_t pack_bwd_elems(int l) {
  const LayerShape s = layer_shape(l);
  return (int64_t)s.CI * kpad(s.CO);
}

int64_t wgrad_scratch_floats(int ci, int co, int cir, int cor, int blocks);

struct NetLayout {
  size_t params, grads, adam_m, adam_v, wf[kLayers], wb[kLayers];
  size_t h[LBS_BLOCKS + 1], z[LBS_BLOCKS + 1], dz[2], dh[2], gout, out;
  size_t wpart, mpart, loss, total;
};

NetLayout net_layout(int64_t npix, bool train) {
  NetLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t P = (size_t)param_count() * 4;
  const size_t act = (size_t)npix * LBS_WIDTH * 2;
  L.params = take(P);
  for (int l = 0; l < kLayers; ++l) L.wf[l] = take(pack_fwd_elems(l) * 2);
  if (train) {
    L.grads = take(P);
    L.adam_m = take(P);
    L.adam_v = take(P);
    for (int l = 1; l < kLayers; ++l) L.wb[l] = take(pack_bwd_elems(l) * 2);
    for (int l = 0; l <= LBS_BLOCKS; ++l) L.h[l] = take(act);
    for (int l = 0; l <= LBS_BLOCKS; ++l) L.z[l] = take(act);
    for (int i = 0; i < 2; ++i) L.dz[i] = take(act);
    for (int i = 0; i < 2; ++i) L.dh[i] = take(act);
    L.gout = take((size_t)npix * LBS_OUT_CHANNELS * 2);
    L.out = take((size_t)npix * LBS_OUT * 4);
    L.wpart = take((size_t)wgrad_scratch_floats(LBS_WIDTH, LBS_WIDTH, LBS_WIDTH, LBS_WIDTH,
                                                kWgradBlocks) * 4);
    L.mpart = take((size_t)kMsePart * 8);
    L.loss = take(8);
  } else {
    // inference: two activation buffers used alternately
    L.h[0] = take(act);
    L.h[1] = take(act);
  }
  L.total = o;
  return L;
}

bool conv_supported(int ci, int co) {
  return (ci == 8 && co == 48) || (ci == 48 && co == 48) || (ci == 48 && co == 16) ||
         (ci == 16 && co == 48);
}
bool wgrad_supported(int ci, int co) {
  return (ci == 8 && co == 48) || (ci == 48 && co == 48) || (ci == 48 && co == 16);
}

int conv_grid(int B, int H, int W, int cap = 0) {
  const int64_t tiles = (int64_t)((W + sg::TW - 1) / sg::TW) * ((H + sg::TR - 1) / sg::TR) * B;
  const int64_t lim = cap > 0 ? cap : kConvGridMax;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, lim));
}

lb_status check_image(int B, int H, int W) {
  if (B < 1 || H < 1 || W < 1) return fail(LB_EINVAL, "B, H, W must be >= 1 (got %d, %d, %d)", B, H, W);
  if ((int64_t)B * H * W * LBS_WIDTH >= ((int64_t)1 << 40))
    return fail(LB_EINVAL, "tensor too large");
  return LB_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

lb_status conv(int mode, int ci, int co, const void* x, const void* wp, const float* bias,
               const void* res, const void* zprev, void* y, void* z, float* yf, int nout, int B,
               int H, int W, hipStream_t st, int blocks = 0) {
  sg::ConvArgs a;
  a.x = (const sg::bf16*)x;
  a.w = (const sg::bf16*)wp;
  a.bias = bias;
  a.res = (const sg::bf16*)res;
  a.zprev = (const sg::bf16*)zprev;
  a.y = (sg::bf16*)y;
  a.z = (sg::bf16*)z;
  a.yf = yf;
  a.nout = nout;
  a.B = B;
  a.H = H;
  a.W = W;
  HIPCHK(sg::launch_conv(ci, co, mode, a, conv_grid(B, H, W, blocks), st));
  return LB_OK;
}

// scratch of a weight gradient: per-workgroup partials, then the FP64
// partials of the reduction's first stage (8-byte aligned)
int64_t wgrad_scratch_floats(int ci, int co, int cir, int cor, int blocks) {
  return (int64_t)blocks * (9 * ci * co + co) + 2 + 2 * 16 * (int64_t)(9 * cir * cor + cor);
}

lb_status wgrad(int ci, int co, int cir, int cor, const void* x, const void* gz, int B, int H,
                int W, float scale, float* part, int blocks, float* dw, float* db, hipStream_t st) {
  sg::WgradArgs a;
  a.x = (const sg::bf16*)x;
  a.gz = (const sg::bf16*)gz;
  a.part = part;
  a.B = B;
  a.H = H;
  a.W = W;
  const int64_t units = (int64_t)((W + sg::WG_SEG - 1) / sg::WG_SEG) *
                        ((H + sg::WG_RC - 1) / sg::WG_RC) * B;
  const int grid = (int)std::min<int64_t>(blocks, units);
  HIPCHK(sg::launch_wgrad(ci, co, a, grid, st));
  uintptr_t t = (uintptr_t)(part + (int64_t)blocks * (9 * ci * co + co));
  t = (t + 7) & ~(uintptr_t)7;
  HIPCHK(sg::launch_wgrad_reduce(part, grid, ci, co, cir, cor, scale, (double*)t, dw, db, st));
  return LB_OK;
}

}  // namespace

struct lbs_net {
  int max_batch = 0, H = 0, W = 0;
  bool train = false;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  NetLayout L{};
  int adam_t = 0;
  bool packed = false;  // forward packs match the parameters
  template <typename T>
  T* at(size_t off) const {
    return (T*)(ws + off);
  }
};

namespace {

lb_status pack_forward(lbs_net* n) {
  for (int l = 0; l < kLayers; ++l) {
    const LayerShape s = layer_shape(l);
    HIPCHK(sg::launch_pack(n->at<float>(n->L.params) + param_offset(l), s.cir, s.cor, s.CI, s.CO, 0,
                           n->at<sg::bf16>(n->L.wf[l]), n->st));
  }
  n->packed = true;
  return LB_OK;
}

const float* bias_of(const lbs_net* n, int l) {
  const LayerShape s = layer_shape(l);
  return n->at<float>(n->L.params) + param_offset(l) + 9 * s.cir * s.cor;
}

}  // namespace

extern "C" {

lb_status lbs_param_count(int64_t* count) {
  if (!count) return fail(LB_EINVAL, "count is NULL");
  *count = param_count();
  return LB_OK;
}

lb_status lbs_workspace_bytes(int32_t max_batch, int32_t H, int32_t W, int32_t train,
                              size_t* bytes) {
  if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
  lb_status r = check_image(max_batch, H, W);
  if (r != LB_OK) return r;
  *bytes = net_layout((int64_t)max_batch * H * W, train != 0).total;
  return LB_OK;
}

lb_status lbs_create(int32_t max_batch, int32_t H, int32_t W, int32_t train, void* dev_ws,
                     size_t ws_bytes, void* hip_stream, lbs_net** out) {
  if (!dev_ws || !out) return fail(LB_EINVAL, "NULL argument");
  lb_status r = check_image(max_batch, H, W);
  if (r != LB_OK) return r;
  if ((uintptr_t)dev_ws % kAlign) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  const NetLayout L = net_layout((int64_t)max_batch * H * W, train != 0);
  if (ws_bytes < L.total) return fail(LB_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  lbs_net* n = new lbs_net();
  n->max_batch = max_batch;
  n->H = H;
  n->W = W;
  n->train = train != 0;
  n->ws = (char*)dev_ws;
  n->st = (hipStream_t)hip_stream;
  n->L = L;
  const size_t P = (size_t)param_count() * 4;
  hipError_t e = hipMemsetAsync(n->ws + L.params, 0, P, n->st);
  if (e == hipSuccess) e = hipStreamSynchronize(n->st);
  if (e != hipSuccess) {
    delete n;
    return fail(LB_EDEVICE, "clearing the parameters failed: %s", hipGetErrorString(e));
  }
  *out = n;
  return LB_OK;
}

lb_status lbs_set_params(lbs_net* n, const float* d_params) {
  if (!n || !d_params) return fail(LB_EINVAL, "NULL argument");
  const size_t P = (size_t)param_count() * 4;
  HIPCHK(hipMemcpyAsync(n->ws + n->L.params, d_params, P, hipMemcpyDeviceToDevice, n->st));
  if (n->train) {
    HIPCHK(hipMemsetAsync(n->ws + n->L.adam_m, 0, P, n->st));
    HIPCHK(hipMemsetAsync(n->ws + n->L.adam_v, 0, P, n->st));
  }
  n->adam_t = 0;
  n->packed = false;
  return LB_OK;
}

lb_status lbs_get_params(lbs_net* n, float* d_params) {
  if (!n || !d_params) return fail(LB_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(d_params, n->ws + n->L.params, (size_t)param_count() * 4,
                        hipMemcpyDeviceToDevice, n->st));
  return LB_OK;
}

lb_status lbs_get_grads(lbs_net* n, float* d_grads) {
  if (!n || !d_grads) return fail(LB_EINVAL, "NULL argument");
  if (!n->train) return fail(LB_ESTATE, "network was created without training buffers");
  HIPCHK(hipMemcpyAsync(d_grads, n->ws + n->L.grads, (size_t)param_count() * 4,
                        hipMemcpyDeviceToDevice, n->st));
  return LB_OK;
}

lb_status lbs_forward(lbs_net* n, int32_t B, const void* d_x, float* d_out) {
  if (!n || !d_x || !d_out) return fail(LB_EINVAL, "NULL argument");
  if (B < 1 || B > n->max_batch) return fail(LB_EINVAL, "B must be in [1, %d] (got %d)", n->max_batch, B);
  if (!aligned16(d_x)) return fail(LB_EINVAL, "d_x must be 16-byte aligned");
  lb_status r;
  if (!n->packed && (r = pack_forward(n)) != LB_OK) return r;
  const int H = n->H, W = n->W;
  // activations alternate between two buffers (training buffers h0, h1 when
  // the network has them)
  void* buf[2] = {n->ws + n->L.h[0], n->ws + n->L.h[1]};
  if ((r = conv(sg::FWD_FIRST, LBS_IN_CHANNELS, LBS_WIDTH, d_x, n->at<void>(n->L.wf[0]),
                bias_of(n, 0), nullptr, nullptr, buf[0], nullptr, nullptr, 0, B, H, W, n->st)) != LB_OK)
    return r;
  int cur = 0;
  if (LBS_BLOCKS == 4 && W % sg::SK_ST == 0) {
    // the four residual layers in one pass, activations kept on chip
    sg::StackArgs sa;
    sa.x = (const sg::bf16*)buf[0];
    for (int l = 1; l <= 4; ++l) {
      sa.w[l - 1] = n->at<sg::bf16>(n->L.wf[l]);
      sa.bias[l - 1] = bias_of(n, l);
    }
    sa.y = (sg::bf16*)buf[1];
    sa.B = B;
    sa.H = H;
    sa.W = W;
    HIPCHK(sg::launch_stack(sa, n->st));
    cur = 1;
  } else {
    for (int l = 1; l <= LBS_BLOCKS; ++l) {
      if ((r = conv(sg::FWD_RES, LBS_WIDTH, LBS_WIDTH, buf[cur], n->at<void>(n->L.wf[l]), bias_of(n, l),
                    buf[cur], nullptr, buf[cur ^ 1], nullptr, nullptr, 0, B, H, W, n->st)) != LB_OK)
        return r;
      cur ^= 1;
    }
  }
  return conv(sg::FWD_OUT, LBS_WIDTH, LBS_OUT_CHANNELS, buf[cur], n->at<void>(n->L.wf[kLayers - 1]),
              bias_of(n, kLayers - 1), nullptr, nullptr, nullptr, nullptr, d_out, LBS_OUT, B, H, W,
              n->st);
}

lb_status lbs_train_step(lbs_net* n, int32_t B, const void* d_x, const float* d_target, float lr,
                         double* d_loss) {
  if (!n || !d_x || !d_target) return fail(LB_EINVAL, "NULL argument");
  if (!n->train) return fail(LB_ESTATE, "network was created without training buffers");
  if (B < 1 || B > n->max_batch) return fail(LB_EINVAL, "B must be in [1, %d] (got %d)", n->max_batch, B);
  if (!aligned16(d_x)) return fail(LB_EINVAL, "d_x must be 16-byte aligned");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(LB_EINVAL, "lr must be > 0");
  const int H = n->H, W = n->W;
  const int64_t npix = (int64_t)B * H * W;
  const NetLayout& L = n->L;
  hipStream_t st = n->st;
  lb_status r;
  if ((r = pack_forward(n)) != LB_OK) return r;
  for (int l = 1; l < kLayers; ++l) {
    const LayerShape s = layer_shape(l);
    HIPCHK(sg::launch_pack(n->at<float>(L.params) + param_offset(l), s.cir, s.cor, s.CI, s.CO, 1,
                           n->at<sg::bf16>(L.wb[l]), st));
  }
  // forward, keeping every activation and pre-activation
  if ((r = conv(sg::FWD_FIRST, LBS_IN_CHANNELS, LBS_WIDTH, d_x, n->at<void>(L.wf[0]), bias_of(n, 0),
                nullptr, nullptr, n->at<void>(L.h[0]), n->at<void>(L.z[0]), nullptr, 0, B, H, W,
                st)) != LB_OK)
    return r;
  for (int l = 1; l <= LBS_BLOCKS; ++l)
    if ((r = conv(sg::FWD_RES, LBS_WIDTH, LBS_WIDTH, n->at<void>(L.h[l - 1]), n->at<void>(L.wf[l]),
                  bias_of(n, l), n->at<void>(L.h[l - 1]), nullptr, n->at<void>(L.h[l]),
                  n->at<void>(L.z[l]), nullptr, 0, B, H, W, st)) != LB_OK)
      return r;
  float* out = n->at<float>(L.out);
  if ((r = conv(sg::FWD_OUT, LBS_WIDTH, LBS_OUT_CHANNELS, n->at<void>(L.h[LBS_BLOCKS]),
                n->at<void>(L.wf[kLayers - 1]), bias_of(n, kLayers - 1), nullptr, nullptr, nullptr,
                nullptr, out, LBS_OUT, B, H, W, st)) != LB_OK)
    return r;
  // loss; the backward pass carries 2 (out - target) and applies the mean's
  // 1 / (npix LBS_OUT) in the gradient reductions
  double* loss = n->at<double>(L.loss);
  HIPCHK(sg::launch_mse(out, d_target, npix, LBS_OUT, LBS_OUT_CHANNELS, n->at<sg::bf16>(L.gout),
                        n->at<double>(L.mpart), loss, st));
  if (d_loss) HIPCHK(hipMemcpyAsync(d_loss, loss, 8, hipMemcpyDeviceToDevice, st));
  const float scale = (float)(1.0 / ((double)npix * LBS_OUT));
  float* grads = n->at<float>(L.grads);
  float* wpart = n->at<float>(L.wpart);
  auto grad_w = [&](int l) { return grads + param_offset(l); };
  auto grad_b = [&](int l) {
    const LayerShape s = layer_shape(l);
    return grads + param_offset(l) + 9 * s.cir * s.cor;
  };
  // output layer
  const int lo = kLayers - 1;
  if ((r = wgrad(LBS_WIDTH, LBS_OUT_CHANNELS, LBS_WIDTH, LBS_OUT, n->at<void>(L.h[LBS_BLOCKS]),
                 n->at<void>(L.gout), B, H, W, scale, wpart, kWgradBlocks, grad_w(lo), grad_b(lo),
                 st)) != LB_OK)
    return r;
  // dL/dh_top = conv^T(gout); dL/dz_top = dL/dh_top SiLU'(z_top)
  int a = 0;
  if ((r = conv(sg::BWD, LBS_OUT_CHANNELS, LBS_WIDTH, n->at<void>(L.gout), n->at<void>(L.wb[lo]),
                nullptr, nullptr, n->at<void>(L.z[LBS_BLOCKS]), n->at<void>(L.dz[a]),
                n->at<void>(L.dh[a]), nullptr, 0, B, H, W, st)) != LB_OK)
    return r;
  // residual blocks, top down: dz[a] = dL/dz_l, dh[a] = dL/dh_l
  for (int l = LBS_BLOCKS; l >= 1; --l) {
    if ((r = wgrad(LBS_WIDTH, LBS_WIDTH, LBS_WIDTH, LBS_WIDTH, n->at<void>(L.h[l - 1]),
                   n->at<void>(L.dz[a]), B, H, W, scale, wpart, kWgradBlocks, grad_w(l), grad_b(l),
                   st)) != LB_OK)
      return r;
    // dL/dh_{l-1} = dL/dh_l + conv^T(dL/dz_l); dL/dz_{l-1} = that SiLU'(z_{l-1})
    if ((r = conv(sg::BWD, LBS_WIDTH, LBS_WIDTH, n->at<void>(L.dz[a]), n->at<void>(L.wb[l]), nullptr,
                  n->at<void>(L.dh[a]), n->at<void>(L.z[l - 1]), n->at<void>(L.dz[a ^ 1]),
                  l > 1 ? n->at<void>(L.dh[a ^ 1]) : nullptr, nullptr, 0, B, H, W, st)) != LB_OK)
      return r;
    a ^= 1;
  }
  // first layer
  if ((r = wgrad(LBS_IN_CHANNELS, LBS_WIDTH, LBS_IN_REAL, LBS_WIDTH, d_x, n->at<void>(L.dz[a]), B, H,
                 W, scale, wpart, kWgradBlocks, grad_w(0), grad_b(0), st)) != LB_OK)
    return r;
  n->adam_t += 1;
  HIPCHK(sg::launch_adam(n->at<float>(L.params), grads, n->at<float>(L.adam_m),
                         n->at<float>(L.adam_v), (int)param_count(), lr, 0.9f, 0.999f, 1e-8f,
                         n->adam_t, st));
  n->packed = false;
  return LB_OK;
}

lb_status lbs_destroy(lbs_net* n) {
  if (!n) return LB_OK;
  (void)hipStreamSynchronize(n->st);
  delete n;
  return LB_OK;
}

// ---- layers -----------------------------------------------------------------

lb_status lbs_pack(const float* d_w, int32_t cir, int32_t cor, int32_t CI, int32_t CO,
                   int32_t transposed, void* d_wpack, void* hip_stream) {
  if (!d_w || !d_wpack) return fail(LB_EINVAL, "NULL argument");
  if (cir < 1 || cor < 1 || cir > CI || cor > CO || CI % 8 || CO % 8 || CI > 64 || CO > 64)
    return fail(LB_EINVAL, "need 1 <= cir <= CI, 1 <= cor <= CO, CI and CO multiples of 8, <= 64");
  HIPCHK(sg::launch_pack(d_w, cir, cor, CI, CO, transposed ? 1 : 0, (sg::bf16*)d_wpack,
                         (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_conv(int32_t mode, int32_t ci, int32_t co, const void* d_x, const void* d_wpack,
                   const float* d_bias, const void* d_res, const void* d_zprev, void* d_y,
                   void* d_z, float* d_yf, int32_t nout, int32_t B, int32_t H, int32_t W,
                   int32_t blocks, void* hip_stream) {
  if (mode < 0 || mode > 3) return fail(LB_EINVAL, "mode must be 0..3 (got %d)", mode);
  if (blocks < 0 || blocks > 4096) return fail(LB_EINVAL, "blocks must be in [0, 4096]");
  if (!conv_supported(ci, co)) return fail(LB_EINVAL, "unsupported channel pair (%d, %d)", ci, co);
  lb_status r = check_image(B, H, W);
  if (r != LB_OK) return r;
  if (!d_x || !d_wpack) return fail(LB_EINVAL, "x and wpack are required");
  if (!aligned16(d_x) || !aligned16(d_wpack) || !aligned16(d_y) || !aligned16(d_z) ||
      !aligned16(d_res) || !aligned16(d_zprev) || !aligned16(d_yf))
    return fail(LB_EINVAL, "tensors must be 16-byte aligned");
  if (mode == sg::FWD_OUT) {
    if (!d_yf) return fail(LB_EINVAL, "output mode needs yf");
    if (nout < 1 || nout > co) return fail(LB_EINVAL, "nout must be in [1, %d]", co);
  } else if (!d_y) {
    return fail(LB_EINVAL, "mode %d needs y", mode);
  }
  if (mode == sg::FWD_RES && !d_res) return fail(LB_EINVAL, "residual mode needs res");
  if (mode == sg::BWD && !d_zprev) return fail(LB_EINVAL, "backward mode needs zprev");
  if (mode == sg::BWD && d_bias) return fail(LB_EINVAL, "backward mode takes no bias");
  return conv(mode, ci, co, d_x, d_wpack, d_bias, d_res, d_zprev, d_y, d_z, d_yf, nout, B, H, W,
              (hipStream_t)hip_stream, blocks);
}

lb_status lbs_wgrad_scratch_floats(int32_t ci, int32_t co, int32_t cir, int32_t cor, int32_t blocks,
                                   int64_t* count) {
  if (!count) return fail(LB_EINVAL, "count is NULL");
  if (!wgrad_supported(ci, co)) return fail(LB_EINVAL, "unsupported channel pair (%d, %d)", ci, co);
  if (cir < 1 || cir > ci || cor < 1 || cor > co) return fail(LB_EINVAL, "need 1 <= cir <= ci, 1 <= cor <= co");
  if (blocks < 1 || blocks > 4096) return fail(LB_EINVAL, "blocks must be in [1, 4096]");
  *count = wgrad_scratch_floats(ci, co, cir, cor, blocks);
  return LB_OK;
}

lb_status lbs_wgrad(int32_t ci, int32_t co, int32_t cir, int32_t cor, const void* d_x,
                    const void* d_gz, int32_t B, int32_t H, int32_t W, float scale, float* d_part,
                    int32_t blocks, float* d_dw, float* d_db, void* hip_stream) {
  if (!wgrad_supported(ci, co)) return fail(LB_EINVAL, "unsupported channel pair (%d, %d)", ci, co);
  if (cir < 1 || cir > ci || cor < 1 || cor > co) return fail(LB_EINVAL, "need 1 <= cir <= ci, 1 <= cor <= co");
  lb_status r = check_image(B, H, W);
  if (r != LB_OK) return r;
  if (!d_x || !d_gz || !d_part || !d_dw) return fail(LB_EINVAL, "NULL argument");
  if (!aligned16(d_x) || !aligned16(d_gz)) return fail(LB_EINVAL, "x and gz must be 16-byte aligned");
  if (blocks < 1 || blocks > 4096) return fail(LB_EINVAL, "blocks must be in [1, 4096]");
  if ((uintptr_t)d_part % 4) return fail(LB_EINVAL, "d_part must be 4-byte aligned");
  return wgrad(ci, co, cir, cor, d_x, d_gz, B, H, W, scale, d_part, blocks, d_dw, d_db,
               (hipStream_t)hip_stream);
}

}  // extern "C"

// Scratch of lbs_wgrad_noalloc: a file-scope device array, one copy per GPU,
// held until the process ends. Its name is a host-side stand-in in host code:
// kernels get the device address that hipGetSymbolAddress returns, looked up
// once per device with that device current.
constexpr int64_t kNoallocScratchFloats = (int64_t)4 << 20;  // 16 MiB
static __device__ __align__(256) float scratch[kNoallocScratchFloats];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
float* g_scratch_ptr[kMaxDevices] = {};

lb_status scratch_of_current_device(float** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LB_EDEVICE, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LB_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return LB_OK;
}
}  // namespace

extern "C" {

lb_status lbs_wgrad_noalloc(int32_t ci, int32_t co, int32_t cir, int32_t cor, const void* d_x,
                            const void* d_gz, int32_t B, int32_t H, int32_t W, float scale,
                            int32_t blocks, float* d_dw, float* d_db, void* hip_stream) {
  if (!wgrad_supported(ci, co)) return fail(LB_EINVAL, "unsupported channel pair (%d, %d)", ci, co);
  if (cir < 1 || cir > ci || cor < 1 || cor > co) return fail(LB_EINVAL, "need 1 <= cir <= ci, 1 <= cor <= co");
  lb_status r = check_image(B, H, W);
  if (r != LB_OK) return r;
  if (!d_x || !d_gz || !d_dw) return fail(LB_EINVAL, "NULL argument");
  if (!aligned16(d_x) || !aligned16(d_gz)) return fail(LB_EINVAL, "x and gz must be 16-byte aligned");
  if (blocks < 1 || blocks > 4096) return fail(LB_EINVAL, "blocks must be in [1, 4096]");
  const int64_t need = wgrad_scratch_floats(ci, co, cir, cor, blocks);
  if (need > kNoallocScratchFloats)
    return fail(LB_EINVAL,
                "blocks = %d needs %lld scratch floats; the static scratch holds %lld: use fewer "
                "blocks or lbs_wgrad with a caller workspace", blocks, (long long)need,
                (long long)kNoallocScratchFloats);
  float* part = nullptr;
  if ((r = scratch_of_current_device(&part)) != LB_OK) return r;
  // every workgroup writes its whole partial block before the reduction
  // reads it, so nothing needs clearing
  return wgrad(ci, co, cir, cor, d_x, d_gz, B, H, W, scale, part, blocks, d_dw, d_db,
               (hipStream_t)hip_stream);
}

lb_status lbs_bias_grad(const void* d_gz, int64_t npix, int32_t C, int32_t nreal, float scale,
                        float* d_part, float* d_db, void* hip_stream) {
  if (!d_gz || !d_part || !d_db) return fail(LB_EINVAL, "NULL argument");
  if (npix < 1 || C < 1 || C > 64 || nreal < 1 || nreal > C)
    return fail(LB_EINVAL, "need npix >= 1, 1 <= nreal <= C <= 64");
  HIPCHK(sg::launch_bias_grad((const sg::bf16*)d_gz, npix, C, nreal, scale, d_part, d_db,
                              (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_mse(const float* d_pred, const float* d_target, int64_t npix, int32_t nout,
                  int32_t CO, void* d_gout, double* d_part, double* d_loss, void* hip_stream) {
  if (!d_pred || !d_target || !d_gout || !d_part || !d_loss) return fail(LB_EINVAL, "NULL argument");
  if (npix < 1 || nout < 1 || nout > CO) return fail(LB_EINVAL, "need npix >= 1, 1 <= nout <= CO");
  HIPCHK(sg::launch_mse(d_pred, d_target, npix, nout, CO, (sg::bf16*)d_gout, d_part, d_loss,
                        (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_adam(float* d_p, const float* d_g, float* d_m, float* d_v, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t t, void* hip_stream) {
  if (!d_p || !d_g || !d_m || !d_v) return fail(LB_EINVAL, "NULL argument");
  if (n < 1 || t < 1) return fail(LB_EINVAL, "need n >= 1 and t >= 1");
  HIPCHK(sg::launch_adam(d_p, d_g, d_m, d_v, n, lr, beta1, beta2, eps, t, (hipStream_t)hip_stream));
  return LB_OK;
}

// ---- fields -----------------------------------------------------------------

static sg::Scales to_scales(const lbs_scales* s) { return {s->n_scale, s->u_scale, s->v_scale, s->t_scale}; }

static lb_status check_scales(const lbs_scales* s) {
  if (!s) return fail(LB_EINVAL, "scales is NULL");
  if (!(s->n_scale != 0.f && s->u_scale != 0.f) || !std::isfinite(s->n_scale) ||
      !std::isfinite(s->u_scale) || !std::isfinite(s->v_scale) || !std::isfinite(s->t_scale))
    return fail(LB_EINVAL, "scales must be finite, n_scale and u_scale nonzero");
  return LB_OK;
}

lb_status lbs_fields_to_input(const double* d_fields, int32_t B, int32_t H, int32_t W,
                              const float* d_vx, const float* d_cond, int32_t walls,
                              const lbs_scales* s, void* d_x, void* hip_stream) {
  if (!d_fields || !d_vx || !d_cond || !d_x) return fail(LB_EINVAL, "NULL argument");
  lb_status r = check_image(B, H, W);
  if (r != LB_OK || (r = check_scales(s)) != LB_OK) return r;
  if (!aligned16(d_x)) return fail(LB_EINVAL, "d_x must be 16-byte aligned");
  HIPCHK(sg::launch_fields_to_input(d_fields, B, H, W, d_vx, d_cond, walls ? 1 : 0, to_scales(s),
                                    (sg::bf16*)d_x, (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_make_target(const double* d_f0, const double* d_f1, int32_t B, int64_t nn,
                          const lbs_scales* s, float* d_target, void* hip_stream) {
  if (!d_f0 || !d_f1 || !d_target) return fail(LB_EINVAL, "NULL argument");
  if (B < 1 || nn < 1) return fail(LB_EINVAL, "need B >= 1, nn >= 1");
  lb_status r = check_scales(s);
  if (r != LB_OK) return r;
  HIPCHK(sg::launch_make_target(d_f0, d_f1, B, nn, to_scales(s), d_target, (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_apply_output(const double* d_f0, const float* d_out, int32_t B, int64_t nn,
                           const lbs_scales* s, double* d_f1, void* hip_stream) {
  if (!d_f0 || !d_out || !d_f1) return fail(LB_EINVAL, "NULL argument");
  if (B < 1 || nn < 1) return fail(LB_EINVAL, "need B >= 1, nn >= 1");
  lb_status r = check_scales(s);
  if (r != LB_OK) return r;
  HIPCHK(sg::launch_apply_output(d_f0, d_out, B, nn, to_scales(s), d_f1, (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_compare(const double* d_a, const double* d_b, int32_t B, int64_t nn, double* d_out,
                      void* hip_stream) {
  if (!d_a || !d_b || !d_out) return fail(LB_EINVAL, "NULL argument");
  if (B < 1 || B > 65535 || nn < 1) return fail(LB_EINVAL, "need 1 <= B <= 65535, nn >= 1");
  HIPCHK(sg::launch_compare(d_a, d_b, B, nn, d_out, (hipStream_t)hip_stream));
  return LB_OK;
}

lb_status lbs_project_mass(double* d_a, const double* d_ref, int32_t B, int64_t nn,
                           const int32_t* d_mask, void* hip_stream) {
  if (!d_a || !d_ref || !d_mask) return fail(LB_EINVAL, "NULL argument");
  if (B < 1 || B > 65535 || nn < 1) return fail(LB_EINVAL, "need 1 <= B <= 65535, nn >= 1");
  HIPCHK(sg::launch_project_mass(d_a, d_ref, B, nn, d_mask, (hipStream_t)hip_stream));
  return LB_OK;
}

}  // extern "C"
