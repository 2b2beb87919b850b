// Learned surrogate kernels for gfx950: 3x3 convolutions as implicit GEMMs on
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), their
// backward passes, the loss, Adam, and the packing between lattice fields and
// network tensors.
//
// Tensors are NHWC bf16: [batch, rows (y), columns (x), channels], channels a
// multiple of 8. A 3x3 convolution wraps around in x (periodic lattice) and
// sees zeros beyond the first and last rows (walls). Weights are kept in FP32
// as w[tap][ci][co], tap = (dy+1)*3 + (dx+1), and packed for the kernels as
// bf16 B-matrices [co][k], k = tap*CI + ci, padded with zeros to a multiple
// of 32 in k.
//
// MFMA operand layout (16x16x32): lane l holds A[m = l%16][k = 8(l/16) .. +7],
// B[k = 8(l/16) .. +7][n = l%16]; the accumulator holds D[m = 4(l/16) + r][n = l%16],
// r = 0..3.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sg_internal.h"

#include <type_traits>

namespace sg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CNT = 64 * TR;  // threads per conv workgroup (TR waves)
constexpr int NTH = 256; // threads per workgroup of the other kernels

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }  // round to nearest even

// SiLU and its derivative with the hardware reciprocal (about 1 ulp in FP32,
// far below the bf16 rounding the results go through) instead of an IEEE
// division, which costs about ten instructions.
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
// r + SiLU(z) with one rounding (the residual layers)
__device__ __forceinline__ float silu_res(float z, float r) { return __builtin_fmaf(z, sigmoid(z), r); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

template <int CI>
__host__ __device__ constexpr int kpad() { return (9 * CI + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// 3x3 convolution (forward, or input-gradient with flipped weights).
// Persistent workgroups: the packed weights are staged in LDS once, then each
// workgroup walks tiles of TR rows x TW columns of one image. Each of its TR
// waves owns one output row: 4 subtiles of 16 pixels by CO/16 subtiles of 16
// output channels, computed as W X^T so that every lane ends with 4
// consecutive channels of one pixel and the epilogue (bias, SiLU, residual,
// bf16 stores) runs straight from the accumulators. The next tile's input is
// loaded into registers while the matrix cores work on the current one.
// Eight waves per workgroup and about 115 KB of LDS: two waves per SIMD.
// ---------------------------------------------------------------------------
template <int CI, int CO>
struct ConvShape {
  static constexpr int K = 9 * CI, KP = kpad<CI>(), NS = CO / 16;
  // LDS pixel stride (elements): padded for conflict-free 16-byte reads, except
  // in the output layer (48 -> 16), whose unpadded tile (78 KB with the
  // weights) lets two workgroups share a CU
  static constexpr int PX = (CI == 48 && CO == 16) ? CI : CI + 8;
  static constexpr int WS = KP + 8;   // LDS weight row stride
  static constexpr int TCOLS = TW + 2, TROWS = TR + 2;
  static constexpr int CH = CI / 8;   // 16-byte chunks per input pixel
  static constexpr int NLD = TROWS * TCOLS * CH;
  static constexpr int PER = (NLD + CNT - 1) / CNT;  // input chunks per thread
};

// The 16-byte chunks a thread loads for every tile: chunk j is input pixel
// (row, col) of the tile (with its 1-pixel halo), channels 8 c .. 8 c + 7.
// These depend only on the thread, so they are worked out once.
template <int CI, int CO>
struct TileChunks {
  int row[ConvShape<CI, CO>::PER], col[ConvShape<CI, CO>::PER], c[ConvShape<CI, CO>::PER];
  __device__ __forceinline__ TileChunks() {
    using S = ConvShape<CI, CO>;
#pragma unroll
    for (int j = 0; j < S::PER; ++j) {
      const int i = threadIdx.x + j * CNT;
      const int pix = i / S::CH;
      c[j] = i % S::CH;
      col[j] = pix % S::TCOLS;
      row[j] = i < S::NLD ? pix / S::TCOLS : -(1 << 20);  // past the last chunk: never loaded
    }
  }
};

template <int CI, int CO>
__device__ __forceinline__ void conv_load_tile(uint4* pre, const bf16* x, const TileChunks<CI, CO>& tc,
                                               int tile, int tilesX, int tilesY, int H, int W) {
  using S = ConvShape<CI, CO>;
  const int tx = tile % tilesX, ty = (tile / tilesX) % tilesY, img = tile / (tilesX * tilesY);
  const int x0 = tx * TW, h0 = ty * TR;
  const bf16* xi = x + (int64_t)img * H * W * CI;
#pragma unroll
  for (int j = 0; j < S::PER; ++j) {
    uint4 v = {0u, 0u, 0u, 0u};
    const int h = h0 - 1 + tc.row[j];
    int xx = x0 - 1 + tc.col[j];  // in [-1, x0 + TW]: periodic in x
    if (W >= S::TCOLS) {
      xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
    } else {
      xx %= W;
      if (xx < 0) xx += W;
    }
    if (h >= 0 && h < H) v = *(const uint4*)(xi + ((int64_t)h * W + xx) * CI + tc.c[j] * 8);
    pre[j] = v;
  }
}

// The first and the output layer (8 input channels; 16 output channels) are
// memory work: held to 128 VGPRs (four waves per SIMD) so that two workgroups
// share a CU and keep twice the loads in flight.
template <int CI, int CO, int MODE>
__global__ __launch_bounds__(CNT, (CI == 8 && MODE == FWD_FIRST) || (CO == 16 && MODE == FWD_OUT) ? 4 : 1)
void conv_kernel(ConvArgs a) {
  using S = ConvShape<CI, CO>;
  constexpr int KP = S::KP, NS = S::NS, PX = S::PX, WS = S::WS, TCOLS = S::TCOLS;
  constexpr int K = S::K;
  __shared__ __attribute__((aligned(16))) bf16 sx[S::TROWS * TCOLS * PX];
  __shared__ __attribute__((aligned(16))) bf16 sw[CO * WS];

  const int tid = threadIdx.x;
  for (int i = tid; i < CO * (KP / 8); i += CNT) {
    const int co = i / (KP / 8), c = i % (KP / 8);
    *(uint4*)&sw[co * WS + c * 8] = ((const uint4*)a.w)[i];
  }

  const int tilesX = (a.W + TW - 1) / TW, tilesY = (a.H + TR - 1) / TR;
  const int ntiles = tilesX * tilesY * a.B;
  const int wave = tid >> 6, lane = tid & 63, lm = lane & 15, lg = lane >> 4;

  // bias of the four output channels 16 ns + 4 lg .. +3 this lane holds
  float bv[NS][4];
#pragma unroll
  for (int ns = 0; ns < NS; ++ns)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = ns * 16 + lg * 4 + r;
      bv[ns][r] = (a.bias && (MODE != FWD_OUT || co < a.nout)) ? a.bias[co] : 0.f;
    }

  const TileChunks<CI, CO> tc;
  uint4 pre[S::PER];
  if (blockIdx.x < ntiles) conv_load_tile<CI, CO>(pre, a.x, tc, blockIdx.x, tilesX, tilesY, a.H, a.W);

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = tile % tilesX;
    const int ty = (tile / tilesX) % tilesY;
    const int img = tile / (tilesX * tilesY);
    const int x0 = tx * TW, h0 = ty * TR;
    __syncthreads();  // the previous tile's readers of sx are done (and sw is staged)
#pragma unroll
    for (int j = 0; j < S::PER; ++j) {
      const int i = tid + j * CNT;
      if (i < S::NLD) *(uint4*)&sx[(tc.row[j] * TCOLS + tc.col[j]) * PX + tc.c[j] * 8] = pre[j];
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles)  // in flight during the matrix work
      conv_load_tile<CI, CO>(pre, a.x, tc, tile + gridDim.x, tilesX, tilesY, a.H, a.W);

    // D = W X^T: the weights are the A operand (rows: output channels), the
    // input pixels the B operand, so lane (lm, lg) ends with channels
    // 16 ns + 4 lg .. +3 of pixel 16 ms + lm of the wave's row
    // (the accumulators start from the bias)
    f32x4 acc[4][NS];
#pragma unroll
    for (int ms = 0; ms < 4; ++ms)
#pragma unroll
      for (int ns = 0; ns < NS; ++ns) acc[ms][ns] = f32x4{bv[ns][0], bv[ns][1], bv[ns][2], bv[ns][3]};

#pragma unroll
    for (int kc = 0; kc < KP / 32; ++kc) {
      const int k = kc * 32 + lg * 8;  // this lane's 8 consecutive k (one tap)
      const bool kv = k < K;
      const int tap = kv ? k / CI : 0, ci0 = kv ? k % CI : 0;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      bf16x8 wfr[NS];
#pragma unroll
      for (int ns = 0; ns < NS; ++ns) wfr[ns] = *(const bf16x8*)&sw[(ns * 16 + lm) * WS + k];
#pragma unroll
      for (int ms = 0; ms < 4; ++ms) {
        bf16x8 xfr = *(const bf16x8*)&sx[((wave + 1 + dy) * TCOLS + (ms * 16 + lm + 1 + dx)) * PX + ci0];
        if (!kv) xfr = bf16x8{};
#pragma unroll
        for (int ns = 0; ns < NS; ++ns)
          acc[ms][ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfr[ns], xfr, acc[ms][ns], 0, 0, 0);
      }
    }

    // Epilogue straight from the accumulators, 8 bytes (4 channels) per lane
    // and store; the four lanes lg of a pixel write 32 contiguous bytes. The
    // inputs of every store (residual, previous pre-activation) are loaded
    // first so their latencies overlap; a residual that is this layer's own
    // input comes from the tile.
    const int h = h0 + wave;
    if (MODE == FWD_OUT) {
      if (h < a.H) {
        if (a.nout == 3 && NS == 1) {
          // the network's three output channels: lanes lg = 0 hold them
          // (channels 0 .. 3 of their pixel), one 12-byte store each, the 16
          // pixels of a subtile contiguous
          if (lg == 0) {
#pragma unroll
            for (int ms = 0; ms < 4; ++ms) {
              const int xx = x0 + ms * 16 + lm;
              if (xx >= a.W) continue;
              float* p = a.yf + (((int64_t)img * a.H + h) * a.W + xx) * 3;
              p[0] = acc[ms][0][0];
              p[1] = acc[ms][0][1];
              p[2] = acc[ms][0][2];
            }
          }
        } else {
#pragma unroll
          for (int ms = 0; ms < 4; ++ms) {
            const int xx = x0 + ms * 16 + lm;
            if (xx >= a.W) continue;
            const int64_t q = ((int64_t)img * a.H + h) * a.W + xx;
#pragma unroll
            for (int ns = 0; ns < NS; ++ns)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int co = ns * 16 + lg * 4 + r;
                if (co < a.nout) a.yf[q * a.nout + co] = acc[ms][ns][r];
              }
          }
        }
      }
    } else {
      const bool res_in_tile = MODE == FWD_RES && a.res == a.x;
      int64_t off[4];
      bool ok[4];
      bf16x4 rr[4][NS], zp[4][NS];
#pragma unroll
      for (int ms = 0; ms < 4; ++ms) {
        const int xx = x0 + ms * 16 + lm;
        ok[ms] = h < a.H && xx < a.W;
        off[ms] = (((int64_t)img * a.H + (ok[ms] ? h : 0)) * a.W + (ok[ms] ? xx : 0)) * CO + lg * 4;
#pragma unroll
        for (int ns = 0; ns < NS; ++ns) {
          rr[ms][ns] = bf16x4{};
          zp[ms][ns] = bf16x4{};
          if (MODE == FWD_RES) {
            if (res_in_tile)
              rr[ms][ns] = *(const bf16x4*)&sx[((wave + 1) * TCOLS + (ms * 16 + lm + 1)) * PX + ns * 16 + lg * 4];
            else if (ok[ms])
              rr[ms][ns] = *(const bf16x4*)(a.res + off[ms] + ns * 16);
          } else if (MODE == BWD && ok[ms]) {
            if (a.res) rr[ms][ns] = *(const bf16x4*)(a.res + off[ms] + ns * 16);
            zp[ms][ns] = *(const bf16x4*)(a.zprev + off[ms] + ns * 16);
          }
        }
      }
#pragma unroll
      for (int ms = 0; ms < 4; ++ms) {
        if (!ok[ms]) continue;
#pragma unroll
        for (int ns = 0; ns < NS; ++ns) {
          bf16x4 yo, zo;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float v = acc[ms][ns][r];
            if (MODE == FWD_FIRST) {
              yo[r] = f2bf(silu(v));
              zo[r] = f2bf(v);
            } else if (MODE == FWD_RES) {
              yo[r] = f2bf(silu_res(v, bf2f(rr[ms][ns][r])));
              zo[r] = f2bf(v);
            } else {  // BWD: v = dL/dh of this layer's input (+ the residual path)
              const float g = v + bf2f(rr[ms][ns][r]);
              zo[r] = f2bf(g);
              yo[r] = f2bf(g * silu_grad(bf2f(zp[ms][ns][r])));
            }
          }
          *(bf16x4*)(a.y + off[ms] + ns * 16) = yo;
          if (a.z) *(bf16x4*)(a.z + off[ms] + ns * 16) = zo;
        }
      }
    }
  }
}

template <int CI, int CO, int MODE>
static hipError_t launch_conv_t(const ConvArgs& a, int grid, hipStream_t st) {
  // persistent: at most the workgroups that fit on the device at once
  static int resident = 0;
  if (!resident) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, conv_kernel<CI, CO, MODE>, CNT, 0) !=
            hipSuccess || per < 1)
      per = 1;
    resident = cus * per;
  }
  hipLaunchKernelGGL((conv_kernel<CI, CO, MODE>), dim3(grid < resident ? grid : resident), dim3(CNT),
                     0, st, a);
  return hipGetLastError();
}

hipError_t launch_conv(int ci, int co, int mode, const ConvArgs& a, int grid, hipStream_t st) {
#define SG_CONV(CI_, CO_)                                                     \
  if (ci == CI_ && co == CO_) {                                               \
    if (mode == FWD_FIRST) return launch_conv_t<CI_, CO_, FWD_FIRST>(a, grid, st); \
    if (mode == FWD_RES) return launch_conv_t<CI_, CO_, FWD_RES>(a, grid, st);     \
    if (mode == FWD_OUT) return launch_conv_t<CI_, CO_, FWD_OUT>(a, grid, st);     \
    if (mode == BWD) return launch_conv_t<CI_, CO_, BWD>(a, grid, st);             \
  }
  SG_CONV(8, 48)
  SG_CONV(48, 48)
  SG_CONV(48, 16)
  SG_CONV(16, 48)
#undef SG_CONV
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// The residual stack h_l = h_(l-1) + SiLU(conv_l(h_(l-1))), l = 1..4, in one
// pass over HBM: h0 is read once and h4 written once, the activations in
// between stay in LDS. A workgroup owns a strip of SK_ST columns of one image
// and marches down its rows. Every layer keeps a ring of four rows of
// SK_ST + 8 pixels (x periodic: the strip and 4 halo columns on each side;
// layer l computes pixels l .. SK_ST + 7 - l of its ring, one fewer on each
// side per layer). Layer l computes row y at step y + 2 l from rows
// y - 1 .. y + 1 of layer l - 1, which were finished by the step before, so
// one barrier per step orders the rings (a slot is rewritten the step after
// its last reader). Rows outside the image are zeros, the walls' padding:
// the loader and every layer write them as such.
//
// Two waves per layer keep that layer's packed weights in registers (42
// fragments of 16 bytes per lane) and split its 16-pixel subtiles 3 + 2
// (layers 1-3: 70, 68, 66 pixels in five subtiles, the fifth overlapping
// the fourth; layer 4: 64 pixels in 2 + 2). The roles are dealt so that
// waves w and w + 4 (the same SIMD when waves go to the SIMDs in turn) pair
// a 3-subtile part with a 2-subtile one. The product, its k order
// and the epilogue are conv_kernel's (W X^T, FP32 accumulation starting from
// the bias, SiLU with the residual from the layer's input added in one FMA,
// bf16 rounding), so the stack gives the same bits as four FWD_RES launches.
//
// Within a step a wave takes its subtiles one after the other and runs the
// epilogue of subtile m between the products of subtile m + 1 (one output
// value per step of k, scheduling fences every two steps), so that its SiLU
// (two transcendental operations per value) runs on the vector unit while the
// matrix cores work; the body is compiled per role (subtile count, layer 4 or
// not) so that it holds no branch the scheduler cannot cross.
// ---------------------------------------------------------------------------
constexpr int SK_RW = SK_ST + 8;        // ring pixels per row
constexpr int SK_PX = 56;               // LDS pixel stride (elements)
constexpr int SK_KP = kpad<48>();       // 448
constexpr int SK_NKC = SK_KP / 32;      // 14 steps of k
constexpr int SK_NT = 512;              // 8 waves
constexpr int SK_LD = SK_RW * 6;        // 16-byte chunks of an input row (432)

__global__ __launch_bounds__(SK_NT) void stack_kernel(StackArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 ring[4][4][SK_RW * SK_PX];
  __shared__ __attribute__((aligned(16))) float sbias[4][48];
  const int tid = threadIdx.x, lane = tid & 63, lm = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the role is scalar
  const int strips = a.W / SK_ST;
  const int img = blockIdx.x / strips, x0 = (blockIdx.x % strips) * SK_ST;

  // role of the wave: layer L (1..4), first (3 subtiles; layer 4: 2) or
  // second part (2 subtiles)
  const int L = (0x43243211 >> (4 * wave)) & 15;
  const bool first = (0x71 >> wave) & 1;
  const int nm = (L < 4 && first) ? 3 : 2;
  const int k0 = first ? 0 : (L < 4 ? 3 : 2);
  int cs[3], wmin[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const int k = k0 + m;
    const bool last = L < 4 && k == 4;
    cs[m] = last ? SK_RW - 16 - L : L + 16 * k;  // first pixel of the subtile
    wmin[m] = last ? L + 64 : 0;                 // pixels below this were written by subtile 3
  }

  bf16x8 wr[3][SK_NKC];
  {
    const bf16* wl = a.w[L - 1];
#pragma unroll
    for (int ns = 0; ns < 3; ++ns)
#pragma unroll
      for (int kc = 0; kc < SK_NKC; ++kc)
        wr[ns][kc] = *(const bf16x8*)&wl[(ns * 16 + lm) * SK_KP + kc * 32 + lg * 8];
  }
  if (tid < 4 * 48) sbias[tid / 48][tid % 48] = a.bias[tid / 48] ? a.bias[tid / 48][tid % 48] : 0.f;
  for (int i = tid; i < 4 * 4 * SK_RW * SK_PX / 8; i += SK_NT)
    ((uint4*)&ring[0][0][0])[i] = uint4{0u, 0u, 0u, 0u};

  // loader: thread tid < 432 moves chunk tid % 6 (8 channels) of ring pixel
  // tid / 6 of every input row
  const int lpx = tid / 6, lch = tid % 6;
  int lx = x0 - 4 + lpx;
  lx = lx < 0 ? lx + a.W : (lx >= a.W ? lx - a.W : lx);
  const bf16* xin = a.x + (int64_t)img * a.H * a.W * 48 + (int64_t)lx * 48 + lch * 8;
  uint4 pre = {0u, 0u, 0u, 0u};
  if (tid < SK_LD && a.H > 0) pre = *(const uint4*)xin;
  __syncthreads();  // the rings are zero

  bf16* const rin = &ring[L - 1][0][0];
  bf16* const rout = &ring[L < 4 ? L : 0][0][0];
  constexpr int SLOT = SK_RW * SK_PX;

  // The march, compiled per role (NM subtiles; LAST: layer 4, which stores
  // to memory) so that a step's body has no branch: the epilogue of subtile
  // m is interleaved with the products of subtile m + 1.
  auto march = [&](auto nmc, auto lastc) {
    constexpr int NM = decltype(nmc)::value;
    constexpr bool LAST = decltype(lastc)::value;
    for (int t = 0; t < a.H + 8; ++t) {
      if (tid < SK_LD) *(uint4*)&ring[0][t & 3][lpx * SK_PX + lch * 8] = pre;
      pre = uint4{0u, 0u, 0u, 0u};
      if (tid < SK_LD && t + 1 < a.H) pre = *(const uint4*)(xin + (int64_t)(t + 1) * a.W * 48);

      const int y = t - 2 * L;
      if (y < 0 || y >= a.H) {
        if (!LAST) {  // the padding row: zeros over the wave's pixels
#pragma unroll
          for (int m = 0; m < NM; ++m) {
            const int c = cs[m] + lm;
            if (c < wmin[m]) continue;
            uint2* o = (uint2*)&rout[(y & 3) * SLOT + c * SK_PX + lg * 12];
            o[0] = uint2{0u, 0u};
            o[1] = uint2{0u, 0u};
            o[2] = uint2{0u, 0u};
          }
        }
      } else {
        auto ldx = [&](int m, int kc) {
          // this lane's 8 consecutive k = 8 j (one tap): j = 6 tap + ci0 / 8
          const int j = 4 * kc + lg;
          const bool kv = j < 54;
          const int tap = kv ? (j * 43) >> 8 : 0;   // j / 6 for j < 56
          const int ci0 = kv ? 8 * (j - 6 * tap) : 0;
          const int ty = (tap * 11) >> 5;           // tap / 3 for tap < 9
          const int dy = ty - 1, dx = tap - 3 * ty - 1;
          const bf16* src = rin + ((y + dy) & 3) * SLOT + (lm + dx) * SK_PX + ci0;
          bf16x8 xfr = *(const bf16x8*)&src[cs[m] * SK_PX];
          if (!kv) xfr = bf16x8{};
          return xfr;
        };
        // products of subtile m into acc (input fragments two steps of k ahead)
        auto products = [&](int m, f32x4* acc) {
#pragma unroll
          for (int ns = 0; ns < 3; ++ns) acc[ns] = *(const f32x4*)&sbias[L - 1][ns * 16 + lg * 4];
          bf16x8 xa = ldx(m, 0), xb = ldx(m, 1);
#pragma unroll
          for (int kc = 0; kc < SK_NKC; ++kc) {
            bf16x8 xn = bf16x8{};
            if (kc + 2 < SK_NKC) xn = ldx(m, kc + 2);
#pragma unroll
            for (int ns = 0; ns < 3; ++ns)
              acc[ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ns][kc], xa, acc[ns], 0, 0, 0);
            xa = xb;
            xb = xn;
          }
        };
        // epilogue of subtile m (the bias is in the accumulators): SiLU and
        // residual, bf16; pixels the overlapping fifth subtile shares with the
        // fourth are written twice, with the same bits
        auto epilogue = [&](int m, const f32x4* acc) {
          const int c = cs[m] + lm;
          const bf16* rrow = rin + (y & 3) * SLOT + c * SK_PX + lg * 4;
#pragma unroll
          for (int ns = 0; ns < 3; ++ns) {
            const bf16x4 rr = *(const bf16x4*)&rrow[ns * 16];
            bf16x4 yo;
#pragma unroll
            for (int r = 0; r < 4; ++r) yo[r] = f2bf(silu_res(acc[ns][r], bf2f(rr[r])));
            if (!LAST)
              *(bf16x4*)&rout[(y & 3) * SLOT + c * SK_PX + ns * 16 + lg * 4] = yo;
            else
              *(bf16x4*)(a.y + (((int64_t)img * a.H + y) * a.W + x0 + c - 4) * 48 + ns * 16 + lg * 4) = yo;
          }
        };
        f32x4 acc[2][3];
        products(0, acc[0]);
        // the products of subtile m + 1 with the epilogue of subtile m in
        // between, one output value per step of k (12 per lane), the order
        // fixed by scheduling fences so that the matrix cores and the vector
        // unit work side by side
#pragma unroll
        for (int m = 0; m + 1 < NM; ++m) {
          f32x4* pa = acc[(m + 1) & 1];
          const f32x4* ea = acc[m & 1];
          const int c = cs[m] + lm;
          const bf16* rrow = rin + (y & 3) * SLOT + c * SK_PX + lg * 4;
          bf16x4 rr, yo;
#pragma unroll
          for (int ns = 0; ns < 3; ++ns) pa[ns] = *(const f32x4*)&sbias[L - 1][ns * 16 + lg * 4];
          bf16x8 xa = ldx(m + 1, 0), xb = ldx(m + 1, 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int kc = 0; kc < SK_NKC; ++kc) {
            bf16x8 xn = bf16x8{};
            if (kc + 2 < SK_NKC) xn = ldx(m + 1, kc + 2);
#pragma unroll
            for (int ns = 0; ns < 3; ++ns)
              pa[ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[ns][kc], xa, pa[ns], 0, 0, 0);
            xa = xb;
            xb = xn;
            if (kc < 12) {
              const int ns = kc >> 2, r = kc & 3;
              if (r == 0) rr = *(const bf16x4*)&rrow[ns * 16];
              yo[r] = f2bf(silu_res(ea[ns][r], bf2f(rr[r])));
              if (r == 3) {
                if (!LAST)
                  *(bf16x4*)&rout[(y & 3) * SLOT + c * SK_PX + ns * 16 + lg * 4] = yo;
                else
                  *(bf16x4*)(a.y + (((int64_t)img * a.H + y) * a.W + x0 + c - 4) * 48 + ns * 16 + lg * 4) = yo;
              }
            }
            if (kc & 1) __builtin_amdgcn_sched_barrier(0);
          }
        }
        epilogue(NM - 1, acc[(NM - 1) & 1]);
      }
      __syncthreads();
    }
  };
  if (L == 4)
    march(std::integral_constant<int, 2>{}, std::integral_constant<bool, true>{});
  else if (nm == 3)
    march(std::integral_constant<int, 3>{}, std::integral_constant<bool, false>{});
  else
    march(std::integral_constant<int, 2>{}, std::integral_constant<bool, false>{});
}

hipError_t launch_stack(const StackArgs& a, hipStream_t st) {
  if (a.B < 1 || a.H < 1 || a.W < SK_ST || a.W % SK_ST) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stack_kernel, dim3(a.B * (a.W / SK_ST)), dim3(SK_NT), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[tap*CI + ci][co] = sum_p x[p + tap][ci] gz[p][co], a GEMM
// with the pixels as the contraction. A persistent workgroup takes work units
// of WG_RC rows of one 64-pixel column segment of one image and marches down
// them. Each input row is loaded once, transposed (pixels contiguous) and
// stored in LDS three times, shifted by dx = -1, 0, 1; three rows stay in a
// ring (row mod 3), so the A operand of tap (dy, dx) for output row h is the
// copy dx of ring row h + dy. The output gradient row is staged transposed
// beside it; the next row's blocks are loaded into registers during the
// matrix work. The workgroup accumulates its share of the 9CI x CO tiles in
// registers; partial sums per workgroup go to `part`, and wgrad_reduce adds
// them in a fixed order.
// ---------------------------------------------------------------------------
template <int CI, int CO>
__global__ __launch_bounds__(NTH) void wgrad_kernel(WgradArgs a) {
  constexpr int M = 9 * CI, MS = (M + 15) / 16, NS = CO / 16;
  constexpr int SEG = WG_SEG, PS = SEG + 8;  // pixels per segment, LDS row stride
  constexpr int MPW = (MS + 3) / 4;          // M-subtiles per wave (strided by 4)
  constexpr int RING = 3 * CI * PS;      // one ring row: three shifted copies
  // Blocks of 8 pixels x 8 channels: eight 16-byte loads, a register
  // transpose, eight 16-byte LDS stores. Block it < NA is (c8, group, dx)
  // of the input row, the rest (c8, group) of the output-gradient row; a
  // thread owns blocks tid + j NTH.
  constexpr int CA = CI / 8, NA = 3 * (SEG / 8) * CA, NB = NA + (SEG / 8) * (CO / 8);
  constexpr int IPT = (NB + NTH - 1) / NTH;
  __shared__ __attribute__((aligned(16))) bf16 sa[3 * RING];  // [row mod 3][dx + 1][ci][p]
  __shared__ __attribute__((aligned(16))) bf16 sg[CO * PS];   // gz^T[co][p]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lm = lane & 15, lg = lane >> 4;

  f32x4 acc[MPW][NS];
#pragma unroll
  for (int i = 0; i < MPW; ++i)
#pragma unroll
    for (int ns = 0; ns < NS; ++ns) acc[i][ns] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;  // bias gradient partial of channel tid (tid < CO)

  // this lane's A rows: m = 16 ms + lm of each of its M-subtiles, as
  // (dy, offset of copy dx and channel ci within a ring row); m >= M is zero
  int a_dy[MPW], a_off[MPW];
  bool a_ok[MPW];
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int m = (wave + 4 * i) * 16 + lm;
    const int tap = m / CI, ci = m % CI;
    a_ok[i] = m < M;
    a_dy[i] = a_ok[i] ? tap / 3 - 1 : 0;
    a_off[i] = a_ok[i] ? ((tap % 3) * CI + ci) * PS : 0;
  }

  const int segX = (a.W + SEG - 1) / SEG;
  const int chunks = (a.H + WG_RC - 1) / WG_RC;
  const int nunits = segX * chunks * a.B;
  uint4 in[IPT][8];
  // blocks of input row hin (zero outside the image) and, if hg >= 0, of
  // output-gradient row hg, of column segment x0 of image img
  auto load = [&](int img, int x0, int hin, int hg) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int it = tid + j * NTH;
#pragma unroll
      for (int q = 0; q < 8; ++q) in[j][q] = uint4{0u, 0u, 0u, 0u};
      if (it < NA) {
        const int c8 = it % CA, t2 = it / CA, g = t2 % (SEG / 8), dx = t2 / (SEG / 8) - 1;
        if (hin >= 0 && hin < a.H) {
          const bf16* xr = a.x + ((int64_t)img * a.H + hin) * a.W * CI + c8 * 8;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int p = g * 8 + q;
            int xx = x0 + p + dx;  // in [-1, W] for the loaded pixels: periodic in x
            xx = xx < 0 ? xx + a.W : (xx >= a.W ? xx - a.W : xx);
            if (x0 + p < a.W) in[j][q] = *(const uint4*)(xr + (int64_t)xx * CI);
          }
        }
      } else if (it < NB && hg >= 0) {
        const int j2 = it - NA, c8 = j2 % (CO / 8), g = j2 / (CO / 8);
        const bf16* gr = a.gz + (((int64_t)img * a.H + hg) * a.W + x0) * CO + c8 * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (x0 + g * 8 + q < a.W) in[j][q] = *(const uint4*)(gr + (int64_t)(g * 8 + q) * CO);
      }
    }
  };
  // transpose the loaded blocks into ring row `slot` (and sg when with_gz):
  // out row (channel) 2w holds the low halves of dword w of the 8 pixels,
  // row 2w + 1 the high halves; dword k of a row packs pixels 2k, 2k + 1
  auto store = [&](int slot, bool with_gz) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      const int it = tid + j * NTH;
      if (it >= (with_gz ? NB : NA)) continue;
      int row0, g;
      bf16* base;
      if (it < NA) {
        const int c8 = it % CA, t2 = it / CA, dx1 = t2 / (SEG / 8);
        g = t2 % (SEG / 8);
        row0 = dx1 * CI + c8 * 8;
        base = sa + slot * RING;
      } else {
        const int j2 = it - NA;
        g = j2 / (CO / 8);
        row0 = (j2 % (CO / 8)) * 8;
        base = sg;
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t e = ((const uint32_t*)&in[j][2 * k])[w];
          const uint32_t o = ((const uint32_t*)&in[j][2 * k + 1])[w];
          lo[k] = __builtin_amdgcn_perm(o, e, 0x05040100u);
          hi[k] = __builtin_amdgcn_perm(o, e, 0x07060302u);
        }
        *(uint4*)&base[(row0 + 2 * w) * PS + g * 8] = uint4{lo[0], lo[1], lo[2], lo[3]};
        *(uint4*)&base[(row0 + 2 * w + 1) * PS + g * 8] = uint4{hi[0], hi[1], hi[2], hi[3]};
      }
    }
  };
  auto slot_of = [](int row) { return ((row % 3) + 3) % 3; };

  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int sx = u % segX, ch = (u / segX) % chunks, img = u / (segX * chunks);
    const int x0 = sx * SEG, h0 = ch * WG_RC, h1 = min(a.H, h0 + WG_RC);
    // the ring's first two rows (h0 - 1, h0)
#pragma unroll 1
    for (int r = h0 - 1; r <= h0; ++r) {
      load(img, x0, r, -1);
      __syncthreads();  // earlier readers of this ring row are done
      store(slot_of(r), false);
    }
    load(img, x0, h0 + 1, h0);
#pragma unroll 1
    for (int h = h0; h < h1; ++h) {
      __syncthreads();  // the previous row's readers of the ring row and sg are done
      store(slot_of(h + 1), true);
      __syncthreads();
      if (h + 1 < h1) load(img, x0, h + 2, h + 1);  // in flight during the matrix work
      if (tid < CO) {  // the bias gradient: 16-byte reads issued together, then added
        uint4 v[SEG / 8];
#pragma unroll
        for (int c = 0; c < SEG / 8; ++c) v[c] = *(const uint4*)&sg[tid * PS + c * 8];
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < SEG / 8; ++c) {
          const bf16x8 e = __builtin_bit_cast(bf16x8, v[c]);
#pragma unroll
          for (int q = 0; q < 8; ++q) t += bf2f(e[q]);
        }
        bsum += t;
      }
      int abase[MPW];
#pragma unroll
      for (int i = 0; i < MPW; ++i) abase[i] = slot_of(h + a_dy[i]) * RING + a_off[i];
#pragma unroll
      for (int kc = 0; kc < SEG / 32; ++kc) {
        const int k = kc * 32 + lg * 8;
        bf16x8 bfr[NS];
#pragma unroll
        for (int ns = 0; ns < NS; ++ns) bfr[ns] = *(const bf16x8*)&sg[(ns * 16 + lm) * PS + k];
#pragma unroll
        for (int i = 0; i < MPW; ++i) {
          const int ms = wave + 4 * i;
          if (ms < MS) {  // uniform per wave
            bf16x8 afr = *(const bf16x8*)&sa[abase[i] + k];
            if (!a_ok[i]) afr = bf16x8{};
#pragma unroll
            for (int ns = 0; ns < NS; ++ns)
              acc[i][ns] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[ns], acc[i][ns], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();  // the last row's readers are done before the next unit's ring rows
  }
  // partial sums of this workgroup: part[block][m][co], then the bias
  // partials part[block][M CO + co]
  float* out = a.part + (int64_t)blockIdx.x * (M * CO + CO);
  if (tid < CO) out[M * CO + tid] = bsum;
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int ms = wave + 4 * i;
    if (ms >= MS) continue;
#pragma unroll
    for (int ns = 0; ns < NS; ++ns)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = ms * 16 + lg * 4 + r, co = ns * 16 + lm;
        if (m < M) out[m * CO + co] = acc[i][ns][r];
      }
  }
}

template <int CI, int CO>
static hipError_t launch_wgrad_t(const WgradArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((wgrad_kernel<CI, CO>), dim3(grid), dim3(NTH), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(int ci, int co, const WgradArgs& a, int grid, hipStream_t st) {
  if (ci == 8 && co == 48) return launch_wgrad_t<8, 48>(a, grid, st);
  if (ci == 48 && co == 48) return launch_wgrad_t<48, 48>(a, grid, st);
  if (ci == 48 && co == 16) return launch_wgrad_t<48, 16>(a, grid, st);
  return hipErrorInvalidValue;
}

// Fixed-order sum of the workgroup partials onto the real channels, in two
// stages (stage 1: kRedGroups consecutive runs of blocks, stage 2: the runs).
// Output element i < 9 cir cor: dw[(tap*cir + ci)*cor + co] from partial
// entry (tap*CI + ci)*CO + co; i >= 9 cir cor: db[co] from entry 9 CI CO + co.
constexpr int kRedGroups = 16;

__device__ __forceinline__ int64_t wgrad_entry(int i, int CI, int CO, int cir, int cor) {
  const int nw = 9 * cir * cor;
  if (i >= nw) return (int64_t)9 * CI * CO + (i - nw);
  const int co = i % cor, ci = (i / cor) % cir, tap = i / (cor * cir);
  return (int64_t)(tap * CI + ci) * CO + co;
}

__global__ void wgrad_reduce1_kernel(const float* __restrict__ part, int nblk, int CI, int CO,
                                     int cir, int cor, double* __restrict__ tmp) {
  const int n = 9 * cir * cor + cor;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int g = blockIdx.y;
  const int per = (nblk + kRedGroups - 1) / kRedGroups;
  const int b0 = g * per, b1 = min(nblk, b0 + per);
  const int64_t stride = (int64_t)9 * CI * CO + CO, j = wgrad_entry(i, CI, CO, cir, cor);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = b0;
  for (; b + 3 < b1; b += 4) {
    s0 += part[b * stride + j];
    s1 += part[(b + 1) * stride + j];
    s2 += part[(b + 2) * stride + j];
    s3 += part[(b + 3) * stride + j];
  }
  for (; b < b1; ++b) s0 += part[b * stride + j];
  tmp[(int64_t)g * n + i] = (s0 + s1) + (s2 + s3);
}

__global__ void wgrad_reduce2_kernel(const double* __restrict__ tmp, int n, int nw, float scale,
                                     float* __restrict__ dw, float* __restrict__ db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
#pragma unroll
  for (int g = 0; g < kRedGroups; ++g) s += tmp[(int64_t)g * n + i];
  if (i < nw)
    dw[i] = (float)(s * scale);
  else if (db)
    db[i - nw] = (float)(s * scale);
}

hipError_t launch_wgrad_reduce(const float* part, int nblk, int CI, int CO, int cir, int cor,
                               float scale, double* tmp, float* dw, float* db, hipStream_t st) {
  const int nw = 9 * cir * cor, n = nw + cor;
  hipLaunchKernelGGL(wgrad_reduce1_kernel, dim3((n + 255) / 256, kRedGroups), dim3(256), 0, st, part,
                     nblk, CI, CO, cir, cor, tmp);
  hipLaunchKernelGGL(wgrad_reduce2_kernel, dim3((n + 255) / 256), dim3(256), 0, st, tmp, n, nw,
                     scale, dw, db);
  return hipGetLastError();
}

// Bias gradient: db[c] = scale * sum_p gz[p][c] in a fixed order: block b
// sums pixels b, b + nb, ... per channel, then one pass adds the block sums.
constexpr int kBiasBlocks = 1024;

__global__ void bias_partial_kernel(const bf16* __restrict__ gz, int64_t npix, int C,
                                    float* __restrict__ part) {
  const int c = threadIdx.x;
  if (c >= C) return;
  double s = 0.0;
  for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) s += (double)bf2f(gz[p * C + c]);
  part[blockIdx.x * C + c] = (float)s;
}

__global__ void bias_final_kernel(const float* __restrict__ part, int nb, int C, int nreal,
                                  float scale, float* __restrict__ db) {
  const int c = threadIdx.x;
  if (c >= nreal) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b * C + c];
  db[c] = (float)(s * scale);
}

hipError_t launch_bias_grad(const bf16* gz, int64_t npix, int C, int nreal, float scale,
                            float* part, float* db, hipStream_t st) {
  hipLaunchKernelGGL(bias_partial_kernel, dim3(kBiasBlocks), dim3(64), 0, st, gz, npix, C, part);
  hipLaunchKernelGGL(bias_final_kernel, dim3(1), dim3(64), 0, st, part, kBiasBlocks, C, nreal,
                     scale, db);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loss: mean squared error over the nout real output channels, FP32 inputs;
// writes the gradient of the summed loss, 2 (pred - target), as bf16 with
// CO channels (zeros past nout), and per-block FP64 partial sums.
// ---------------------------------------------------------------------------
__global__ void mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                           int64_t npix, int nout, int CO, bf16* __restrict__ gout,
                           double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
       p += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < CO; ++c) {
      float g = 0.f;
      if (c < nout) {
        const float d = pred[p * nout + c] - target[p * nout + c];
        s += (double)d * d;
        g = 2.f * d;
      }
      gout[p * CO + c] = f2bf(g);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One wave: lane l adds part[l], part[l + 64], ... in order, then the 64 lane
// sums are added pairwise in a fixed tree, so the result does not vary from
// run to run.
__global__ void sum_partials_kernel(const double* __restrict__ part, int n, double scale,
                                    double* __restrict__ out) {
  const int l = threadIdx.x;
  double s = 0.0;
  for (int i = l; i < n; i += 64) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (l == 0) *out = s * scale;
}

hipError_t launch_mse(const float* pred, const float* target, int64_t npix, int nout, int CO,
                      bf16* gout, double* part, double* loss, hipStream_t st) {
  const int nb = 512;
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, pred, target, npix, nout, CO, gout, part);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, part, nb,
                     1.0 / ((double)npix * nout), loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adam on FP32 master parameters (Kingma and Ba), step t counted from 1.
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight packing: FP32 w[tap][ci][co] (ci < cir, co < cor real channels) into
// bf16 B-matrices. Forward: wp[co][tap*CI + ci]. Input gradient (transposed
// convolution, flipped taps): wp[ci][tap'*CO + co] = w[8 - tap'][ci][co].
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const float* __restrict__ w, int cir, int cor, int CI, int CO,
                            int transposed, bf16* __restrict__ wp) {
  // forward: rows = CO, k over 9*CI; transposed: rows = CI, k over 9*CO
  const int rows = transposed ? CI : CO;
  const int kin = transposed ? CO : CI;
  const int KPd = (9 * kin + 31) / 32 * 32;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * KPd) return;
  const int row = i / KPd, k = i % KPd;
  float v = 0.f;
  if (k < 9 * kin) {
    const int tap = k / kin, c = k % kin;
    if (!transposed) {
      if (c < cir && row < cor) v = w[(tap * cir + c) * cor + row];
    } else {
      if (row < cir && c < cor) v = w[((8 - tap) * cir + row) * cor + c];
    }
  }
  wp[i] = f2bf(v);
}

hipError_t launch_pack(const float* w, int cir, int cor, int CI, int CO, int transposed, bf16* wp,
                       hipStream_t st) {
  const int rows = transposed ? CI : CO;
  const int kin = transposed ? CO : CI;
  const int n = rows * ((9 * kin + 31) / 32 * 32);
  hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, cir, cor, CI, CO,
                     transposed, wp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fields <-> network tensors, batched over instances of one size (nn = H*W
// nodes). Moments are FP64 blocks [B][3][H][W] (n, u_x, u_y).
// Input channels (8, bf16): (n - 1) s_n, u_x s_u, u_y s_u, V(x) s_v, wall speed
// s_u on the wall rows (-U on row 0, +U on row H-1, 0 elsewhere), (T - 0.9) s_t,
// 0, 0. Target / output channels (3, FP32): change over the chunk,
// (dn s_n, du_x s_u, du_y s_u).
// ---------------------------------------------------------------------------
__global__ void fields_to_input_kernel(const double* __restrict__ mom, int B, int H, int W,
                                       const float* __restrict__ vx, const float* __restrict__ cond,
                                       int walls, Scales s, bf16* __restrict__ x) {
  const int64_t nn = (int64_t)H * W;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < (int64_t)B * nn;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(g / nn);
    const int64_t k = g - (int64_t)b * nn;
    const int h = (int)(k / W), xx = (int)(k % W);
    const double* m = mom + (int64_t)b * 3 * nn;
    const float uwall = cond[2 * b], temp = cond[2 * b + 1];
    float c[8];
    c[0] = (float)((m[k] - 1.0) * s.n);
    c[1] = (float)(m[nn + k] * s.u);
    c[2] = (float)(m[2 * nn + k] * s.u);
    c[3] = vx[(int64_t)b * W + xx] * s.v;
    c[4] = walls ? (h == 0 ? -uwall * s.u : (h == H - 1 ? uwall * s.u : 0.f)) : 0.f;
    c[5] = (temp - 0.9f) * s.t;
    c[6] = 0.f;
    c[7] = 0.f;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = f2bf(c[j]);
    *(bf16x8*)(x + g * 8) = v;
  }
}

static int grid_1d(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

hipError_t launch_fields_to_input(const double* mom, int B, int H, int W, const float* vx,
                                  const float* cond, int walls, Scales s, bf16* x, hipStream_t st) {
  hipLaunchKernelGGL(fields_to_input_kernel, dim3(grid_1d((int64_t)B * H * W)), dim3(256), 0, st,
                     mom, B, H, W, vx, cond, walls, s, x);
  return hipGetLastError();
}

// target[b][k][c] = (fields1 - fields0) scaled
__global__ void make_target_kernel(const double* __restrict__ m0, const double* __restrict__ m1,
                                   int B, int64_t nn, Scales s, float* __restrict__ target) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < (int64_t)B * nn;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = g / nn, k = g - b * nn, o = b * 3 * nn + k;
    target[g * 3 + 0] = (float)((m1[o] - m0[o]) * s.n);
    target[g * 3 + 1] = (float)((m1[o + nn] - m0[o + nn]) * s.u);
    target[g * 3 + 2] = (float)((m1[o + 2 * nn] - m0[o + 2 * nn]) * s.u);
  }
}

hipError_t launch_make_target(const double* m0, const double* m1, int B, int64_t nn, Scales s,
                              float* target, hipStream_t st) {
  hipLaunchKernelGGL(make_target_kernel, dim3(grid_1d(B * nn)), dim3(256), 0, st, m0, m1, B, nn, s,
                     target);
  return hipGetLastError();
}

// predicted fields (FP64) = fields0 + output / scales
__global__ void apply_output_kernel(const double* __restrict__ m0, const float* __restrict__ out,
                                    int B, int64_t nn, Scales s, double* __restrict__ m1) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < (int64_t)B * nn;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = g / nn, k = g - b * nn, o = b * 3 * nn + k;
    m1[o] = m0[o] + (double)out[g * 3 + 0] / s.n;
    m1[o + nn] = m0[o + nn] + (double)out[g * 3 + 1] / s.u;
    m1[o + 2 * nn] = m0[o + 2 * nn] + (double)out[g * 3 + 2] / s.u;
  }
}

hipError_t launch_apply_output(const double* m0, const float* out, int B, int64_t nn, Scales s,
                               double* m1, hipStream_t st) {
  hipLaunchKernelGGL(apply_output_kernel, dim3(grid_1d(B * nn)), dim3(256), 0, st, m0, out, B, nn,
                     s, m1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-instance comparisons of two field blocks [B][3][nn], one workgroup per
// instance, fixed reduction order (deterministic): out[b][0..5] = (sum n_a,
// sum n_b, max |n_a - n_b| / n_b, count of nodes where n_a is not finite or
// outside (0, 3), sum (n_a - n_b)^2, sum n_b^2).
// ---------------------------------------------------------------------------
constexpr int kCmpBS = 256;

__global__ __launch_bounds__(kCmpBS) void compare_kernel(const double* __restrict__ a,
                                                         const double* __restrict__ bref,
                                                         int64_t nn, double* __restrict__ out) {
  const int b = blockIdx.x;
  const double* na = a + (int64_t)b * 3 * nn;
  const double* nb = bref + (int64_t)b * 3 * nn;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = threadIdx.x; k < nn; k += kCmpBS) {
    const double x = na[k], y = nb[k];
    v[0] += x;
    v[1] += y;
    const double e = fabs(x - y) / y;
    v[2] = (e > v[2] || e != e) ? e : v[2];  // NaN propagates
    v[3] += (x > 0.0 && x < 3.0) ? 0.0 : 1.0;
    v[4] += (x - y) * (x - y);
    v[5] += y * y;
  }
  __shared__ double red[6][kCmpBS];
#pragma unroll
  for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = v[j];
  __syncthreads();
  for (int o = kCmpBS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double u = red[j][threadIdx.x + o];
        if (j == 2) {
          if (u > red[2][threadIdx.x] || u != u) red[2][threadIdx.x] = u;
        } else {
          red[j][threadIdx.x] += u;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[6 * b + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_compare(const double* a, const double* b, int B, int64_t nn, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(compare_kernel, dim3(B), dim3(kCmpBS), 0, st, a, b, nn, out);
  return hipGetLastError();
}

// Mass projection: n_a += (sum n_ref - sum n_a) / nn for the instances with
// mask[b] != 0, so that the total density of a equals that of ref (FP64,
// fixed reduction order).
__global__ __launch_bounds__(kCmpBS) void project_mass_kernel(double* __restrict__ a,
                                                              const double* __restrict__ ref,
                                                              int64_t nn,
                                                              const int32_t* __restrict__ mask) {
  const int b = blockIdx.x;
  if (!mask[b]) return;
  double* na = a + (int64_t)b * 3 * nn;
  const double* nr = ref + (int64_t)b * 3 * nn;
  double d = 0;
  for (int64_t k = threadIdx.x; k < nn; k += kCmpBS) d += nr[k] - na[k];
  __shared__ double red[kCmpBS];
  red[threadIdx.x] = d;
  __syncthreads();
  for (int o = kCmpBS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double shift = red[0] / (double)nn;
  for (int64_t k = threadIdx.x; k < nn; k += kCmpBS) na[k] += shift;
}

hipError_t launch_project_mass(double* a, const double* ref, int B, int64_t nn, const int32_t* mask,
                               hipStream_t st) {
  hipLaunchKernelGGL(project_mass_kernel, dim3(B), dim3(kCmpBS), 0, st, a, ref, nn, mask);
  return hipGetLastError();
}

}  // namespace sg
