// Host-side helpers shared by the single-lattice and batched C ABI code.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "lb_internal.h"
#include "lbvdw.h"

using lbk::Desc;
using lbk::ReduceOut;
using lbk::Tile;

namespace lbh {

extern thread_local std::string g_err;

inline lb_status fail(lb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return lbh::fail(LB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline lb_status validate(const lb_params* p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (p->Lx < 1) return fail(LB_EINVAL, "Lx must be >= 1 (got %d)", p->Lx);
  if (p->Ly < 4) return fail(LB_EINVAL, "Ly must be >= 4 (got %d)", p->Ly);
  // the nine population planes of one buffer must stay below 2 GiB (32-bit
  // buffer offsets in the step kernel, range-checked without wrapping)
  if ((int64_t)p->Lx * p->Ly * 9 * (p->fp32 ? 4 : 8) >= ((int64_t)1 << 31))
    return fail(LB_EINVAL, "9*Lx*Ly*(4|8) bytes must be < 2 GiB (FP32: < 59652323 nodes)");
  if (p->y_periodic != 0 && p->y_periodic != 1) return fail(LB_EINVAL, "y_periodic must be 0 or 1");
  if (p->fp32 < 0 || p->fp32 > 2) return fail(LB_EINVAL, "fp32 must be 0, 1 or 2 (got %d)", p->fp32);
  if (!(p->T > 0.0 && p->T <= 1.5)) return fail(LB_EINVAL, "T must be in (0, 1.5] (got %g)", p->T);
  if (!(std::sqrt(3.0) * p->tau > 0.5) || !std::isfinite(p->tau))
    return fail(LB_EINVAL, "need sqrt(3)*tau > 1/2 (got tau=%g)", p->tau);
  if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa)) return fail(LB_EINVAL, "kappa must be >= 0");
  if (!std::isfinite(p->N) || !std::isfinite(p->Q)) return fail(LB_EINVAL, "N, Q must be finite");
  if (!(std::fabs(p->U) < 0.3)) return fail(LB_EINVAL, "|U| must be < 0.3 (got %g)", p->U);
  if (p->check_every < 0) return fail(LB_EINVAL, "check_every must be >= 0");
  if (p->drift_correct != 0 && p->drift_correct != 1) return fail(LB_EINVAL, "drift_correct must be 0 or 1");
  if (p->collision != 0 && p->collision != 1) return fail(LB_EINVAL, "collision must be 0 or 1");
  if (p->fext_x)
    for (int x = 0; x < p->Lx; ++x)
      if (!std::isfinite(p->fext_x[x])) return fail(LB_EINVAL, "fext_x[%d] is not finite", x);
  return LB_OK;
}

// Workspace layout of one lattice, all offsets 256-byte aligned.
struct Layout {
  size_t desc, red, tiles, tiles1, fext, part, mom, stage, S0, S1, total;
  int max_tiles;
};

constexpr int kMinRows = 8;

inline Layout layout_for(const lb_params* p, size_t base = 0) {
  const size_t nn = (size_t)p->Lx * p->Ly;
  const size_t rs = p->fp32 ? sizeof(float) : sizeof(double);
  Layout L;
  const int strips = (p->Lx + 49) / 50;  // narrowest strip: 64 threads, two steps
  const int chunks = (p->Ly + kMinRows - 1) / kMinRows;
  L.max_tiles = strips * chunks;
  size_t o = base;
  L.desc = o; o = align_up(o + sizeof(Desc));
  L.red = o; o = align_up(o + sizeof(ReduceOut));
  L.tiles = o; o = align_up(o + sizeof(Tile) * (size_t)L.max_tiles);
  L.tiles1 = o; o = align_up(o + sizeof(Tile) * (size_t)L.max_tiles);
  L.fext = o; o = align_up(o + sizeof(double) * (size_t)p->Lx);  // FP32 or FP64 table
  L.part = o; o = align_up(o + sizeof(double) * 6 * (size_t)lbk::reduce_blocks((int64_t)nn));
  L.mom = o; o = align_up(o + sizeof(double) * 3 * nn);
  L.stage = o; o = align_up(o + sizeof(double) * nn);
  L.S0 = o; o = align_up(o + rs * 9 * nn);
  L.S1 = o; o = align_up(o + rs * 9 * nn);
  L.total = o - base;
  return L;
}

// Precision of a parameter set: lbk::kFP64, kFP32 or kFP32SR.
inline int prec_of(const lb_params* p) { return p->fp32; }
// FP64 arithmetic (FP64, or FP32 storage with stochastic rounding).
inline bool arith64(const lb_params* p) { return p->fp32 != lbk::kFP32; }

// Strip width: one strip per row for narrow lattices; 512-thread strips
// (one workgroup per CU) once the lattice fills the device with them.
inline int default_threads(const lb_params* p) {
  if (p->Lx + 6 <= 64) return 64;
  // FP64 arithmetic (two waves per SIMD): 256-thread strips once the lattice is large
  if (arith64(p)) return ((int64_t)p->Lx * p->Ly >= ((int64_t)1 << 22) && p->Lx + 6 > 128) ? 256 : 128;
  if (p->Lx + 6 <= 128) return 128;
  if (p->Lx + 6 <= 256) return 256;
  if (p->Lx + 6 <= 320) return 320;  // one strip per row (e.g. 256-wide lattices)
  if ((int64_t)p->Lx * p->Ly >= ((int64_t)1 << 22)) return 512;
  return 256;
}

// Workgroups of the step kernel that fit on the device at once: FP32 runs at
// 3 waves per SIMD (about 140 VGPRs), FP64 arithmetic at 2.
inline int resident_slots(const lb_params* p, int threads) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  const int waves_per_cu = (arith64(p) ? 2 : 3) * 4;
  return cus * std::max(1, waves_per_cu / ((threads + 63) / 64));
}

// Rows per chunk for a target number of chunks: a height of `mod` mod 8 so
// the kernel's 8-row unrolled march has no idle tail (2 for the one-step
// kernel, whose march is rows + 6 long; 0 for the two-step kernel, rows + 16).
inline int rows_for_chunks(int Ly, int chunks, int mod = 2) {
  int rows = (Ly + std::max(chunks, 1) - 1) / std::max(chunks, 1);
  rows = ((std::max(rows, 8 + mod) - mod + 7) / 8) * 8 + mod;
  return std::min(rows, Ly);
}

// Rows per chunk: as few chunks as fill the resident workgroups `rounds`
// times.
inline int default_rows(const lb_params* p, int threads, int rounds = 1) {
  const int strips = (p->Lx + threads - 7) / (threads - 6);
  return rows_for_chunks(p->Ly, rounds * resident_slots(p, threads) / strips);
}

// Two-step kernel (FP32): strips of threads-14 columns. One workgroup's LDS
// rings take 288 (threads + 2) bytes, so 8, 4, 2 or 2 workgroups of 64, 128,
// 192 or 256 threads fit on a CU (160 KB of LDS); at most 256 VGPRs allow 2
// waves per SIMD.
inline bool fused_threads_ok(int threads) {
  return threads == 64 || threads == 128 || threads == 192 || threads == 256;
}

inline int fused_resident_slots(int threads) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  const int by_lds = (160 * 1024) / (288 * (threads + 2));
  const int by_vgpr = 8 / (threads / 64);
  return cus * std::max(1, std::min(by_lds, by_vgpr));
}

inline int fused_default_rows(const lb_params* p, int threads, int rounds = 1) {
  const int strips = (p->Lx + threads - 15) / (threads - 14);
  return rows_for_chunks(p->Ly, rounds * fused_resident_slots(threads) / strips, 0);
}

// Tiles of one lattice: strips of `threads - 2 halo` columns (halo 3 for the
// one-step kernel, 7 for the two-step kernel), chunks of `rows` rows (the
// last one ragged) or, with `balanced` and Ly a multiple of 8, as many
// chunks with heights that are multiples of 8 and differ by at most 8, or,
// with `short_ends`, the rows the last chunk would lack taken from the first
// and the last chunk alike (the two-step kernel runs the chunks at the walls
// in its slower general body, the others in the wall-free one);
// strip-major so consecutive tiles are vertical neighbours. Odd chunks march
// downwards (sign bit of inst), so two neighbouring chunks reach their
// shared boundary rows at the same time and share those loads in L2.
inline std::vector<Tile> make_tiles(int inst, int Lx, int Ly, int threads, int rows,
                                    int halo = 3, bool balanced = false, bool short_ends = false) {
  std::vector<int> y0s;
  const int nch = (Ly + rows - 1) / rows;
  if (short_ends && nch >= 3) {
    const int spare = nch * rows - Ly;  // < rows
    const int s1 = (spare / 2) / 8 * 8;
    y0s.push_back(0);
    for (int j = 1, y = rows - s1; j < nch; ++j, y += rows) y0s.push_back(y);
  } else if (balanced && Ly % 8 == 0 && rows >= 8) {
    const int n = (Ly + rows - 1) / rows, units = Ly / 8;
    for (int j = 0, y = 0; j < n; ++j) {
      y0s.push_back(y);
      y += 8 * (units / n + (j < units % n ? 1 : 0));
    }
  } else {
    for (int y0 = 0; y0 < Ly; y0 += rows) y0s.push_back(y0);
  }
  y0s.push_back(Ly);
  std::vector<Tile> t;
  const int w = threads - 2 * halo;
  for (int x0 = 0; x0 < Lx; x0 += w)
    for (size_t j = 0; j + 1 < y0s.size(); ++j) {
      const int code = (j & 1) ? (int)((unsigned)inst | 0x80000000u) : inst;
      t.push_back({code, x0, y0s[j], std::min(Ly, y0s[j + 1])});
    }
  return t;
}

}  // namespace lbh

