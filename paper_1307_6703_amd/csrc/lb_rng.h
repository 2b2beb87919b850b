// Counter-based random numbers and unbiased rounding to float, for the
// stochastic-rounding precision of the lattice kernels (lb_device.hip,
// d17_device.hip). Device functions only.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace lbrng {

// Counter-based random numbers for the stochastic rounding: the pcg4d hash of
// Jarzynski and Olano ("Hash Functions for GPU Rendering", JCGT 9(3), 2020),
// applied to (column, row, step, 0), so every node, step and population gets
// its own draw and the stream does not depend on the launch shape.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 pcg4d(U4 v) {
  v.x = v.x * 1664525u + 1013904223u;
  v.y = v.y * 1664525u + 1013904223u;
  v.z = v.z * 1664525u + 1013904223u;
  v.w = v.w * 1664525u + 1013904223u;
  v.x += v.y * v.w;
  v.y += v.z * v.x;
  v.z += v.x * v.y;
  v.w += v.y * v.z;
  v.x ^= v.x >> 16;
  v.y ^= v.y >> 16;
  v.z ^= v.z >> 16;
  v.w ^= v.w >> 16;
  v.x += v.y * v.w;
  v.y += v.z * v.x;
  v.z += v.x * v.y;
  v.w += v.y * v.z;
  return v;
}

// Nine 14-bit draws from one hash: two from the low 28 bits of each word,
// the ninth from the words' top 4 bits.
__device__ __forceinline__ void draws14(U4 h, uint32_t q[9]) {
  q[0] = h.x & 0x3fffu; q[1] = (h.x >> 14) & 0x3fffu;
  q[2] = h.y & 0x3fffu; q[3] = (h.y >> 14) & 0x3fffu;
  q[4] = h.z & 0x3fffu; q[5] = (h.z >> 14) & 0x3fffu;
  q[6] = h.w & 0x3fffu; q[7] = (h.w >> 14) & 0x3fffu;
  q[8] = ((h.x >> 28) | ((h.y >> 28) << 4) | ((h.z >> 28) << 8) | ((h.w >> 30) << 12)) & 0x3fffu;
}

// Unbiased rounding of v to float. The magnitude goes to its nearest float
// or to the neighbouring float on the other side of it, the latter with
// probability |remainder| / gap, so the expected result is v (up to the
// 14-bit resolution of the draw q, a bias below 2^-15 of a float ulp).
__device__ __forceinline__ float round_stochastic(double v, uint32_t q) {
  const double a = fabs(v);
  const float fn = (float)a;          // nearest, ties to even
  const double r = a - (double)fn;    // exact
  const uint32_t b = __float_as_uint(fn);
  // r < 0 implies fn > 0, so b - 1 stays a finite non-negative float
  const float fo = __uint_as_float(r > 0.0 ? b + 1u : b - 1u);
  const double gap = fabs((double)fo - (double)fn);
  const float m = ((double)q + 0.5) * (1.0 / 16384.0) * gap < fabs(r) ? fo : fn;
  return v < 0.0 ? -m : m;
}

}  // namespace lbrng
