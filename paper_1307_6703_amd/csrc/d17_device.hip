// Device code of the D2Q17 variant of the lattice Boltzmann step for a van der
// Waals fluid (Coclite, Gonnella, Lamura, arXiv:1307.6703): the third-order
// model with seventeen velocities that the remark after Eq.(nav) names as the
// way to remove the u*^3 term of the Navier-Stokes equation. Periodic
// lattices; gfx950.
//
// The step is the paper's (pull streaming, density, the force of Eq.(force2)
// with Eq.(eqstate) and Eq.(periodicforce) from the stencils of Eq.(xstencil)
// and Eq.(laplstencil), velocity u* of Eq.(newvel), BGK collision with a
// forcing term, Eq.(evoleq)); the equilibrium and the forcing term are their
// Hermite expansions carried to third order:
//   f_eq_i = w^_i n + w_i n E_i(u),
//   E_i = a1 c.u + (s^2/2)(c.u)^2 - (s/2) u^2 + (s^3/6)(c.u)^3 - (s^2/2)(c.u) u^2,
//   F_i = w_i (1 - omega/2) [a1 c.F + s^2 (c.u)(c.F) - s u.F
//         + (s^3/2)(c.F)(c.u)^2 - (s^2/2)(c.F) u^2 - s^2 (u.F)(c.u)],
// with s = r^2 = (125 + 5 sqrt(193))/72 the lattice's scale (its sound speed
// squared is 1/s), w^_i = w_i [1 + (T-1)(s |c_i|^2 - 2)/2] the rest-state
// weights and a1 = s [1 + (T-1)(s |c_i|^2 - 4)/2]. Both are expansions in the
// same polynomials, so with j = n u the collision's new part is one sum:
//   omega n E_i + (1 - omega/2) F_i-part
//     = a1 c.B + (s^2/2) c.A.c - (s/2) tr A + (s^3/6) C:ccc - (s^2/2) c.v,
//   B = omega j + p F,  A = omega j u + p (u F + F u),
//   C = omega j u u + p (F u u + u F u + u u F),  v_a = C_abb,
// p = 1 - omega/2. The terms of A are even in c and the others odd, so the
// two directions of each pair share them.
//
// Lattice units (dx = dt = 1, c_i integer); the host converts the paper's
// tau (tau_l = r tau), kappa and F_ext (divided by s). Populations are stored
// as deviations g_i = f_i - w^_i nbar (nbar = 0 in FP64 mode).
//
// Kernel design. A workgroup of NT threads owns a strip of NT - 4 columns and
// a chunk of rows; thread t works on column x0 - 2 + t and marches along y
// (upwards in even chunks, downwards in odd ones, so that neighbouring chunks
// read the rows they share at about the same time, on the same XCD in the
// tile order below; this order measured faster, although the L2 counters show
// the shared rows fetched again, largely from the Infinity Cache). Each
// iteration takes one row a through three stages (d = the march direction):
//   A (row a):     the 17 pulled values S_i(x - c_i) (loaded one iteration
//                  ahead into a register ring), density deviation and raw
//                  momentum;
//   B (row a-d):   Laplacian of n and the pressure term p^i - p^w;
//   C (row a-2d):  force from the gradients of both, u*, collision, store.
// The density deviations and the B results live in three-row LDS rings; the
// pulled values wait two rows in registers. Two barriers per row. The pull
// reaches three rows and columns: every load comes straight from the
// population array (periodic wrap), no halo exchange.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "d17_internal.h"
#include "lb_rng.h"

namespace d17k {

// Velocity set: 0 rest; 1-4 (1,0), (0,1), (-1,0), (0,-1); 5-8 (1,1), (-1,1),
// (-1,-1), (1,-1); 9-12 twice those diagonals; 13-16 three times the axis
// vectors. Direction i + 2 is the opposite of i for i = 1, 2, 5, 6, 9, 10,
// 13, 14.
__host__ __device__ constexpr int cx17(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1
         : (i == 3 || i == 6 || i == 7) ? -1
         : (i == 9 || i == 12) ? 2
         : (i == 10 || i == 11) ? -2
         : i == 13 ? 3
         : i == 15 ? -3
                   : 0;
}
__host__ __device__ constexpr int cy17(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1
         : (i == 4 || i == 7 || i == 8) ? -1
         : (i == 9 || i == 10) ? 2
         : (i == 11 || i == 12) ? -2
         : i == 14 ? 3
         : i == 16 ? -3
                   : 0;
}
__host__ __device__ constexpr int shell17(int i) {
  return i == 0 ? 0 : i <= 4 ? 1 : i <= 8 ? 2 : i <= 12 ? 3 : 4;
}

// The quadrature of degree 7: s from 75 v^2 - 125 v + 36 = 0 (v = 1/s), the
// shell weights from the conditions of order 4 and 6.
void lattice17(int cx[17], int cy[17], double w[17], double* s_out) {
  const double s = (125.0 + 5.0 * std::sqrt(193.0)) / 72.0;
  const double v = 1.0 / s, v2 = v * v, v3 = v2 * v;
  const double ws[5] = {0.0, 9.0 * v2 / 8.0 - 0.75 * v3, v2 / 3.0 - 0.25 * v3,
                        (3.0 * v3 - v2) / 192.0, (6.0 * v3 - v2) / 648.0};
  const double w0 = 1.0 - 4.0 * (ws[1] + ws[2] + ws[3] + ws[4]);
  for (int i = 0; i < 17; ++i) {
    if (cx) cx[i] = cx17(i);
    if (cy) cy[i] = cy17(i);
    if (w) w[i] = i == 0 ? w0 : ws[shell17(i)];
  }
  if (s_out) *s_out = s;
}

double rest_weight17(int i, double T) {
  double w[17], s;
  lattice17(nullptr, nullptr, w, &s);
  const double cc = (double)(cx17(i) * cx17(i) + cy17(i) * cy17(i));
  return w[i] * (1.0 + 0.5 * (T - 1.0) * (s * cc - 2.0));
}

// Buffer loads and stores: the population array as one buffer resource, the
// plane and row as a scalar byte offset, the column as a per-lane byte
// offset (no per-lane 64-bit address arithmetic). The host keeps each array
// below 2 GiB, so the offsets never wrap 32 bits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int num_records) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, num_records,
                                           0x00020000);
}
__device__ __forceinline__ float ld(float*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double ld(double*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
// FP64 populations are stored non-temporally (the nt bit): the written planes
// then do not displace the rows the neighbouring chunks still read
// (8192 x 1024: 531 -> 502 us per step); for FP32 it measured slower.
__device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 2);
}

template <typename A>
__device__ __forceinline__ A rcp(A x) { return (A)1 / x; }
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Per-lattice constants in the arithmetic precision, converted on the host
// and passed as a kernel argument, so they stay in scalar registers.
template <typename A>
struct K17 {
  A nbar, T, ps, keep, pre, om, kap, N, M, Q, Rw, Q4R, h1, h2, h3, half;
  A w[5], wr[5], owr[5], a1[5];
};

template <typename A>
static K17<A> make_k17(const Desc17& d) {
  K17<A> k;
  k.nbar = (A)d.nbar;
  k.T = (A)d.T;
  k.ps = (A)d.ps;
  k.keep = (A)(1.0 - d.omega);
  k.pre = (A)(1.0 - 0.5 * d.omega);
  k.om = (A)d.omega;
  k.kap = (A)d.kappa_l;
  k.N = (A)d.N;
  k.M = (A)d.M;
  k.Q = (A)d.Q;
  k.Rw = (A)d.R;
  k.Q4R = (A)(4.0 * (d.Q + d.R));
  k.h1 = (A)d.h1;
  k.h2 = (A)d.h2;
  k.h3 = (A)d.h3;
  k.half = (A)0.5;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    k.w[j] = (A)d.w[j];
    k.wr[j] = (A)d.wr[j];
    k.owr[j] = (A)d.owr[j];
    k.a1[j] = (A)d.a1[j];
  }
  return k;
}

// The 17 values node (x, a) pulls: slot i holds S_i(x - c_i, a - c_y,i).
// ra: the row wrapped into [0, Ly); vcol[c + 3]: byte offset of column
// x - c wrapped; rb, pb: bytes per row and per plane. Ly >= 4, so one
// conditional wrap brings ra - c_y into range.
template <typename S, typename A>
__device__ __forceinline__ void pull17(A (&g)[17], __amdgpu_buffer_rsrc_t src, int ra, int Ly,
                                       uint32_t rb, uint32_t pb, const int (&vcol)[7]) {
  uint32_t ro[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    int r = ra - (k - 3);
    r = r < 0 ? r + Ly : (r >= Ly ? r - Ly : r);
    ro[k] = (uint32_t)r * rb;
  }
#pragma unroll
  for (int i = 0; i < 17; ++i)
    g[i] = (A)ld((S*)nullptr, src, vcol[cx17(i) + 3], (int)(ro[cy17(i) + 3] + (uint32_t)i * pb));
}

// Collision of one node (the file header's sum), in place on the pulled
// deviations g; dn = n - nbar, j = momentum with the half force, F = force.
template <typename A>
__device__ __forceinline__ void collide17(A (&g)[17], const K17<A>& k, A n, A dn, A jx, A jy,
                                          A rn, A Fx, A Fy) {
  const A ux = jx * rn, uy = jy * rn;
  const A om = k.om, p = k.pre;
  const A Bx = om * jx + p * Fx, By = om * jy + p * Fy;
  const A Axx = om * jx * ux + (p + p) * ux * Fx;
  const A Ayy = om * jy * uy + (p + p) * uy * Fy;
  const A Axy = om * jx * uy + p * (ux * Fy + uy * Fx);
  const A pFx = p * Fx, pFy = p * Fy;
  const A Cxxx = (om * jx + (pFx + pFx + pFx)) * ux * ux;
  const A Cyyy = (om * jy + (pFy + pFy + pFy)) * uy * uy;
  const A Cxxy = (om * jx + (pFx + pFx)) * ux * uy + pFy * ux * ux;
  const A Cxyy = (om * jy + (pFy + pFy)) * ux * uy + pFx * uy * uy;
  const A vx = Cxxx + Cxyy, vy = Cxxy + Cyyy;
  const A tr = k.h1 * (Axx + Ayy);
  g[0] = k.keep * g[0] + k.owr[0] * dn - k.w[0] * tr;
#pragma unroll
  for (int i = 1; i < 17; ++i) {
    const int q = (i - 1) & 3;
    if (q >= 2) continue;  // i + 2 is the opposite of i (q = 0, 1)
    const A a = (A)cx17(i), b = (A)cy17(i);
    const int sh = shell17(i);
    const A ev = k.h2 * (a * a * Axx + (a + a) * b * Axy + b * b * Ayy) - tr;
    const A od = k.a1[sh] * (a * Bx + b * By) +
                 k.h3 * (a * a * a * Cxxx + (A)3 * a * a * b * Cxxy + (A)3 * a * b * b * Cxyy +
                         b * b * b * Cyyy) -
                 k.h2 * (a * vx + b * vy);
    const A base = k.owr[sh] * dn + k.w[sh] * ev;
    const A wod = k.w[sh] * od;
    g[i] = k.keep * g[i] + base + wod;
    g[i + 2] = k.keep * g[i + 2] + base - wod;
  }
  (void)n;
}

// One row iteration of the march (stages A, B, C of the file header). K: the
// register slot holding row a's pulled values; row a - 2's are in slot
// (K + 2) & 3, and row a + 1's are loaded into slot (K + 1) & 3.
template <typename S, typename A, int NT, int K, bool SR>
__device__ __forceinline__ void iter17(
    int it, int nit, int dir, int a, int q, const Desc17& d, const K17<A>& k, A (&g)[4][17],
    A (&mx)[4], A (&my)[4], A (&nR)[3][NT], A (&PR)[3][NT], A (&LR)[3][NT],
    __amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst, uint32_t rb, uint32_t pb,
    const int (&vcol)[7], int voff_own, bool own, A shift, A fx, int flags, double* mom,
    int xs, uint32_t rstep) {
  const int t = threadIdx.x;
  const int Ly = d.Ly;
  // A: row a
  {
    A (&v)[17] = g[K];
    if (flags & kApplyShift) {
#pragma unroll
      for (int i = 0; i < 17; ++i) v[i] += k.wr[shell17(i)] * shift;
    }
    A s0 = v[0], sx = (A)0, sy = (A)0;
#pragma unroll
    for (int i = 1; i < 17; ++i) {
      s0 += v[i];
      if (cx17(i)) sx += (A)cx17(i) * v[i];
      if (cy17(i)) sy += (A)cy17(i) * v[i];
    }
    nR[q][t] = s0;
    mx[K] = sx;
    my[K] = sy;
  }
  if (it + 1 < nit) {
    int ra = a + dir;
    ra = ra < 0 ? ra + Ly : (ra >= Ly ? ra - Ly : ra);
    pull17<S, A>(g[(K + 1) & 3], src, ra, Ly, rb, pb, vcol);
  }
  const int q1 = q == 0 ? 2 : q - 1;  // row a - dir
  const int q2 = q == 2 ? 0 : q + 1;  // row a - 2 dir (and a + dir)
  __syncthreads();
  // B: row a - dir
  if (it >= 2 && t >= 1 && t <= NT - 2) {
    const A c = nR[q1][t];
    // grouped by rows, so a march in the other direction rounds the same
    const A L = k.Q * ((nR[q1][t + 1] + nR[q1][t - 1]) + (nR[q][t] + nR[q2][t])) +
                k.Rw * ((nR[q][t + 1] + nR[q][t - 1]) + (nR[q2][t + 1] + nR[q2][t - 1])) -
                k.Q4R * c;
    const A n = k.nbar + c;
    LR[q1][t] = L;
    PR[q1][t] = n * n * ((A)1.125 - k.T * rcp((A)3 - n)) * k.ps;
  }
  __syncthreads();
  // C: row r = a - 2 dir; B's rows r - dir, r, r + dir are in slots q, q2, q1
  // (the y differences are taken along the march and carry its sign; every
  // sum over the two neighbour rows is grouped by row, so both march
  // directions round the same)
  if (it >= 4 && t >= 2 && t <= NT - 3) {
    const int r = a - 2 * dir;
    const A dn = nR[q2][t];
    const A n = k.nbar + dn;
    const A sy = (A)dir;
    const A gPx = k.N * (PR[q2][t + 1] - PR[q2][t - 1]) +
                  k.M * ((PR[q1][t + 1] - PR[q1][t - 1]) + (PR[q][t + 1] - PR[q][t - 1]));
    const A gPy = sy * (k.N * (PR[q1][t] - PR[q][t]) +
                        k.M * ((PR[q1][t + 1] - PR[q][t + 1]) + (PR[q1][t - 1] - PR[q][t - 1])));
    const A gLx = k.N * (LR[q2][t + 1] - LR[q2][t - 1]) +
                  k.M * ((LR[q1][t + 1] - LR[q1][t - 1]) + (LR[q][t + 1] - LR[q][t - 1]));
    const A gLy = sy * (k.N * (LR[q1][t] - LR[q][t]) +
                        k.M * ((LR[q1][t + 1] - LR[q][t + 1]) + (LR[q1][t - 1] - LR[q][t - 1])));
    const A Fx = gPx + k.kap * n * gLx + fx;
    const A Fy = gPy + k.kap * n * gLy;
    constexpr int KC = (K + 2) & 3;
    const A jx = mx[KC] + k.half * Fx, jy = my[KC] + k.half * Fy;
    const A rn = rcp(n);
    collide17<A>(g[KC], k, n, dn, jx, jy, rn, Fx, Fy);
    if (own) {
      const uint32_t ro = (uint32_t)r * rb;
      if constexpr (SR) {
        // 17 draws of 14 bits from two hashes of (column, row, step, 0 | 1)
        uint32_t q[18];
        lbrng::draws14(lbrng::pcg4d(lbrng::U4{(uint32_t)xs, (uint32_t)r, rstep, 0u}), q);
        lbrng::draws14(lbrng::pcg4d(lbrng::U4{(uint32_t)xs, (uint32_t)r, rstep, 1u}), q + 9);
#pragma unroll
        for (int i = 0; i < 17; ++i)
          st(lbrng::round_stochastic((double)g[KC][i], q[i]), dst, voff_own,
             (int)(ro + (uint32_t)i * pb));
      } else {
#pragma unroll
        for (int i = 0; i < 17; ++i) st((S)g[KC][i], dst, voff_own, (int)(ro + (uint32_t)i * pb));
      }
      if (flags & kWriteMoments) {
        const int64_t o = (int64_t)r * d.Lx + xs;
        const int64_t nn = (int64_t)d.Lx * Ly;
        mom[o] = (double)n;
        mom[nn + o] = (double)(jx * rn);
        mom[2 * nn + o] = (double)(jy * rn);
      }
    }
  }
}

template <typename S, typename A, int NT, bool SR>
__global__ __launch_bounds__(NT) void step17_kernel(Desc17 d, K17<A> k, int parity, int rows,
                                                    int chunks, int flags, double* mom,
                                                    uint32_t rstep) {
  __shared__ A nR[3][NT];
  __shared__ A PR[3][NT];
  __shared__ A LR[3][NT];
  const int t = threadIdx.x;
  const int Lx = d.Lx, Ly = d.Ly;
  // Workgroups are dealt round-robin over the 8 XCDs; each XCD takes a
  // contiguous run of tiles in row-of-chunks order (all strips of a chunk row,
  // then the next chunk row), so neighbouring strips, which share the cache
  // lines at their edges, run together on one XCD; odd chunks march
  // downwards, so the rows two neighbouring chunks both read are read at
  // about the same time.
  const int nb = gridDim.x, b = blockIdx.x;
  const int qb = nb >> 3, rm = nb & 7, xcd = b & 7;
  const int tile = xcd * qb + (xcd < rm ? xcd : rm) + (b >> 3);
  const int strips = nb / chunks;
  const int chunk = tile / strips, strip = tile - chunk * strips;
  const int x0 = strip * (NT - 4);
  const int y0 = chunk * rows;
  const int y1 = min(y0 + rows, Ly);
  const int dir = (chunk & 1) ? -1 : 1;
  const int xu = x0 - 2 + t;  // unwrapped column
  int xs = xu % Lx;
  if (xs < 0) xs += Lx;
  int vcol[7];
#pragma unroll
  for (int c = -3; c <= 3; ++c) {
    int v = (xs - c) % Lx;
    if (v < 0) v += Lx;
    vcol[c + 3] = v * (int)sizeof(S);
  }
  const bool own = t >= 2 && t <= NT - 3 && xu < Lx;
  const uint32_t pb = (uint32_t)Lx * sizeof(S), rb = 17u * pb;
  const int nbytes = (int)(rb * (uint32_t)Ly);
  const __amdgpu_buffer_rsrc_t src = rsrc(d.S[parity], nbytes);
  const __amdgpu_buffer_rsrc_t dst = rsrc(d.S[parity ^ 1], nbytes);
  const A fx = (A)d.fext[xs];
  const A shift = (flags & kApplyShift) ? (A)*d.shift : (A)0;

  A g[4][17];
  A mx[4], my[4];
  // rows y0 - 2 .. y1 + 1 in the march direction
  const int nit = y1 - y0 + 4;
  const int ab = dir > 0 ? y0 - 2 : y1 + 1;
  {
    const int ra = ab < 0 ? ab + Ly : (ab >= Ly ? ab - Ly : ab);
    pull17<S, A>(g[0], src, ra, Ly, rb, pb, vcol);
  }
  int q = 0;  // LDS ring slot of row a: it mod 3
  for (int it = 0; it < nit; it += 4) {
    const int a = ab + dir * it;
    iter17<S, A, NT, 0, SR>(it, nit, dir, a, q, d, k, g, mx, my, nR, PR, LR, src, dst, rb, pb, vcol,
                        vcol[3], own, shift, fx, flags, mom, xs, rstep);
    q = q == 2 ? 0 : q + 1;
    if (it + 1 >= nit) break;
    iter17<S, A, NT, 1, SR>(it + 1, nit, dir, a + dir, q, d, k, g, mx, my, nR, PR, LR, src, dst, rb,
                        pb, vcol, vcol[3], own, shift, fx, flags, mom, xs, rstep);
    q = q == 2 ? 0 : q + 1;
    if (it + 2 >= nit) break;
    iter17<S, A, NT, 2, SR>(it + 2, nit, dir, a + 2 * dir, q, d, k, g, mx, my, nR, PR, LR, src, dst,
                        rb, pb, vcol, vcol[3], own, shift, fx, flags, mom, xs, rstep);
    q = q == 2 ? 0 : q + 1;
    if (it + 3 >= nit) break;
    iter17<S, A, NT, 3, SR>(it + 3, nit, dir, a + 3 * dir, q, d, k, g, mx, my, nR, PR, LR, src, dst,
                        rb, pb, vcol, vcol[3], own, shift, fx, flags, mom, xs, rstep);
    q = q == 2 ? 0 : q + 1;
  }
}

template <typename S, typename A, bool SR>
static hipError_t launch_t(int threads, int rows, const Desc17& d, int parity, int flags,
                           double* mom, uint32_t rstep, hipStream_t st) {
  const int64_t strips = (d.Lx + threads - 5) / (threads - 4);
  const int64_t chunks = (d.Ly + rows - 1) / rows;
  if (strips * chunks > INT32_MAX) return hipErrorInvalidValue;
  const int grid = (int)(strips * chunks);
  const K17<A> k = make_k17<A>(d);
  switch (threads) {
    case 64:
      step17_kernel<S, A, 64, SR>
          <<<grid, 64, 0, st>>>(d, k, parity, rows, (int)chunks, flags, mom, rstep);
      break;
    case 128:
      step17_kernel<S, A, 128, SR>
          <<<grid, 128, 0, st>>>(d, k, parity, rows, (int)chunks, flags, mom, rstep);
      break;
    case 256:
      step17_kernel<S, A, 256, SR>
          <<<grid, 256, 0, st>>>(d, k, parity, rows, (int)chunks, flags, mom, rstep);
      break;
    case 512:
      step17_kernel<S, A, 512, SR>
          <<<grid, 512, 0, st>>>(d, k, parity, rows, (int)chunks, flags, mom, rstep);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step17(int prec, int threads, int rows, const Desc17& d, int parity, int flags,
                         double* mom, uint32_t rstep, hipStream_t st) {
  if (rows < 1) return hipErrorInvalidValue;
  switch (prec) {
    case 0:
      return launch_t<double, double, false>(threads, rows, d, parity, flags, mom, rstep, st);
    case 1:
      return launch_t<float, float, false>(threads, rows, d, parity, flags, mom, rstep, st);
    case 2:
      return launch_t<float, double, true>(threads, rows, d, parity, flags, mom, rstep, st);
    default:
      return hipErrorInvalidValue;
  }
}

// ---- initial state, checks, population transfer ---------------------------

template <typename S>
__global__ void init17_kernel(Desc17 d, int parity, const double* n0, const double* ux0,
                              const double* uy0) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(k / d.Lx), x = (int)(k - (int64_t)y * d.Lx);
    const double n = n0[k];
    const double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
    const double uu = ux * ux + uy * uy;
    S* out = (S*)d.S[parity] + (int64_t)y * 17 * d.Lx + x;
#pragma unroll
    for (int i = 0; i < 17; ++i) {
      const int sh = shell17(i);
      const double cu = cx17(i) * ux + cy17(i) * uy;
      const double E = d.a1[sh] * cu + d.h2 * cu * cu - d.h1 * uu + d.h3 * cu * cu * cu -
                       d.h2 * cu * uu;
      const double f = d.wr[sh] * n + d.w[sh] * n * E;
      out[(int64_t)i * d.Lx] = (S)(f - d.wr[sh] * d.nbar);
    }
  }
}

hipError_t launch_init17(bool fp32, const Desc17& d, int parity, const double* n0,
                         const double* ux, const double* uy, hipStream_t st) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const int blocks = (int)std::min<int64_t>((nn + 255) / 256, 4096);
  if (fp32)
    init17_kernel<float><<<blocks, 256, 0, st>>>(d, parity, n0, ux, uy);
  else
    init17_kernel<double><<<blocks, 256, 0, st>>>(d, parity, n0, ux, uy);
  return hipGetLastError();
}

int reduce17_blocks(int64_t nn) { return (int)std::min<int64_t>((nn + 1023) / 1024, 1024); }

// Per-block FP64 partials: mass, jx, jy, min n, max n, non-finite nodes, in
// a fixed order for a given grid.
template <typename S>
__global__ __launch_bounds__(256) void reduce17_kernel(Desc17 d, int parity, double* part,
                                                       int add_shift) {
  __shared__ double sm[6][256];
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const double sh = add_shift ? *d.shift : 0.0;
  double m = 0.0, jx = 0.0, jy = 0.0, lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < nn; k += (int64_t)gridDim.x * 256) {
    const int y = (int)(k / d.Lx), x = (int)(k - (int64_t)y * d.Lx);
    const S* row = (const S*)d.S[parity] + (int64_t)y * 17 * d.Lx + x;
    double n = d.nbar + sh, px = 0.0, py = 0.0;
#pragma unroll
    for (int i = 0; i < 17; ++i) {
      const double v = (double)row[(int64_t)i * d.Lx];
      n += v;
      px += cx17(i) * v;
      py += cy17(i) * v;
    }
    if (!std::isfinite(n) || !std::isfinite(px) || !std::isfinite(py)) {
      bad += 1.0;
      continue;
    }
    m += n;
    jx += px;
    jy += py;
    lo = fmin(lo, n);
    hi = fmax(hi, n);
  }
  const int t = threadIdx.x;
  sm[0][t] = m;
  sm[1][t] = jx;
  sm[2][t] = jy;
  sm[3][t] = lo;
  sm[4][t] = hi;
  sm[5][t] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sm[0][t] += sm[0][t + w];
      sm[1][t] += sm[1][t + w];
      sm[2][t] += sm[2][t + w];
      sm[3][t] = fmin(sm[3][t], sm[3][t + w]);
      sm[4][t] = fmax(sm[4][t], sm[4][t + w]);
      sm[5][t] += sm[5][t + w];
    }
    __syncthreads();
  }
  if (t < 6) part[blockIdx.x * 6 + t] = sm[t][0];
}

hipError_t launch_reduce17(bool fp32, const Desc17& d, int parity, double* part, int add_shift,
                           hipStream_t st) {
  const int nb = reduce17_blocks((int64_t)d.Lx * d.Ly);
  if (fp32)
    reduce17_kernel<float><<<nb, 256, 0, st>>>(d, parity, part, add_shift);
  else
    reduce17_kernel<double><<<nb, 256, 0, st>>>(d, parity, part, add_shift);
  return hipGetLastError();
}

__global__ void reduce17_final_kernel(const double* part, int nb, int64_t nn, Reduce17* out,
                                      int mode, int drift) {
  if (threadIdx.x != 0) return;
  double m = 0.0, jx = 0.0, jy = 0.0, lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    m += part[b * 6 + 0];
    jx += part[b * 6 + 1];
    jy += part[b * 6 + 2];
    lo = fmin(lo, part[b * 6 + 3]);
    hi = fmax(hi, part[b * 6 + 4]);
    bad += part[b * 6 + 5];
  }
  out->mass = m;
  out->jx = jx;
  out->jy = jy;
  out->nmin = lo;
  out->nmax = hi;
  out->nonfinite = bad;
  if (mode == 1) {
    out->mass_ref = m;
    out->has_ref = 1u;
    out->shift = 0.0;
    out->status = 0u;
    return;
  }
  if (mode == 0) {
    const bool fail = bad > 0.0 || !(lo > 0.0) || !(hi < 3.0);
    if (fail) out->status |= 1u;
    out->shift = (drift && out->has_ref && !fail) ? (out->mass_ref - m) / (double)nn : 0.0;
  }
}

hipError_t launch_reduce17_final(const double* part, int nb, int64_t nn, Reduce17* out, int mode,
                                 int drift, hipStream_t st) {
  reduce17_final_kernel<<<1, 64, 0, st>>>(part, nb, nn, out, mode, drift);
  return hipGetLastError();
}

template <typename S>
__global__ void get_pops17_kernel(Desc17 d, int parity, int plane, double* f, int add_shift) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const double base = d.wr[shell17(plane)] * (d.nbar + (add_shift ? *d.shift : 0.0));
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(k / d.Lx), x = (int)(k - (int64_t)y * d.Lx);
    f[k] = (double)((const S*)d.S[parity])[((int64_t)y * 17 + plane) * d.Lx + x] + base;
  }
}

template <typename S>
__global__ void set_pops17_kernel(Desc17 d, int parity, int plane, const double* f) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const double base = d.wr[shell17(plane)] * d.nbar;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(k / d.Lx), x = (int)(k - (int64_t)y * d.Lx);
    ((S*)d.S[parity])[((int64_t)y * 17 + plane) * d.Lx + x] = (S)(f[k] - base);
  }
}

hipError_t launch_get_pops17(bool fp32, const Desc17& d, int parity, int plane, double* f,
                             int add_shift, hipStream_t st) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const int blocks = (int)std::min<int64_t>((nn + 255) / 256, 4096);
  if (fp32)
    get_pops17_kernel<float><<<blocks, 256, 0, st>>>(d, parity, plane, f, add_shift);
  else
    get_pops17_kernel<double><<<blocks, 256, 0, st>>>(d, parity, plane, f, add_shift);
  return hipGetLastError();
}

hipError_t launch_set_pops17(bool fp32, const Desc17& d, int parity, int plane, const double* f,
                             hipStream_t st) {
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const int blocks = (int)std::min<int64_t>((nn + 255) / 256, 4096);
  if (fp32)
    set_pops17_kernel<float><<<blocks, 256, 0, st>>>(d, parity, plane, f);
  else
    set_pops17_kernel<double><<<blocks, 256, 0, st>>>(d, parity, plane, f);
  return hipGetLastError();
}

}  // namespace d17k
