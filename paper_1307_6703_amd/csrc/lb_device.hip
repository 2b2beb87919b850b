// Device code: the fused lattice Boltzmann step for a van der Waals fluid
// (Coclite, Gonnella, Lamura, arXiv:1307.6703, Sec. II) for gfx950, one step
// per launch (step_kernel) or two with the intermediate populations kept on
// chip (step2_kernel), plus the initial-state, reduction and
// population-conversion kernels.
//
// Lattice units throughout (dx = dt = 1, c_i in {0,+-1}^2); the host converts
// the paper's tau and kappa. Populations are stored as g_i = f_i - w^_i nbar,
// where w^_i = w_i [1 + (T-1)(3|c_i|^2-2)/2] are the rest-state weights; nbar
// is 0 in FP64 mode (g = f) and the mean density in FP32 mode, so the stored
// values are small deviations that keep FP32 resolution.
//
// Three precisions: FP64 storage and arithmetic; FP32 storage and
// arithmetic; FP32 storage with FP64 arithmetic, where each stored value is
// rounded stochastically (up or down with the probabilities that make the
// expected stored value the exact one). Rounding to nearest repeats the same
// error every step once a pattern is steady, and the lattice integrates that
// bias over the relaxation time of its slowest modes; unbiased rounding turns
// it into noise that does not accumulate.
//
// Step kernel design. A workgroup of NT threads owns a strip of NT-6 columns
// and a chunk of rows; thread t works on column x0-3+t. It marches along y:
// each iteration loads one new row (9 coalesced pulls per node) and moves four
// pipeline stages forward by one row:
//   A (row a):   pull streaming, density n (n-hat at walls), raw momentum;
//   B (row a-1): Laplacian of n and the pressure term p^i - p^w;
//   C (row a-2): force F and momentum j* = sum f c + F/2 (wall value at walls);
//   D (row a-3): grad n and div(j*), wall rule, equilibrium, forcing, BGK
//                collision, store.
// n, L, P, j* live in small LDS rings (radius-1 stencils on each stage give
// the radius-3 dependence of the step); the pulled populations and F wait
// in register rings. Ghost rows beyond the walls mirror the field (neutral
// wetting): scalars and x-components even, y-components odd.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lb_internal.h"

namespace lbk {

// D2Q9 in the order 0 rest, E, N, W, S, NE, NW, SW, SE (Sec. II).
__host__ __device__ constexpr int cx(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : i == 1 ? 3 : i == 2 ? 4 : i == 3 ? 1 : i == 4 ? 2 : i == 5 ? 7 : i == 6 ? 8 : i == 7 ? 5 : 6;
}

// Rest-state weights w^_i = w_i [1 + (T-1)(3|c_i|^2 - 2)/2]: the equilibrium
// of Eq.(eqfunc) at u = 0 is w^_i n.
__host__ __device__ inline double rest_weight_hd(int i, double T) {
  if (i == 0) return 4.0 / 9.0 * (2.0 - T);
  if (i <= 4) return (T + 1.0) / 18.0;
  return (2.0 * T - 1.0) / 36.0;
}

double rest_weight(int i, double T) { return rest_weight_hd(i, T); }

// Populations are stored row-interleaved: the nine planes of one lattice row
// are adjacent, S[(9 y + i) Lx + x]. Index of population i at node k = y Lx + x.
__device__ __forceinline__ int64_t pidx(int i, int64_t k, int64_t y, int Lx) {
  return k + (8 * y + i) * (int64_t)Lx;
}

// Per-lattice constants of the stages in the storage precision. The y
// stencils are taken along the march ("ahead" minus "behind"); Ny and My
// carry the march direction's sign, so the results are d/dy.
template <typename R>
struct Sten {
  R nbar, T, kap3, third, N, M, Q, Rw, Q4R, Ny, My, Ub, Ut;
};

template <typename R>
__device__ __forceinline__ Sten<R> make_sten(const Desc& d, int dir) {
  Sten<R> c;
  c.nbar = (R)d.nbar;
  c.T = (R)d.T;
  c.kap3 = (R)d.kappa3;
  c.third = (R)(1.0 / 3.0);
  c.N = (R)d.N;
  c.M = (R)d.M;
  c.Q = (R)d.Q;
  c.Rw = (R)d.R;
  c.Q4R = (R)(4.0 * (d.Q + d.R));
  c.Ny = (R)(dir * d.N);
  c.My = (R)(dir * d.M);
  c.Ub = (R)(-d.U);
  c.Ut = (R)d.U;
  return c;
}

// Equilibrium (Eq.(eqfunc)) and forcing (Eq.(forceterm), Eq.(coeff)) in
// lattice units, followed by BGK relaxation (Eq.(evoleq)), on deviations:
//   g_i <- (1 - omega) g_i + omega geq_i + F_i,
//   geq_i = w^_i dn + w_i n [3 c.u + 9/2 (c.u)^2 - 3/2 u^2],
//   F_i   = w_i s [3 c.F + X:(3 c c - I)/2],  s = 1 - omega/2,
//   X = 3 (u F + F u) + (1 - T)(u grad n + grad n u + D I).
// Both are expansions in the same Hermite polynomials, so omega geq_i + F_i
// = omega w^_i dn + w_i [3 B.c_i + 9/2 A:(c_i c_i - I/3)] with
//   B = omega j + s F,   A = omega n u u + (s/3) X,
// j = n u. Per direction pair the even part comes from A (and dn), the odd
// part from B.
template <typename R>
struct Coll {
  R keep, om, s;             // 1 - omega, omega, s
  R k1, k2, k3;              // 2 s, 2 s (1 - T)/3, s (1 - T)/3
  R owr0, owra, owrd;        // omega w^_i
  R w0t15, wa3, wa15, wd3, wd9;  // 3/2 w_0, 3 w_a, 3/2 w_a, 3 w_d, 9 w_d
};

template <typename R>
__device__ __forceinline__ Coll<R> make_coll(const Desc& d) {
  Coll<R> c;
  const double om = d.omega, s = 1.0 - 0.5 * d.omega, oneT = 1.0 - d.T;
  c.keep = (R)(1.0 - om);
  c.om = (R)om;
  c.s = (R)s;
  c.k1 = (R)(2.0 * s);
  c.k2 = (R)(2.0 / 3.0 * s * oneT);
  c.k3 = (R)(s / 3.0 * oneT);
  c.owr0 = (R)(om * rest_weight_hd(0, d.T));
  c.owra = (R)(om * rest_weight_hd(1, d.T));
  c.owrd = (R)(om * rest_weight_hd(5, d.T));
  c.w0t15 = (R)(1.5 * 4.0 / 9.0);
  c.wa3 = (R)(3.0 / 9.0);
  c.wa15 = (R)(1.5 / 9.0);
  c.wd3 = (R)(3.0 / 36.0);
  c.wd9 = (R)(9.0 / 36.0);
  return c;
}

// A_xx = u_x (omega n u_x + 2 s F_x + 2 s (1-T)/3 dn_x) + s (1-T)/3 D, and
// so on; the even part of direction i is w_i [9/2 A:c c - 3/2 tr A].
template <typename R>
__device__ __forceinline__ void collide(R g[9], const Coll<R>& c, R n, R dn, R jx, R jy, R rn,
                                        R Fx, R Fy, R dnx, R dny, R D) {
  const R ux = jx * rn, uy = jy * rn;
  const R on = c.om * n;
  const R Axx = ux * (on * ux + c.k1 * Fx + c.k2 * dnx) + c.k3 * D;
  const R Ayy = uy * (on * uy + c.k1 * Fy + c.k2 * dny) + c.k3 * D;
  const R Axy = ux * (on * uy + c.s * Fy + c.k3 * dny) + uy * (c.s * Fx + c.k3 * dnx);
  const R Bx = c.om * jx + c.s * Fx, By = c.om * jy + c.s * Fy;
  const R tr = Axx + Ayy;
  const R da = c.owra * dn, dd = c.owrd * dn;
  g[0] = c.keep * g[0] + (c.owr0 * dn - c.w0t15 * tr);
  {
    const R es = da + c.wa3 * Axx - c.wa15 * Ayy, ea = c.wa3 * Bx;
    g[1] = c.keep * g[1] + (es + ea);
    g[3] = c.keep * g[3] + (es - ea);
  }
  {
    const R es = da + c.wa3 * Ayy - c.wa15 * Axx, ea = c.wa3 * By;
    g[2] = c.keep * g[2] + (es + ea);
    g[4] = c.keep * g[4] + (es - ea);
  }
  {
    const R t = dd + c.wd3 * tr, x = c.wd9 * Axy;
    const R e5 = t + x, e6 = t - x;
    const R a5 = c.wd3 * (Bx + By), a6 = c.wd3 * (By - Bx);
    g[5] = c.keep * g[5] + (e5 + a5);
    g[7] = c.keep * g[7] + (e5 - a5);
    g[6] = c.keep * g[6] + (e6 + a6);
    g[8] = c.keep * g[8] + (e6 - a6);
  }
}

// Row index of the lattice a pipeline row maps to, and the parity applied
// to y-components there (mirror about the wall nodes, or periodic wrap).
struct RowMap {
  int phys;   // physical row
  int wall;   // 0 bulk, 1 lower wall (row 0), 2 upper wall (row Ly-1)
  int ysgn;   // +1, or -1 on a mirrored ghost row
};

__device__ __forceinline__ RowMap map_row(int a, int Ly, int periodic) {
  RowMap m;
  m.ysgn = 1;
  if (periodic) {
    int r = a % Ly;
    m.phys = r < 0 ? r + Ly : r;
    m.wall = 0;
  } else {
    int r = a;
    if (r < 0) { r = -r; m.ysgn = -1; }
    else if (r > Ly - 1) { r = 2 * (Ly - 1) - r; m.ysgn = -1; }
    m.phys = r;
    m.wall = (r == 0) ? 1 : (r == Ly - 1 ? 2 : 0);
  }
  return m;
}

// Buffer loads and stores: one buffer resource per population array
// (uniform); the plane and row as a scalar byte offset and the column as a
// per-lane byte offset, so no per-lane 64-bit address arithmetic is needed.
// The hardware range check compares scalar + lane offset with num_records
// (the array's size): a lane that must not touch memory uses a lane offset
// equal to num_records, a row that must not touch memory uses a resource
// with num_records = 0, and the hardware drops the store / returns 0. The
// host keeps every array below 2 GiB, so the two offsets never wrap 32 bits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int num_records) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, num_records,
                                           0x00020000);
}
__device__ __forceinline__ float buf_ld(float*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_ld(double*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 0);
}

template <typename R>
__device__ __forceinline__ R fast_rcp(R x) { return (R)1 / x; }
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Values the stages pass to each other through LDS.
template <typename R>
struct Pair {
  R x, y;
};

template <typename R>
struct Mom {
  R jx, jy;
};

template <typename R>
struct Quad {
  R jx, jy, Fx, Fy;
};

// Pull the nine values a node of physical row `m.phys` needs (Eq.(evoleq)):
// slot i holds S_i(x - c_i). At a wall node the three slots whose source lies
// outside the lattice hold instead the node's own post-collision populations
// that would leave it (lower wall: S4, S7, S8 in slots 2, 5, 6; upper wall:
// S2, S5, S6 in slots 4, 7, 8), so that the sum of the slots is n-hat.
// Row map for loads: full reflection for rows beyond the tile's ghost range
// (rows that are loaded but never stored), so every row index maps into the
// lattice.
__device__ __forceinline__ RowMap map_row_any(int a, int Ly, int periodic) {
  if (periodic || (a >= -3 && a <= Ly + 2)) return map_row(a, Ly, periodic);
  RowMap m;
  const int P = 2 * (Ly - 1);
  int r = a % P;
  if (r < 0) r += P;
  m.ysgn = 1;
  if (r > Ly - 1) r = P - r;
  m.phys = r;
  m.wall = (r == 0) ? 1 : (r == Ly - 1 ? 2 : 0);
  return m;
}

template <typename R>
__device__ __forceinline__ void pull_row(R v[9], __amdgpu_buffer_rsrc_t S, uint32_t pbytes,
                                         uint32_t rb, int Ly, int periodic, const RowMap& m, int vc,
                                         int vm, int vp) {
  // source rows y - c_y (wrapped when periodic); at a wall node the slots
  // whose source lies outside take the node's own outgoing populations
  int rs = m.phys - 1, rn = m.phys + 1;
  if (periodic) {
    rs = rs < 0 ? rs + Ly : rs;
    rn = rn >= Ly ? rn - Ly : rn;
  }
  const bool lo = m.wall == 1, hi = m.wall == 2;
  const uint32_t o_s = (uint32_t)(lo ? m.phys : rs) * rb;  // row of c_y = +1 sources
  const uint32_t o_0 = (uint32_t)m.phys * rb;
  const uint32_t o_n = (uint32_t)(hi ? m.phys : rn) * rb;  // row of c_y = -1 sources
  // lower wall: slots 2, 5, 6 read own S4, S7, S8; upper: 4, 7, 8 read own S2, S5, S6
  const int v5 = lo ? vc : vm, v6 = lo ? vc : vp, v7 = hi ? vc : vp, v8 = hi ? vc : vm;
  const uint32_t p2 = lo ? 4u : 2u, p5 = lo ? 7u : 5u, p6 = lo ? 8u : 6u;
  const uint32_t p4 = hi ? 2u : 4u, p7 = hi ? 5u : 7u, p8 = hi ? 6u : 8u;
  v[0] = buf_ld((R*)nullptr, S, vc, (int)(0u * pbytes + o_0));
  v[1] = buf_ld((R*)nullptr, S, vm, (int)(1u * pbytes + o_0));
  v[2] = buf_ld((R*)nullptr, S, vc, (int)(p2 * pbytes + o_s));
  v[3] = buf_ld((R*)nullptr, S, vp, (int)(3u * pbytes + o_0));
  v[4] = buf_ld((R*)nullptr, S, vc, (int)(p4 * pbytes + o_n));
  v[5] = buf_ld((R*)nullptr, S, v5, (int)(p5 * pbytes + o_s));
  v[6] = buf_ld((R*)nullptr, S, v6, (int)(p6 * pbytes + o_s));
  v[7] = buf_ld((R*)nullptr, S, v7, (int)(p7 * pbytes + o_n));
  v[8] = buf_ld((R*)nullptr, S, v8, (int)(p8 * pbytes + o_n));
}

// ---- stage arithmetic, shared by the one-step and two-step kernels --------

// Stage B at one node: the Laplacian of n (Eq.(laplstencil)) and the pressure
// term p^i - p^w = n T - 3 n T / (3 - n) + 9 n^2 / 8 = n^2 (9/8 - T / (3 - n))
// (Eq.(eqstate)), from the density deviations of the rows behind the node
// (nb), at it (n0) and ahead of it (na) in the march.
template <typename R>
__device__ __forceinline__ Pair<R> stage_lp(const R* nb, const R* n0, const R* na, int u,
                                            const Sten<R>& c) {
  const R dn = n0[u];
  const R L = c.Q * ((n0[u + 1] + n0[u - 1]) + (na[u] + nb[u])) +
              c.Rw * ((na[u + 1] + na[u - 1]) + (nb[u + 1] + nb[u - 1])) - c.Q4R * dn;
  const R n = c.nbar + dn;
  const R P = n * n * ((R)1.125 - c.T * fast_rcp<R>((R)3 - n));
  return Pair<R>{L, P};
}

// Stage C force at one node in lattice units (Eq.(force2), Eq.(periodicforce)):
// F = [grad(p^i - p^w) + kappa n grad(Laplacian n) + F_ext] / 3, from the
// (Laplacian, pressure term) rows behind (Bk), at (Md) and ahead (Ah). The
// gradient stencil (Eq.(xstencil)): d/dx = N (E - W) + M (d1 + d2),
// d/dy = dir [N (A - B) + M (d1 - d2)], d1 = AE - BW, d2 = BE - AW.
template <typename R>
__device__ __forceinline__ void stage_force(const Pair<R>* Bk, const Pair<R>* Md,
                                            const Pair<R>* Ah, int u, R n, R fx3,
                                            const Sten<R>& c, R& Fx, R& Fy) {
  const Pair<R> aE = Ah[u + 1], aW = Ah[u - 1], aC = Ah[u];
  const Pair<R> bE = Bk[u + 1], bW = Bk[u - 1], bC = Bk[u];
  const Pair<R> mE = Md[u + 1], mW = Md[u - 1];
  const R Ld1 = aE.x - bW.x, Ld2 = bE.x - aW.x;
  const R Pd1 = aE.y - bW.y, Pd2 = bE.y - aW.y;
  const R gLx = c.N * (mE.x - mW.x) + c.M * (Ld1 + Ld2);
  const R gLy = c.Ny * (aC.x - bC.x) + c.My * (Ld1 - Ld2);
  const R gPx = c.N * (mE.y - mW.y) + c.M * (Pd1 + Pd2);
  const R gPy = c.Ny * (aC.y - bC.y) + c.My * (Pd1 - Pd2);
  const R kn = c.kap3 * n;
  Fx = c.third * gPx + kn * gLx + fx3;
  Fy = c.third * gPy + kn * gLy;
}

// Stage C momentum j* = sum_i f_i c_i + F/2 (Eq.(newvel)) of the pulled
// populations v of a node; a wall node carries the wall's momentum n U.
// ysgn = -1 on a mirrored ghost row (y-components odd).
template <typename R>
__device__ __forceinline__ void stage_mom(const R v[9], int wall, int ysgn, R n, R Fx, R Fy,
                                          const Sten<R>& c, R& jx, R& jy) {
  const R px = (v[1] - v[3]) + (v[5] - v[6]) + (v[8] - v[7]);
  R py = (v[2] - v[4]) + (v[5] - v[8]) + (v[6] - v[7]);
  if (ysgn < 0) py = -py;
  // selects, not branches: wall is uniform, both values are cheap
  jx = wall ? n * (wall == 1 ? c.Ub : c.Ut) : px + (R)0.5 * Fx;
  jy = wall ? (R)0 : py + (R)0.5 * Fy;
}

// Stage D gradients (Eq.(coeff)): grad n and D = d/dx j*_x + d/dy j*_y, from
// the density rows behind / at / ahead of the node and the j* rows behind (Jb),
// at (J0) and ahead (Ja). sb and sa multiply the y-components read from Jb and
// Ja: -1 where that row stands for the mirror image of the other across a
// wall, else 1.
template <typename R, typename J>
__device__ __forceinline__ void stage_grad(const R* nb, const R* n0, const R* na, const J* Jb,
                                           const J* J0, const J* Ja, int u, R sb, R sa,
                                           const Sten<R>& c, R& dnx, R& dny, R& D) {
  const R nd1 = na[u + 1] - nb[u - 1], nd2 = nb[u + 1] - na[u - 1];
  dnx = c.N * (n0[u + 1] - n0[u - 1]) + c.M * (nd1 + nd2);
  dny = c.Ny * (na[u] - nb[u]) + c.My * (nd1 - nd2);
  // the y-derivative of j*_y as sa Ta - sb Tb: the rows ahead and behind
  // each carry their mirror sign once
  const R Ta = c.Ny * Ja[u].jy + c.My * (Ja[u + 1].jy + Ja[u - 1].jy);
  const R Tb = c.Ny * Jb[u].jy + c.My * (Jb[u + 1].jy + Jb[u - 1].jy);
  const R mEx = J0[u + 1].jx, mWx = J0[u - 1].jx;
  D = c.N * (mEx - mWx) + c.M * ((Ja[u + 1].jx - Ja[u - 1].jx) + (Jb[u + 1].jx - Jb[u - 1].jx)) +
      (sa * Ta - sb * Tb);
}

// Moving-wall rule (Sec. II) for the populations of a wall node whose source
// lies outside the lattice: lower wall (wall 1, speed Ub) as printed, upper
// wall (2, speed Ut) by mirror.
template <typename R>
__device__ __forceinline__ void stage_wall(R g[9], int wall, R dn, R n, R Fx, R Fy,
                                           const Sten<R>& c) {
  if (wall == 1) {
    const R h = (R)0.5 * (g[1] - g[3]);
    g[2] = g[4];
    g[5] = g[7] - h - (R)0.25 * (Fx + Fy) + (R)0.5 * n * c.Ub;
    g[6] = g[8] + h + (R)0.25 * (Fx - Fy) - (R)0.5 * n * c.Ub;
    g[0] = dn - (g[1] + g[3]) - (R)2 * (g[4] + g[7] + g[8]) + (R)0.5 * Fy;
  } else if (wall == 2) {
    const R h = (R)0.5 * (g[1] - g[3]);
    g[4] = g[2];
    g[7] = g[5] + h + (R)0.25 * (Fx + Fy) - (R)0.5 * n * c.Ut;
    g[8] = g[6] - h - (R)0.25 * (Fx - Fy) + (R)0.5 * n * c.Ut;
    g[0] = dn - (g[1] + g[3]) - (R)2 * (g[2] + g[5] + g[6]) - (R)0.5 * Fy;
  }
}

// Density deviation of a node: the sum of its pulled slots (n-hat at walls).
template <typename R>
__device__ __forceinline__ R slot_sum(const R v[9]) {
  return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])) + v[8];
}

// ---------------------------------------------------------------------------
// Two time steps per launch (FP32). A workgroup of NT threads owns a strip of
// NT-14 columns; thread t works on column x0-7+t. The first step runs the
// pipeline of step_kernel over the columns and rows the second step needs (4
// more on each side) and keeps its post-collision populations in a ring of
// four rows instead of storing them (populations 1, 3, 5-8, which move along
// x, in LDS; 0, 2 and 4 in the thread's registers); the second step pulls
// from that ring, runs the same four stages 9 rows behind the first, and
// stores. Each population in HBM is read and written once per two steps.
//
// The second step has no ghost rows: at a wall row its stages read the
// mirror image of the row inside the lattice where the first step reads a
// ghost row (the same values, y-components negated), so both kernels give
// the same bits. Its rows run from S2 to E2 in march order, its outputs plus
// three rows on each side, cut at a wall; the first step's outputs run one
// row further on each side that is not a wall.
//
// Per iteration k, four phases with barriers after the first three:
//   1: A1 (row k of the first step's pipeline), A2 (second step row k-9);
//   2: B1, B2;  3: C1, C2;  4: D1 (into the ring), D2 (to HBM).
// A2 reads ring rows k-10 .. k-8, which D1 wrote at least two iterations
// earlier, so phase 4 needs no barrier before the next phase 1; D1 then
// writes row k-6 over row k-10, which A2 read in phase 1 of the same
// iteration. Ring slots are row mod ring size, so those of the second step
// are the first step's shifted by 9.
// ---------------------------------------------------------------------------
// One tile of the two-step kernel. YB: 1 the lattice has walls, 2 it is
// periodic in y, or every row of the tile's pipeline lies at least one row
// inside the walls (then the rows map as if periodic, which there is the
// identity, and no wall rule applies: the same arithmetic on the same values
// as the walls body, so the same bits); 0 read per lattice.
// Regularised collision (Sec. II names the step that re-projects the
// post-collision populations onto the Hermite space): the non-equilibrium
// part h = g - geq is replaced by its projection onto the Hermite
// polynomials of order <= 2 before it relaxes,
//   g_i <- geq_i + (1 - omega) P[h]_i + F_i,
//   P[h]_i = w_i [a0 + 3 a1.c_i + 9/2 a2 : (c_i c_i - I/3)],
// a0 = sum h, a1 = sum h c, a2 = sum h (c c - I/3); geq and F as in collide,
// formed separately here.
template <typename R>
struct CollReg {
  R keep, oneT, s3;          // 1 - omega, 1 - T, 3 s
  R wr0, wra, wrd;           // w^_i
  R w0, wa, wd;              // w_i
  R w0s, was, wds;           // w_i s
};

template <typename R>
__device__ __forceinline__ CollReg<R> make_coll_reg(const Desc& d) {
  CollReg<R> c;
  const double s = 1.0 - 0.5 * d.omega;
  c.keep = (R)(1.0 - d.omega);
  c.oneT = (R)(1.0 - d.T);
  c.s3 = (R)(3.0 * s);
  c.wr0 = (R)rest_weight_hd(0, d.T);
  c.wra = (R)rest_weight_hd(1, d.T);
  c.wrd = (R)rest_weight_hd(5, d.T);
  c.w0 = (R)(4.0 / 9.0);
  c.wa = (R)(1.0 / 9.0);
  c.wd = (R)(1.0 / 36.0);
  c.w0s = (R)(4.0 / 9.0 * s);
  c.was = (R)(1.0 / 9.0 * s);
  c.wds = (R)(1.0 / 36.0 * s);
  return c;
}

template <typename R>
__device__ __forceinline__ void collide_reg(R g[9], const CollReg<R>& c, R n, R dn, R jx, R jy,
                                            R rn, R Fx, R Fy, R dnx, R dny, R D) {
  const R ux = jx * rn, uy = jy * rn;
  const R usq = (R)1.5 * (ux * ux + uy * uy);
  const R Xxx = (R)6 * ux * Fx + c.oneT * ((R)2 * ux * dnx + D);
  const R Xyy = (R)6 * uy * Fy + c.oneT * ((R)2 * uy * dny + D);
  const R Xxy = (R)3 * (ux * Fy + uy * Fx) + c.oneT * (ux * dny + uy * dnx);
  const R trX = Xxx + Xyy;
  // equilibrium deviations and forcing, by direction
  R eq[9], fo[9];
  eq[0] = c.wr0 * dn - c.w0 * (n * usq);
  fo[0] = -c.w0s * ((R)0.5 * trX);
  {
    const R e = c.wra * dn + c.wa * (n * ((R)4.5 * ux * ux - usq)), a = (R)3 * c.wa * jx;
    const R fs = c.was * (Xxx - (R)0.5 * Xyy), fa = c.wa * c.s3 * Fx;
    eq[1] = e + a; eq[3] = e - a; fo[1] = fs + fa; fo[3] = fs - fa;
  }
  {
    const R e = c.wra * dn + c.wa * (n * ((R)4.5 * uy * uy - usq)), a = (R)3 * c.wa * jy;
    const R fs = c.was * (Xyy - (R)0.5 * Xxx), fa = c.wa * c.s3 * Fy;
    eq[2] = e + a; eq[4] = e - a; fo[2] = fs + fa; fo[4] = fs - fa;
  }
  {
    const R cu = ux + uy;
    const R e = c.wrd * dn + c.wd * (n * ((R)4.5 * cu * cu - usq)), a = (R)3 * c.wd * (jx + jy);
    const R fs = c.wds * (trX + (R)3 * Xxy), fa = c.wd * c.s3 * (Fx + Fy);
    eq[5] = e + a; eq[7] = e - a; fo[5] = fs + fa; fo[7] = fs - fa;
  }
  {
    const R cu = uy - ux;
    const R e = c.wrd * dn + c.wd * (n * ((R)4.5 * cu * cu - usq)), a = (R)3 * c.wd * (jy - jx);
    const R fs = c.wds * (trX - (R)3 * Xxy), fa = c.wd * c.s3 * (Fy - Fx);
    eq[6] = e + a; eq[8] = e - a; fo[6] = fs + fa; fo[8] = fs - fa;
  }
  R h[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) h[i] = g[i] - eq[i];
  const R a0 = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
  const R a1x = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
  const R a1y = (h[2] - h[4]) + (h[5] - h[8]) + (h[6] - h[7]);
  const R dg = (h[5] + h[6]) + (h[7] + h[8]);
  const R a2xx = (h[1] + h[3]) + dg - a0 * (R)(1.0 / 3.0);
  const R a2yy = (h[2] + h[4]) + dg - a0 * (R)(1.0 / 3.0);
  const R a2xy = (h[5] - h[6]) + (h[7] - h[8]);
  // P[h] by direction, times 1 - omega: w_i [a0 + 3 a1.c + 9/2 a2:(cc - I/3)]
  const R k0 = c.keep * c.w0, ka = c.keep * c.wa, kd = c.keep * c.wd;
  g[0] = eq[0] + k0 * (a0 - (R)1.5 * (a2xx + a2yy)) + fo[0];
  {
    const R s = a0 + (R)3 * a2xx - (R)1.5 * a2yy, t = (R)3 * a1x;
    g[1] = eq[1] + ka * (s + t) + fo[1];
    g[3] = eq[3] + ka * (s - t) + fo[3];
  }
  {
    const R s = a0 + (R)3 * a2yy - (R)1.5 * a2xx, t = (R)3 * a1y;
    g[2] = eq[2] + ka * (s + t) + fo[2];
    g[4] = eq[4] + ka * (s - t) + fo[4];
  }
  {
    const R s = a0 + (R)3 * (a2xx + a2yy), x9 = (R)9 * a2xy;
    const R t5 = (R)3 * (a1x + a1y), t6 = (R)3 * (a1y - a1x);
    g[5] = eq[5] + kd * (s + x9 + t5) + fo[5];
    g[7] = eq[7] + kd * (s + x9 - t5) + fo[7];
    g[6] = eq[6] + kd * (s - x9 + t6) + fo[6];
    g[8] = eq[8] + kd * (s - x9 - t6) + fo[8];
  }
}

template <int NT, bool MOM, int YB, bool REG>
__device__ __forceinline__ void step2_tile(const Desc& __restrict__ d, const Tile& tile, int dir,
                                           int parity, int flags, float (&nR)[8][NT + 2],
                                           Pair<float> (&LP)[4][NT + 2], Mom<float> (&JR)[4][NT + 2],
                                           float (&nR2)[8][NT + 2], Pair<float> (&LP2)[4][NT + 2],
                                           Mom<float> (&JR2)[4][NT + 2], float (&O)[4][6][NT + 2]) {
  using R = float;
  const int Lx = d.Lx, Ly = d.Ly, periodic = YB == 0 ? d.periodic : (YB == 2 ? 1 : 0);
  const int64_t nn = (int64_t)Lx * Ly;
  const int rowb = 9 * Lx * (int)sizeof(R);
  const int arrb = (int)(9 * nn * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t Sin = make_rsrc(d.S[parity], arrb);
  const __amdgpu_buffer_rsrc_t Sout = make_rsrc(d.S[parity ^ 1], arrb);
  const __amdgpu_buffer_rsrc_t Snone = make_rsrc(d.S[parity ^ 1], 0);
  const R* __restrict__ fext3 = (const R*)d.fext3;
  const Coll<R> cl = make_coll<R>(d);
  const CollReg<R> clr = make_coll_reg<R>(d);
  const Sten<R> c = make_sten<R>(d, dir);
  R shift = (R)0;
  if ((flags & kApplyShift) && d.shift) shift = (R)(*d.shift);
  const R sh0 = shift * (R)rest_weight_hd(0, d.T), sha = shift * (R)rest_weight_hd(1, d.T),
          shd = shift * (R)rest_weight_hd(5, d.T);

  const int t = threadIdx.x;
  const int W = min(NT - 14, Lx - tile.x0);  // columns this strip updates
  int xc = (tile.x0 - 7 + t) % Lx;
  if (xc < 0) xc += Lx;
  const int xm = xc == 0 ? Lx - 1 : xc - 1;
  const int xp = xc == Lx - 1 ? 0 : xc + 1;
  // lanes of the first step's pulls, of its force stage (the column force
  // table), and of the second step's stores
  const bool actA = t < W + 14;
  const bool actC = t >= 2 && t < W + 12;
  const bool act2D = t >= 7 && t < W + 7;
  const int vc = actA ? xc * (int)sizeof(R) : arrb;
  const int vm = actA ? xm * (int)sizeof(R) : arrb;
  const int vp = actA ? xp * (int)sizeof(R) : arrb;
  const R fx3 = actC ? fext3[xc] : (R)0;
  const uint32_t pbytes = (uint32_t)Lx * (uint32_t)sizeof(R);

  // Rows in march order. S1 is the first step's first output row (relative
  // index 0); rel(y) = dir (y - S1).
  int S2, E2, ofirst, olast;
  bool ws = false, we = false;
  if (dir > 0) {
    S2 = tile.y0 - 3;
    E2 = tile.y1 + 2;
    if (!periodic) {
      S2 = max(S2, 0);
      E2 = min(E2, Ly - 1);
      ws = S2 == 0;
      we = E2 == Ly - 1;
    }
    ofirst = tile.y0;
    olast = tile.y1 - 1;
  } else {
    S2 = tile.y1 + 2;
    E2 = tile.y0 - 3;
    if (!periodic) {
      S2 = min(S2, Ly - 1);
      E2 = max(E2, 0);
      ws = S2 == Ly - 1;
      we = E2 == 0;
    }
    ofirst = tile.y1 - 1;
    olast = tile.y0;
  }
  const int S1 = ws ? S2 : S2 - dir;
  const int E1 = we ? E2 : E2 + dir;
  const int K1 = dir * (E1 - S1) + 1 + 6;  // first step: pipeline rows S1-3 .. E1+3
  const int a0 = S1 - 3 * dir;
  // second step, relative rows: first and last of its pipeline, and of its
  // outputs
  const int r2s = dir * (S2 - S1), r2e = dir * (E2 - S1);
  const int rds = dir * (ofirst - S1), rde = dir * (olast - S1);
  const int K = rde + 13;  // D2 runs on relative row k - 12

  const int u = t + 1;

  // one row in flight: an iteration of two steps outlasts the load latency,
  // and the registers are scarce (two rows measured the same)
  constexpr int P = 1;
  R f[4][9], f2[4][9], pf[P][9];
  R Fr[2][2], Fr2[2][2];  // (F_x, F_y) of the row stage C last finished
  R Or[4][3];             // populations 0, 2, 4 of the ring rows
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f[s][i] = (R)0;
      f2[s][i] = (R)0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) Or[s][i] = (R)0;
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      Fr[s][i] = (R)0;
      Fr2[s][i] = (R)0;
    }

#pragma unroll
  for (int j = 0; j < P; ++j)
    pull_row<R>(pf[j], j < K1 ? Sin : Snone, pbytes, (uint32_t)rowb, Ly, periodic,
                map_row_any(a0 + dir * j, Ly, periodic), vc, vm, vp);

  // Every stage runs on every lane and iteration, valid or not: a ring
  // write lands in the slot of a row that no valid stage still needs, and
  // valid stages read only rows and columns that valid stages wrote, so the
  // idle work is harmless; without branches around the stages the compiler
  // can interleave the two steps' instructions. Stores go through the
  // buffers' range checks.
  for (int kb = 0; kb < K; kb += 8) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = kb + s;
      const int a = a0 + dir * k;
      // ---- phase 1: A2 (relative row k-9) pulls from the ring (rows k-10,
      // k-9, k-8); A1 (row a) takes the row loaded P iterations ago ---------
      {
        const int y = S1 + dir * (k - 9);
        const bool lo = !periodic && y == 0, hi = !periodic && y == Ly - 1;
        constexpr int ps = NT + 2;  // plane stride; planes 0..5 hold populations 1, 3, 5, 6, 7, 8
        const R* Ob = &O[(s + 2) & 3][0][0];
        const R* Oc = &O[(s + 3) & 3][0][0];
        const R* Oa = &O[s & 3][0][0];
        const R* Os = dir > 0 ? Ob : Oa;  // row y - 1 (sources with c_y = +1)
        const R* On = dir > 0 ? Oa : Ob;  // row y + 1 (sources with c_y = -1)
        const R* rb = Or[(s + 2) & 3];
        const R* rc = Or[(s + 3) & 3];
        const R* ra = Or[s & 3];
        const R s2 = dir > 0 ? rb[1] : ra[1];  // population 2 of row y - 1
        const R n4 = dir > 0 ? ra[2] : rb[2];  // population 4 of row y + 1
        R* v = f2[(s + 3) & 3];
        v[0] = rc[0];
        v[1] = Oc[0 * ps + u - 1];
        v[3] = Oc[1 * ps + u + 1];
        if (lo || hi) {  // a wall row (uniform): the node's own outgoing populations
          v[2] = lo ? rc[2] : s2;
          v[5] = lo ? Oc[4 * ps + u] : Os[2 * ps + u - 1];
          v[6] = lo ? Oc[5 * ps + u] : Os[3 * ps + u + 1];
          v[4] = hi ? rc[1] : n4;
          v[7] = hi ? Oc[2 * ps + u] : On[4 * ps + u + 1];
          v[8] = hi ? Oc[3 * ps + u] : On[5 * ps + u - 1];
        } else {
          v[2] = s2;
          v[5] = Os[2 * ps + u - 1];
          v[6] = Os[3 * ps + u + 1];
          v[4] = n4;
          v[7] = On[4 * ps + u + 1];
          v[8] = On[5 * ps + u - 1];
        }
        nR2[(s + 7) & 7][u] = slot_sum<R>(v);
      }
      {
        R* v = f[s & 3];
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = pf[s % P][i];
        if (shift != (R)0) {
          v[0] += sh0;
#pragma unroll
          for (int i = 1; i <= 4; ++i) v[i] += sha;
#pragma unroll
          for (int i = 5; i <= 8; ++i) v[i] += shd;
        }
        nR[s][u] = slot_sum<R>(v);
      }
      {
        const RowMap mp = map_row_any(a + P * dir, Ly, periodic);
        const __amdgpu_buffer_rsrc_t Sp = (k + P < K1) ? Sin : Snone;
        if (mp.wall == 0)  // interior rows (uniform): no wall slots
          pull_row<R>(pf[s % P], Sp, pbytes, (uint32_t)rowb, Ly, periodic, RowMap{mp.phys, 0, 1}, vc,
                      vm, vp);
        else
          pull_row<R>(pf[s % P], Sp, pbytes, (uint32_t)rowb, Ly, periodic, mp, vc, vm, vp);
      }
      __syncthreads();
      // ---- phase 2: B1 (row a - dir), B2 (relative row k-10) -----------------
      LP[(s + 3) & 3][u] = stage_lp<R>(nR[(s + 6) & 7], nR[(s + 7) & 7], nR[s], u, c);
      {
        const int r = k - 10;
        const R* bh = nR2[(s + 5) & 7];
        const R* ah = nR2[(s + 7) & 7];
        if (ws && r == r2s) bh = ah;  // behind the first row: its mirror
        if (we && r == r2e) ah = bh;
        LP2[(s + 2) & 3][u] = stage_lp<R>(bh, nR2[(s + 6) & 7], ah, u, c);
      }
      __syncthreads();
      // ---- phase 3: C1 (row a - 2 dir), C2 (relative row k-11) ---------------
      {
        const int r = k - 11;
        const Pair<R>* bh = LP2[s & 3];
        const Pair<R>* ah = LP2[(s + 2) & 3];
        if (ws && r == r2s) bh = ah;
        if (we && r == r2e) ah = bh;
        const R n1 = c.nbar + nR[(s + 6) & 7][u];
        const R n2 = c.nbar + nR2[(s + 5) & 7][u];
        R Fx1, Fy1, jx1, jy1, Fx2, Fy2, jx2, jy2;
        stage_force<R>(LP[(s + 1) & 3], LP[(s + 2) & 3], LP[(s + 3) & 3], u, n1, fx3, c, Fx1, Fy1);
        stage_force<R>(bh, LP2[(s + 1) & 3], ah, u, n2, fx3, c, Fx2, Fy2);
        const RowMap m = map_row(a - 2 * dir, Ly, periodic);
        const int y = S1 + dir * r;
        const int wall2 = periodic ? 0 : (y == 0 ? 1 : (y == Ly - 1 ? 2 : 0));
        // interior rows (uniform) take the body without the wall selects
        if (m.wall == 0 && m.ysgn > 0)
          stage_mom<R>(f[(s + 2) & 3], 0, 1, n1, Fx1, Fy1, c, jx1, jy1);
        else
          stage_mom<R>(f[(s + 2) & 3], m.wall, m.ysgn, n1, Fx1, Fy1, c, jx1, jy1);
        if (wall2 == 0)
          stage_mom<R>(f2[(s + 1) & 3], 0, 1, n2, Fx2, Fy2, c, jx2, jy2);
        else
          stage_mom<R>(f2[(s + 1) & 3], wall2, 1, n2, Fx2, Fy2, c, jx2, jy2);
        JR[(s + 2) & 3][u] = Mom<R>{jx1, jy1};
        JR2[(s + 1) & 3][u] = Mom<R>{jx2, jy2};
        Fr[s & 1][0] = Fx1;
        Fr[s & 1][1] = Fy1;
        Fr2[(s + 1) & 1][0] = Fx2;
        Fr2[(s + 1) & 1][1] = Fy2;
      }
      __syncthreads();
      // ---- phase 4: D1 (row a - 3 dir) into the ring, D2 (relative row k-12)
      // to HBM ---------------------------------------------------------------
      if (k >= 6 && k < K1) {
        const int dd1 = a - 3 * dir;
        R g1[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g1[i] = f[(s + 1) & 3][i];
        R dnx1, dny1, D1;
        stage_grad<R>(nR[(s + 4) & 7], nR[(s + 5) & 7], nR[(s + 6) & 7], JR[s & 3],
                      JR[(s + 1) & 3], JR[(s + 2) & 3], u, (R)1, (R)1, c, dnx1, dny1, D1);
        const Mom<R> m1 = JR[(s + 1) & 3][u];
        const R Fx1 = Fr[(s + 1) & 1][0], Fy1 = Fr[(s + 1) & 1][1];
        const R dn1 = nR[(s + 5) & 7][u];
        const R n1 = c.nbar + dn1;
        const R rn1 = fast_rcp<R>(n1);
        const int wall1 = periodic ? 0 : (dd1 == 0 ? 1 : (dd1 == Ly - 1 ? 2 : 0));
        stage_wall<R>(g1, wall1, dn1, n1, Fx1, Fy1, c);
        if constexpr (REG)
          collide_reg<R>(g1, clr, n1, dn1, m1.jx, m1.jy, rn1, Fx1, Fy1, dnx1, dny1, D1);
        else
          collide<R>(g1, cl, n1, dn1, m1.jx, m1.jy, rn1, Fx1, Fy1, dnx1, dny1, D1);
        R* o = &O[(s + 2) & 3][0][0];
        constexpr int ps = NT + 2;
        o[0 * ps + u] = g1[1];
        o[1 * ps + u] = g1[3];
        o[2 * ps + u] = g1[5];
        o[3 * ps + u] = g1[6];
        o[4 * ps + u] = g1[7];
        o[5 * ps + u] = g1[8];
        Or[(s + 2) & 3][0] = g1[0];
        Or[(s + 2) & 3][1] = g1[2];
        Or[(s + 2) & 3][2] = g1[4];
      }
      {
        const int r = k - 12;
        const int dd2 = S1 + dir * r;
        const bool valid2 = r >= rds && r <= rde;
        R g2[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g2[i] = f2[s & 3][i];
        R n2 = (R)1, ux2 = (R)0, uy2 = (R)0;
        if (valid2) {
          const R* bh = nR2[(s + 3) & 7];
          const R* ah = nR2[(s + 5) & 7];
          const Mom<R>* Jb = JR2[(s + 3) & 3];
          const Mom<R>* Ja = JR2[(s + 1) & 3];
          R sb = (R)1, sa = (R)1;
          if (ws && r == r2s) { bh = ah; Jb = Ja; sb = (R)-1; }
          if (we && r == r2e) { ah = bh; Ja = Jb; sa = (R)-1; }
          R dnx2, dny2, D2;
          stage_grad<R>(bh, nR2[(s + 4) & 7], ah, Jb, JR2[s & 3], Ja, u, sb, sa, c, dnx2, dny2, D2);
          const Mom<R> m2 = JR2[s & 3][u];
          const R Fx2 = Fr2[s & 1][0], Fy2 = Fr2[s & 1][1];
          const R dn2 = nR2[(s + 4) & 7][u];
          n2 = c.nbar + dn2;
          const R rn2 = fast_rcp<R>(n2);
          ux2 = m2.jx * rn2;
          uy2 = m2.jy * rn2;
          const int wall2 = periodic ? 0 : (dd2 == 0 ? 1 : (dd2 == Ly - 1 ? 2 : 0));
          stage_wall<R>(g2, wall2, dn2, n2, Fx2, Fy2, c);
          if constexpr (REG)
            collide_reg<R>(g2, clr, n2, dn2, m2.jx, m2.jy, rn2, Fx2, Fy2, dnx2, dny2, D2);
          else
            collide<R>(g2, cl, n2, dn2, m2.jx, m2.jy, rn2, Fx2, Fy2, dnx2, dny2, D2);
        }
        // output rows lie in [0, Ly) (y0 .. y1-1 of the tile), periodic or not
        const __amdgpu_buffer_rsrc_t so = valid2 ? Sout : Snone;
        const int yy = valid2 ? dd2 : 0;
        const uint32_t roff = (uint32_t)yy * (uint32_t)rowb;
        const int vst = act2D ? vc : arrb;
#pragma unroll
        for (int i = 0; i < 9; ++i) buf_st(g2[i], so, vst, (int)((uint32_t)i * pbytes + roff));
        if (MOM) {
          const int momb = (int)(3 * nn * 8);
          const __amdgpu_buffer_rsrc_t mo = make_rsrc(d.mom, valid2 ? momb : 0);
          const int vo = act2D ? xc * 8 : momb;
          const int ro = yy * Lx * 8;
          buf_st((double)n2, mo, vo, ro);
          buf_st((double)ux2, mo, vo, (int)(nn * 8) + ro);
          buf_st((double)uy2, mo, vo, (int)(2 * nn * 8) + ro);
        }
      }
    }
  }
}

// YB: 1 every lattice of the launch has walls (tiles whose pipeline stays at
// least one row inside the walls take the wall-free body), 2 every lattice is
// periodic in y, 0 read per lattice.
template <int NT, bool MOM, int YB, bool REG>
__global__ __launch_bounds__(NT, 2) void step2_kernel(const Desc* __restrict__ descs,
                                                      const Tile* __restrict__ tiles, int ntiles,
                                                      int parity, int flags) {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, rm = nb & 7, xcd = b & 7;
  const int logical = xcd * q + (xcd < rm ? xcd : rm) + (b >> 3);
  if (logical >= ntiles) return;  // uniform per block
  const Tile tile = tiles[logical];
  const int inst = tile.inst & 0x7fffffff;
  const int dir = (tile.inst < 0) ? -1 : 1;
  const Desc& d = descs[inst];
  // LDS rings: 288 (NT + 2) bytes, so eight 64-thread, four 128-thread or
  // two 256-thread workgroups fit on a CU. The force F goes from stage C to
  // stage D of the next iteration in registers; of the first step's
  // post-collision populations only those that move along x (1, 3, 5, 6, 7,
  // 8) go through LDS (O, planes in that order), populations 0, 2 and 4 stay
  // in the thread's registers.
  __shared__ float nR[8][NT + 2];
  __shared__ Pair<float> LP[4][NT + 2];
  __shared__ Mom<float> JR[4][NT + 2];
  __shared__ float nR2[8][NT + 2];
  __shared__ Pair<float> LP2[4][NT + 2];
  __shared__ Mom<float> JR2[4][NT + 2];
  __shared__ float O[4][6][NT + 2];
  // inner: the first step's pipeline rows, y0 - 7 .. y1 + 6, lie within
  // [1, Ly - 2], so none is a wall or ghost row and their pulls read rows
  // 0 .. Ly - 1 as they are
  if (YB == 1 && NT == 256 && tile.y0 >= 8 && tile.y1 <= d.Ly - 8)
    step2_tile<NT, MOM, 2, REG>(d, tile, dir, parity, flags, nR, LP, JR, nR2, LP2, JR2, O);
  else
    step2_tile<NT, MOM, YB, REG>(d, tile, dir, parity, flags, nR, LP, JR, nR2, LP2, JR2, O);
}

template <int NT, int YB, bool REG>
static void launch_step2_y(const Desc* dd, const Tile* dt, int ntiles, int parity, int flags,
                           hipStream_t st) {
  if (flags & kWriteMoments)
    hipLaunchKernelGGL((step2_kernel<NT, true, YB, REG>), dim3(ntiles), dim3(NT), 0, st, dd, dt,
                       ntiles, parity, flags);
  else
    hipLaunchKernelGGL((step2_kernel<NT, false, YB, REG>), dim3(ntiles), dim3(NT), 0, st, dd, dt,
                       ntiles, parity, flags);
}

template <int NT, bool REG>
static hipError_t launch_step2_t(const Desc* dd, const Tile* dt, int ntiles, int parity,
                                 int flags, hipStream_t st) {
  if (flags & kYWalls)
    launch_step2_y<NT, 1, REG>(dd, dt, ntiles, parity, flags, st);
  else if (flags & kYPeriodic)
    launch_step2_y<NT, 2, REG>(dd, dt, ntiles, parity, flags, st);
  else
    launch_step2_y<NT, 0, REG>(dd, dt, ntiles, parity, flags, st);
  return hipGetLastError();
}

template <bool REG>
static hipError_t launch_step2_r(int threads, const Desc* d_descs, const Tile* d_tiles,
                                 int ntiles, int parity, int flags, hipStream_t stream) {
  if (threads == 64) return launch_step2_t<64, REG>(d_descs, d_tiles, ntiles, parity, flags, stream);
  if (threads == 128) return launch_step2_t<128, REG>(d_descs, d_tiles, ntiles, parity, flags, stream);
  if (threads == 192) return launch_step2_t<192, REG>(d_descs, d_tiles, ntiles, parity, flags, stream);
  if (threads == 256) return launch_step2_t<256, REG>(d_descs, d_tiles, ntiles, parity, flags, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_step2(int threads, bool reg, const Desc* d_descs, const Tile* d_tiles,
                        int ntiles, int parity, int flags, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  return reg ? launch_step2_r<true>(threads, d_descs, d_tiles, ntiles, parity, flags, stream)
             : launch_step2_r<false>(threads, d_descs, d_tiles, ntiles, parity, flags, stream);
}

// ---------------------------------------------------------------------------
// ---- one-step kernel: step_kernel in three precisions, the stochastic
// rounding and the regularised collision. The code above this section is
// everything the two-step kernel compiles from.
// ---------------------------------------------------------------------------

// Population stores of the one-step kernel: FP64 values with the
// non-temporal bit, so the written planes do not displace rows that
// neighbouring chunks still read; FP32 values as they are.
__device__ __forceinline__ void pop_st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  buf_st(v, r, voff, soff);
}
__device__ __forceinline__ void pop_st(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, 2);
}

}  // namespace lbk

#include "lb_rng.h"

namespace lbk {

using lbrng::draws14;
using lbrng::pcg4d;
using lbrng::round_stochastic;
using lbrng::U4;

// Rows of populations in flight ahead of stage A, and the waves per SIMD the
// register budget is sized for (FP32; FP64 always sizes for one wave). Two
// rows at 3 waves per SIMD (about 140 VGPRs, no spills) measured fastest on
// the 8192 x 2048 lattice: one 512-thread workgroup per CU, 255 workgroups.
#ifndef LB_PREFETCH
#define LB_PREFETCH 2
#endif
#ifndef LB_WAVES_PER_SIMD
#define LB_WAVES_PER_SIMD 3
#endif
constexpr int kPrefetch = LB_PREFETCH;
static_assert(kPrefetch == 1 || kPrefetch == 2 || kPrefetch == 4, "prefetch depth must divide 8");

// S: storage type of the populations, R: arithmetic type. S = float with
// R = double stores through round_stochastic. REG: regularised collision.
template <typename S, typename R, int NT, bool MOM, bool REG>
__global__ __launch_bounds__(NT, sizeof(R) == 4 ? LB_WAVES_PER_SIMD : 1) void step_kernel(
    const Desc* __restrict__ descs, const Tile* __restrict__ tiles, int ntiles, int parity,
    int flags) {
  constexpr bool kSR = sizeof(S) < sizeof(R);
  // Workgroups are dealt round-robin over the 8 XCDs; give each XCD a
  // contiguous run of tiles so vertically adjacent chunks share its L2.
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, rm = nb & 7, xcd = b & 7;
  const int logical = xcd * q + (xcd < rm ? xcd : rm) + (b >> 3);
  if (logical >= ntiles) return;  // uniform per block
  const Tile tile = tiles[logical];
  const int inst = tile.inst & 0x7fffffff;
  const int dir = (tile.inst < 0) ? -1 : 1;  // march direction along y
  const Desc& d = descs[inst];
  const int Lx = d.Lx, Ly = d.Ly, periodic = d.periodic;
  const int64_t nn = (int64_t)Lx * Ly;
  const int rowb = 9 * Lx * (int)sizeof(S);        // bytes of one row (nine planes)
  const int arrb = (int)(9 * nn * (int64_t)sizeof(S));  // bytes of the nine planes (< 2 GiB)
  const __amdgpu_buffer_rsrc_t Sin = make_rsrc(d.S[parity], arrb);
  const __amdgpu_buffer_rsrc_t Sout = make_rsrc(d.S[parity ^ 1], arrb);
  const __amdgpu_buffer_rsrc_t Snone = make_rsrc(d.S[parity ^ 1], 0);  // drops every access
  const R* __restrict__ fext3 = (const R*)d.fext3;
  const Coll<R> cl = make_coll<R>(d);
  const CollReg<R> clr = make_coll_reg<R>(d);
  const Sten<R> c = make_sten<R>(d, dir);
  // Stochastic rounding: this launch's step number comes from the counter of
  // the buffer it reads; the workgroup of the lattice's first tile writes the
  // next one into the counter of the buffer it writes (read by the next
  // launch, untouched by this one).
  uint32_t rstep = 0;
  if constexpr (kSR) {
    rstep = d.rng[parity];
    if (tile.x0 == 0 && tile.y0 == 0 && threadIdx.x == 0) d.rng[parity ^ 1] = rstep + 1u;
  }
  R shift = (R)0;
  if ((flags & kApplyShift) && d.shift) shift = (R)(*d.shift);
  const R sh0 = shift * (R)rest_weight_hd(0, d.T), sha = shift * (R)rest_weight_hd(1, d.T),
          shd = shift * (R)rest_weight_hd(5, d.T);

  const int t = threadIdx.x;
  const int W = min(NT - 6, Lx - tile.x0);  // columns this strip updates
  int xc = (tile.x0 - 3 + t) % Lx;
  if (xc < 0) xc += Lx;
  const int xm = xc == 0 ? Lx - 1 : xc - 1;  // source of c_x = +1
  const int xp = xc == Lx - 1 ? 0 : xc + 1;  // source of c_x = -1
  const bool actA = t < W + 6;
  const bool actB = t >= 1 && t < W + 5;
  const bool actC = t >= 2 && t < W + 4;
  const bool actD = t >= 3 && t < W + 3;
  // per-lane byte offsets; lanes outside the strip use the array bound (dropped)
  const int vc = actA ? xc * (int)sizeof(S) : arrb;
  const int vm = actA ? xm * (int)sizeof(S) : arrb;
  const int vp = actA ? xp * (int)sizeof(S) : arrb;
  const R fx3 = actC ? fext3[xc] : (R)0;
  const uint32_t pbytes = (uint32_t)Lx * (uint32_t)sizeof(S);  // plane stride within a row

  // LDS rings indexed by pipeline row j (row a_j = a_0 + dir j): slot j % 8
  // for n, j % 4 for the others. With the loop unrolled by 8 every slot is a
  // compile-time offset. One padding entry on each side keeps the stencil
  // reads of edge lanes inside the arrays.
  __shared__ R nR[8][NT + 2];          // density deviation dn
  __shared__ Pair<R> LP[4][NT + 2];    // (Laplacian of n, p^i - p^w)
  __shared__ Quad<R> JR[4][NT + 2];    // (j*_x, j*_y, F_x, F_y)
  const int u = t + 1;                 // padded column index

  constexpr int P = kPrefetch;
  R f[4][9];     // pulled populations, slot j % 4
  S pf[P][9];    // the next P rows' pulled populations, in flight (slot j % P)
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 9; ++i) f[s][i] = (R)0;

  const int y0 = tile.y0, y1 = tile.y1;
  // Pipeline rows j = 0 .. K-1 are rows y0-3 .. y1+2 in march order. At
  // iteration k: A on row j = k, B on k-1, C on k-2, D on k-3. Valid: A for
  // k < K, B for 2 <= k < K, C for 4 <= k < K, D for 6 <= k < K. Iterations
  // past K (at most 7, only when the chunk height is not 2 mod 8) run with
  // their memory accesses dropped. Every load and store is issued on every
  // iteration, outside branches, so the compiler can count them exactly
  // when it waits for the prefetched row.
  const int K = (y1 - y0) + 6;
  const int a0 = dir > 0 ? y0 - 3 : y1 + 2;

#pragma unroll
  for (int j = 0; j < P; ++j)
    pull_row<S>(pf[j], j < K ? Sin : Snone, pbytes, (uint32_t)rowb, Ly, periodic,
                map_row_any(a0 + dir * j, Ly, periodic), vc, vm, vp);

  for (int kb = 0; kb < K; kb += 8) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = kb + s;
      const int a = a0 + dir * k;
      // ---- stage A: row a (its loads were issued P iterations ago) -----------
      if (k < K) {
        R* v = f[s & 3];
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = (R)pf[s % P][i];
        if (shift != (R)0) {
          v[0] += sh0;
#pragma unroll
          for (int i = 1; i <= 4; ++i) v[i] += sha;
#pragma unroll
          for (int i = 5; i <= 8; ++i) v[i] += shd;
        }
        nR[s][u] = slot_sum<R>(v);
      }
      // prefetch row a + P dir into the slot just consumed (dropped past the
      // last pipeline row)
      pull_row<S>(pf[s % P], (k + P < K) ? Sin : Snone, pbytes, (uint32_t)rowb, Ly, periodic,
                  map_row_any(a + P * dir, Ly, periodic), vc, vm, vp);
      __syncthreads();
      // ---- stage B: row a - dir: Laplacian and pressure term -----------------
      if (k >= 2 && k < K && actB)
        LP[(s + 3) & 3][u] = stage_lp<R>(nR[(s + 6) & 7], nR[(s + 7) & 7], nR[s], u, c);
      __syncthreads();
      // ---- stage C: row a - 2 dir: force and j* ------------------------------
      if (k >= 4 && k < K && actC) {
        const R n = c.nbar + nR[(s + 6) & 7][u];
        R Fx, Fy, jx, jy;
        stage_force<R>(LP[(s + 1) & 3], LP[(s + 2) & 3], LP[(s + 3) & 3], u, n, fx3, c, Fx, Fy);
        // momentum of the pulled populations of this row, still in the ring
        const RowMap m = map_row(a - 2 * dir, Ly, periodic);
        stage_mom<R>(f[(s + 2) & 3], m.wall, m.ysgn, n, Fx, Fy, c, jx, jy);
        JR[(s + 2) & 3][u] = Quad<R>{jx, jy, Fx, Fy};
      }
      __syncthreads();
      // ---- stage D: row a - 3 dir: walls, collision, store -------------------
      const int dd = a - 3 * dir;
      const bool validD = k >= 6 && k < K;
      // rows without a valid D stage store nothing (their stores are dropped)
      R g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = f[(s + 1) & 3][i];
      R n = (R)1, ux = (R)0, uy = (R)0;
      if (validD) {
        R dnx, dny, D;
        stage_grad<R>(nR[(s + 4) & 7], nR[(s + 5) & 7], nR[(s + 6) & 7], JR[s & 3],
                      JR[(s + 1) & 3], JR[(s + 2) & 3], u, (R)1, (R)1, c, dnx, dny, D);
        const Quad<R> mC = JR[(s + 1) & 3][u];
        const R dn = nR[(s + 5) & 7][u];
        n = c.nbar + dn;
        const R rn = fast_rcp<R>(n);
        ux = mC.jx * rn;
        uy = mC.jy * rn;
        const int wall = periodic ? 0 : (dd == 0 ? 1 : (dd == Ly - 1 ? 2 : 0));
        stage_wall<R>(g, wall, dn, n, mC.Fx, mC.Fy, c);
        if constexpr (REG)
          collide_reg<R>(g, clr, n, dn, mC.jx, mC.jy, rn, mC.Fx, mC.Fy, dnx, dny, D);
        else
          collide<R>(g, cl, n, dn, mC.jx, mC.jy, rn, mC.Fx, mC.Fy, dnx, dny, D);
      }
      {
        const __amdgpu_buffer_rsrc_t so = validD ? Sout : Snone;
        const uint32_t roff = validD ? (uint32_t)dd * (uint32_t)rowb : 0u;
        const int vst = actD ? vc : arrb;
        if constexpr (kSR) {
          uint32_t q[9];
          draws14(pcg4d(U4{(uint32_t)xc, (uint32_t)dd, rstep, 0u}), q);
#pragma unroll
          for (int i = 0; i < 9; ++i)
            buf_st(round_stochastic(g[i], q[i]), so, vst, (int)((uint32_t)i * pbytes + roff));
        } else {
#pragma unroll
          for (int i = 0; i < 9; ++i) pop_st(g[i], so, vst, (int)((uint32_t)i * pbytes + roff));
        }
        if (MOM) {
          const int momb = (int)(3 * nn * 8);
          const __amdgpu_buffer_rsrc_t mo = make_rsrc(d.mom, validD ? momb : 0);
          const int vo = actD ? xc * 8 : momb;
          const int ro = validD ? dd * Lx * 8 : 0;
          buf_st((double)n, mo, vo, ro);
          buf_st((double)ux, mo, vo, (int)(nn * 8) + ro);
          buf_st((double)uy, mo, vo, (int)(2 * nn * 8) + ro);
        }
      }
    }
  }
}

template <typename S, typename R, int NT, bool REG>
static hipError_t launch_step_t(const Desc* dd, const Tile* dt, int ntiles, int parity, int flags,
                                hipStream_t st) {
  if (flags & kWriteMoments)
    hipLaunchKernelGGL((step_kernel<S, R, NT, true, REG>), dim3(ntiles), dim3(NT), 0, st, dd, dt,
                       ntiles, parity, flags);
  else
    hipLaunchKernelGGL((step_kernel<S, R, NT, false, REG>), dim3(ntiles), dim3(NT), 0, st, dd,
                       dt, ntiles, parity, flags);
  return hipGetLastError();
}

template <typename S, typename R, bool REG>
static hipError_t launch_step_p(int threads, const Desc* dd, const Tile* dt, int ntiles,
                                int parity, int flags, hipStream_t st) {
  if (threads == 64) return launch_step_t<S, R, 64, REG>(dd, dt, ntiles, parity, flags, st);
  if (threads == 128) return launch_step_t<S, R, 128, REG>(dd, dt, ntiles, parity, flags, st);
  if (threads == 256) return launch_step_t<S, R, 256, REG>(dd, dt, ntiles, parity, flags, st);
  if (threads == 320) return launch_step_t<S, R, 320, REG>(dd, dt, ntiles, parity, flags, st);
  if constexpr (sizeof(R) == 4)
    if (threads == 512) return launch_step_t<S, R, 512, REG>(dd, dt, ntiles, parity, flags, st);
  return hipErrorInvalidValue;
}

template <typename S, typename R>
static hipError_t launch_step_c(bool reg, int threads, const Desc* dd, const Tile* dt, int ntiles,
                                int parity, int flags, hipStream_t st) {
  return reg ? launch_step_p<S, R, true>(threads, dd, dt, ntiles, parity, flags, st)
             : launch_step_p<S, R, false>(threads, dd, dt, ntiles, parity, flags, st);
}

hipError_t launch_step(int prec, bool reg, int threads, const Desc* d_descs, const Tile* d_tiles,
                       int ntiles, int parity, int flags, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == kFP32)
    return launch_step_c<float, float>(reg, threads, d_descs, d_tiles, ntiles, parity, flags, stream);
  if (prec == kFP32SR)
    return launch_step_c<float, double>(reg, threads, d_descs, d_tiles, ntiles, parity, flags,
                                        stream);
  if (prec == kFP64)
    return launch_step_c<double, double>(reg, threads, d_descs, d_tiles, ntiles, parity, flags,
                                         stream);
  return hipErrorInvalidValue;
}

// ---- initial state: S(0) = f_eq(n0, u0; T) (Eq.(eqfunc)) as deviations ----
template <typename R>
__global__ void init_kernel(const Desc* __restrict__ desc, int parity, const double* __restrict__ n0,
                            const double* __restrict__ ux0, const double* __restrict__ uy0,
                            int64_t nn) {
  const Desc& d = *desc;
  R* S = (R*)d.S[parity];
  if (d.rng && blockIdx.x == 0 && threadIdx.x == 0) d.rng[parity] = 0u;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double n = n0[k];
    const double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
    const double usq = 1.5 * (ux * ux + uy * uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double cu = cx(i) * ux + cy(i) * uy;
      const double wr = rest_weight_hd(i, d.T);
      const double g = wr * (n - d.nbar) + w[i] * n * (3.0 * cu + 4.5 * cu * cu - usq);
      S[pidx(i, k, k / d.Lx, d.Lx)] = (R)g;
    }
    if (d.mom) {
      d.mom[k] = n;
      d.mom[nn + k] = ux;
      d.mom[2 * nn + k] = uy;
    }
  }
}

static int grid_for(int64_t nn, int bs) {
  int64_t g = (nn + bs - 1) / bs;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

hipError_t launch_init(bool fp32, const Desc* d_desc, int parity, const double* d_n0,
                       const double* d_ux, const double* d_uy, int64_t nn, hipStream_t stream) {
  if (fp32)
    hipLaunchKernelGGL(init_kernel<float>, dim3(grid_for(nn, 256)), dim3(256), 0, stream, d_desc,
                       parity, d_n0, d_ux, d_uy, nn);
  else
    hipLaunchKernelGGL(init_kernel<double>, dim3(grid_for(nn, 256)), dim3(256), 0, stream, d_desc,
                       parity, d_n0, d_ux, d_uy, nn);
  return hipGetLastError();
}

// ---- FP64 checks: mass, momentum, min/max density, non-finite count ------
// Node density and momentum of the stored post-collision populations,
// accumulated in FP64. Wavefront reduction by DPP-backed shuffles, then
// across the block's waves in LDS; one partial per block. The partials are
// combined in a fixed order by reduce_final, so results are deterministic.
constexpr int kRedBS = 256;
constexpr int kRedMaxBlocks = 1024;

__host__ __device__ inline int reduce_blocks_hd(int64_t nn) {
  int64_t g = (nn + kRedBS * 8 - 1) / (kRedBS * 8);
  if (g < 1) g = 1;
  if (g > kRedMaxBlocks) g = kRedMaxBlocks;
  return (int)g;
}

int reduce_blocks(int64_t nn) { return reduce_blocks_hd(nn); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Partial sums of workgroup blk of nblk over the nodes of one lattice.
template <typename R>
__device__ __forceinline__ void reduce_partial(const Desc& d, int parity, int64_t nn, int blk,
                                               int nblk, int add_shift, double* __restrict__ part) {
  const R* S = (const R*)d.S[parity];
  double m = 0, jx = 0, jy = 0, mn = 1e300, mx = -1e300, bad = 0;
  const double base = d.nbar + ((add_shift && d.shift) ? *d.shift : 0.0);
  double wr[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) wr[i] = rest_weight_hd(i, d.T) * base;
  for (int64_t k = blk * (int64_t)kRedBS + threadIdx.x; k < nn; k += (int64_t)nblk * kRedBS) {
    double rho = 0, px = 0, py = 0;
    const int64_t y = k / d.Lx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double f = (double)S[pidx(i, k, y, d.Lx)] + wr[i];
      rho += f;
      px += cx(i) * f;
      py += cy(i) * f;
    }
    if (!isfinite(rho) || !isfinite(px) || !isfinite(py)) {
      bad += 1;
    } else {
      m += rho;
      jx += px;
      jy += py;
      mn = fmin(mn, rho);
      mx = fmax(mx, rho);
    }
  }
  __shared__ double red[6][kRedBS / 64];
  m = wave_sum(m); jx = wave_sum(jx); jy = wave_sum(jy); bad = wave_sum(bad);
  mn = wave_min(mn); mx = wave_max(mx);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = m; red[1][wv] = jx; red[2][wv] = jy; red[3][wv] = mn; red[4][wv] = mx; red[5][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0, a1 = 0, a2 = 0, a3 = 1e300, a4 = -1e300, a5 = 0;
    for (int w = 0; w < kRedBS / 64; ++w) {
      a0 += red[0][w]; a1 += red[1][w]; a2 += red[2][w];
      a3 = fmin(a3, red[3][w]); a4 = fmax(a4, red[4][w]); a5 += red[5][w];
    }
    double* o = part + blk * 6;
    o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3; o[4] = a4; o[5] = a5;
  }
}

template <typename R>
__global__ __launch_bounds__(kRedBS) void reduce_kernel(const Desc* __restrict__ desc, int parity,
                                                        int64_t nn, double* __restrict__ part,
                                                        int add_shift) {
  reduce_partial<R>(*desc, parity, nn, blockIdx.x, gridDim.x, add_shift, part);
}

// The same for the lattices list[0 .. gridDim.y): workgroup (b, j) computes
// partial b of lattice list[j] into part + 6 part_off[list[j]] (the grid is
// as wide as the largest lattice needs; the others exit early).
template <typename R>
__global__ __launch_bounds__(kRedBS) void reduce_batch_kernel(const Desc* __restrict__ descs,
                                                              int parity,
                                                              const int32_t* __restrict__ list,
                                                              const int64_t* __restrict__ part_off,
                                                              double* __restrict__ part) {
  const int i = list[blockIdx.y];
  const Desc& d = descs[i];
  const int64_t nn = (int64_t)d.Lx * d.Ly;
  const int nb = reduce_blocks_hd(nn);
  if ((int)blockIdx.x >= nb) return;  // uniform per workgroup
  reduce_partial<R>(d, parity, nn, blockIdx.x, nb, 0, part + 6 * part_off[i]);
}

hipError_t launch_reduce(bool fp32, const Desc* d_desc, int parity, int64_t nn, double* d_part,
                         int add_shift, hipStream_t stream) {
  const int nb = reduce_blocks(nn);
  if (fp32)
    hipLaunchKernelGGL(reduce_kernel<float>, dim3(nb), dim3(kRedBS), 0, stream, d_desc, parity, nn,
                       d_part, add_shift);
  else
    hipLaunchKernelGGL(reduce_kernel<double>, dim3(nb), dim3(kRedBS), 0, stream, d_desc, parity, nn,
                       d_part, add_shift);
  return hipGetLastError();
}

// Combine the partials in a fixed order (the same state always gives the
// same bits): thread t sums partials t, t + 256, ... in order, then the
// wavefront and workgroup reductions run in a fixed tree. mode 0: check
// (update the sticky status and the drift shift); 1: set the reference
// mass; 2: report only.
__device__ __forceinline__ void reduce_final_body(const double* __restrict__ part, int nb,
                                                  int64_t nn, ReduceOut* __restrict__ out,
                                                  int mode, int drift) {
  double m = 0, jx = 0, jy = 0, mn = 1e300, mx = -1e300, bad = 0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const double* q = part + 6 * b;
    m += q[0]; jx += q[1]; jy += q[2];
    mn = fmin(mn, q[3]); mx = fmax(mx, q[4]); bad += q[5];
  }
  __shared__ double red[6][4];
  m = wave_sum(m); jx = wave_sum(jx); jy = wave_sum(jy); bad = wave_sum(bad);
  mn = wave_min(mn); mx = wave_max(mx);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = m; red[1][wv] = jx; red[2][wv] = jy; red[3][wv] = mn; red[4][wv] = mx; red[5][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  m = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
  jx = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
  jy = ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3]));
  mn = fmin(fmin(red[3][0], red[3][1]), fmin(red[3][2], red[3][3]));
  mx = fmax(fmax(red[4][0], red[4][1]), fmax(red[4][2], red[4][3]));
  bad = ((red[5][0] + red[5][1]) + (red[5][2] + red[5][3]));
  out->mass = m; out->jx = jx; out->jy = jy; out->nmin = mn; out->nmax = mx; out->nonfinite = bad;
  const bool fail = bad > 0 || !(mn > 0.0) || !(mx < 3.0);
  if (mode == 1) {
    out->mass_ref = m;
    out->has_ref = 1u;
    out->status = fail ? 1u : 0u;
    out->shift = 0.0;
  } else if (mode == 0) {
    if (fail) out->status |= 1u;
    out->shift = (drift && out->has_ref && !fail) ? (out->mass_ref - m) / (double)nn : 0.0;
  }
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ part, int nb,
                                                           int64_t nn, ReduceOut* __restrict__ out,
                                                           int mode, int drift) {
  reduce_final_body(part, nb, nn, out, mode, drift);
}

// One workgroup per lattice of the list (the periodic check, mode 0).
__global__ __launch_bounds__(256) void reduce_final_batch_kernel(
    const Desc* __restrict__ descs, const int32_t* __restrict__ list,
    const int64_t* __restrict__ part_off, const double* __restrict__ part,
    ReduceOut* __restrict__ reds, int drift) {
  const int i = list[blockIdx.x];
  const int64_t nn = (int64_t)descs[i].Lx * descs[i].Ly;
  reduce_final_body(part + 6 * part_off[i], reduce_blocks_hd(nn), nn, reds + i, 0, drift);
}

hipError_t launch_check_batch(bool fp32, const Desc* d_descs, int parity, const int32_t* d_list,
                              int n, int max_blocks, const int64_t* d_part_off, double* d_part,
                              ReduceOut* d_reds, int drift, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(reduce_batch_kernel<float>, dim3(max_blocks, n), dim3(kRedBS), 0, st, d_descs,
                       parity, d_list, d_part_off, d_part);
  else
    hipLaunchKernelGGL(reduce_batch_kernel<double>, dim3(max_blocks, n), dim3(kRedBS), 0, st, d_descs,
                       parity, d_list, d_part_off, d_part);
  hipLaunchKernelGGL(reduce_final_batch_kernel, dim3(n), dim3(256), 0, st, d_descs, d_list,
                     d_part_off, d_part, d_reds, drift);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* d_part, int nb, int64_t nn, ReduceOut* d_out,
                               int mode, int drift, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, stream, d_part, nb, nn, d_out,
                     mode, drift);
  return hipGetLastError();
}

// ---- population conversion (checkpoint / inspection) ----------------------
template <typename R>
__global__ void get_pops_kernel(const Desc* __restrict__ desc, int parity, int p0, int p1,
                                int64_t nn, double* __restrict__ out, int add_shift) {
  const Desc& d = *desc;
  const R* S = (const R*)d.S[parity];
  const double base = d.nbar + ((add_shift && d.shift) ? *d.shift : 0.0);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x)
    for (int i = p0; i < p1; ++i)
      out[(int64_t)(i - p0) * nn + k] =
          (double)S[pidx(i, k, k / d.Lx, d.Lx)] + rest_weight_hd(i, d.T) * base;
}

template <typename R>
__global__ void set_pops_kernel(const Desc* __restrict__ desc, int parity, int p0, int p1,
                                int64_t nn, const double* __restrict__ in, uint32_t step) {
  const Desc& d = *desc;
  R* S = (R*)d.S[parity];
  if (d.rng && blockIdx.x == 0 && threadIdx.x == 0) d.rng[parity] = step;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x)
    for (int i = p0; i < p1; ++i)
      S[pidx(i, k, k / d.Lx, d.Lx)] =
          (R)(in[(int64_t)(i - p0) * nn + k] - rest_weight_hd(i, d.T) * d.nbar);
}

hipError_t launch_get_pops(bool fp32, const Desc* d_desc, int parity, int p0, int p1, int64_t nn,
                           double* d_f, int add_shift, hipStream_t stream) {
  if (fp32)
    hipLaunchKernelGGL(get_pops_kernel<float>, dim3(grid_for(nn, 256)), dim3(256), 0, stream,
                       d_desc, parity, p0, p1, nn, d_f, add_shift);
  else
    hipLaunchKernelGGL(get_pops_kernel<double>, dim3(grid_for(nn, 256)), dim3(256), 0, stream,
                       d_desc, parity, p0, p1, nn, d_f, add_shift);
  return hipGetLastError();
}

hipError_t launch_set_pops(bool fp32, const Desc* d_desc, int parity, int p0, int p1, int64_t nn,
                           const double* d_f, int64_t step, hipStream_t stream) {
  if (fp32)
    hipLaunchKernelGGL(set_pops_kernel<float>, dim3(grid_for(nn, 256)), dim3(256), 0, stream,
                       d_desc, parity, p0, p1, nn, d_f, (uint32_t)step);
  else
    hipLaunchKernelGGL(set_pops_kernel<double>, dim3(grid_for(nn, 256)), dim3(256), 0, stream,
                       d_desc, parity, p0, p1, nn, d_f, (uint32_t)step);
  return hipGetLastError();
}

// ---- batch helpers for the learned surrogate --------------------------------
// Gather the moments of every instance (all the same size) into one block
// [count][3][Ly][Lx]; scatter fields back as equilibrium populations (the
// re-entry of Eq.(eqfunc) at u = u*) for the instances with mask != 0.
__global__ void gather_moments_kernel(const Desc* __restrict__ descs, int64_t nn,
                                      double* __restrict__ out) {
  const int i = blockIdx.y;
  const double* mom = descs[i].mom;
  double* o = out + (int64_t)i * 3 * nn;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 3 * nn;
       k += (int64_t)gridDim.x * blockDim.x)
    o[k] = mom[k];
}

// Re-entry of instance i (mask[i] != 0) at the fields [i][3][nn] (n, u*_x,
// u*_y): with from == null its populations become the equilibrium of
// Eq.(eqfunc) at those fields; otherwise they gain f_eq(fields) - f_eq(from)
// and keep their non-equilibrium part (with fields == from, bit for bit
// unchanged). The fields become the instance's moments.
template <typename R>
__global__ void scatter_eq_kernel(const Desc* __restrict__ descs, ReduceOut* __restrict__ red,
                                  int parity, int64_t nn, const double* __restrict__ fields,
                                  const double* __restrict__ from, const int32_t* __restrict__ mask) {
  const int i = blockIdx.y;
  if (!mask[i]) return;  // uniform per block
  const Desc& d = descs[i];
  // a drift shift measured on a replaced state does not apply to the new
  // one; an added equilibrium difference keeps the state's mass error
  if (!from && blockIdx.x == 0 && threadIdx.x == 0) red[i].shift = 0.0;
  R* S = (R*)d.S[parity];
  const double* f = fields + (int64_t)i * 3 * nn;
  const double* f0 = from ? from + (int64_t)i * 3 * nn : nullptr;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  auto feq = [&](int q, double n, double ux, double uy) {
    const double cu = cx(q) * ux + cy(q) * uy;
    return rest_weight_hd(q, d.T) * (n - d.nbar) +
           w[q] * n * (3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
  };
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nn;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double n = f[k], ux = f[nn + k], uy = f[2 * nn + k];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      R& s = S[pidx(q, k, k / d.Lx, d.Lx)];
      if (f0)
        s = (R)((double)s + (feq(q, n, ux, uy) - feq(q, f0[k], f0[nn + k], f0[2 * nn + k])));
      else
        s = (R)feq(q, n, ux, uy);
    }
    d.mom[k] = n;
    d.mom[nn + k] = ux;
    d.mom[2 * nn + k] = uy;
  }
}

hipError_t launch_gather_moments(const Desc* d_descs, int count, int64_t nn, double* out,
                                 hipStream_t st) {
  hipLaunchKernelGGL(gather_moments_kernel, dim3(grid_for(3 * nn, 256), count), dim3(256), 0, st,
                     d_descs, nn, out);
  return hipGetLastError();
}

hipError_t launch_scatter_eq(bool fp32, const Desc* d_descs, ReduceOut* d_red, int count,
                             int parity, int64_t nn, const double* fields, const double* from,
                             const int32_t* d_mask, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(scatter_eq_kernel<float>, dim3(grid_for(nn, 256), count), dim3(256), 0, st,
                       d_descs, d_red, parity, nn, fields, from, d_mask);
  else
    hipLaunchKernelGGL(scatter_eq_kernel<double>, dim3(grid_for(nn, 256), count), dim3(256), 0, st,
                       d_descs, d_red, parity, nn, fields, from, d_mask);
  return hipGetLastError();
}

}  // namespace lbk
