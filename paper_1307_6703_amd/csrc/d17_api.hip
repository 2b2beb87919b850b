// C ABI of the D2Q17 variant (include/lbd2q17.h): parameter checks, workspace
// layout, state bookkeeping and kernel launches. The arithmetic of the step
// lives in d17_device.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "d17_internal.h"
#include "lb_host.h"
#include "lbd2q17.h"

using d17k::Desc17;
using d17k::Reduce17;
using lbh::fail;

struct lb17_handle {
  lb_params p;
  hipStream_t st;
  Desc17 d;
  bool fp32;        // FP32 storage (fp32 = 1 or 2)
  int prec;         // lb_params.fp32
  double* fext;     // device, Lx values (F_ext,x / s)
  double* part;     // device, reduce partials
  Reduce17* red;    // device
  double* mom;      // device, n, ux, uy planes
  int parity;
  int64_t step;
  bool has_state, moments_valid, unstable, pending_shift;
  int threads, rows;  // 0: default
};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double scale_s() {
  double s;
  d17k::lattice17(nullptr, nullptr, nullptr, &s);
  return s;
}

lb_status validate17(const lb_params* p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (p->Lx < 1) return fail(LB_EINVAL, "Lx must be >= 1 (got %d)", p->Lx);
  if (p->Ly < 4) return fail(LB_EINVAL, "Ly must be >= 4 (got %d)", p->Ly);
  if (p->y_periodic != 1)
    return fail(LB_EINVAL, "D2Q17 lattices are periodic in y (the wall rule is D2Q9's)");
  if (p->U != 0.0) return fail(LB_EINVAL, "D2Q17 lattices have no walls: U must be 0");
  if (p->collision != 0) return fail(LB_EINVAL, "D2Q17 lattices collide with BGK only");
  if (p->fp32 < 0 || p->fp32 > 2) return fail(LB_EINVAL, "fp32 must be 0, 1 or 2 (got %d)", p->fp32);
  if ((int64_t)p->Lx * p->Ly * 17 * (p->fp32 ? 4 : 8) >= ((int64_t)1 << 31))
    return fail(LB_EINVAL, "17*Lx*Ly*(4|8) bytes must be < 2 GiB");
  if (!(p->T > 0.0 && p->T <= 1.5)) return fail(LB_EINVAL, "T must be in (0, 1.5] (got %g)", p->T);
  if (!(std::sqrt(scale_s()) * p->tau > 0.5) || !std::isfinite(p->tau))
    return fail(LB_EINVAL, "need sqrt(s)*tau > 1/2 (got tau=%g)", p->tau);
  if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa)) return fail(LB_EINVAL, "kappa must be >= 0");
  if (!std::isfinite(p->N) || !std::isfinite(p->Q)) return fail(LB_EINVAL, "N, Q must be finite");
  if (p->check_every < 0) return fail(LB_EINVAL, "check_every must be >= 0");
  if (p->drift_correct != 0 && p->drift_correct != 1)
    return fail(LB_EINVAL, "drift_correct must be 0 or 1");
  if (p->fext_x)
    for (int x = 0; x < p->Lx; ++x)
      if (!std::isfinite(p->fext_x[x])) return fail(LB_EINVAL, "fext_x[%d] is not finite", x);
  return LB_OK;
}

struct Layout17 {
  size_t red, fext, part, mom, S0, S1, total;
};

Layout17 layout17(const lb_params* p) {
  const size_t nn = (size_t)p->Lx * p->Ly;
  const size_t rs = p->fp32 ? 4 : 8;
  Layout17 L;
  size_t o = 0;
  L.red = o;
  o = up(o + sizeof(Reduce17));
  L.fext = o;
  o = up(o + (size_t)p->Lx * 8);
  L.part = o;
  o = up(o + (size_t)d17k::reduce17_blocks((int64_t)nn) * 6 * 8);
  L.mom = o;
  o = up(o + 3 * nn * 8);
  L.S0 = o;
  o = up(o + 17 * nn * rs);
  L.S1 = o;
  o = up(o + 17 * nn * rs);
  L.total = o;
  return L;
}

int64_t nodes(const lb17_handle* h) { return (int64_t)h->p.Lx * h->p.Ly; }

// Default launch, from measurements on 8192 x 2048 (FP32) and 8192 x 1024
// (FP64): wide strips where the lattice is wide (512 threads for FP32
// arithmetic, 256 for FP64 arithmetic, whose registers allow fewer waves),
// narrower ones for narrow lattices; rows so that the grid holds about 4096
// (FP32) or 2048 (FP64 arithmetic) workgroups, in multiples of 8, at least 8.
// Neighbouring chunks share the rows they both read through the cache
// (alternating march directions).
void launch_shape(const lb17_handle* h, int* threads, int* rows) {
  const int Lx = h->p.Lx;
  const bool a32 = h->prec == 1;  // FP32 arithmetic
  int t = h->threads;
  if (!t) t = Lx >= 2048 ? (a32 ? 512 : 256) : Lx >= 256 ? 256 : Lx >= 96 ? 128 : 64;
  int r = h->rows;
  if (!r) {
    const int strips = (Lx + t - 5) / (t - 4);
    const int chunks = std::max(1, (a32 ? 4096 : 2048) / strips);
    r = (h->p.Ly + chunks - 1) / chunks;
    r = std::max(8, r / 8 * 8);
  }
  *threads = t;
  *rows = std::min(r, h->p.Ly);
}

lb_status read_status(lb17_handle* h, Reduce17* out = nullptr) {
  Reduce17 r;
  HIPCHK(hipMemcpyAsync(&r, h->red, sizeof r, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (r.status & 1u) h->unstable = true;
  if (out) *out = r;
  return LB_OK;
}

lb_status enqueue_check(lb17_handle* h, int mode) {
  const int nb = d17k::reduce17_blocks(nodes(h));
  HIPCHK(d17k::launch_reduce17(h->fp32, h->d, h->parity, h->part, h->pending_shift ? 1 : 0, h->st));
  HIPCHK(d17k::launch_reduce17_final(h->part, nb, nodes(h), h->red, mode,
                                     h->p.drift_correct && h->fp32, h->st));
  return LB_OK;
}

// A fresh state in S[parity]: reference mass, counters.
lb_status fresh_state(lb17_handle* h, int64_t step) {
  h->step = step;
  h->unstable = false;
  h->pending_shift = false;
  h->has_state = true;
  Reduce17 z;
  std::memset(&z, 0, sizeof z);
  HIPCHK(hipMemcpyAsync(h->red, &z, sizeof z, hipMemcpyHostToDevice, h->st));
  lb_status r = enqueue_check(h, 1);
  if (r != LB_OK) return r;
  HIPCHK(hipStreamSynchronize(h->st));
  return LB_OK;
}

void fill_desc(lb17_handle* h, char* ws, const Layout17& L) {
  const lb_params& p = h->p;
  Desc17& d = h->d;
  std::memset(&d, 0, sizeof d);
  d.S[0] = ws + L.S0;
  d.S[1] = ws + L.S1;
  d.fext = h->fext;
  d.shift = &h->red->shift;
  d.Lx = p.Lx;
  d.Ly = p.Ly;
  d.nbar = 0.0;
  const double s = scale_s();
  d.T = p.T;
  d.omega = 1.0 / (std::sqrt(s) * p.tau);
  d.kappa_l = p.kappa / s;
  d.N = p.N;
  d.M = (1.0 - 2.0 * p.N) / 4.0;
  d.Q = p.Q;
  d.R = (1.0 - p.Q) / 2.0;
  d.ps = 1.0 / s;
  double w[17];
  d17k::lattice17(nullptr, nullptr, w, nullptr);
  const int rep[5] = {0, 1, 5, 9, 13};  // one direction per shell
  const double cc[5] = {0.0, 1.0, 2.0, 8.0, 9.0};
  for (int k = 0; k < 5; ++k) {
    d.w[k] = w[rep[k]];
    d.wr[k] = w[rep[k]] * (1.0 + 0.5 * (p.T - 1.0) * (s * cc[k] - 2.0));
    d.owr[k] = d.omega * d.wr[k];
    d.a1[k] = s * (1.0 + 0.5 * (p.T - 1.0) * (s * cc[k] - 4.0));
  }
  d.h1 = 0.5 * s;
  d.h2 = 0.5 * s * s;
  d.h3 = s * s * s / 6.0;
}

// nsteps steps in the current launch shape; the last one writes the moments.
lb_status step_impl17(lb17_handle* h, int64_t nsteps) {
  int threads, rows;
  launch_shape(h, &threads, &rows);
  for (int64_t k = 0; k < nsteps; ++k) {
    int flags = (k == nsteps - 1) ? d17k::kWriteMoments : 0;
    if (h->pending_shift) flags |= d17k::kApplyShift;
    HIPCHK(d17k::launch_step17(h->prec, threads, rows, h->d, h->parity, flags, h->mom,
                               (uint32_t)h->step, h->st));
    h->parity ^= 1;
    h->pending_shift = false;
    h->step += 1;
    if (h->p.check_every > 0 && h->step % h->p.check_every == 0) {
      lb_status r = enqueue_check(h, 0);
      if (r != LB_OK) return r;
      h->pending_shift = h->p.drift_correct && h->fp32;
    }
  }
  if (nsteps > 0) h->moments_valid = true;
  return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb17_lattice(int32_t cx[17], int32_t cy[17], double w[17], double* s) {
  int ix[17], iy[17];
  d17k::lattice17(ix, iy, w, s);
  for (int i = 0; i < 17; ++i) {
    if (cx) cx[i] = ix[i];
    if (cy) cy[i] = iy[i];
  }
  return LB_OK;
}

lb_status lb17_workspace_bytes(const lb_params* p, size_t* bytes) {
  lb_status r = validate17(p);
  if (r != LB_OK) return r;
  if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
  *bytes = layout17(p).total;
  return LB_OK;
}

lb_status lb17_create(const lb_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                      lb17_handle** out) {
  lb_status r = validate17(p);
  if (r != LB_OK) return r;
  if (!out) return fail(LB_EINVAL, "out is NULL");
  if (!dev_ws || ((uintptr_t)dev_ws % kAlign)) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  const Layout17 L = layout17(p);
  if (ws_bytes < L.total) return fail(LB_ENOMEM, "workspace too small (%zu < %zu)", ws_bytes, L.total);
  lb17_handle* h = new (std::nothrow) lb17_handle();
  if (!h) return fail(LB_ENOMEM, "out of host memory");
  h->p = *p;
  h->p.fext_x = nullptr;
  h->st = (hipStream_t)hip_stream;
  h->fp32 = p->fp32 != 0;
  h->prec = p->fp32;
  char* ws = (char*)dev_ws;
  h->red = (Reduce17*)(ws + L.red);
  h->fext = (double*)(ws + L.fext);
  h->part = (double*)(ws + L.part);
  h->mom = (double*)(ws + L.mom);
  fill_desc(h, ws, L);
  std::vector<double> fx(p->Lx, 0.0);
  const double s = scale_s();
  if (p->fext_x)
    for (int x = 0; x < p->Lx; ++x) fx[x] = p->fext_x[x] / s;
  hipError_t e = hipMemcpyAsync(h->fext, fx.data(), fx.size() * 8, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) {
    delete h;
    return fail(LB_EDEVICE, "fext upload failed: %s", hipGetErrorString(e));
  }
  *out = h;
  return LB_OK;
}

lb_status lb17_init_lattice(lb17_handle* h, const double* n0, const double* ux0,
                            const double* uy0) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!n0) return fail(LB_EINVAL, "n0 is NULL");
  const int64_t nn = nodes(h);
  double sum = 0.0;
  for (int64_t k = 0; k < nn; ++k) {
    if (!(n0[k] > 0.0 && n0[k] < 3.0)) return fail(LB_EINVAL, "n0[%lld] outside (0, 3)", (long long)k);
    sum += n0[k];
  }
  for (const double* u : {ux0, uy0})
    if (u)
      for (int64_t k = 0; k < nn; ++k)
        if (!std::isfinite(u[k])) return fail(LB_EINVAL, "initial velocity is not finite");
  h->d.nbar = h->fp32 ? sum / (double)nn : 0.0;
  HIPCHK(hipMemcpyAsync(h->mom, n0, nn * 8, hipMemcpyHostToDevice, h->st));
  if (ux0) HIPCHK(hipMemcpyAsync(h->mom + nn, ux0, nn * 8, hipMemcpyHostToDevice, h->st));
  else HIPCHK(hipMemsetAsync(h->mom + nn, 0, nn * 8, h->st));
  if (uy0) HIPCHK(hipMemcpyAsync(h->mom + 2 * nn, uy0, nn * 8, hipMemcpyHostToDevice, h->st));
  else HIPCHK(hipMemsetAsync(h->mom + 2 * nn, 0, nn * 8, h->st));
  h->parity = 0;
  HIPCHK(d17k::launch_init17(h->fp32, h->d, 0, h->mom, h->mom + nn, h->mom + 2 * nn, h->st));
  lb_status r = fresh_state(h, 0);
  if (r != LB_OK) return r;
  h->moments_valid = true;
  return LB_OK;
}

lb_status lb17_init_lattice_device(lb17_handle* h, const double* d_n0, const double* d_ux0,
                                   const double* d_uy0) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!d_n0) return fail(LB_EINVAL, "n0 is NULL");
  const int64_t nn = nodes(h);
  // stage the fields in the moment planes, then check them on the host
  // (the bounds and the mean density)
  HIPCHK(hipMemcpyAsync(h->mom, d_n0, nn * 8, hipMemcpyDeviceToDevice, h->st));
  if (d_ux0) HIPCHK(hipMemcpyAsync(h->mom + nn, d_ux0, nn * 8, hipMemcpyDeviceToDevice, h->st));
  else HIPCHK(hipMemsetAsync(h->mom + nn, 0, nn * 8, h->st));
  if (d_uy0) HIPCHK(hipMemcpyAsync(h->mom + 2 * nn, d_uy0, nn * 8, hipMemcpyDeviceToDevice, h->st));
  else HIPCHK(hipMemsetAsync(h->mom + 2 * nn, 0, nn * 8, h->st));
  std::vector<double> n0(nn), u(2 * nn);
  HIPCHK(hipMemcpyAsync(n0.data(), h->mom, nn * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(u.data(), h->mom + nn, 2 * nn * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  double sum = 0.0;
  for (int64_t k = 0; k < nn; ++k) {
    if (!(n0[k] > 0.0 && n0[k] < 3.0)) return fail(LB_EINVAL, "n0[%lld] outside (0, 3)", (long long)k);
    sum += n0[k];
  }
  for (int64_t k = 0; k < 2 * nn; ++k)
    if (!std::isfinite(u[k])) return fail(LB_EINVAL, "initial velocity is not finite");
  h->d.nbar = h->fp32 ? sum / (double)nn : 0.0;
  h->parity = 0;
  HIPCHK(d17k::launch_init17(h->fp32, h->d, 0, h->mom, h->mom + nn, h->mom + 2 * nn, h->st));
  lb_status r = fresh_state(h, 0);
  if (r != LB_OK) return r;
  h->moments_valid = true;
  return LB_OK;
}

lb_status lb17_get_moments_device(lb17_handle* h, double* d_n, double* d_ux, double* d_uy) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!h->moments_valid) return fail(LB_ESTATE, "no moments: init the lattice or take a step");
  const int64_t nn = nodes(h);
  if (d_n) HIPCHK(hipMemcpyAsync(d_n, h->mom, nn * 8, hipMemcpyDeviceToDevice, h->st));
  if (d_ux) HIPCHK(hipMemcpyAsync(d_ux, h->mom + nn, nn * 8, hipMemcpyDeviceToDevice, h->st));
  if (d_uy) HIPCHK(hipMemcpyAsync(d_uy, h->mom + 2 * nn, nn * 8, hipMemcpyDeviceToDevice, h->st));
  return LB_OK;
}

lb_status lb17_step_n(lb17_handle* h, int64_t nsteps) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  if (h->unstable) return fail(LB_ESTATE, "a stability check failed; restart the lattice");
  return step_impl17(h, nsteps);
}

lb_status lb17_get_moments(lb17_handle* h, double* n, double* ux, double* uy) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!h->moments_valid) return fail(LB_ESTATE, "no moments: init the lattice or take a step");
  const int64_t nn = nodes(h);
  if (n) HIPCHK(hipMemcpyAsync(n, h->mom, nn * 8, hipMemcpyDeviceToHost, h->st));
  if (ux) HIPCHK(hipMemcpyAsync(ux, h->mom + nn, nn * 8, hipMemcpyDeviceToHost, h->st));
  if (uy) HIPCHK(hipMemcpyAsync(uy, h->mom + 2 * nn, nn * 8, hipMemcpyDeviceToHost, h->st));
  lb_status r = read_status(h);
  if (r != LB_OK) return r;
  if (h->unstable) return fail(LB_EUNSTABLE, "a stability check failed");
  return LB_OK;
}

lb_status lb17_reduce(lb17_handle* h, double out[6]) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!out) return fail(LB_EINVAL, "out is NULL");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  lb_status r = enqueue_check(h, 2);
  if (r != LB_OK) return r;
  Reduce17 ro;
  if ((r = read_status(h, &ro)) != LB_OK) return r;
  out[0] = ro.mass;
  out[1] = ro.jx;
  out[2] = ro.jy;
  out[3] = ro.nmin;
  out[4] = ro.nmax;
  out[5] = ro.nonfinite;
  if (h->unstable) return fail(LB_EUNSTABLE, "a stability check failed");
  return LB_OK;
}

lb_status lb17_get_populations(lb17_handle* h, double* f) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!f) return fail(LB_EINVAL, "f is NULL");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  const int64_t nn = nodes(h);
  // the buffer the next step writes stages one FP64 plane at a time
  double* stage = (double*)h->d.S[h->parity ^ 1];
  for (int i = 0; i < 17; ++i) {
    HIPCHK(d17k::launch_get_pops17(h->fp32, h->d, h->parity, i, stage, h->pending_shift ? 1 : 0,
                                   h->st));
    HIPCHK(hipMemcpyAsync(f + i * nn, stage, nn * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  return LB_OK;
}

lb_status lb17_set_populations(lb17_handle* h, const double* f, int64_t step) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!f) return fail(LB_EINVAL, "f is NULL");
  if (step < 0) return fail(LB_EINVAL, "step must be >= 0");
  const int64_t nn = nodes(h);
  double sum = 0.0;
  for (int64_t k = 0; k < 17 * nn; ++k) {
    if (!std::isfinite(f[k])) return fail(LB_EINVAL, "f has a non-finite value");
    sum += f[k];
  }
  h->parity = 0;
  h->d.nbar = h->fp32 ? sum / (double)nn : 0.0;
  double* stage = (double*)h->d.S[1];
  for (int i = 0; i < 17; ++i) {
    HIPCHK(hipMemcpyAsync(stage, f + i * nn, nn * 8, hipMemcpyHostToDevice, h->st));
    HIPCHK(d17k::launch_set_pops17(h->fp32, h->d, 0, i, stage, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  h->moments_valid = false;
  return fresh_state(h, step);
}

lb_status lb17_set_launch(lb17_handle* h, int32_t threads, int32_t rows) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512)
    return fail(LB_EINVAL, "threads must be 0, 64, 128, 256 or 512 (got %d)", threads);
  if (rows < 0) return fail(LB_EINVAL, "rows must be >= 0");
  h->threads = threads;
  h->rows = rows;
  return LB_OK;
}

lb_status lb17_get_launch(lb17_handle* h, int32_t* threads, int32_t* rows, int32_t* blocks) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  int t, r;
  launch_shape(h, &t, &r);
  if (threads) *threads = t;
  if (rows) *rows = r;
  if (blocks) *blocks = ((h->p.Lx + t - 5) / (t - 4)) * ((h->p.Ly + r - 1) / r);
  return LB_OK;
}

lb_status lb17_autotune(lb17_handle* h, int32_t nsteps, int32_t* threads, int32_t* rows,
                        double* ms_per_step) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (nsteps < 1) return fail(LB_EINVAL, "nsteps must be >= 1");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  if (h->unstable) return fail(LB_ESTATE, "a stability check failed; restart the lattice");
  // candidates: every strip width up to about twice the lattice width, and
  // for each the default chunk height and a few fixed ones
  std::vector<std::pair<int, int>> cand;
  const int t0 = h->threads, r0 = h->rows;
  for (int t : {64, 128, 256, 512}) {
    if (t > 64 && h->p.Lx + 4 <= t / 2) continue;
    h->threads = t;
    h->rows = 0;
    int dt, dr;
    launch_shape(h, &dt, &dr);
    std::vector<int> rs = {dr, 8, 16, 32, 64};
    std::sort(rs.begin(), rs.end());
    rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
    for (int rw : rs)
      if (rw <= h->p.Ly) cand.push_back({t, rw});
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = 1e300;
  int bt = t0, br = r0;
  lb_status r = LB_OK;
  for (const auto& c : cand) {
    h->threads = c.first;
    h->rows = c.second;
    if ((r = step_impl17(h, 1)) != LB_OK) break;  // warm-up
    if (hipEventRecord(e0, h->st) != hipSuccess) { r = fail(LB_EDEVICE, "event record failed"); break; }
    if ((r = step_impl17(h, nsteps)) != LB_OK) break;
    if (hipEventRecord(e1, h->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      r = fail(LB_EDEVICE, "event sync failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms / nsteps < best) {
      best = ms / nsteps;
      bt = c.first;
      br = c.second;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->threads = bt;
  h->rows = br;
  if (r != LB_OK) return r;
  if (threads) *threads = bt;
  if (rows) *rows = br;
  if (ms_per_step) *ms_per_step = best;
  return LB_OK;
}

lb_status lb17_get_step(lb17_handle* h, int64_t* step) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!step) return fail(LB_EINVAL, "step is NULL");
  *step = h->step;
  return LB_OK;
}

lb_status lb17_destroy(lb17_handle* h) {
  if (!h) return LB_OK;
  hipError_t e = hipStreamSynchronize(h->st);
  delete h;
  if (e != hipSuccess) return fail(LB_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
  return LB_OK;
}

}  // extern "C"
