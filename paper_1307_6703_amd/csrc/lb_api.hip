// Host side of the C ABI declared in include/lbvdw.h: parameter checks,
// workspace layout, tiling, step scheduling, checks and checkpoints. Every
// step of the method runs in the kernels of lb_device.hip.
#include <hip/hip_runtime.h>

#include <cstring>

#include "lb_host.h"

namespace lbh {
thread_local std::string g_err;
}  // namespace lbh

using namespace lbh;

struct lb_handle {
  lb_params p{};
  std::vector<double> fext;  // host copy
  char* ws = nullptr;
  Layout L{};
  hipStream_t st = nullptr;
  int device = 0;
  Desc hdesc{};  // host mirror of the device descriptor
  Desc* ddesc = nullptr;
  ReduceOut* dred = nullptr;
  Tile* dtiles = nullptr;   // tiles of the current launch shape
  Tile* dtiles1 = nullptr;  // one-step tiles for single steps of a two-step shape
  double* dpart = nullptr;
  double* dmom = nullptr;
  double* dstage = nullptr;
  int parity = 0;
  int64_t step = 0;
  bool has_state = false;
  bool moments_valid = false;
  bool unstable = false;
  bool pending_shift = false;
  int threads = 128, rows = 16, ntiles = 0;
  int fuse = 1;  // steps per launch of the current shape
  int threads1 = 128, ntiles1 = 0;
};

namespace {

bool fp32_of(const lb_handle* h) { return h->p.fp32 != 0; }  // FP32 storage
int prec(const lb_handle* h) { return prec_of(&h->p); }
int64_t nodes(const lb_handle* h) { return (int64_t)h->p.Lx * h->p.Ly; }

lb_status upload_desc(lb_handle* h) {
  HIPCHK(hipMemcpyAsync(h->ddesc, &h->hdesc, sizeof(Desc), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return LB_OK;
}

// Upload the tiles of a shape; fuse = steps per launch (1 or 2).
lb_status upload_tiles(lb_handle* h, Tile* dst, int threads, int rows, int fuse, int* ntiles) {
  std::vector<Tile> t = make_tiles(0, h->p.Lx, h->p.Ly, threads, rows, fuse == 2 ? 7 : 3, false,
                                   fuse == 2 && !h->p.y_periodic);
  if ((int)t.size() > h->L.max_tiles) return fail(LB_EINVAL, "too many tiles for the workspace");
  HIPCHK(hipMemcpyAsync(dst, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  *ntiles = (int)t.size();
  return LB_OK;
}

lb_status set_tiles(lb_handle* h, int threads, int rows, int fuse = 1) {
  if (fuse == 2) {
    if (prec(h) != lbk::kFP32)
      return fail(LB_EINVAL, "two steps per launch need FP32 storage and arithmetic (fp32 = 1)");
    if (!fused_threads_ok(threads))
      return fail(LB_EINVAL, "two steps per launch: threads must be 64, 128, 192 or 256 (got %d)", threads);
  } else if (threads != 64 && threads != 128 && threads != 256 && threads != 320 &&
             !(threads == 512 && prec(h) == lbk::kFP32)) {
    return fail(LB_EINVAL, "threads must be 64, 128, 256, 320 or 512 (fp32 = 1 only) (got %d)", threads);
  }
  if (rows < 1) return fail(LB_EINVAL, "rows must be >= 1");
  rows = std::max(std::min(rows, h->p.Ly), std::min(kMinRows, h->p.Ly));
  int nt = 0;
  lb_status r = upload_tiles(h, h->dtiles, threads, rows, fuse, &nt);
  if (r != LB_OK) return r;
  if (fuse == 2) {  // single steps (odd counts, steps before a check) use the default shape
    const int t1 = default_threads(&h->p);
    if ((r = upload_tiles(h, h->dtiles1, t1, default_rows(&h->p, t1), 1, &h->ntiles1)) != LB_OK)
      return r;
    h->threads1 = t1;
  }
  h->threads = threads;
  h->rows = rows;
  h->ntiles = nt;
  h->fuse = fuse;
  return LB_OK;
}

// Read the sticky status word; sets h->unstable.
lb_status read_status(lb_handle* h, ReduceOut* out = nullptr) {
  ReduceOut r;
  HIPCHK(hipMemcpyAsync(&r, h->dred, sizeof r, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (out) *out = r;
  if (r.status & 1u) h->unstable = true;
  return LB_OK;
}

lb_status enqueue_check(lb_handle* h, int mode) {
  const int nb = lbk::reduce_blocks(nodes(h));
  HIPCHK(lbk::launch_reduce(fp32_of(h), h->ddesc, h->parity, nodes(h), h->dpart,
                            (mode == 2 && h->pending_shift) ? 1 : 0, h->st));
  HIPCHK(lbk::launch_reduce_final(h->dpart, nb, nodes(h), h->dred, mode,
                                  mode == 0 ? h->p.drift_correct : 0, h->st));
  return LB_OK;
}

lb_status after_restart(lb_handle* h) {
  h->unstable = false;
  h->pending_shift = false;
  lb_status s = enqueue_check(h, 1);
  if (s != LB_OK) return s;
  s = read_status(h);
  if (s != LB_OK) return s;
  if (h->unstable) return fail(LB_EUNSTABLE, "initial state has non-finite values or n outside (0, 3)");
  h->has_state = true;
  return LB_OK;
}

// With a two-step shape, pairs of steps run as one launch unless a check
// falls after the first of them or one step is left; those run alone.
lb_status step_impl(lb_handle* h, int64_t nsteps, bool moments_last) {
  const int ce = h->p.check_every;
  for (int64_t s = 0; s < nsteps;) {
    const bool pair = h->fuse == 2 && nsteps - s >= 2 && !(ce > 0 && (h->step + 1) % ce == 0);
    const int n = pair ? 2 : 1;
    int flags = 0;
    if (moments_last && s + n == nsteps) flags |= lbk::kWriteMoments;
    if (h->pending_shift) flags |= lbk::kApplyShift;
    if (pair)
      HIPCHK(lbk::launch_step2(h->threads, h->p.collision != 0, h->ddesc, h->dtiles, h->ntiles, h->parity,
                               flags | (h->p.y_periodic ? lbk::kYPeriodic : lbk::kYWalls), h->st));
    else if (h->fuse == 2)
      HIPCHK(lbk::launch_step(prec(h), h->p.collision != 0, h->threads1, h->ddesc, h->dtiles1, h->ntiles1, h->parity,
                              flags, h->st));
    else
      HIPCHK(lbk::launch_step(prec(h), h->p.collision != 0, h->threads, h->ddesc, h->dtiles, h->ntiles, h->parity,
                              flags, h->st));
    h->pending_shift = false;
    h->parity ^= 1;
    h->step += n;
    s += n;
    if (h->p.check_every > 0 && h->step % h->p.check_every == 0) {
      lb_status r = enqueue_check(h, 0);
      if (r != LB_OK) return r;
      h->pending_shift = h->p.drift_correct != 0;
    }
  }
  return LB_OK;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

lb_status lb_workspace_bytes(const lb_params* p, size_t* bytes) {
  lb_status s = validate(p);
  if (s != LB_OK) return s;
  if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
  *bytes = layout_for(p).total;
  return LB_OK;
}

lb_status lb_create(const lb_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream,
                    lb_handle** out) {
  lb_status s = validate(p);
  if (s != LB_OK) return s;
  if (!out) return fail(LB_EINVAL, "out is NULL");
  if (!dev_ws) return fail(LB_EINVAL, "workspace is NULL");
  if ((uintptr_t)dev_ws % kAlign) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  Layout L = layout_for(p);
  if (ws_bytes < L.total)
    return fail(LB_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  lb_handle* h = new lb_handle();
  h->p = *p;
  h->p.fext_x = nullptr;
  h->L = L;
  h->ws = (char*)dev_ws;
  h->st = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(LB_EDEVICE, "no current HIP device");
  }
  h->ddesc = (Desc*)(h->ws + L.desc);
  h->dred = (ReduceOut*)(h->ws + L.red);
  h->dtiles = (Tile*)(h->ws + L.tiles);
  h->dtiles1 = (Tile*)(h->ws + L.tiles1);
  h->dpart = (double*)(h->ws + L.part);
  h->dmom = (double*)(h->ws + L.mom);
  h->dstage = (double*)(h->ws + L.stage);
  const double tau_l = std::sqrt(3.0) * p->tau;
  Desc& d = h->hdesc;
  d.S[0] = h->ws + L.S0;
  d.S[1] = h->ws + L.S1;
  d.fext3 = h->ws + L.fext;
  d.mom = h->dmom;
  d.shift = &h->dred->shift;
  d.rng = h->dred->rng_step;
  d.Lx = p->Lx;
  d.Ly = p->Ly;
  d.periodic = p->y_periodic;
  d.reg = p->collision;
  d.nbar = 0.0;
  d.T = p->T;
  d.omega = 1.0 / tau_l;
  d.kappa3 = p->kappa / 3.0;
  d.N = p->N;
  d.M = (1.0 - 2.0 * p->N) / 4.0;
  d.Q = p->Q;
  d.R = (1.0 - p->Q) / 2.0;
  d.U = p->U;
  // external force table, converted to lattice units (F_l = F_p / 3)
  h->fext.assign(p->Lx, 0.0);
  if (p->fext_x) std::copy(p->fext_x, p->fext_x + p->Lx, h->fext.begin());
  lb_status r = LB_OK;
  auto cleanup = [&](lb_status e) { delete h; return e; };
  if (prec_of(p) == lbk::kFP32) {
    std::vector<float> f3(p->Lx);
    for (int x = 0; x < p->Lx; ++x) f3[x] = (float)(h->fext[x] / 3.0);
    if (hipMemcpyAsync(h->ws + L.fext, f3.data(), f3.size() * 4, hipMemcpyHostToDevice, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
      return cleanup(fail(LB_EDEVICE, "uploading the force table failed"));
  } else {
    std::vector<double> f3(p->Lx);
    for (int x = 0; x < p->Lx; ++x) f3[x] = h->fext[x] / 3.0;
    if (hipMemcpyAsync(h->ws + L.fext, f3.data(), f3.size() * 8, hipMemcpyHostToDevice, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
      return cleanup(fail(LB_EDEVICE, "uploading the force table failed"));
  }
  ReduceOut z;
  std::memset(&z, 0, sizeof z);
  if (hipMemcpyAsync(h->dred, &z, sizeof z, hipMemcpyHostToDevice, h->st) != hipSuccess)
    return cleanup(fail(LB_EDEVICE, "clearing the check block failed"));
  if ((r = upload_desc(h)) != LB_OK) return cleanup(r);
  // default shape: two steps per launch for FP32 lattices of at least 2^20
  // nodes whose strips are mostly interior columns, else one step per launch;
  // 256-thread strips where their columns exceed Lx by at most 3% (wider
  // strips stream longer pieces of each row), else 128
  if (prec_of(p) == lbk::kFP32 && (int64_t)p->Lx * p->Ly >= ((int64_t)1 << 20) &&
      p->Lx >= 256) {
    const int64_t cols256 = (int64_t)((p->Lx + 241) / 242) * 242;
    const int th = cols256 * 100 <= (int64_t)p->Lx * 103 ? 256 : 128;
    if ((r = set_tiles(h, th, fused_default_rows(p, th), 2)) != LB_OK) return cleanup(r);
  } else {
    const int th = default_threads(p);
    if ((r = set_tiles(h, th, default_rows(p, th))) != LB_OK) return cleanup(r);
  }
  *out = h;
  return LB_OK;
}

static lb_status init_common(lb_handle* h, const double* d_n0, const double* d_ux,
                             const double* d_uy, double nbar) {
  h->hdesc.nbar = h->p.fp32 ? nbar : 0.0;
  lb_status r = upload_desc(h);
  if (r != LB_OK) return r;
  h->parity = 0;
  h->step = 0;
  HIPCHK(lbk::launch_init(fp32_of(h), h->ddesc, 0, d_n0, d_ux, d_uy, nodes(h), h->st));
  r = after_restart(h);
  if (r != LB_OK) return r;
  h->moments_valid = true;
  return LB_OK;
}

lb_status lb_init_lattice(lb_handle* h, const double* n0, const double* ux0, const double* uy0) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!n0) return fail(LB_EINVAL, "n0 is NULL");
  const int64_t nn = nodes(h);
  double sum = 0.0;
  for (int64_t k = 0; k < nn; ++k) {
    if (!(n0[k] > 0.0 && n0[k] < 3.0))
      return fail(LB_EINVAL, "n0[%lld] = %g is outside (0, 3)", (long long)k, n0[k]);
    sum += n0[k];
    if (ux0 && !std::isfinite(ux0[k])) return fail(LB_EINVAL, "ux0[%lld] is not finite", (long long)k);
    if (uy0 && !std::isfinite(uy0[k])) return fail(LB_EINVAL, "uy0[%lld] is not finite", (long long)k);
  }
  // stage the fields in the moments buffer; the init kernel reads them there
  HIPCHK(hipMemcpyAsync(h->dmom, n0, nn * 8, hipMemcpyHostToDevice, h->st));
  if (ux0) HIPCHK(hipMemcpyAsync(h->dmom + nn, ux0, nn * 8, hipMemcpyHostToDevice, h->st));
  if (uy0) HIPCHK(hipMemcpyAsync(h->dmom + 2 * nn, uy0, nn * 8, hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  lb_status r = init_common(h, h->dmom, ux0 ? h->dmom + nn : nullptr, uy0 ? h->dmom + 2 * nn : nullptr,
                            sum / (double)nn);
  return r;
}

lb_status lb_init_lattice_device(lb_handle* h, const double* d_n0, const double* d_ux0,
                                 const double* d_uy0) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!d_n0) return fail(LB_EINVAL, "n0 is NULL");
  const int64_t nn = nodes(h);
  // the mean density (FP32 reference) comes from the FP64 reduction of the
  // initial state built with nbar = 0 first
  std::vector<double> n0(nn);
  HIPCHK(hipMemcpyAsync(n0.data(), d_n0, nn * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  double sum = 0.0;
  for (int64_t k = 0; k < nn; ++k) {
    if (!(n0[k] > 0.0 && n0[k] < 3.0))
      return fail(LB_EINVAL, "n0[%lld] = %g is outside (0, 3)", (long long)k, n0[k]);
    sum += n0[k];
  }
  return init_common(h, d_n0, d_ux0, d_uy0, sum / (double)nn);
}

lb_status lb_step_n(lb_handle* h, int64_t nsteps) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state: call lb_init_lattice first");
  if (h->unstable) return fail(LB_ESTATE, "lattice was flagged unstable; restart it");
  if (nsteps == 0) return LB_OK;
  lb_status r = step_impl(h, nsteps, true);
  if (r != LB_OK) return r;
  h->moments_valid = true;
  return LB_OK;
}

lb_status lb_get_moments_device(lb_handle* h, double* d_n, double* d_ux, double* d_uy) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!h->moments_valid) return fail(LB_ESTATE, "no moments: init the lattice or take a step");
  const int64_t nn = nodes(h);
  if (d_n) HIPCHK(hipMemcpyAsync(d_n, h->dmom, nn * 8, hipMemcpyDeviceToDevice, h->st));
  if (d_ux) HIPCHK(hipMemcpyAsync(d_ux, h->dmom + nn, nn * 8, hipMemcpyDeviceToDevice, h->st));
  if (d_uy) HIPCHK(hipMemcpyAsync(d_uy, h->dmom + 2 * nn, nn * 8, hipMemcpyDeviceToDevice, h->st));
  return LB_OK;
}

lb_status lb_get_moments(lb_handle* h, double* n, double* ux, double* uy) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!h->moments_valid) return fail(LB_ESTATE, "no moments: init the lattice or take a step");
  const int64_t nn = nodes(h);
  if (n) HIPCHK(hipMemcpyAsync(n, h->dmom, nn * 8, hipMemcpyDeviceToHost, h->st));
  if (ux) HIPCHK(hipMemcpyAsync(ux, h->dmom + nn, nn * 8, hipMemcpyDeviceToHost, h->st));
  if (uy) HIPCHK(hipMemcpyAsync(uy, h->dmom + 2 * nn, nn * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  lb_status r = read_status(h);
  if (r != LB_OK) return r;
  if (h->unstable) return fail(LB_EUNSTABLE, "a stability check failed");
  return LB_OK;
}

lb_status lb_reduce(lb_handle* h, double out[6]) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!out) return fail(LB_EINVAL, "out is NULL");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  lb_status r = enqueue_check(h, 2);
  if (r != LB_OK) return r;
  ReduceOut ro;
  if ((r = read_status(h, &ro)) != LB_OK) return r;
  out[0] = ro.mass; out[1] = ro.jx; out[2] = ro.jy;
  out[3] = ro.nmin; out[4] = ro.nmax; out[5] = ro.nonfinite;
  if (h->unstable) return fail(LB_EUNSTABLE, "a stability check failed");
  return LB_OK;
}

lb_status lb_get_populations(lb_handle* h, double* f) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!f) return fail(LB_EINVAL, "f is NULL");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  const int64_t nn = nodes(h);
  for (int i = 0; i < 9; ++i) {
    HIPCHK(lbk::launch_get_pops(fp32_of(h), h->ddesc, h->parity, i, i + 1, nn, h->dstage,
                                h->pending_shift ? 1 : 0, h->st));
    HIPCHK(hipMemcpyAsync(f + i * nn, h->dstage, nn * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  return LB_OK;
}

lb_status lb_set_populations(lb_handle* h, const double* f, int64_t step) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (!f) return fail(LB_EINVAL, "f is NULL");
  if (step < 0) return fail(LB_EINVAL, "step must be >= 0");
  const int64_t nn = nodes(h);
  double mass = 0.0;
  for (int64_t k = 0; k < 9 * nn; ++k) {
    if (!std::isfinite(f[k])) return fail(LB_EINVAL, "f[%lld] is not finite", (long long)k);
    mass += f[k];
  }
  h->hdesc.nbar = h->p.fp32 ? mass / (double)nn : 0.0;
  lb_status r = upload_desc(h);
  if (r != LB_OK) return r;
  h->parity = 0;
  for (int i = 0; i < 9; ++i) {
    HIPCHK(hipMemcpyAsync(h->dstage, f + i * nn, nn * 8, hipMemcpyHostToDevice, h->st));
    HIPCHK(lbk::launch_set_pops(fp32_of(h), h->ddesc, 0, i, i + 1, nn, h->dstage, step, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  h->step = step;
  h->moments_valid = false;
  return after_restart(h);
}

lb_status lb_set_checks(lb_handle* h, int32_t check_every, int32_t drift_correct) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (check_every < 0) return fail(LB_EINVAL, "check_every must be >= 0");
  if (drift_correct != 0 && drift_correct != 1) return fail(LB_EINVAL, "drift_correct must be 0 or 1");
  h->p.check_every = check_every;
  h->p.drift_correct = drift_correct;
  return LB_OK;
}

lb_status lb_get_step(lb_handle* h, int64_t* step) {
  if (!h || !step) return fail(LB_EINVAL, "NULL argument");
  *step = h->step;
  return LB_OK;
}

lb_status lb_destroy(lb_handle* h) {
  if (!h) return LB_OK;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return LB_OK;
}

lb_status lb_set_launch(lb_handle* h, int32_t threads, int32_t rows) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (threads == 0) threads = default_threads(&h->p);
  if (rows == 0) rows = default_rows(&h->p, threads);
  return set_tiles(h, threads, rows, 1);
}

lb_status lb_set_launch_fused(lb_handle* h, int32_t threads, int32_t rows) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (threads == 0) threads = 128;
  if (rows == 0) rows = fused_default_rows(&h->p, threads);
  return set_tiles(h, threads, rows, 2);
}

lb_status lb_get_steps_per_launch(lb_handle* h, int32_t* steps) {
  if (!h || !steps) return fail(LB_EINVAL, "NULL argument");
  *steps = h->fuse;
  return LB_OK;
}

lb_status lb_get_launch(lb_handle* h, int32_t* threads, int32_t* rows, int32_t* blocks) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (threads) *threads = h->threads;
  if (rows) *rows = h->rows;
  if (blocks) *blocks = h->ntiles;
  return LB_OK;
}

lb_status lb_autotune(lb_handle* h, int32_t nsteps, int32_t* threads, int32_t* rows,
                      double* ms_per_step) {
  if (!h) return fail(LB_EINVAL, "handle is NULL");
  if (nsteps < 1) return fail(LB_EINVAL, "nsteps must be >= 1");
  if (!h->has_state) return fail(LB_ESTATE, "lattice has no state");
  if (h->unstable) return fail(LB_ESTATE, "lattice was flagged unstable");
  // candidate shapes (threads, rows, steps per launch): strip widths up to
  // one strip per row, and for each the chunk heights that fill the resident
  // workgroups once or twice, plus a few fixed heights; with FP32 storage the
  // two-step kernel's shapes too
  struct Cand {
    int t, rw, fuse;
  };
  std::vector<Cand> cand;
  for (int t : {128, 256, 512}) {
    if (t == 512 && prec(h) != lbk::kFP32) continue;
    if (t > 128 && h->p.Lx + 6 <= t / 2) continue;
    std::vector<int> rs = {default_rows(&h->p, t, 1), default_rows(&h->p, t, 2), 16, 64};
    std::sort(rs.begin(), rs.end());
    rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
    for (int rw : rs)
      if (rw <= h->p.Ly) cand.push_back({t, rw, 1});
  }
  if (prec(h) == lbk::kFP32)
    for (int t : {64, 128, 192, 256}) {
      if (t > 128 && h->p.Lx + 14 <= t / 2) continue;
      std::vector<int> rs = {fused_default_rows(&h->p, t, 1), fused_default_rows(&h->p, t, 2), 32};
      std::sort(rs.begin(), rs.end());
      rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
      for (int rw : rs)
        if (rw <= h->p.Ly) cand.push_back({t, rw, 2});
    }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = 1e300;
  int bt = h->threads, br = h->rows, bf = h->fuse;
  lb_status r = LB_OK;
  for (const auto& c : cand) {
    const int t = c.t, rw = c.rw;
    {
      if ((r = set_tiles(h, t, rw, c.fuse)) != LB_OK) break;
      if ((r = step_impl(h, c.fuse, false)) != LB_OK) break;  // warm-up
      if (hipEventRecord(e0, h->st) != hipSuccess) { r = fail(LB_EDEVICE, "event record failed"); break; }
      if ((r = step_impl(h, nsteps, false)) != LB_OK) break;
      if (hipEventRecord(e1, h->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        r = fail(LB_EDEVICE, "event sync failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / nsteps;
      if (per < best) { best = per; bt = t; br = h->rows; bf = c.fuse; }
    }
    if (r != LB_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != LB_OK) return r;
  h->moments_valid = false;
  if ((r = set_tiles(h, bt, br, bf)) != LB_OK) return r;
  if (threads) *threads = bt;
  if (rows) *rows = br;
  if (ms_per_step) *ms_per_step = best;
  return LB_OK;
}

}  // extern "C"
