// Host side of the batched C ABI (include/lbvdw.h): many independent
// lattices of uneven size advance together. One step of the batch is one
// launch of the step kernel over the tiles of every instance (the tile table
// names the instance; each instance has its own descriptor, populations,
// force table and checks). Runs of steps are recorded once into a HIP graph
// and replayed.
#include <hip/hip_runtime.h>

#include <cstring>
#include <numeric>

#include "lb_host.h"

using namespace lbh;

namespace {

struct Inst {
  lb_params p{};
  size_t base = 0;  // offset of the instance's region in the workspace
  Layout L{};
  bool has_state = false;
  bool moments_valid = false;
};

// Shared part of the batch workspace.
struct BatchLayout {
  size_t descs, reds, tiles, tiles1, sub_tiles, part, part_off, list_all, list_sub, inst0, total;
  int max_tiles;
  std::vector<int64_t> off;  // partial-sum block offset of each instance
};

BatchLayout batch_layout(int count, const lb_params* p, std::vector<Inst>* insts) {
  BatchLayout B;
  int max_tiles = 0;
  int64_t sum_red = 0;
  B.off.resize(count);
  for (int i = 0; i < count; ++i) {
    const int strips = (p[i].Lx + 49) / 50;  // narrowest strip: 64 threads, two steps
    const int chunks = (p[i].Ly + 7) / 8;
    max_tiles += strips * chunks;
    B.off[i] = sum_red;
    sum_red += lbk::reduce_blocks((int64_t)p[i].Lx * p[i].Ly);
  }
  size_t o = 0;
  B.descs = o; o = align_up(o + sizeof(Desc) * count);
  B.reds = o; o = align_up(o + sizeof(ReduceOut) * count);
  B.tiles = o; o = align_up(o + sizeof(Tile) * (size_t)max_tiles);
  B.tiles1 = o; o = align_up(o + sizeof(Tile) * (size_t)max_tiles);
  B.sub_tiles = o; o = align_up(o + sizeof(Tile) * (size_t)max_tiles);
  B.part = o; o = align_up(o + sizeof(double) * 6 * (size_t)sum_red);
  B.part_off = o; o = align_up(o + sizeof(int64_t) * count);
  B.list_all = o; o = align_up(o + sizeof(int32_t) * count);
  B.list_sub = o; o = align_up(o + sizeof(int32_t) * count);
  B.inst0 = o;
  for (int i = 0; i < count; ++i) {
    Layout L = layout_for(&p[i], o);
    if (insts) {
      (*insts)[i].base = o;
      (*insts)[i].L = L;
    }
    o += L.total;
  }
  B.total = o;
  B.max_tiles = max_tiles;
  return B;
}

constexpr int kGraphSteps = 64;

}  // namespace

struct lb_batch {
  int count = 0;
  bool fp32 = false;  // FP32 storage
  int prec = 0;       // lbk::Prec of every instance
  int reg = 0;        // regularised collision (every instance)
  int yflags = 0;     // lbk::kYWalls / kYPeriodic when every instance has that y boundary
  int check_every = 0, drift = 0;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  BatchLayout B{};
  std::vector<Inst> inst;
  std::vector<Desc> hdesc;
  Desc* ddesc = nullptr;
  ReduceOut* dred = nullptr;
  Tile* dtiles = nullptr;   // tiles of the current launch shape
  Tile* dtiles1 = nullptr;  // one-step tiles for single steps of a two-step shape
  Tile* dsub = nullptr;     // tile table of the last subset step
  double* dpart = nullptr;
  int threads = 256, rows = 64, ntiles = 0;
  int fuse = 1;  // steps per launch of the current shape
  int threads1 = 128, rows1 = 16, ntiles1 = 0;
  int parity = 0;
  int64_t step = 0;
  bool pending_shift = false;
  bool unstable_any = false;
  std::vector<int> unstable;
  std::vector<char> dropped;  // instances taken out of the steps (lb_batch_drop_unstable)
  // batched checks: partial-sum offsets, the list of checked instances (all
  // live ones, or the last subset), its length and widest reduction
  int64_t* dpoff = nullptr;
  int32_t* dlist_all = nullptr;
  int32_t* dlist_sub = nullptr;
  int n_all = 0, nb_all = 1, n_sub = 0, nb_sub = 1;
  // graphs of kGraphSteps steps, keyed by the pending-shift state at entry;
  // recorded on a private stream (the caller's may be the null stream, which
  // cannot be captured) and replayed on the caller's
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t rec = nullptr;
  int exec_threads = 0, exec_rows = 0;
};

namespace {

int64_t inst_nodes(const lb_batch* b, int i) { return (int64_t)b->inst[i].p.Lx * b->inst[i].p.Ly; }

void drop_graphs(lb_batch* b) {
  for (auto& e : b->exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
}

// Upload the instances with mask[i] != 0 (all when mask is NULL) that have a
// state and are not dropped as a check list; returns its length and the
// widest reduction among them.
lb_status upload_list(lb_batch* b, const int32_t* mask, int32_t* dlist, int* n, int* nb) {
  std::vector<int32_t> l;
  int w = 1;
  for (int i = 0; i < b->count; ++i)
    if ((!mask || mask[i]) && b->inst[i].has_state && !b->dropped[i]) {
      l.push_back(i);
      w = std::max(w, lbk::reduce_blocks(inst_nodes(b, i)));
    }
  if (!l.empty()) {
    HIPCHK(hipMemcpyAsync(dlist, l.data(), l.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->st));
    HIPCHK(hipStreamSynchronize(b->st));  // l is a host temporary
  }
  *n = (int)l.size();
  *nb = w;
  return LB_OK;
}

// Tiles of the instances with mask[i] != 0 (all when mask is NULL), largest
// instances first: the dispatcher hands out tiles in order, so the
// long-running ones start early. Chunk heights are balanced within each
// instance, so no short ragged chunk finishes early beside full ones.
std::vector<Tile> tile_list(const lb_batch* b, int threads, int rows, const int32_t* mask,
                            int halo = 3) {
  std::vector<int> order;
  for (int i = 0; i < b->count; ++i)
    if ((!mask || mask[i]) && !b->dropped[i]) order.push_back(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return inst_nodes(b, x) > inst_nodes(b, y); });
  std::vector<Tile> all;
  for (int i : order) {
    const int r = std::max(std::min(rows, b->inst[i].p.Ly), std::min(8, b->inst[i].p.Ly));
    std::vector<Tile> t = make_tiles(i, b->inst[i].p.Lx, b->inst[i].p.Ly, threads, r, halo, true);
    all.insert(all.end(), t.begin(), t.end());
  }
  return all;
}

// Default launch shape of a batch: 128-thread strips (64 when every instance
// is that narrow), which measured fastest for batches of many small lattices
// (many short tiles keep more workgroups in flight than wide strips), and a
// chunk height that makes the tiles of all instances fill the resident
// workgroups about once. lb_batch_autotune refines it.
void default_batch_launch(const lb_batch* b, int* threads, int* rows) {
  int t = 64;
  for (int i = 0; i < b->count; ++i)
    if (b->inst[i].p.Lx + 6 > 64) t = 128;
  int64_t strip_rows = 0;
  for (int i = 0; i < b->count; ++i)
    strip_rows += (int64_t)((b->inst[i].p.Lx + t - 7) / (t - 6)) * b->inst[i].p.Ly;
  const int slots = resident_slots(&b->inst[0].p, t);
  const int64_t want = (strip_rows + slots - 1) / std::max(slots, 1);
  int r = (int)std::min<int64_t>(std::max<int64_t>(want, 10), 1 << 20);
  r = ((r - 2 + 7) / 8) * 8 + 2;
  *threads = t;
  *rows = r;
}

lb_status upload_tiles(lb_batch* b, Tile* dst, int threads, int rows, int fuse, int* ntiles) {
  std::vector<Tile> all = tile_list(b, threads, rows, nullptr, fuse == 2 ? 7 : 3);
  if ((int)all.size() > b->B.max_tiles) return fail(LB_EINVAL, "too many tiles for the workspace");
  HIPCHK(hipMemcpyAsync(dst, all.data(), all.size() * sizeof(Tile), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  *ntiles = (int)all.size();
  return LB_OK;
}

// Launch shape (fuse = steps per launch). A two-step shape keeps the default
// one-step shape for single steps (before a check that splits a pair, the
// last of an odd count, subset steps).
lb_status batch_tiles(lb_batch* b, int threads, int rows, int fuse = 1) {
  if (fuse == 2) {
    if (b->prec != lbk::kFP32)
      return fail(LB_EINVAL, "two steps per launch need FP32 storage and arithmetic (fp32 = 1)");
    if (!fused_threads_ok(threads))
      return fail(LB_EINVAL, "two steps per launch: threads must be 64, 128, 192 or 256 (got %d)", threads);
  } else if (threads != 64 && threads != 128 && threads != 256 && threads != 320 &&
             !(threads == 512 && b->prec == lbk::kFP32)) {
    return fail(LB_EINVAL, "threads must be 64, 128, 256, 320 or 512 (fp32 = 1 only) (got %d)", threads);
  }
  if (rows < 1) return fail(LB_EINVAL, "rows must be >= 1");
  int nt = 0;
  lb_status r = upload_tiles(b, b->dtiles, threads, rows, fuse, &nt);
  if (r != LB_OK) return r;
  if (fuse == 2) {
    int t1 = 0, r1 = 0;
    default_batch_launch(b, &t1, &r1);
    if ((r = upload_tiles(b, b->dtiles1, t1, r1, 1, &b->ntiles1)) != LB_OK) return r;
    b->threads1 = t1;
    b->rows1 = r1;
  }
  b->threads = threads;
  b->rows = rows;
  b->ntiles = nt;
  b->fuse = fuse;
  drop_graphs(b);
  return LB_OK;
}

lb_status enqueue_checks(lb_batch* b, int mode, int only = -1, const int32_t* mask = nullptr) {
  if (mode == 0 && only < 0) {
    // periodic check of all live instances, or of the subset last uploaded
    const bool sub = mask != nullptr;
    HIPCHK(lbk::launch_check_batch(b->fp32, b->ddesc, b->parity, sub ? b->dlist_sub : b->dlist_all,
                                   sub ? b->n_sub : b->n_all, sub ? b->nb_sub : b->nb_all, b->dpoff,
                                   b->dpart, b->dred, b->drift, b->st));
    return LB_OK;
  }
  for (int i = 0; i < b->count; ++i) {
    if (only >= 0 && i != only) continue;
    if (mask && !mask[i]) continue;
    if (!b->inst[i].has_state || b->dropped[i]) continue;
    const int64_t nn = inst_nodes(b, i);
    HIPCHK(lbk::launch_reduce(b->fp32, b->ddesc + i, b->parity, nn, b->dpart,
                              (mode == 2 && b->pending_shift) ? 1 : 0, b->st));
    HIPCHK(lbk::launch_reduce_final(b->dpart, lbk::reduce_blocks(nn), nn, b->dred + i, mode,
                                    mode == 0 ? b->drift : 0, b->st));
  }
  return LB_OK;
}

// Enqueue `n` steps eagerly (also used while recording a graph). With a
// two-step shape, pairs of steps are one launch unless a check falls after
// the first of them or one step is left. dry: advance the counters exactly
// as the launches would, without launching (after a graph replay).
lb_status enqueue_steps(lb_batch* b, int64_t n, bool moments_last, bool dry = false) {
  const int ce = b->check_every;
  for (int64_t s = 0; s < n;) {
    const bool pair = b->fuse == 2 && n - s >= 2 && !(ce > 0 && (b->step + 1) % ce == 0);
    const int k = pair ? 2 : 1;
    int flags = 0;
    if (moments_last && s + k == n) flags |= lbk::kWriteMoments;
    if (b->pending_shift) flags |= lbk::kApplyShift;
    if (!dry) {
      if (pair)
        HIPCHK(lbk::launch_step2(b->threads, b->reg != 0, b->ddesc, b->dtiles, b->ntiles, b->parity,
                                 flags | b->yflags, b->st));
      else if (b->fuse == 2)
        HIPCHK(lbk::launch_step(b->prec, b->reg != 0, b->threads1, b->ddesc, b->dtiles1, b->ntiles1, b->parity,
                                flags, b->st));
      else
        HIPCHK(lbk::launch_step(b->prec, b->reg != 0, b->threads, b->ddesc, b->dtiles, b->ntiles, b->parity,
                                flags, b->st));
    }
    b->pending_shift = false;
    b->parity ^= 1;
    b->step += k;
    s += k;
    if (ce > 0 && b->step % ce == 0) {
      if (!dry) {
        lb_status r = enqueue_checks(b, 0);
        if (r != LB_OK) return r;
      }
      b->pending_shift = b->drift != 0;
    }
  }
  return LB_OK;
}

// A graph run must start where its recording started: even parity, a step
// count on the check grid, and the same pending-shift state.
bool graph_aligned(const lb_batch* b) {
  if (b->parity != 0) return false;
  if (b->check_every > 0 && b->step % b->check_every != 0) return false;
  return true;
}

lb_status replay(lb_batch* b) {
  const int key = b->pending_shift ? 1 : 0;
  if (!b->exec[key]) {
    hipGraph_t g;
    const int par0 = b->parity;
    const int64_t step0 = b->step;
    const bool pend0 = b->pending_shift;
    if (!b->rec) HIPCHK(hipStreamCreateWithFlags(&b->rec, hipStreamNonBlocking));
    hipStream_t user = b->st;
    b->st = b->rec;
    HIPCHK(hipStreamBeginCapture(b->rec, hipStreamCaptureModeThreadLocal));
    lb_status r = enqueue_steps(b, kGraphSteps, false);
    hipError_t e = hipStreamEndCapture(b->rec, &g);
    b->st = user;
    // recording did not run anything: restore the counters
    b->parity = par0;
    b->step = step0;
    b->pending_shift = pend0;
    if (r != LB_OK) return r;
    if (e != hipSuccess) return fail(LB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LB_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  HIPCHK(hipGraphLaunch(b->exec[key], b->st));
  // advance the counters exactly as the recorded steps do
  return enqueue_steps(b, kGraphSteps, false, true);
}

lb_status read_batch_status(lb_batch* b) {
  std::vector<ReduceOut> r(b->count);
  HIPCHK(hipMemcpyAsync(r.data(), b->dred, sizeof(ReduceOut) * b->count, hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  for (int i = 0; i < b->count; ++i)
    if ((r[i].status & 1u) && !b->dropped[i]) {
      b->unstable[i] = 1;
      b->unstable_any = true;
    }
  return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_batch_workspace_bytes(int32_t count, const lb_params* p, size_t* bytes) {
  if (count < 1) return fail(LB_EINVAL, "count must be >= 1");
  if (!p || !bytes) return fail(LB_EINVAL, "NULL argument");
  for (int i = 0; i < count; ++i) {
    lb_status s = validate(&p[i]);
    if (s != LB_OK) return s;
  }
  *bytes = batch_layout(count, p, nullptr).total;
  return LB_OK;
}

lb_status lb_batch_create(int32_t count, const lb_params* p, void* dev_ws, size_t ws_bytes,
                          void* hip_stream, lb_batch** out) {
  if (count < 1) return fail(LB_EINVAL, "count must be >= 1");
  if (!p || !out || !dev_ws) return fail(LB_EINVAL, "NULL argument");
  if ((uintptr_t)dev_ws % kAlign) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
  for (int i = 0; i < count; ++i) {
    lb_status s = validate(&p[i]);
    if (s != LB_OK) return s;
    if (p[i].fp32 != p[0].fp32) return fail(LB_EINVAL, "all instances must share fp32");
    if (p[i].collision != p[0].collision) return fail(LB_EINVAL, "all instances must share collision");
    if (p[i].check_every != p[0].check_every || p[i].drift_correct != p[0].drift_correct)
      return fail(LB_EINVAL, "all instances must share check_every and drift_correct");
  }
  lb_batch* b = new lb_batch();
  b->count = count;
  b->fp32 = p[0].fp32 != 0;
  b->prec = prec_of(&p[0]);
  b->reg = p[0].collision;
  {
    int np = 0;
    for (int i = 0; i < count; ++i) np += p[i].y_periodic != 0;
    b->yflags = np == count ? lbk::kYPeriodic : (np == 0 ? lbk::kYWalls : 0);
  }
  b->check_every = p[0].check_every;
  b->drift = p[0].drift_correct;
  b->inst.resize(count);
  b->B = batch_layout(count, p, &b->inst);
  if (ws_bytes < b->B.total) {
    size_t need = b->B.total;
    delete b;
    return fail(LB_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  b->ws = (char*)dev_ws;
  b->st = (hipStream_t)hip_stream;
  b->ddesc = (Desc*)(b->ws + b->B.descs);
  b->dred = (ReduceOut*)(b->ws + b->B.reds);
  b->dtiles = (Tile*)(b->ws + b->B.tiles);
  b->dtiles1 = (Tile*)(b->ws + b->B.tiles1);
  b->dsub = (Tile*)(b->ws + b->B.sub_tiles);
  b->dpart = (double*)(b->ws + b->B.part);
  b->dpoff = (int64_t*)(b->ws + b->B.part_off);
  b->dlist_all = (int32_t*)(b->ws + b->B.list_all);
  b->dlist_sub = (int32_t*)(b->ws + b->B.list_sub);
  b->hdesc.resize(count);
  b->unstable.assign(count, 0);
  b->dropped.assign(count, 0);
  auto cleanup = [&](lb_status e) { delete b; return e; };
  for (int i = 0; i < count; ++i) {
    Inst& I = b->inst[i];
    I.p = p[i];
    I.p.fext_x = nullptr;
    Desc& d = b->hdesc[i];
    d.S[0] = b->ws + I.L.S0;
    d.S[1] = b->ws + I.L.S1;
    d.fext3 = b->ws + I.L.fext;
    d.mom = (double*)(b->ws + I.L.mom);
    d.shift = &b->dred[i].shift;
    d.rng = b->dred[i].rng_step;
    d.Lx = p[i].Lx;
    d.Ly = p[i].Ly;
    d.periodic = p[i].y_periodic;
    d.reg = p[i].collision;
    d.nbar = 0.0;
    d.T = p[i].T;
    d.omega = 1.0 / (std::sqrt(3.0) * p[i].tau);
    d.kappa3 = p[i].kappa / 3.0;
    d.N = p[i].N;
    d.M = (1.0 - 2.0 * p[i].N) / 4.0;
    d.Q = p[i].Q;
    d.R = (1.0 - p[i].Q) / 2.0;
    d.U = p[i].U;
    std::vector<double> f(p[i].Lx, 0.0);
    if (p[i].fext_x)
      for (int x = 0; x < p[i].Lx; ++x) f[x] = p[i].fext_x[x] / 3.0;
    hipError_t e;
    if (b->prec == lbk::kFP32) {
      std::vector<float> f32(f.begin(), f.end());
      e = hipMemcpyAsync(b->ws + I.L.fext, f32.data(), f32.size() * 4, hipMemcpyHostToDevice, b->st);
      if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    } else {
      e = hipMemcpyAsync(b->ws + I.L.fext, f.data(), f.size() * 8, hipMemcpyHostToDevice, b->st);
      if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    }
    if (e != hipSuccess) return cleanup(fail(LB_EDEVICE, "uploading a force table failed"));
  }
  std::vector<ReduceOut> z(count);
  std::memset(z.data(), 0, sizeof(ReduceOut) * count);
  if (hipMemcpyAsync(b->dpoff, b->B.off.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, b->st) != hipSuccess ||
      hipMemcpyAsync(b->dred, z.data(), sizeof(ReduceOut) * count, hipMemcpyHostToDevice, b->st) != hipSuccess ||
      hipMemcpyAsync(b->ddesc, b->hdesc.data(), sizeof(Desc) * count, hipMemcpyHostToDevice, b->st) != hipSuccess ||
      hipStreamSynchronize(b->st) != hipSuccess)
    return cleanup(fail(LB_EDEVICE, "uploading descriptors failed"));
  int dt = 0, dr = 0;
  default_batch_launch(b, &dt, &dr);
  lb_status r = batch_tiles(b, dt, dr);
  if (r != LB_OK) return cleanup(r);
  *out = b;
  return LB_OK;
}

lb_status lb_batch_init(lb_batch* b, int32_t idx, const double* n0, const double* ux0,
                        const double* uy0) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (idx < 0 || idx >= b->count) return fail(LB_EINVAL, "index %d out of range", idx);
  if (!n0) return fail(LB_EINVAL, "n0 is NULL");
  if (b->step != 0 || b->parity != 0)
    return fail(LB_ESTATE, "instances can only be initialised before the batch steps");
  Inst& I = b->inst[idx];
  const int64_t nn = inst_nodes(b, idx);
  double sum = 0.0;
  for (int64_t k = 0; k < nn; ++k) {
    if (!(n0[k] > 0.0 && n0[k] < 3.0))
      return fail(LB_EINVAL, "n0[%lld] = %g is outside (0, 3)", (long long)k, n0[k]);
    sum += n0[k];
  }
  double* mom = (double*)(b->ws + I.L.mom);
  HIPCHK(hipMemcpyAsync(mom, n0, nn * 8, hipMemcpyHostToDevice, b->st));
  if (ux0) HIPCHK(hipMemcpyAsync(mom + nn, ux0, nn * 8, hipMemcpyHostToDevice, b->st));
  if (uy0) HIPCHK(hipMemcpyAsync(mom + 2 * nn, uy0, nn * 8, hipMemcpyHostToDevice, b->st));
  b->hdesc[idx].nbar = b->fp32 ? sum / (double)nn : 0.0;
  HIPCHK(hipMemcpyAsync(b->ddesc + idx, &b->hdesc[idx], sizeof(Desc), hipMemcpyHostToDevice, b->st));
  HIPCHK(lbk::launch_init(b->fp32, b->ddesc + idx, 0, mom, ux0 ? mom + nn : nullptr,
                          uy0 ? mom + 2 * nn : nullptr, nn, b->st));
  I.has_state = true;
  lb_status r = upload_list(b, nullptr, b->dlist_all, &b->n_all, &b->nb_all);
  if (r != LB_OK) return r;
  r = enqueue_checks(b, 1, idx);
  if (r != LB_OK) return r;
  if ((r = read_batch_status(b)) != LB_OK) return r;
  if (b->unstable[idx]) return fail(LB_EUNSTABLE, "initial state of instance %d is invalid", idx);
  I.moments_valid = true;
  return LB_OK;
}

lb_status lb_batch_step_n(lb_batch* b, int64_t nsteps) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
  for (int i = 0; i < b->count; ++i)
    if (!b->inst[i].has_state) return fail(LB_ESTATE, "instance %d has no state", i);
  if (b->unstable_any) return fail(LB_ESTATE, "an instance was flagged unstable");
  if (nsteps == 0) return LB_OK;
  int64_t left = nsteps;
  lb_status r;
  // recorded runs where the step count is on the check grid; eager steps up
  // to the next point where a recorded run can start; the last step is
  // always eager (it writes the moments)
  while (left > 1) {
    if (left > kGraphSteps && graph_aligned(b)) {
      if ((r = replay(b)) != LB_OK) return r;
      left -= kGraphSteps;
    } else {
      int64_t k = left - 1;
      if (b->check_every > 0)
        k = std::min<int64_t>(k, b->check_every - b->step % b->check_every);
      else if (b->parity != 0)
        k = 1;
      if ((r = enqueue_steps(b, k, false)) != LB_OK) return r;
      left -= k;
    }
  }
  if ((r = enqueue_steps(b, left, true)) != LB_OK) return r;
  for (auto& I : b->inst) I.moments_valid = true;
  return LB_OK;
}

lb_status lb_batch_get_moments(lb_batch* b, int32_t idx, double* n, double* ux, double* uy) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (idx < 0 || idx >= b->count) return fail(LB_EINVAL, "index %d out of range", idx);
  if (!b->inst[idx].moments_valid) return fail(LB_ESTATE, "instance %d has no moments", idx);
  const int64_t nn = inst_nodes(b, idx);
  const double* mom = (const double*)(b->ws + b->inst[idx].L.mom);
  if (n) HIPCHK(hipMemcpyAsync(n, mom, nn * 8, hipMemcpyDeviceToHost, b->st));
  if (ux) HIPCHK(hipMemcpyAsync(ux, mom + nn, nn * 8, hipMemcpyDeviceToHost, b->st));
  if (uy) HIPCHK(hipMemcpyAsync(uy, mom + 2 * nn, nn * 8, hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  lb_status r = read_batch_status(b);
  if (r != LB_OK) return r;
  if (b->unstable[idx]) return fail(LB_EUNSTABLE, "instance %d failed a stability check", idx);
  return LB_OK;
}

lb_status lb_batch_reduce(lb_batch* b, int32_t idx, double out[6]) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (idx < 0 || idx >= b->count) return fail(LB_EINVAL, "index %d out of range", idx);
  if (!out) return fail(LB_EINVAL, "out is NULL");
  if (!b->inst[idx].has_state) return fail(LB_ESTATE, "instance %d has no state", idx);
  lb_status r = enqueue_checks(b, 2, idx);
  if (r != LB_OK) return r;
  ReduceOut ro;
  HIPCHK(hipMemcpyAsync(&ro, b->dred + idx, sizeof ro, hipMemcpyDeviceToHost, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  out[0] = ro.mass; out[1] = ro.jx; out[2] = ro.jy;
  out[3] = ro.nmin; out[4] = ro.nmax; out[5] = ro.nonfinite;
  if (ro.status & 1u) {
    b->unstable[idx] = 1;
    b->unstable_any = true;
    return fail(LB_EUNSTABLE, "instance %d failed a stability check", idx);
  }
  return LB_OK;
}

lb_status lb_batch_status(lb_batch* b, int32_t* per_instance) {
  if (!b || !per_instance) return fail(LB_EINVAL, "NULL argument");
  lb_status r = read_batch_status(b);
  if (r != LB_OK) return r;
  for (int i = 0; i < b->count; ++i) per_instance[i] = b->unstable[i] ? LB_EUNSTABLE : LB_OK;
  return LB_OK;
}

lb_status lb_batch_set_launch(lb_batch* b, int32_t threads, int32_t rows) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  int dt = 0, dr = 0;
  default_batch_launch(b, &dt, &dr);
  if (threads == 0) threads = dt;
  if (rows == 0) rows = dr;
  return batch_tiles(b, threads, rows, 1);
}

lb_status lb_batch_set_launch_fused(lb_batch* b, int32_t threads, int32_t rows) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (threads == 0) threads = 128;
  if (rows == 0) rows = 64;
  return batch_tiles(b, threads, rows, 2);
}

lb_status lb_batch_get_steps_per_launch(lb_batch* b, int32_t* steps) {
  if (!b || !steps) return fail(LB_EINVAL, "NULL argument");
  *steps = b->fuse;
  return LB_OK;
}

lb_status lb_batch_autotune(lb_batch* b, int32_t nsteps, int32_t* threads, int32_t* rows,
                            double* ms_per_step) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  if (nsteps < 1) return fail(LB_EINVAL, "nsteps must be >= 1");
  for (int i = 0; i < b->count; ++i)
    if (!b->inst[i].has_state) return fail(LB_ESTATE, "instance %d has no state", i);
  if (b->unstable_any) return fail(LB_ESTATE, "an instance was flagged unstable");
  // (threads, rows, steps per launch); the two-step kernel's shapes with FP32
  struct Cand {
    int t, rw, fuse;
  };
  std::vector<Cand> cand;
  for (int t : {128, 256, 512})
    for (int rw : {16, 32, 64, 128, 256})
      if (t != 512 || b->prec == lbk::kFP32) cand.push_back({t, rw, 1});
  if (b->prec == lbk::kFP32)
    for (int t : {64, 128, 192, 256})
      for (int rw : {16, 32, 48, 64, 128, 256}) cand.push_back({t, rw, 2});
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = 1e300;
  int bt = b->threads, br = b->rows, bf = b->fuse;
  lb_status r = LB_OK;
  for (const Cand& c : cand) {
    const int t = c.t, rw = c.rw;
    if (r != LB_OK) break;
    if ((r = batch_tiles(b, t, rw, c.fuse)) != LB_OK) break;
    if ((r = enqueue_steps(b, c.fuse, false)) != LB_OK) break;
    if (hipEventRecord(e0, b->st) != hipSuccess) { r = fail(LB_EDEVICE, "event record failed"); break; }
    if ((r = enqueue_steps(b, nsteps, false)) != LB_OK) break;
    if (hipEventRecord(e1, b->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      r = fail(LB_EDEVICE, "event sync failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms / nsteps < best) { best = ms / nsteps; bt = t; br = rw; bf = c.fuse; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != LB_OK) return r;
  for (auto& I : b->inst) I.moments_valid = false;
  if ((r = batch_tiles(b, bt, br, bf)) != LB_OK) return r;
  if (threads) *threads = bt;
  if (rows) *rows = br;
  if (ms_per_step) *ms_per_step = best;
  return LB_OK;
}

static lb_status same_size(const lb_batch* b) {
  for (int i = 1; i < b->count; ++i)
    if (b->inst[i].p.Lx != b->inst[0].p.Lx || b->inst[i].p.Ly != b->inst[0].p.Ly)
      return fail(LB_EINVAL, "all instances must have the same size for this call");
  return LB_OK;
}

lb_status lb_batch_get_moments_device(lb_batch* b, double* dev_out) {
  if (!b || !dev_out) return fail(LB_EINVAL, "NULL argument");
  lb_status r = same_size(b);
  if (r != LB_OK) return r;
  for (int i = 0; i < b->count; ++i)
    if (!b->inst[i].moments_valid) return fail(LB_ESTATE, "instance %d has no moments", i);
  HIPCHK(lbk::launch_gather_moments(b->ddesc, b->count, inst_nodes(b, 0), dev_out, b->st));
  return LB_OK;
}

static lb_status reenter(lb_batch* b, const double* dev_fields, const double* dev_from,
                         const int32_t* mask) {
  if (!b || !dev_fields || !mask) return fail(LB_EINVAL, "NULL argument");
  lb_status r = same_size(b);
  if (r != LB_OK) return r;
  std::vector<int32_t> m(mask, mask + b->count);
  bool any = false;
  for (int i = 0; i < b->count; ++i) {
    m[i] = m[i] ? 1 : 0;
    if (m[i] && !b->inst[i].has_state) return fail(LB_ESTATE, "instance %d has no state", i);
    any = any || m[i];
  }
  if (!any) return LB_OK;
  // the mask travels in the sub-tile table's region (no step is in flight
  // that reads it: stream order)
  int32_t* dmask = (int32_t*)b->dsub;
  if ((size_t)b->count * sizeof(int32_t) > (size_t)b->B.max_tiles * sizeof(Tile))
    return fail(LB_EINVAL, "batch too large for the mask buffer");
  HIPCHK(hipMemcpyAsync(dmask, m.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice, b->st));
  HIPCHK(lbk::launch_scatter_eq(b->fp32, b->ddesc, b->dred, b->count, b->parity, inst_nodes(b, 0),
                                dev_fields, dev_from, dmask, b->st));
  HIPCHK(hipStreamSynchronize(b->st));  // m is a host temporary
  for (int i = 0; i < b->count; ++i)
    if (m[i]) b->inst[i].moments_valid = true;
  return LB_OK;
}

lb_status lb_batch_set_equilibrium_device(lb_batch* b, const double* dev_fields,
                                          const int32_t* mask) {
  return reenter(b, dev_fields, nullptr, mask);
}

lb_status lb_batch_shift_equilibrium_device(lb_batch* b, const double* dev_from,
                                            const double* dev_fields, const int32_t* mask) {
  if (!dev_from) return fail(LB_EINVAL, "NULL argument");
  return reenter(b, dev_fields, dev_from, mask);
}

lb_status lb_batch_step_subset(lb_batch* b, int64_t nsteps, const int32_t* mask) {
  if (!b || !mask) return fail(LB_EINVAL, "NULL argument");
  if (nsteps < 0 || nsteps % 2) return fail(LB_EINVAL, "nsteps must be even and >= 0 (got %lld)",
                                            (long long)nsteps);
  if (b->unstable_any) return fail(LB_ESTATE, "an instance was flagged unstable");
  bool any = false;
  for (int i = 0; i < b->count; ++i)
    if (mask[i]) {
      if (!b->inst[i].has_state) return fail(LB_ESTATE, "instance %d has no state", i);
      any = true;
    }
  if (!any || nsteps == 0) return LB_OK;
  // Every launch flips the buffer parity once, and the subset must end on
  // the batch's parity, so it takes an even number of launches: with the
  // two-step shape, pairs of steps, and when their count is odd, two single
  // steps (one-step shape) in place of one pair.
  int64_t pairs = 0, singles = nsteps;
  if (b->fuse == 2) {
    pairs = nsteps / 2;
    singles = 0;
    if (pairs % 2) {
      pairs -= 1;
      singles = 2;
    }
  }
  lb_status lr = upload_list(b, mask, b->dlist_sub, &b->n_sub, &b->nb_sub);
  if (lr != LB_OK) return lr;
  int64_t launch = 0;
  const int64_t launches = singles + pairs;
  for (int kind = 1; kind <= 2; ++kind) {
    const int64_t n = kind == 1 ? singles : pairs;
    if (n == 0) continue;
    const int th = kind == 2 ? b->threads : (b->fuse == 2 ? b->threads1 : b->threads);
    const int rw = kind == 2 ? b->rows : (b->fuse == 2 ? b->rows1 : b->rows);
    std::vector<Tile> t = tile_list(b, th, rw, mask, kind == 2 ? 7 : 3);
    if ((int)t.size() > b->B.max_tiles) return fail(LB_EINVAL, "too many tiles for the workspace");
    // stream order: the copy waits for earlier launches that read the table
    HIPCHK(hipMemcpyAsync(b->dsub, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice, b->st));
    HIPCHK(hipStreamSynchronize(b->st));  // t is a host temporary
    for (int64_t s = 0; s < n; ++s, ++launch) {
      const int flags = (launch == launches - 1) ? lbk::kWriteMoments : 0;
      const int par = b->parity ^ (int)(launch & 1);
      if (kind == 2)
        HIPCHK(lbk::launch_step2(th, b->reg != 0, b->ddesc, b->dsub, (int)t.size(), par,
                                 flags | b->yflags, b->st));
      else
        HIPCHK(lbk::launch_step(b->prec, b->reg != 0, th, b->ddesc, b->dsub, (int)t.size(), par, flags, b->st));
    }
  }
  lb_status r = enqueue_checks(b, 0, -1, mask);
  if (r != LB_OK) return r;
  for (int i = 0; i < b->count; ++i)
    if (mask[i]) b->inst[i].moments_valid = true;
  return LB_OK;
}

lb_status lb_batch_drop_unstable(lb_batch* b, int32_t* dropped) {
  if (!b) return fail(LB_EINVAL, "batch is NULL");
  lb_status r = read_batch_status(b);
  if (r != LB_OK) return r;
  int n = 0;
  for (int i = 0; i < b->count; ++i) {
    if (b->unstable[i] && !b->dropped[i]) b->dropped[i] = 1;
    n += b->dropped[i];
  }
  if (n == b->count) return fail(LB_ESTATE, "every instance is unstable");
  b->unstable_any = false;
  if ((r = upload_list(b, nullptr, b->dlist_all, &b->n_all, &b->nb_all)) != LB_OK) return r;
  // rebuild the tile table without the dropped instances (drops the graphs)
  if ((r = batch_tiles(b, b->threads, b->rows, b->fuse)) != LB_OK) return r;
  if (dropped) *dropped = n;
  return LB_OK;
}

lb_status lb_batch_destroy(lb_batch* b) {
  if (!b) return LB_OK;
  (void)hipStreamSynchronize(b->st);
  drop_graphs(b);
  if (b->rec) (void)hipStreamDestroy(b->rec);
  delete b;
  return LB_OK;
}

}  // extern "C"
