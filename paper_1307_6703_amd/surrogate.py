"""Learned surrogate of the lattice Boltzmann step, audited by the lattice.

Binding of include/lbsurrogate.h (argument marshalling: every convolution,
gradient, loss, optimiser step, field conversion and comparison runs in the
library's HIP kernels) plus the host logic that drives it:

* ``generate_data``: training pairs from batched lattice runs (fields at the
  start of a chunk of K steps and their change over the chunk);
* ``train``: minibatch Adam on those pairs;
* ``SurrogateRun``: advances a batch of lattices chunk by chunk. Each chunk
  the network predicts every trusted instance; a rotating subset of them,
  any untrusted instance and any prediction that fails the FP64 mass or
  range check are stepped by the lattice instead (``lb_batch_step_subset``),
  and the audited predictions are compared with the lattice's own result;
  an audit above the density tolerance makes the instance untrusted for a
  while. Accepted predictions are projected onto the exact mass and
  re-enter the lattice by adding the change of the equilibrium populations
  of Eq.(eqfunc) (the populations keep their non-equilibrium part).

The paper has no surrogate; the lattice's equations stay the reference
throughout.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import lbvdw
from .lbvdw import Batch, _check, _require, load_library

IN_CHANNELS, IN_REAL, WIDTH, BLOCKS, OUT, OUT_CHANNELS = 8, 6, 48, 4, 3, 16
FWD_FIRST, FWD_RES, FWD_OUT, BWD = 0, 1, 2, 3


class lbs_scales(ctypes.Structure):
    _fields_ = [("n_scale", ctypes.c_float), ("u_scale", ctypes.c_float),
                ("v_scale", ctypes.c_float), ("t_scale", ctypes.c_float)]


# n - 1 in [-0.7, 0.8] -> about +-1.5; |u| <= 0.1 -> 1; force density of
# the potential <= 0.004 -> 0.8; T - 0.9 in [-0.05, 0.08] -> 0.8
DEFAULT_SCALES = (2.0, 10.0, 200.0, 10.0)


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def param_count() -> int:
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.lbs_param_count(ctypes.byref(n)))
    return n.value


def layer_shapes():
    """(cir, cor) of each layer in parameter order."""
    return [(IN_REAL, WIDTH)] + [(WIDTH, WIDTH)] * BLOCKS + [(WIDTH, OUT)]


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights for the SiLU layers, residual branches scaled by
    0.2 (each block starts close to the identity), a small output layer,
    zero biases; flat FP32 in the library's parameter order."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l, (ci, co) in enumerate(layer_shapes()):
        std = np.sqrt(2.0 / (9 * ci))
        if 1 <= l <= BLOCKS:
            std *= 0.2
        if l == BLOCKS + 1:
            std = 0.1 * np.sqrt(1.0 / (9 * ci))
        parts.append(g.normal(0.0, std, size=9 * ci * co))
        parts.append(np.zeros(co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == param_count()
    return p


def split_params(p: np.ndarray):
    """Flat parameters -> [(w[3,3,ci,co], b[co]), ...] (FP64), the layout of
    the FP64 reference layers."""
    out, o = [], 0
    for ci, co in layer_shapes():
        w = np.asarray(p[o:o + 9 * ci * co], dtype=np.float64).reshape(3, 3, ci, co)
        o += 9 * ci * co
        b = np.asarray(p[o:o + co], dtype=np.float64)
        o += co
        out.append((w, b))
    return out


class Net:
    """The network in a device workspace (lbs_create)."""

    def __init__(self, max_batch: int, H: int, W: int, train: bool = False, device="cuda",
                 stream=None):
        import torch
        lib = load_library()
        self.max_batch, self.H, self.W, self.train_mode = int(max_batch), int(H), int(W), bool(train)
        nbytes = ctypes.c_size_t()
        _check(lib.lbs_workspace_bytes(self.max_batch, self.H, self.W, int(train), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib.lbs_create(self.max_batch, self.H, self.W, int(train), ctypes.c_void_p(base + off),
                              nbytes.value, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.device = self.workspace.device
        self.nparams = param_count()
        self._loss = torch.zeros(1, dtype=torch.float64, device=device)

    def set_params(self, p):
        import torch
        t = torch.as_tensor(np.asarray(p, dtype=np.float32)).to(self.device) \
            if not isinstance(p, torch.Tensor) else p.to(self.device, torch.float32).contiguous()
        _require(t, torch.float32, self.nparams)
        _check(load_library().lbs_set_params(self._h, _vp(t)))
        torch.cuda.current_stream().synchronize()  # t may be a temporary

    def params(self):
        import torch
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(load_library().lbs_get_params(self._h, _vp(t)))
        return t

    def grads(self):
        import torch
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(load_library().lbs_get_grads(self._h, _vp(t)))
        return t

    def _check_x(self, x, B):
        import torch
        _require(x, torch.bfloat16, B * self.H * self.W * IN_CHANNELS)

    def forward(self, x, out=None):
        import torch
        B = x.shape[0]
        self._check_x(x, B)
        if out is None:
            out = torch.empty((B, self.H, self.W, OUT), dtype=torch.float32, device=self.device)
        _require(out, torch.float32, B * self.H * self.W * OUT)
        _check(load_library().lbs_forward(self._h, int(B), _vp(x), _vp(out)))
        return out

    def train_step(self, x, target, lr: float):
        """One Adam step; returns the device FP64 loss (before the update)."""
        import torch
        B = x.shape[0]
        self._check_x(x, B)
        _require(target, torch.float32, B * self.H * self.W * OUT)
        _check(load_library().lbs_train_step(self._h, int(B), _vp(x), _vp(target), float(lr),
                                         _vp(self._loss)))
        return self._loss

    def close(self):
        if getattr(self, "_h", None) is not None and lbvdw._lib is not None:
            load_library().lbs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- layers ---------------------------------------------------------------

def kpad(kin: int) -> int:
    return (9 * kin + 31) // 32 * 32


def pack(w, cir, cor, CI, CO, transposed=False):
    """FP32 device weights [9*cir*cor] -> packed bf16 matrix."""
    import torch
    rows, kin = (CI, CO) if transposed else (CO, CI)
    out = torch.empty(rows * kpad(kin), dtype=torch.bfloat16, device=w.device)
    _require(w, torch.float32, 9 * cir * cor)
    _check(load_library().lbs_pack(_vp(w), cir, cor, CI, CO, int(bool(transposed)), _vp(out), _stream()))
    return out


def conv(mode, ci, co, x, wpack, bias=None, res=None, zprev=None, want_z=False, nout=0, blocks=0):
    """One convolution (lbs_conv). Returns (y, z) for modes 0, 1, 3 and the
    FP32 output for mode 2. blocks > 0 caps the persistent grid."""
    import torch
    B, H, W, _ = x.shape
    y = z = yf = None
    if mode == FWD_OUT:
        yf = torch.empty((B, H, W, nout), dtype=torch.float32, device=x.device)
    else:
        y = torch.empty((B, H, W, co), dtype=torch.bfloat16, device=x.device)
        if want_z:
            z = torch.empty_like(y)
    _check(load_library().lbs_conv(mode, ci, co, _vp(x), _vp(wpack), _vp(bias), _vp(res), _vp(zprev),
                               _vp(y), _vp(z), _vp(yf), int(nout), B, H, W, int(blocks),
                               _stream()))
    return yf if mode == FWD_OUT else (y, z)


def wgrad(ci, co, cir, cor, x, gz, scale=1.0, blocks=512):
    """Weight and bias gradients (lbs_wgrad): (dw [9*cir*cor], db [cor])."""
    import torch
    B, H, W, _ = x.shape
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.lbs_wgrad_scratch_floats(ci, co, cir, cor, int(blocks), ctypes.byref(n)))
    part = torch.empty(n.value, dtype=torch.float32, device=x.device)
    dw = torch.empty(9 * cir * cor, dtype=torch.float32, device=x.device)
    db = torch.empty(cor, dtype=torch.float32, device=x.device)
    _check(lib.lbs_wgrad(ci, co, cir, cor, _vp(x), _vp(gz), B, H, W, float(scale), _vp(part),
                         int(blocks), _vp(dw), _vp(db), _stream()))
    return dw, db


def bias_grad(gz, nreal, scale=1.0):
    import torch
    C = gz.shape[-1]
    npix = gz.numel() // C
    part = torch.empty(1024 * C, dtype=torch.float32, device=gz.device)
    db = torch.empty(nreal, dtype=torch.float32, device=gz.device)
    _check(load_library().lbs_bias_grad(_vp(gz), npix, C, nreal, float(scale), _vp(part), _vp(db), _stream()))
    return db


def mse(pred, target, CO=OUT_CHANNELS):
    import torch
    nout = pred.shape[-1]
    npix = pred.numel() // nout
    gout = torch.empty(pred.shape[:-1] + (CO,), dtype=torch.bfloat16, device=pred.device)
    part = torch.empty(512, dtype=torch.float64, device=pred.device)
    loss = torch.empty(1, dtype=torch.float64, device=pred.device)
    _check(load_library().lbs_mse(_vp(pred), _vp(target), npix, nout, CO, _vp(gout), _vp(part), _vp(loss),
                              _stream()))
    return loss, gout


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(load_library().lbs_adam(_vp(p), _vp(g), _vp(m), _vp(v), p.numel(), float(lr), float(b1),
                               float(b2), float(eps), int(t), _stream()))


def _scales(s):
    return lbs_scales(*(s if s is not None else DEFAULT_SCALES))


def fields_to_input(fields, vx, cond, walls=True, scales=None, out=None):
    """fields [B,3,H,W] FP64, vx [B,W] FP32, cond [B,2] FP32 -> x [B,H,W,8] bf16."""
    import torch
    B, _, H, W = fields.shape
    if out is None:
        out = torch.empty((B, H, W, IN_CHANNELS), dtype=torch.bfloat16, device=fields.device)
    sc = _scales(scales)
    _check(load_library().lbs_fields_to_input(_vp(fields), B, H, W, _vp(vx), _vp(cond), int(bool(walls)),
                                          ctypes.byref(sc), _vp(out), _stream()))
    return out


def make_target(f0, f1, scales=None, out=None):
    import torch
    B, _, H, W = f0.shape
    if out is None:
        out = torch.empty((B, H, W, OUT), dtype=torch.float32, device=f0.device)
    sc = _scales(scales)
    _check(load_library().lbs_make_target(_vp(f0), _vp(f1), B, H * W, ctypes.byref(sc), _vp(out), _stream()))
    return out


def apply_output(f0, out, scales=None, f1=None):
    import torch
    B, _, H, W = f0.shape
    if f1 is None:
        f1 = torch.empty_like(f0)
    sc = _scales(scales)
    _check(load_library().lbs_apply_output(_vp(f0), _vp(out), B, H * W, ctypes.byref(sc), _vp(f1), _stream()))
    return f1


def compare(a, b, out=None):
    """Per instance (sum n_a, sum n_b, max |n_a - n_b| / n_b, bad nodes of a,
    sum (n_a - n_b)^2, sum n_b^2)."""
    import torch
    B, _, H, W = a.shape
    if out is None:
        out = torch.empty((B, 6), dtype=torch.float64, device=a.device)
    _check(load_library().lbs_compare(_vp(a), _vp(b), B, H * W, _vp(out), _stream()))
    return out


def project_mass(a, ref, mask_dev):
    B, _, H, W = a.shape
    _check(load_library().lbs_project_mass(_vp(a), _vp(ref), B, H * W, _vp(mask_dev), _stream()))


# ---- data, training, audited runs --------------------------------------------

def _batch_for(draws, check_every=100, drift=True, shape=None):
    specs = [dict(Lx=w.Lx, Ly=w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                  fext=w.fext()) for w in draws]
    b = Batch(specs, fp32=True, check_every=check_every, drift_correct=drift)
    for i, w in enumerate(draws):
        b.init(i, w.n0())
    if shape is not None:
        b.set_launch(shape[0], shape[1], steps_per_launch=shape[2])
    return b


# Launch shape (threads, rows, steps per launch) of the lattice runs of the
# experiment: two steps per launch in one-wave strips of 50 columns and
# chunks of 32 rows. On 256 lattices of 256 x 128 it is the fastest shape of
# the full batch (127 us per step against 159 with the default one-step
# shape; 64 or 128 rows are within 1-3%), and its short chunks keep a
# subset of the instances (the audits) filling the device. Results do not
# depend on the shape.
LATTICE_SHAPE = (64, 32, 2)


def conditions(draws, device="cuda"):
    """Per-instance network conditions: force table [B,W] and (U, T) [B,2]."""
    import torch
    vx = torch.tensor(np.stack([w.fext() for w in draws]), dtype=torch.float32, device=device)
    cond = torch.tensor([[w.U, w.T] for w in draws], dtype=torch.float32, device=device)
    return vx.contiguous(), cond.contiguous()


def screen(draws, steps: int, keep: Optional[int] = None):
    """The draws whose lattices pass every stability check over `steps`
    steps (a stiff quench under strong shear can fail), in order, at most
    `keep` of them."""
    b = _batch_for(draws)
    b.step(steps)
    status = b.status()
    b.close()
    ok = [w for w, s in zip(draws, status) if s == 0]
    return ok[:keep] if keep is not None else ok


def generate_data(draws, warmup: int, chunks: int, K: int = 50, scales=None, shape=None):
    """Run the lattices of `draws` (one size) for `warmup` steps, then record
    `chunks` chunks of K steps: inputs [chunks*B,H,W,8] bf16 and targets
    [chunks*B,H,W,3] FP32, ordered chunk-major (a run of consecutive samples
    spans different instances)."""
    import torch
    B = len(draws)
    H, W = draws[0].Ly, draws[0].Lx
    b = _batch_for(draws, shape=shape)
    vx, cond = conditions(draws)
    x = torch.empty((chunks * B, H, W, IN_CHANNELS), dtype=torch.bfloat16, device="cuda")
    tgt = torch.empty((chunks * B, H, W, OUT), dtype=torch.float32, device="cuda")
    f = [torch.empty((B, 3, H, W), dtype=torch.float64, device="cuda") for _ in range(2)]
    if warmup:
        b.step(warmup)
    b.moments_device(f[0])
    for c in range(chunks):
        fields_to_input(f[c % 2], vx, cond, True, scales, out=x[c * B:(c + 1) * B])
        b.step(K)
        b.moments_device(f[(c + 1) % 2])
        make_target(f[c % 2], f[(c + 1) % 2], scales, out=tgt[c * B:(c + 1) * B])
    torch.cuda.synchronize()
    status = b.status()
    b.close()
    return x, tgt, status


def train(net: Net, x, tgt, iters: int, batch: int = 16, lr: float = 1e-3, seed: int = 0,
          log_every: int = 100, time_limit: Optional[float] = None):
    """Minibatch Adam with a cosine learning-rate decay over the iterations
    or, with a time limit that ends training first, over the time (the
    schedule follows whichever is further along). Minibatches are contiguous
    runs of `batch` samples at random offsets. Returns [(iteration, loss)]
    sampled every log_every iterations (the loss of that iteration's
    minibatch); the time is read there too."""
    import torch
    g = np.random.Generator(np.random.PCG64(seed))
    n = x.shape[0]
    hist = []
    t0 = time.perf_counter()
    tfrac = 0.0  # fraction of the time limit used, as of the last log point
    for it in range(iters):
        s = int(g.integers(0, n - batch + 1))
        frac = max(it / iters, tfrac)
        cur = lr * 0.5 * (1.0 + np.cos(np.pi * min(frac, 1.0)))
        loss = net.train_step(x[s:s + batch], tgt[s:s + batch], max(cur, lr * 0.02))
        if it % log_every == 0 or it == iters - 1:
            hist.append((it, float(loss.item())))
            if time_limit is not None:
                el = time.perf_counter() - t0
                tfrac = el / time_limit
                if el > time_limit:
                    break
    torch.cuda.synchronize()
    return hist


def dataset_loss(net: Net, x, tgt, batch: int) -> float:
    """Mean loss of the network over every sample of (x, tgt), in minibatches
    of at most `batch` (forward passes only)."""
    n, tot = x.shape[0], 0.0
    for s in range(0, n, batch):
        e = min(n, s + batch)
        loss, _ = mse(net.forward(x[s:e]), tgt[s:e])
        tot += float(loss.item()) * (e - s)
    return tot / n


def persistence_loss(tgt, batch: int) -> float:
    """Mean loss over tgt of the prediction that nothing changes (zero
    output), the baseline a trained network's dataset loss compares with."""
    import torch
    n, tot = tgt.shape[0], 0.0
    for s in range(0, n, batch):
        e = min(n, s + batch)
        loss, _ = mse(torch.zeros_like(tgt[s:e]), tgt[s:e])
        tot += float(loss.item()) * (e - s)
    return tot / n


@dataclass
class RunStats:
    chunks: int = 0
    lattice_chunks: int = 0       # instance-chunks stepped by the lattice
    surrogate_chunks: int = 0     # instance-chunks taken from the network
    audits: int = 0
    audit_failures: int = 0
    mass_rejects: int = 0
    audit_errors: List[float] = field(default_factory=list)

    @property
    def fallback_rate(self) -> float:
        tot = self.lattice_chunks + self.surrogate_chunks
        return self.lattice_chunks / tot if tot else 0.0


class SurrogateRun:
    """Advance a batch of same-size lattices chunk by chunk with the network,
    audited by the lattice (see the module docstring).

    An instance is trusted after `need` consecutive audits within `tol`
    (relative density error against the lattice's own chunk: the maximum
    over nodes of |dn| / n for norm "max", the root-mean-square ratio
    ||dn||_2 / ||n||_2 for norm "rms"); until
    then it runs on the lattice with its predictions audited every chunk.
    A trusted instance is audited once every `audit_every` chunks (rotating)
    and goes back on probation when an audit fails. mass_tol bounds the
    relative change of the total density of a raw prediction: beyond it the
    chunk falls back to the lattice (the workload's fallback rule: mass drift
    above 1e-4). Predictions that pass are then projected onto the exact FP64
    mass, so the run's own mass drift stays at rounding level. The "rms" norm
    lets large local errors through (runs re-entered from such predictions
    have diverged) and is kept for measurement only; the evaluation uses
    "max".

    predictor "persist" replaces the network by the prediction that nothing
    changes over the chunk (same audit, tolerance and re-entry): the
    baseline that shows what the network itself adds.

    reentry "shift" adds f_eq(prediction) - f_eq(chunk start) to the
    populations, so they keep their non-equilibrium part (an accepted
    persistence prediction then leaves the lattice exactly as it was);
    "eq" replaces them by f_eq(prediction).

    budget (a run-level tolerance, or None) replaces the rotation: the
    error of an instance's last passed audit stands for the error of each
    chunk taken from the predictor after it, these add up until the next
    audit, and a trusted instance is audited when the next chunk would take
    the sum beyond the budget, or after audit_every chunks at most. An
    audited chunk runs on the lattice, so the sum starts again from zero."""

    def __init__(self, net: Optional[Net], batch: Batch, draws, K: int = 50, tol: float = 1e-2,
                 mass_tol: float = 1e-4, audit_every: int = 8, need: int = 1, norm: str = "max",
                 scales=None, predictor: str = "net", reentry: str = "shift",
                 budget: Optional[float] = None):
        import torch
        if norm not in ("max", "rms"):
            raise ValueError("norm must be 'max' or 'rms'")
        if budget is not None and not budget >= 0:
            raise ValueError("budget must be None or >= 0")
        self.budget = budget
        if predictor not in ("net", "persist") or (predictor == "net" and net is None):
            raise ValueError("predictor must be 'net' (with a network) or 'persist'")
        if reentry not in ("shift", "eq"):
            raise ValueError("reentry must be 'shift' or 'eq'")
        self.norm, self.predictor, self.reentry = norm, predictor, reentry
        self.net, self.b, self.K = net, batch, int(K)
        self.tol, self.mass_tol = tol, mass_tol
        self.audit_every, self.need = int(audit_every), int(need)
        self.scales = scales
        self.B = batch.count
        H, W = batch.shapes[0]
        self.vx, self.cond = conditions(draws)
        dev = "cuda"
        self.f0 = torch.empty((self.B, 3, H, W), dtype=torch.float64, device=dev)
        self.f1 = torch.empty_like(self.f0)
        self.flb = torch.empty_like(self.f0)
        self.x = torch.empty((self.B, H, W, IN_CHANNELS), dtype=torch.bfloat16, device=dev)
        self.out = torch.empty((self.B, H, W, OUT), dtype=torch.float32, device=dev)
        self.cmp = torch.empty((self.B, 6), dtype=torch.float64, device=dev)
        self.passes = np.zeros(self.B, dtype=np.int64)
        self.est = np.zeros(self.B)            # error of the last passed audit
        self.spent = np.zeros(self.B)          # estimated error taken since then
        self.since = np.zeros(self.B, dtype=np.int64)  # chunks since the last audit
        self.stats = RunStats()

    def chunk(self):
        import torch
        c = self.stats.chunks
        B = self.B
        b = self.b
        b.moments_device(self.f0)
        if self.predictor == "net":
            fields_to_input(self.f0, self.vx, self.cond, True, self.scales, out=self.x)
            self.net.forward(self.x, self.out)
            apply_output(self.f0, self.out, self.scales, self.f1)
        else:
            self.f1.copy_(self.f0)
        raw = compare(self.f1, self.f0, self.cmp).cpu().numpy()
        mass_drift = np.abs(raw[:, 0] - raw[:, 1]) / raw[:, 1]
        bad = (raw[:, 3] > 0) | ~(mass_drift <= self.mass_tol)
        trusted = self.passes >= self.need
        if self.budget is None:
            due = (np.arange(B) % self.audit_every) == (c % self.audit_every)
        else:
            due = (self.spent + self.est > self.budget) | (self.since + 1 >= self.audit_every)
        audit = ~bad & (~trusted | due)
        lattice = bad | audit | ~trusted
        accept = ~lattice
        self.stats.mass_rejects += int(bad.sum())
        self.passes[bad] = 0
        # project every prediction that is used or audited
        proj = torch.from_numpy((~bad).astype(np.int32)).to(self.f0.device)
        project_mass(self.f1, self.f0, proj)
        b.step_subset(self.K, lattice.astype(np.int32))
        if audit.any():
            b.moments_device(self.flb)
            cm = compare(self.f1, self.flb, self.cmp).cpu().numpy()
            err = cm[:, 2] if self.norm == "max" else np.sqrt(cm[:, 4] / cm[:, 5])
            for i in np.nonzero(audit)[0]:
                self.stats.audits += 1
                self.stats.audit_errors.append(float(err[i]))
                if err[i] <= self.tol:
                    self.passes[i] += 1
                    self.est[i] = float(err[i])
                else:
                    self.stats.audit_failures += 1
                    self.passes[i] = 0
        if self.reentry == "shift":
            b.shift_equilibrium(self.f0, self.f1, accept.astype(np.int32))
        else:
            b.set_equilibrium(self.f1, accept.astype(np.int32))
        # chunks on the lattice are exact; accepted ones add their estimate
        self.spent = np.where(lattice, 0.0, self.spent + self.est)
        self.since = np.where(lattice, 0, self.since + 1)
        self.stats.lattice_chunks += int(lattice.sum())
        self.stats.surrogate_chunks += int(accept.sum())
        self.stats.chunks += 1
        return accept


FLOPS_PER_NODE = 2 * 9 * (IN_REAL * WIDTH + BLOCKS * WIDTH * WIDTH + WIDTH * OUT)


def _audited_eval(net, test, start, eval_chunks, K, tol, audit_every, log, shape=None,
                  scales=None):
    """One evaluation window: the lattice alone from step `start` for
    eval_chunks * K steps, then the same span from the same state with the
    audited network (max and RMS norms) and with the persistence baseline,
    re-entering accepted chunks by shift (the default) and, for the
    baseline, also as pure equilibria; both predictors also with audits
    spaced by a run-level error budget equal to the tolerance. Every variant
    audits with the max norm and falls back on a raw mass drift above 1e-4."""
    import torch
    n = len(test)
    steps = eval_chunks * K
    ref = _batch_for(test, shape=shape)
    ref.step(start)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ref.step(steps)
    torch.cuda.synchronize()
    t_lb = time.perf_counter() - t2
    fr = ref.moments_device()
    ref.close()
    win = {"start_step": start, "steps": steps, "lattice_seconds": round(t_lb, 4)}
    # (key, norm, predictor, re-entry, run-level budget, longest audit gap);
    # the control fails every audit, so every chunk runs on the lattice
    # (subset steps, which skip the drift shift the reference applies): it
    # measures how far the lattice alone drifts from the reference through
    # the same machinery
    for key, norm, pred, reentry, budget, gap in (
            ("lattice_control", "max", "persist", "shift", None, audit_every),
            ("audit_max", "max", "net", "shift", None, audit_every),
            ("persist_max", "max", "persist", "shift", None, audit_every),
            ("persist_max_eq_reentry", "max", "persist", "eq", None, audit_every),
            ("audit_max_budget", "max", "net", "shift", tol, 2 * audit_every),
            ("persist_max_budget", "max", "persist", "shift", tol, 2 * audit_every)):
        sgb = _batch_for(test, shape=shape)
        sgb.step(start)
        m0 = np.array([sgb.reduce(i)["mass"] for i in range(n)])
        run = SurrogateRun(net, sgb, test, K=K, tol=-1.0 if key == "lattice_control" else tol,
                           audit_every=gap, norm=norm, predictor=pred, reentry=reentry,
                           budget=budget, scales=scales)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(eval_chunks):
            run.chunk()
        torch.cuda.synchronize()
        t_sg = time.perf_counter() - t3
        fs = sgb.moments_device()
        c = compare(fs, fr).cpu().numpy()
        alive = np.array(sgb.status()) == 0
        max_err = np.where(alive, c[:, 2], np.inf)
        rms_err = np.where(alive, np.sqrt(c[:, 4] / c[:, 5]), np.inf)
        m1 = np.array([sgb.reduce(i)["mass"] if alive[i] else np.nan for i in range(n)])
        st = run.stats
        err_final = max_err if norm == "max" else rms_err
        win[key] = {
            "surrogate_seconds": round(t_sg, 4), "speedup": round(t_lb / t_sg, 3),
            "fallback_rate": round(st.fallback_rate, 4), "audits": st.audits,
            "audit_failures": st.audit_failures, "mass_rejects": st.mass_rejects,
            "audit_error_median": float(np.median(st.audit_errors)) if st.audit_errors else None,
            "final_error_max_norm": {"max": float(max_err.max()), "median": float(np.median(max_err))},
            "final_error_rms": {"max": float(rms_err.max()), "median": float(np.median(rms_err))},
            "final_frac_within_tol": float(np.mean(err_final <= tol)),
            "mass_drift_max": float(np.nanmax(np.abs(m1 - m0) / m0)),
            "diverged": int((~alive).sum()),
        }
        log(f"eval[start {start}, {key}]: lattice {t_lb * 1e3:.1f} ms, run {t_sg * 1e3:.1f} ms, "
            f"fallback {st.fallback_rate:.3f}, audit err median {win[key]['audit_error_median']}, "
            f"final within tol {win[key]['final_frac_within_tol']:.3f}, diverged {(~alive).sum()}")
        sgb.close()
    return win, fr


def experiment(H: int = 128, W: int = 256, train_count: int = 256, train_seed: int = 2024,
               test_count: int = 256, test_seed: int = 99,
               train_windows=((300, 12), (8000, 12)), eval_starts=(300, 10000),
               K: int = 50, iters: int = 10**7, batch: int = 16,
               lr: float = 2e-3, train_seconds: float = 60.0, eval_chunks: int = 20,
               audit_every: int = 8, tol: float = 1e-2, scales=None, log=None):
    """Train on lattice data recorded in the windows (start step, chunks),
    then advance `test_count` fresh lattices (other draws) by
    eval_chunks * K steps from each step of eval_starts, several times from
    the same state: with the lattice alone, with the audited network and
    with the audited persistence baseline. Returns timings, errors against
    the lattice-only run and the fallback statistics."""
    import torch
    import lbsynth as ls

    def say(*a):
        if log:
            log(" ".join(str(v) for v in a))

    out = {"size": f"{W}x{H}", "K": K,
           "scales": list(scales if scales is not None else DEFAULT_SCALES)}
    t0 = time.perf_counter()
    raw = ls.surrogate_draws(train_count, seed=train_seed, Lx=W, Ly=H)
    draws = screen(raw, max(s + c * K for s, c in train_windows))
    shape = LATTICE_SHAPE
    xs, ts, spans = [], [], []
    for s, c in train_windows:
        x, tgt, status = generate_data(draws, s, c, K, scales=scales, shape=shape)
        assert all(v == 0 for v in status)
        spans.append((sum(v.shape[0] for v in xs), x.shape[0]))
        xs.append(x)
        ts.append(tgt)
    x, tgt = torch.cat(xs), torch.cat(ts)
    del xs, ts
    out["train_samples"] = int(x.shape[0])
    out["train_windows"] = [{"start_step": s, "chunks": c} for s, c in train_windows]
    out["train_draws_dropped_unstable"] = len(raw) - len(draws)
    say(f"data: {x.shape[0]} samples in {time.perf_counter() - t0:.1f} s")
    net_t = Net(batch, H, W, train=True)
    net_t.set_params(init_params(0))
    loss0 = dataset_loss(net_t, x, tgt, batch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = train(net_t, x, tgt, iters, batch, lr, log_every=200, time_limit=train_seconds)
    t_train = time.perf_counter() - t1
    its = hist[-1][0] + 1
    loss1 = dataset_loss(net_t, x, tgt, batch)
    per_window = [dataset_loss(net_t, x[a:a + m], tgt[a:a + m], batch) for a, m in spans]
    persist = [persistence_loss(tgt[a:a + m], batch) for a, m in spans]
    out["train"] = {"iterations": its, "batch": batch, "seconds": round(t_train, 1),
                    "dataset_loss_before": loss0, "dataset_loss_after": loss1,
                    "dataset_loss_after_per_window": per_window,
                    "persistence_loss_per_window": persist,
                    "minibatch_loss_curve": [(it, round(l, 7))
                                             for it, l in hist[:: max(1, len(hist) // 20)]],
                    "train_tflops": round(3 * FLOPS_PER_NODE * H * W * batch * its / t_train / 1e12, 1)}
    say(f"train: {its} iterations in {t_train:.1f} s, loss over the {x.shape[0]} samples "
        f"{loss0:.3e} -> {loss1:.3e} (per window {', '.join(f'{v:.3e}' for v in per_window)}; "
        f"persistence {', '.join(f'{v:.3e}' for v in persist)})")
    params = net_t.params().clone()
    net_t.close()
    del x, tgt, net_t
    torch.cuda.empty_cache()

    raw = ls.surrogate_draws(test_count + test_count // 4, seed=test_seed, Lx=W, Ly=H)
    test = screen(raw, max(eval_starts) + eval_chunks * K, keep=test_count)
    out["test_draws_dropped_unstable"] = raw.index(test[-1]) + 1 - len(test)
    test_count = len(test)
    net = Net(test_count, H, W)
    net.set_params(params)
    out["eval"] = {"instances": test_count, "tol": tol, "audit_every": audit_every,
                   "lattice_launch": {"threads": shape[0], "rows": shape[1],
                                      "steps_per_launch": shape[2]},
                   "windows": []}
    say(f"lattice launch shape: {shape}")
    fr = None
    for start in eval_starts:
        win, fr = _audited_eval(net, test, start, eval_chunks, K, tol, audit_every, say, shape,
                                scales)
        out["eval"]["windows"].append(win)
    # forward throughput on the whole test batch
    vx, cond = conditions(test)
    xin = fields_to_input(fr, vx, cond, True, scales)
    yo = torch.empty((test_count, H, W, OUT), dtype=torch.float32, device="cuda")
    for _ in range(3):  # warm-up: the first calls after the lattice runs are slower
        net.forward(xin, yo)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        net.forward(xin, yo)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = FLOPS_PER_NODE * H * W * test_count
    out["forward"] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 1),
                      "peak_bf16_tflops": 2500.0, "frac": round(flops / (ms * 1e-3) / 1e12 / 2500.0, 4),
                      "gflop_per_instance": round(FLOPS_PER_NODE * H * W / 1e9, 3)}
    net.close()
    return out
