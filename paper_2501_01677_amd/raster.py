"""Python boundary of libpgsag: a batch of masked renders over caller-owned
torch buffers, and the autograd function around it.

PyTorch provides device memory and the stream; every step of the forward
and backward pass runs in the library's HIP kernels.  A ``Batch`` owns the
output planes, the upstream-gradient planes, the parameter-gradient arrays,
the workspace and the device copy of the packed descriptor; the Gaussian
parameters and masks stay owned by the caller and must outlive the batch.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
import math

import numpy as np
import torch

from . import _abi as A

OUTPUTS = (("rgb", 3), ("normal", 3), ("dist", 1), ("depth", 1), ("alpha", 1), ("n_contrib", 1))
# upstream-gradient planes: the outputs' and that of the soft contributor
# count (the sum of the blended alphas; the GC-load term's gradient)
GRAD_OUTPUTS = ("rgb", "normal", "dist", "depth", "alpha", "count")
_CHANNELS = dict(OUTPUTS, count=1)
# the differentiable outputs of the autograd function
DIFF_OUTPUTS = ("rgb", "normal", "dist", "depth", "alpha")
PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@dataclass
class RenderConfig:
    tile: int = 16
    persistent: bool = False
    queue_chunk: int = 1
    workgroups_per_cu: int = 4
    alpha_min: float = 1.0 / 255.0
    t_min: float = 1e-4
    alpha_max: float = 0.99
    dilation: float = 0.3
    z_near: float = 0.2
    fov_clamp: float = 1.3
    logit_min: float = float(np.float32(-math.log(254.0)))
    depth_guard: float = 1e-6
    bg: tuple = (0.0, 0.0, 0.0)
    bwd_reduce: int = 0  # 0: matrix-core per-record sums, 1: wave lane exchanges
    deterministic: bool = False  # bit-reproducible gradients (segmented reduction, no float atomics)

    def to_c(self) -> A.Config:
        c = A.Config()
        c.tile, c.persistent, c.queue_chunk = self.tile, int(self.persistent), self.queue_chunk
        c.workgroups_per_cu = self.workgroups_per_cu
        for k in ("alpha_min", "t_min", "alpha_max", "dilation", "z_near", "fov_clamp", "logit_min",
                  "depth_guard"):
            setattr(c, k, getattr(self, k))
        c.bg = (C.c_float * 3)(*self.bg)
        c.bwd_reduce = int(self.bwd_reduce)
        c.deterministic = int(bool(self.deterministic))
        return c


@dataclass
class LossConfig:
    """Weights of the training losses (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 11)."""
    lambda_rgb: float = 1.0
    lambda_normal: float = 0.01
    boundary_weight: float = 0.1
    lambda_load: float = 0.0
    normal_norm: int = 1
    normal_eps: float = 1e-6
    load_term: int = 0  # 0: tile-count variance (value only), 1: Eq. 9 GC-load through the soft count

    def to_c(self) -> A.LossConfig:
        c = A.LossConfig()
        for k in ("lambda_rgb", "lambda_normal", "boundary_weight", "lambda_load", "normal_norm", "normal_eps",
                  "load_term"):
            setattr(c, k, getattr(self, k))
        return c


class CapacityError(RuntimeError):
    pass


class DeviceError(RuntimeError):
    """The device reported that the outputs of the last forward are invalid
    (a bounded wait of a single-pass scan gave up)."""


# largest pair capacity the library plans for (pgsag_plan: 1..2^30-1)
MAX_PAIR_CAPACITY = (1 << 30) - 1


def _capacity(want):
    want = int(want)
    if want > MAX_PAIR_CAPACITY:
        raise CapacityError(f"{want} (tile, Gaussian) pairs needed; the library plans at most {MAX_PAIR_CAPACITY}")
    return max(1, want)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_camera(cam) -> A.Camera:
    c = A.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.R = (C.c_float * 9)(*np.asarray(cam.R, np.float32).reshape(-1).tolist())
    c.t = (C.c_float * 3)(*np.asarray(cam.t, np.float32).reshape(-1).tolist())
    return c


def gaussians_to_device(gs, device="cuda"):
    """scenes.GaussianSet (numpy) -> dict of contiguous float32 device tensors."""
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in gs.arrays().items()}
    d["sh_degree"] = gs.sh_degree
    return d


class Batch:
    """A batch of renders of one or more Gaussian sets (one launch per stage).

    sets:    list of dicts with device tensors means [3,n], log_scales [3,n],
             quats [4,n], opacity_logits [n], sh [K,3,n] and int sh_degree.
    renders: list of dicts with set (int), camera (width, height, fx, fy, cx,
             cy, R, t attributes) and mask (device uint8 [H,W] or None).
    """

    def __init__(self, sets, renders, cfg: RenderConfig | None = None, pair_capacity=None,
                 want_grads=True, outputs=tuple(n for n, _ in OUTPUTS), grad_outputs=GRAD_OUTPUTS,
                 device="cuda", grads=None):
        self.lib = A.lib()
        self.cfg = cfg or RenderConfig()
        self.sets = sets
        self.renders = renders
        self.device = device
        self.want_grads = want_grads
        self.out = []
        self.gout = []
        for rd in renders:
            cam = rd["camera"]
            H, W = int(cam.height), int(cam.width)
            o = {}
            for name, c in OUTPUTS:
                if name in outputs:
                    dt = torch.int32 if name == "n_contrib" else torch.float32
                    o[name] = torch.empty((c, H, W) if c > 1 else (H, W), dtype=dt, device=device)
            self.out.append(o)
            g = {}
            if want_grads:
                for name in grad_outputs:
                    c = _CHANNELS[name]
                    g[name] = torch.zeros((c, H, W) if c > 1 else (H, W), dtype=torch.float32, device=device)
            self.gout.append(g)
        self.grads = []
        if want_grads:
            if grads is not None:       # caller-owned gradient tensors (e.g. views of one flat buffer)
                self.grads = list(grads)
            else:
                for s in sets:
                    self.grads.append({k: torch.zeros_like(s[k]) for k in PARAMS})
        n_rec = sum(int(sets[rd["set"]]["means"].shape[1]) for rd in renders)
        if pair_capacity is None:
            pair_capacity = min(max(1 << 16, 8 * n_rec), MAX_PAIR_CAPACITY)
        self.generation = 0  # forwards run so far (the autograd function checks it)
        self._pack(_capacity(pair_capacity))

    # ------------------------------------------------------------ packing
    def _c_arrays(self):
        gs = (A.Gaussians * len(self.sets))()
        gr = (A.Grads * len(self.sets))()
        for i, s in enumerate(self.sets):
            gs[i].n = int(s["means"].shape[1])
            gs[i].sh_degree = int(s["sh_degree"])
            for k in PARAMS:
                t = s[k]
                assert t.dtype == torch.float32 and t.is_contiguous(), k
                setattr(gs[i], k, _p(t))
            if self.want_grads:
                for k in PARAMS:
                    setattr(gr[i], k, _p(self.grads[i][k]))
        rs = (A.Render * len(self.renders))()
        for i, rd in enumerate(self.renders):
            rs[i].set = int(rd["set"])
            rs[i].cam = make_camera(rd["camera"])
            m = rd.get("mask")
            if m is not None:
                assert m.dtype == torch.uint8 and m.is_contiguous()
            rs[i].mask = _p(m)
            for name, _ in OUTPUTS:
                setattr(rs[i].out, name, _p(self.out[i].get(name)))
            for name in GRAD_OUTPUTS:
                setattr(rs[i].gout, name, _p(self.gout[i].get(name)))
        return gs, gr, rs

    def _pack(self, capacity):
        cfg = self.cfg.to_c()
        gs, gr, rs = self._c_arrays()
        info = A.PlanInfo()
        A.check(self.lib.pgsag_plan(C.byref(cfg), gs, len(self.sets), rs, len(self.renders), capacity,
                                    C.byref(info)), "pgsag_plan")
        self.info = info
        self.host_desc = (C.c_uint8 * info.desc_bytes)()
        A.check(self.lib.pgsag_pack(C.byref(cfg), gs, gr if self.want_grads else None, len(self.sets), rs,
                                    len(self.renders), capacity, self.host_desc, info.desc_bytes),
                "pgsag_pack")
        self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=self.device)
        host = torch.frombuffer(bytearray(bytes(self.host_desc)), dtype=torch.uint8)
        self.dev_desc = host.to(self.device)
        lay = A.Layout()
        A.check(self.lib.pgsag_layout_of(self.host_desc, C.byref(lay)), "pgsag_layout_of")
        self.layout = lay
        self.capacity = capacity

    def repack(self):
        """Re-reads parameter / buffer pointers (after replacing tensors)."""
        self._pack(self.capacity)

    # ------------------------------------------------------------- passes
    def _events(self, events):
        if events is None:
            return None
        arr = (C.c_void_p * len(events))(*[C.c_void_p(e) for e in events])
        return arr

    def forward(self, stream=None, events=None, check_overflow=True):
        """Renders every view.  With check_overflow the status word is read
        (a stream synchronisation) and the batch replans and reruns once if
        the pair capacity was too small."""
        for _ in range(3):
            A.check(self.lib.pgsag_forward(self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                           int(self.info.workspace_bytes), _stream(stream),
                                           self._events(events)), "pgsag_forward")
            self.generation += 1
            if not check_overflow:
                return self.out
            st = self.check_status(stream)
            if not st.overflow:
                return self.out
            self._pack(_capacity(max(st.pairs_needed * 5 // 4, 1024)))
        raise CapacityError("pair capacity overflow persists after replanning")

    def check_status(self, stream=None):
        """Reads the status word of the last forward (a stream
        synchronisation) and raises DeviceError if the device reported its
        results invalid; returns the status (overflow is left to the caller)."""
        st = self.status(stream)
        if st.error:
            raise DeviceError(f"device reported invalid binning results (error word {st.error}); "
                              "the outputs of the last forward are invalid")
        return st

    def fit_capacity(self, slack=1.25, stream=None):
        """Replans the pair capacity to slack x what the last forward needed."""
        st = self.check_status(stream)
        want = _capacity(max(1024, st.pairs_needed * slack))
        if want != self.capacity:
            self._pack(want)
        return st

    def backward(self, gouts=None, stream=None, events=None):
        """Gradients of sum(gout * out) with respect to the raw parameters.
        ``gouts``: list (per render) of dicts name -> tensor, copied into the
        batch's gradient planes (missing names keep their current values)."""
        if not self.want_grads:
            raise RuntimeError("batch was built without gradients")
        if gouts is not None:
            for i, g in enumerate(gouts):
                for name, t in g.items():
                    if t is None:
                        self.gout[i][name].zero_()
                    else:
                        self.gout[i][name].copy_(t.reshape(self.gout[i][name].shape))
        A.check(self.lib.pgsag_backward(self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                        int(self.info.workspace_bytes), _stream(stream),
                                        self._events(events)), "pgsag_backward")
        return self.grads

    def backward_adam(self, lr, state, m_offset, v_offset, b1=0.9, b2=0.999, eps=1e-8, write_grads=False,
                      stream=None, events=None):
        """Backward pass with the Adam update of every parameter folded in:
        parameters updated in place, moments at the gradient tensors' storage
        plus m_offset / v_offset floats, step count in ``state``."""
        if not self.want_grads:
            raise RuntimeError("batch was built without gradients")
        cfg = A.AdamConfig()
        cfg.lr, cfg.b1, cfg.b2, cfg.eps = lr, b1, b2, eps
        cfg.step_state = state.data_ptr()
        cfg.m_offset, cfg.v_offset = int(m_offset), int(v_offset)
        cfg.write_grads = int(bool(write_grads))
        A.check(self.lib.pgsag_backward_adam(self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                             int(self.info.workspace_bytes), C.byref(cfg), _stream(stream),
                                             self._events(events)), "pgsag_backward_adam")

    def binning(self, stream=None):
        A.check(self.lib.pgsag_binning(self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                       int(self.info.workspace_bytes), _stream(stream)), "pgsag_binning")

    def status(self, stream=None):
        st = A.Status()
        A.check(self.lib.pgsag_read_status(self.host_desc, _p(self.workspace), C.byref(st),
                                           _stream(stream)), "pgsag_read_status")
        return st

    def load_stats(self, weights=None, stream=None):
        out = torch.empty((len(self.renders), 4), dtype=torch.float32, device=self.device)
        warr = None
        if weights is not None:
            warr = (C.c_void_p * len(self.renders))(*[None if w is None else w.data_ptr() for w in weights])
        A.check(self.lib.pgsag_load_stats(self.host_desc, _p(self.dev_desc), _p(self.workspace), warr,
                                          _p(out), _stream(stream)), "pgsag_load_stats")
        return out

    def loss(self, gt, lc: LossConfig | None = None, out=None, stream=None, weights=None):
        """Loss of the last forward against ground-truth images gt[r]
        (float32 [3,H,W]); writes dL/d(rgb, normal, depth) (and, with the
        GC-load term, dL/d(soft count)) into the batch's gradient planes.
        ``weights``: per render the Eq. 9 pixel weights (float32 [H,W]) or
        None (= 1).  Returns device float [n_renders, 4] = (total, L_rgb,
        L_ban, load term)."""
        lc = lc or LossConfig()
        if out is None:
            out = torch.empty((len(self.renders), 4), dtype=torch.float32, device=self.device)
        for t in gt:
            assert t.dtype == torch.float32 and t.is_contiguous()
        arr = (C.c_void_p * len(self.renders))(*[t.data_ptr() for t in gt])
        warr = None
        if weights is not None:
            for w in weights:
                assert w is None or (w.dtype == torch.float32 and w.is_contiguous())
            warr = (C.c_void_p * len(self.renders))(*[None if w is None else w.data_ptr() for w in weights])
        A.check(self.lib.pgsag_loss(C.byref(lc.to_c()), self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                    int(self.info.workspace_bytes), arr, warr, _p(out), _stream(stream)),
                "pgsag_loss")
        return out

    def luminance_weights(self, render, gt, out=None, stream=None):
        """Eq. 9 per-pixel weights of render `render` from its ground truth."""
        cam = self.renders[render]["camera"]
        if out is None:
            out = torch.empty((int(cam.height), int(cam.width)), dtype=torch.float32, device=self.device)
        assert gt.dtype == torch.float32 and gt.is_contiguous()
        A.check(self.lib.pgsag_luminance_weights(self.host_desc, _p(self.dev_desc), _p(self.workspace),
                                                 int(self.info.workspace_bytes), render, _p(gt), _p(out),
                                                 _stream(stream)), "pgsag_luminance_weights")
        return out

    # ------------------------------------------------------ workspace views
    def view(self, name, dtype, count, cols=None):
        off = getattr(self.layout, name)
        itemsize = torch.tensor([], dtype=dtype).element_size()
        n = count * (cols or 1)
        t = self.workspace[off:off + n * itemsize].view(dtype)
        return t.view(count, cols) if cols else t


def adam_step(params, grads, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    """Fused Adam update in place over matching float32 device tensors."""
    L = A.lib()
    for t in (params, grads, m, v):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == params.numel()
    A.check(L.pgsag_adam_step(_p(params), _p(grads), _p(m), _p(v), params.numel(), lr, b1, b2, eps, step,
                              _stream(stream)), "pgsag_adam_step")


class _RasterizeFn(torch.autograd.Function):
    """The backward reads the per-pixel state the batch's workspace holds
    and the parameter tensors as they are then, so it is only valid for the
    batch's latest forward with unchanged parameters: the forward generation
    and the parameters' version counters are saved and checked."""

    @staticmethod
    def forward(ctx, batch, *flat):
        batch.forward()
        ctx.batch = batch
        ctx.generation = batch.generation
        ctx.versions = [t._version for t in flat]
        ctx.flat = flat
        outs = []
        for o in batch.out:
            for name in DIFF_OUTPUTS:
                outs.append(o[name].clone())
            outs.append(o["n_contrib"].clone())
        ctx.mark_non_differentiable(*outs[len(DIFF_OUTPUTS)::len(DIFF_OUTPUTS) + 1])
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        batch = ctx.batch
        if batch.generation != ctx.generation:
            raise RuntimeError("the batch ran another forward since this output was rendered; "
                               "its backward would differentiate the newer forward")
        if [t._version for t in ctx.flat] != ctx.versions:
            raise RuntimeError("a Gaussian parameter tensor was modified in place between "
                               "the forward and the backward")
        per = len(DIFF_OUTPUTS) + 1
        gouts = []
        for i in range(len(batch.renders)):
            g = {}
            for j, name in enumerate(DIFF_OUTPUTS):
                gi = grads[i * per + j]
                g[name] = None if gi is None else gi.contiguous()
            g["count"] = None  # no soft-count gradient through autograd (zeroed)
            gouts.append(g)
        batch.backward(gouts)
        res = [None]
        for s in batch.grads:
            res += [s[k].clone() for k in PARAMS]
        return tuple(res)


class MaskedRasterizer:
    """Differentiable masked rendering of fixed Gaussian sets and views.

    ``rasterizer()`` returns, per render, a dict of rgb [3,H,W], normal
    [3,H,W], dist, depth, alpha [H,W] (differentiable) and n_contrib (int32).
    Gradients flow to the parameter tensors of ``sets`` (which should have
    requires_grad set by the caller)."""

    def __init__(self, sets, renders, cfg: RenderConfig | None = None, pair_capacity=None):
        self.batch = Batch(sets, renders, cfg, pair_capacity, want_grads=True)

    def __call__(self):
        flat = []
        for s in self.batch.sets:
            flat += [s[k] for k in PARAMS]
        outs = _RasterizeFn.apply(self.batch, *flat)
        per = len(DIFF_OUTPUTS) + 1
        res = []
        for i in range(len(self.batch.renders)):
            d = {name: outs[i * per + j] for j, name in enumerate(DIFF_OUTPUTS)}
            d["n_contrib"] = outs[i * per + len(DIFF_OUTPUTS)]
            res.append(d)
        return res


def adam_step_device(params, grads, m, v, lr, state, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    """Fused Adam update with the step count in ``state`` (device int32 [4],
    state[0] = steps taken, incremented by this call), so a captured graph
    replays with the right bias corrections."""
    L = A.lib()
    for t in (params, grads, m, v):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.numel() == params.numel()
    assert state.dtype == torch.int32 and state.numel() >= 4
    A.check(L.pgsag_adam_step_device(_p(params), _p(grads), _p(m), _p(v), params.numel(), lr, b1, b2, eps,
                                     _p(state), _stream(stream)), "pgsag_adam_step_device")


def _param_sizes(n, sh_degree):
    K = (sh_degree + 1) ** 2
    return (("means", (3, n)), ("log_scales", (3, n)), ("quats", (4, n)), ("opacity_logits", (n,)),
            ("sh", (K, 3, n)))


class Trainer:
    """One optimisation step over a batch of renders: forward, the loss of
    Sec. 4.2-4.3 against ground-truth images, backward, and one fused Adam
    update over every raw parameter of every set.  Parameters live in one
    flat device buffer, gradients and Adam moments in three equal slices of
    another; the per-set tensors are views into them.  With ``fused`` (the
    default) the update runs inside the backward projection kernel
    (pgsag_backward_adam; the gradients are then stored only with
    ``keep_grads``), otherwise as a separate fused Adam launch.  ``step`` is capturable: ``capture``
    records it once into a HIP graph and ``replay`` runs it."""

    def __init__(self, sets, renders, gt, cfg: RenderConfig | None = None, lc: LossConfig | None = None,
                 lr=1e-3, betas=(0.9, 0.999), eps=1e-8, pair_capacity=None, device="cuda", fused=True,
                 keep_grads=False, weights=None):
        total = 0
        for s in sets:
            for _, shp in _param_sizes(int(s["means"].shape[1]), int(s["sh_degree"])):
                total += int(np.prod(shp))
        self.total = total
        self.fused = fused
        self.keep_grads = keep_grads
        self.P = torch.empty(total, dtype=torch.float32, device=device)
        # gradients, first and second moments: three equal slices of one
        # buffer, so the fused update finds the moments at fixed offsets
        self.GMV = torch.zeros(3 * total, dtype=torch.float32, device=device)
        self.G = self.GMV[:total]
        self.m = self.GMV[total:2 * total]
        self.v = self.GMV[2 * total:]
        self.state = torch.zeros(4, dtype=torch.int32, device=device)
        self.params, grads = [], []
        off = 0
        for s in sets:
            n = int(s["means"].shape[1])
            pv, gv = {"sh_degree": int(s["sh_degree"])}, {}
            for k, shp in _param_sizes(n, int(s["sh_degree"])):
                c = int(np.prod(shp))
                pv[k] = self.P[off:off + c].view(shp)
                pv[k].copy_(s[k].reshape(shp))
                gv[k] = self.G[off:off + c].view(shp)
                off += c
            self.params.append(pv)
            grads.append(gv)
        self.batch = Batch(self.params, renders, cfg, pair_capacity=pair_capacity, device=device, grads=grads)
        self.gt = list(gt)
        self.weights = None if weights is None else list(weights)  # Eq. 9 pixel weights per render
        self.lc = lc or LossConfig()
        self.lr, self.betas, self.eps = lr, betas, eps
        self.loss_out = torch.zeros((len(renders), 4), dtype=torch.float32, device=device)
        self.graph = None

    def fit(self, slack=1.25):
        """Runs one forward with the overflow check and sizes the pair
        capacity to slack x what it needed (no parameter update)."""
        self.batch.forward()
        self.batch.fit_capacity(slack)

    def step(self, stream=None):
        b = self.batch
        b.forward(stream=stream, check_overflow=False)
        b.loss(self.gt, self.lc, out=self.loss_out, stream=stream, weights=self.weights)
        if self.fused:
            b.backward_adam(self.lr, self.state, self.total, 2 * self.total, self.betas[0], self.betas[1], self.eps,
                            write_grads=self.keep_grads, stream=stream)
        else:
            b.backward(stream=stream)
            adam_step_device(self.P, self.G, self.m, self.v, self.lr, self.state, self.betas[0], self.betas[1],
                             self.eps, stream=stream)
        return self.loss_out

    def capture(self):
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.step()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.loss_out

    def overflowed(self):
        """Whether the last step's forward ran out of pair capacity (then
        that step is invalid: fit() again).  Raises DeviceError if the device
        reported the step's binning invalid."""
        return bool(self.batch.check_status().overflow)
