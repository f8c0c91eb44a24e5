"""Learned warm start for the lid-driven cavity (not part of the paper).

A small convolutional network (the fixed topology documented with
modil_cnn_desc in include/modil.h) maps the rasterised measurements and the
Reynolds number of an instance to the three coarsest-but-one multigrid
levels (32^2, 16^2, 8^2 for a 128^2 grid) of its converged solution.  The
iteration then starts from levels (0, 0, y32, y16, y8) instead of zero.

Training targets are canonical: the over-parameterised decomposition makes
the levels a solve ends with depend on its path, so each target level is the
block average of the converged fine field minus what the coarser targets
already explain after interpolation.

The network runs in the library's HIP kernels; this module only allocates
device memory and sequences the calls.
"""
import ctypes
import dataclasses

import numpy as np
import torch
import torch.nn.functional as F

from . import _lib as L
from .modil import Context


def _p(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


@dataclasses.dataclass
class NetConfig:
    batch: int = 64
    size: int = 128
    n_obs: int = 64
    width1: int = 48
    width2: int = 64
    width3: int = 64
    out_ch: int = 3
    re_center: float = 550.0
    re_scale: float = 450.0

    def to_c(self):
        d = L.CnnDesc()
        for k in ("batch", "size", "n_obs", "width1", "width2", "width3", "out_ch"):
            setattr(d, k, int(getattr(self, k)))
        d.re_center, d.re_scale = float(self.re_center), float(self.re_scale)
        return d


class WarmStartNet:
    """Parameters, buffers and the library handle of one network."""

    def __init__(self, cfg: NetConfig, device="cuda", seed=0):
        self.cfg = cfg
        self.device = torch.device(device)
        d = cfg.to_c()
        self.lay = L.CnnLayout()
        L.check(L.lib().modil_cnn_layout(ctypes.byref(d), ctypes.byref(self.lay)))
        nb = int(self.lay.workspace_bytes)
        self._ws_raw = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        sh = (-self._ws_raw.data_ptr()) % 256
        self._ws = self._ws_raw[sh:sh + nb]
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        L.check(L.lib().modil_cnn_create(ctypes.byref(d), _p(self._ws), nb,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        n = int(self.lay.n_params)
        self.master = self.init_params(seed)
        self.bf16 = torch.empty(n, dtype=torch.int16, device=self.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.step_count = 0
        self.sync_bf16()
        B = cfg.batch
        self.img = torch.empty((B, int(self.lay.img_size)), dtype=torch.float32, device=self.device)
        self.acts = torch.empty((B, int(self.lay.act_size)), dtype=torch.float32, device=self.device)
        self.out = torch.empty((B, int(self.lay.out_size)), dtype=torch.float32, device=self.device)
        self.loss = torch.empty((), dtype=torch.float64, device=self.device)

    def layer_shapes(self):
        c = self.cfg
        return [(c.width1, 4, 4), (c.width2, c.width1, 3), (c.width3, c.width2, 3),
                (c.out_ch, c.width1, 3), (c.out_ch, c.width2, 3), (c.out_ch, c.width3, 3)]

    def init_params(self, seed):
        """He-normal weights, zero biases (host-side draw, seeded)."""
        g = np.random.default_rng(seed)
        out = np.zeros(int(self.lay.n_params), dtype=np.float32)
        for i, (co, ci, k) in enumerate(self.layer_shapes()):
            w0 = int(self.lay.w_offset[i])
            std = np.sqrt(2.0 / (ci * k * k)) if i < 3 else np.sqrt(1.0 / (ci * k * k))
            out[w0:w0 + co * ci * k * k] = g.normal(0.0, std, co * ci * k * k)
        return torch.tensor(out, device=self.device)

    def sync_bf16(self):
        L.check(L.lib().modil_cnn_to_bf16(self.h, _p(self.master), _p(self.bf16)))

    def rasterize(self, idx, u, v, re, batch=None):
        """idx [B][n_obs] int32, u, v [B][n_obs] float32, re [B] float32 (device)."""
        B = idx.shape[0] if batch is None else batch
        L.check(L.lib().modil_cnn_rasterize(self.h, B, _p(idx), _p(u), _p(v), _p(re), _p(self.img)))
        return self.img[:B]

    def forward(self, batch):
        L.check(L.lib().modil_cnn_forward(self.h, batch, _p(self.bf16), _p(self.img), _p(self.acts),
                                          _p(self.out)))
        return self.out[:batch]

    def loss_backward(self, batch, target):
        L.check(L.lib().modil_cnn_loss_backward(self.h, batch, _p(self.bf16), _p(self.img),
                                                _p(self.acts), _p(self.out), _p(target),
                                                _p(self.loss), _p(self.grad)))
        return self.loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        hp = L.AdamHP(lr, beta1, beta2, eps)
        L.check(L.lib().modil_cnn_adam(self.h, _p(self.master), _p(self.bf16), _p(self.m), _p(self.v),
                                       _p(self.grad), ctypes.byref(hp), self.step_count))

    def split(self, out):
        """Head maps of a batch of outputs: [(B, C, s/4, s/4), (B, C, s/8, s/8), (B, C, s/16, s/16)]."""
        c, s = self.cfg.out_ch, self.cfg.size
        res, o = [], 0
        for q in (s // 4, s // 8, s // 16):
            n = c * q * q
            res.append(out[:, o:o + n].view(-1, c, q, q))
            o += n
        return res

    def close(self):
        if getattr(self, "h", None):
            L.lib().modil_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------- level targets
def _prolonged(levels):
    """M(levels) of cavity fields through the library: levels is a list of
    [B, 3, n_l, n_l] tensors, finest first; returns [B, 3, n_0, n_0] (float64)."""
    from .modil import ProblemSpec
    B, n = levels[0].shape[0], levels[0].shape[-1]
    spec = ProblemSpec("cavity", (n, n), (1.0, 1.0), len(levels), dtype="f64", batch=B, max_meas=0)
    ctx = Context(spec, device=levels[0].device)
    pack = ctx.new_pack()
    for b in range(B):
        for lv, src in zip(ctx.level_views(pack, b), levels):
            for f in range(3):
                lv[f].copy_(src[b, f])
    out = ctx.prolong(pack).view(B, 3, n, n).clone()
    ctx.close()
    return out


def canonical_targets(fine):
    """fine [B, 3, N, N] converged (u, v, p) -> y at N/4, N/8, N/16.

    p is taken relative to its mean (the loss is invariant under p + c).
    y_c = A_c(fine) - T(coarser part), coarsest first, with A_c the block
    average; the interpolation T(...) is the library's prolongation of the
    decomposition (levels below the target set to zero on the finer ones).
    """
    f = fine.clone().double()
    f[:, 2] -= f[:, 2].mean(dim=(-1, -2), keepdim=True)
    a8 = F.avg_pool2d(f, 16)
    a16 = F.avg_pool2d(f, 8)
    a32 = F.avg_pool2d(f, 4)
    y8 = a8
    y16 = a16 - _prolonged([torch.zeros_like(a16), y8])
    y32 = a32 - _prolonged([torch.zeros_like(a32), y16, y8])
    return y32, y16, y8


def warm_levels(ctx: Context, theta, y32, y16, y8):
    """Write levels (0, 0, y32, y16, y8) of every instance into the pack theta."""
    theta.zero_()
    for b in range(ctx.spec.batch):
        lv = ctx.level_views(theta, b)
        for f in range(3):
            lv[2][f].copy_(y32[b, f])
            lv[3][f].copy_(y16[b, f])
            lv[4][f].copy_(y8[b, f])
    return theta


# ------------------------------------------------------------ the pipeline
def cavity_context(res, dtype="f32", n=128, levels=5):
    """A batched lid-driven-cavity context (forward problem, no data term)."""
    from .modil import ProblemSpec
    spec = ProblemSpec("cavity", (n, n), (1.0, 1.0), levels, dtype=dtype, batch=len(res),
                       max_meas=0, re=float(res[0]), w_pde=1.0)
    ctx = Context(spec)
    for b, re in enumerate(res):
        ctx.set_reynolds(b, float(re))
    return ctx


def fine_fields(ctx, theta):
    """[B, 3, N, N] fine (u, v, p) of a pack."""
    fine = ctx.prolong(theta)
    n = ctx.spec.dims
    return fine.view(ctx.spec.batch, 3, n[0], n[1])


def instances(seeds, n=128, n_obs=64):
    """Reynolds numbers and observed cells of the cavity instances with these seeds."""
    from . import synth
    re = np.array([synth.cavity_reynolds(s) for s in seeds])
    idx = np.stack([synth.cavity_points(s, (n, n), n_obs) for s in seeds]).astype(np.int32)
    return re, idx


def observe(fine, idx):
    """u, v of the fine fields at the observed cells: two [B, n_obs] float32 tensors."""
    B = fine.shape[0]
    flat = fine.reshape(B, 3, -1)
    ii = torch.as_tensor(idx, dtype=torch.long, device=fine.device)
    return (torch.gather(flat[:, 0], 1, ii).float().contiguous(),
            torch.gather(flat[:, 1], 1, ii).float().contiguous())


def predict(net, re, idx, u_obs, v_obs):
    """Head maps (y32, y16, y8) for a batch of instances.  Up to the network's
    batch capacity the maps are views of its output buffer (and its
    activations stay in place for loss_backward); larger batches are run in
    chunks and returned as new tensors."""
    B = len(re)
    cap = net.cfg.batch
    if B > cap:
        parts = []
        for s in range(0, B, cap):
            e = min(B, s + cap)
            y = predict(net, re[s:e], idx[s:e], u_obs[s:e].contiguous(), v_obs[s:e].contiguous())
            parts.append([t.clone() for t in y])
        return [torch.cat([p[k] for p in parts]) for k in range(3)]
    dev = net.device
    net.rasterize(torch.as_tensor(idx, device=dev), u_obs, v_obs,
                  torch.as_tensor(np.asarray(re, dtype=np.float32), device=dev), batch=B)
    return net.split(net.forward(B))


def _take(ctx, dst, src, which):
    """Copy the instances b with which[b] of pack src into pack dst."""
    for b in range(ctx.spec.batch):
        if which[b]:
            for ld, ls in zip(ctx.level_views(dst, b), ctx.level_views(src, b)):
                for fd, fs in zip(ld, ls):
                    fd.copy_(fs)
    return dst


def choose_start(ctx, cold, warm):
    """Fallback rule at the start: keep the warm start only where its residual
    metric is below the cold start's; returns (theta, used_warm[B])."""
    rc = ctx.residual_metric(cold).cpu().numpy()
    rw = ctx.residual_metric(warm).cpu().numpy()
    use = rw < rc
    return _take(ctx, cold.clone(), warm, use), use


def solve_with_fallback(ctx, cold, warm, lr, max_iters, checkpoint, r_target=1e-6, check_every=50):
    """mODIL from the warm start, judged by cold-start mODIL.

    The warm start is used only where its residual metric is below the cold
    start's (choose_start).  Both runs then go on to iteration `checkpoint`
    (a multiple of check_every); every instance whose warm run has not
    brought its residual below the cold run's at that iteration continues
    from the cold run's state (parameters and Adam moments), the others from
    the warm run's.  Returns (result, used_at_start, kept_at_checkpoint): the
    SolveResult of the continued run, whose `iterations` holds, per instance,
    the first checked iteration with r <= r_target of the run it kept.
    """
    from .solve import solve
    assert checkpoint % check_every == 0
    start, use0 = choose_start(ctx, cold, warm)
    rw = solve(ctx, start, lr, checkpoint, r_target=r_target, check_every=check_every,
               stop_when_done=False)
    rc = solve(ctx, cold, lr, checkpoint, r_target=r_target, check_every=check_every,
               stop_when_done=False)
    keep = use0 & (rw.r_final < rc.r_final)
    back = ~keep
    theta = _take(ctx, rw.theta.clone(), rc.theta, back)
    m = _take(ctx, rw.moments[0].clone(), rc.moments[0], back)
    v = _take(ctx, rw.moments[1].clone(), rc.moments[1], back)
    out = solve(ctx, theta, lr, max_iters, r_target=r_target, check_every=check_every,
                moments=(m, v), it0=checkpoint)
    early = np.where(keep, _first_hits(rw, r_target), _first_hits(rc, r_target))
    out.iterations = np.where(early >= 0, early, out.iterations)
    return out, use0, keep


def _first_hits(res, target):
    it = np.full(len(res.r_final), -1)
    for i, r in res.r_history:
        it[(it < 0) & (r <= target)] = i
    return it
