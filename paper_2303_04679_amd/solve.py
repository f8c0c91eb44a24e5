"""Iterate the mODIL step until the residual metric reaches a target.

Runs a batch of independent instances at once (one parameter pack); every
`check_every` iterations the residual metric r of every instance (RMS of the
cell-integrated PDE residual, in FP64) is evaluated on the device and copied
to the host, the first iteration at which an instance reaches r <= r_target
is recorded, and the loop ends when all instances have converged or the
iteration cap is reached.  An optional monitor (for instance the error
against a reference solution) is evaluated at the same checks with its own
target; then an instance has converged once both targets are met.  The
learning rate may follow a schedule.
"""
import dataclasses
import math
import time
from typing import Callable, Optional

import numpy as np
import torch

from .modil import Context


@dataclasses.dataclass
class SolveResult:
    iterations: np.ndarray      # first checked iteration with r <= target (-1: not reached)
    r_final: np.ndarray         # residual metric at the end
    r_history: list             # (iteration, r[batch]) every check
    seconds: float              # wall time of the loop (device synchronised)
    theta: torch.Tensor         # final parameter pack
    iters_run: int              # iteration count at the end (it0 included)
    iterations_monitor: Optional[np.ndarray] = None  # first check with monitor <= target
    monitor_history: Optional[list] = None           # (iteration, monitor[batch]) every check
    moments: Optional[tuple] = None                  # Adam (m, v) at the end


def cosine_lr(lr0, lr_min, total):
    """Cosine decay from lr0 to lr_min over `total` iterations, then lr_min."""
    def f(t):
        if t >= total:
            return lr_min
        return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * t / total))
    return f


def solve(ctx: Context, theta: torch.Tensor, lr: float | Callable[[int], float], max_iters: int,
          r_target: float = 1e-6, check_every: int = 50, betas=(0.9, 0.999), eps=1e-8,
          log: Optional[Callable[[int, np.ndarray], None]] = None,
          monitor: Optional[Callable[[torch.Tensor], np.ndarray]] = None,
          monitor_target: float = 0.0, moments: Optional[tuple] = None, it0: int = 0,
          stop_when_done: bool = True) -> SolveResult:
    """Adam iterations it0 .. max_iters from theta (and Adam moments `moments`,
    zero if None); iteration numbers (steps of the bias correction, checks,
    the schedule) continue from it0."""
    B = ctx.spec.batch
    a = theta.clone()
    b = ctx.new_pack()
    m, v = (ctx.new_pack(), ctx.new_pack()) if moments is None else (moments[0].clone(), moments[1].clone())
    r_dev = torch.empty((B,), dtype=torch.float64, device=ctx.device)
    r_host = torch.empty((B,), dtype=torch.float64, pin_memory=True)
    iters = np.full(B, -1, dtype=np.int64)
    iters_m = np.full(B, -1 if monitor else 0, dtype=np.int64)
    hist, mhist = [], []
    lr_f = lr if callable(lr) else (lambda t: lr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = it0
    while True:
        if it % check_every == 0:
            ctx.residual_metric(a, out=r_dev)
            r_host.copy_(r_dev, non_blocking=True)
            torch.cuda.current_stream(ctx.device).synchronize()
            r = r_host.numpy().copy()
            hist.append((it, r))
            newly = (iters < 0) & (r <= r_target)
            iters[newly] = it
            if monitor:
                e = np.asarray(monitor(a), dtype=np.float64)
                mhist.append((it, e))
                iters_m[(iters_m < 0) & (e <= monitor_target)] = it
            if log:
                log(it, r)
            done = np.all(iters >= 0) and np.all(iters_m >= 0) and stop_when_done
            if done or it >= max_iters or not np.all(np.isfinite(r)):
                break
        ctx.step(a, b, m, v, it + 1, lr=lr_f(it), beta1=betas[0], beta2=betas[1], eps=eps)
        a, b = b, a
        it += 1
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return SolveResult(iters, hist[-1][1], hist, secs, a, it,
                       iters_m if monitor else None, mhist if monitor else None, (m, v))
