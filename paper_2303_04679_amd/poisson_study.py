"""The Poisson study of Section 3.1 on the GPU: convergence of mODIL with Adam
and with L-BFGS against the number of multigrid levels.

    python -m paper_2303_04679_amd.poisson_study --out poisson_study.json

Zero-Dirichlet Poisson problem on [0, 1]^d, d = 1, 2, 3, N = 32 cells per
axis, L = 1 .. 5 levels (32 down to 2 cells), with both discretizations of the
section: cell-based values (Dirichlet condition by quadratic extrapolation
through the wall) and node-based values (N + 1 nodes per axis, the condition
imposed on the boundary nodes directly).  The right-hand side is the
discrete Laplacian of u_ref(x) = g(prod_i 5 (1 - x_i) x_i),
g(v) = (v^5 / (1 + v^5))^(1/5), so u_ref solves the discrete problem exactly.
Initial guess zero.  Adam: step 0.005, 400 iterations; L-BFGS: 50 pairs, 400
iterations.  The error is the RMS difference of the fine field from u_ref
after every iteration.  Everything runs in FP64 through the library.
"""
import argparse
import json
import time

import numpy as np
import torch

from .modil import LBFGS, Context, ProblemSpec


def u_ref(n, d, centering="cell"):
    x = (np.arange(n) + 0.5) / n if centering == "cell" else np.arange(n + 1) / n
    grids = np.meshgrid(*([x] * d), indexing="ij")
    v = np.ones((x.size,) * d)
    for g in grids:
        v = v * 5.0 * (1.0 - g) * g
    return (v ** 5 / (1.0 + v ** 5)) ** 0.2


def laplacian(u, h):
    """Cell-based 2nd-order Laplacian with ghost = -2 u_0 + u_1 / 3 at both walls."""
    out = np.zeros_like(u)
    for a in range(u.ndim):
        v = np.moveaxis(u, a, 0)
        lo = -2.0 * v[:1] + v[1:2] / 3.0
        hi = -2.0 * v[-1:] + v[-2:-1] / 3.0
        p = np.concatenate([lo, v, hi], axis=0)
        out += np.moveaxis((p[2:] - 2.0 * p[1:-1] + p[:-2]) / (h * h), 0, a)
    return out


def laplacian_nodes(u, h):
    """Finite-difference Laplacian at the interior nodes (0 on the boundary nodes)."""
    out = np.zeros_like(u)
    inner = tuple(slice(1, -1) for _ in range(u.ndim))
    for a in range(u.ndim):
        lo = tuple(slice(0, -2) if b == a else slice(1, -1) for b in range(u.ndim))
        hi = tuple(slice(2, None) if b == a else slice(1, -1) for b in range(u.ndim))
        out[inner] += (u[hi] - 2.0 * u[inner] + u[lo]) / (h * h)
    return out


def problem(n, d, L, centering="cell"):
    ctx = Context(ProblemSpec("poisson", (n,) * d, (1.0,) * d, L, dtype="f64", w_pde=1.0,
                              centering=centering))
    ur = u_ref(n, d, centering)
    f = laplacian(ur, 1.0 / n) if centering == "cell" else laplacian_nodes(ur, 1.0 / n)
    ctx.set_field("forcing0", torch.tensor(f.ravel(), dtype=torch.float64, device=ctx.device))
    return ctx, torch.tensor(ur, dtype=torch.float64, device=ctx.device)


def rms_error(ctx, theta, ur):
    """RMS error of the fine field; node-based boundary values are the imposed zeros."""
    u = ctx.fine_views(ctx.prolong(theta))[0]
    if ctx.spec.centering == "node":
        inner = tuple(slice(1, -1) for _ in range(u.dim()))
        d = torch.zeros_like(u)
        d[inner] = u[inner] - ur[inner]
        return float(torch.sqrt((d ** 2).mean()))
    return float(torch.sqrt(((u - ur) ** 2).mean()))


def check_exact(ctx, ur):
    """The library's loss vanishes at u_ref placed on the finest level."""
    th = ctx.new_pack()
    ctx.level_views(th)[0][0].copy_(ur)
    return float(ctx.loss(th).sum())


def run_adam(ctx, ur, iters, lr):
    a, b, m, v = ctx.new_pack(), ctx.new_pack(), ctx.new_pack(), ctx.new_pack()
    err = [rms_error(ctx, a, ur)]
    for t in range(1, iters + 1):
        ctx.step(a, b, m, v, t, lr=lr)
        a, b = b, a
        err.append(rms_error(ctx, a, ur))
    return err


def run_lbfgs(ctx, ur, iters, history):
    th = ctx.new_pack()
    lb = LBFGS(ctx, history=history)
    err, evals = [rms_error(ctx, th, ur)], [0]
    for _ in range(iters):
        info = lb.step(th)
        err.append(rms_error(ctx, th, ur))
        evals.append(evals[-1] + info["evals"])
        if info["status"] == 2 or info["loss"] == 0.0:
            break
    lb.close()
    return err, evals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--iters", type=int, default=400)
    ap.add_argument("--lr", type=float, default=0.005)
    ap.add_argument("--history", type=int, default=50)
    args = ap.parse_args()
    res = {"n": args.n, "iters": args.iters, "lr": args.lr, "history": args.history, "runs": []}
    t0 = time.time()
    for centering in ("cell", "node"):
        for d in (1, 2, 3):
            for L in range(1, 6):
                ctx, ur = problem(args.n, d, L, centering)
                exact = check_exact(ctx, ur)
                ea = run_adam(ctx, ur, args.iters, args.lr)
                el, ev = run_lbfgs(ctx, ur, args.iters, args.history)
                res["runs"].append({"centering": centering, "d": d, "L": L,
                                    "loss_at_reference": exact, "adam": ea,
                                    "lbfgs": el, "lbfgs_evals": ev})
                print(f"[poisson] {centering} d={d} L={L}: loss(u_ref) {exact:.1e}  "
                      f"adam err {ea[-1]:.2e}  lbfgs err {el[-1]:.2e} after {len(el) - 1} "
                      f"iterations ({ev[-1]} evaluations)", flush=True)
                ctx.close()
    res["seconds"] = time.time() - t0
    json.dump(res, open(args.out, "w"))


if __name__ == "__main__":
    main()
