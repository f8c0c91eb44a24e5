"""The Burgers reconstruction of Section 3.2 on the GPU: mODIL with L-BFGS
(six levels) against ODIL with L-BFGS (one level).

    python -m paper_2303_04679_amd.burgers_study --out burgers_study.json

Unit space-time domain (x, t) in [0, 1]^2, 64 x 64 cells, inviscid Burgers
with the first-order upwind flux.  The reference solution comes from the
initial condition u = (1 - cos 6 pi x) / 2 marched row by row with the same
discrete residual (implicit time level; the zero Dirichlet condition as a
ghost value 0 beyond each wall, so the upwind flux lets the wave leave).  The reference values are imposed at 84
points spaced evenly along the edges of a centred square (the paper gives the
number of points, not the rectangle; three sizes are run: sides 0.95, 0.75 and
1/3 of the domain), with weight 1/84 each; the loss has no smoothing term.  A
second run adds uniform noise U[0, 0.05] to the imposed values.  Initial guess
zero.  The error is the RMS difference from the reference over the whole grid
and over the cells inside the square.
"""
import argparse
import json
import time

import numpy as np
import torch

from . import synth
from .modil import LBFGS, Context, ProblemSpec


def upwind_flux(a, b):
    """Murman-Roe flux of f = u^2 / 2 between states a (left) and b (right)."""
    return 0.25 * (a * a + b * b) - 0.5 * np.abs(0.5 * (a + b)) * (b - a)


def reference(n, x):
    """Rows t_k = k / n of the implicit upwind scheme from (1 - cos 6 pi x) / 2."""
    dt, dx = 1.0 / n, 1.0 / n
    rows = [0.5 * (1.0 - np.cos(6.0 * np.pi * x))]
    for _ in range(n - 1):
        prev = rows[-1]
        u = prev.copy()
        for _ in range(50):  # Newton on r(u) = (u - prev)/dt + (F_{i+1/2} - F_{i-1/2})/dx
            # faces -1/2 .. n-1/2; the zero Dirichlet condition as a ghost value 0
            # outside each wall, so the wall faces carry the upwind flux
            ue = np.concatenate([[0.0], u, [0.0]])
            a, b = ue[:-1], ue[1:]
            flux = upwind_flux(a, b)
            r = (u - prev) / dt + (flux[1:] - flux[:-1]) / dx
            m = 0.5 * (a + b)
            s = np.sign(m)
            dFa = 0.5 * a - 0.25 * s * (b - a) + 0.5 * np.abs(m)
            dFb = 0.5 * b - 0.25 * s * (b - a) - 0.5 * np.abs(m)
            J = np.eye(n) / dt
            for k in range(n + 1):  # face k - 1/2 between cells k - 1 and k
                if k - 1 >= 0:
                    J[k - 1, k - 1] += dFa[k] / dx
                    if k < n:
                        J[k - 1, k] += dFb[k] / dx
                if k < n:
                    if k - 1 >= 0:
                        J[k, k - 1] -= dFa[k] / dx
                    J[k, k] -= dFb[k] / dx
            du = np.linalg.solve(J, -r)
            u = u + du
            if np.max(np.abs(du)) < 1e-14:
                break
        rows.append(u)
    return np.stack(rows)


def rectangle_cells(n, frac, points=84):
    """Cells of `points` points spaced evenly along the edges of the square of
    side `frac` centred in the unit domain (starting at a corner), as flat
    indices (row t, column x), and the mask of the cells inside the square."""
    lo, side = 0.5 - 0.5 * frac, frac
    cells = []
    for k in range(points):
        s = 4.0 * side * k / points
        e, r = int(s // side), s % side
        x, t = [(lo + r, lo), (lo + side, lo + r), (lo + side - r, lo + side), (lo, lo + side - r)][e]
        cells.append((min(int(t * n), n - 1), min(int(x * n), n - 1)))
    idx = np.array([t * n + x for t, x in cells], dtype=np.int32)
    if np.unique(idx).size != idx.size:
        raise ValueError("points closer than a cell")
    c = (np.arange(n) + 0.5) / n
    inside = ((c[:, None] > lo) & (c[:, None] < lo + side) & (c[None, :] > lo) & (c[None, :] < lo + side))
    return np.sort(idx), inside


def run(n, L, ref, idx, vals, inside, iters, history):
    spec = ProblemSpec("burgers", (n, n), (1.0, 1.0), L, dtype="f64", max_meas=len(idx),
                       w_pde=1.0, w_reg=0.0)
    ctx = Context(spec)
    ctx.set_measurements(0, idx, vals, 1.0 / len(idx))
    th = ctx.new_pack()
    lb = LBFGS(ctx, history=history)
    refd = torch.tensor(ref, dtype=torch.float64, device=ctx.device)
    ins = torch.tensor(inside, device=ctx.device)

    def err():
        d2 = (ctx.fine_views(ctx.prolong(th))[0] - refd) ** 2
        return float(torch.sqrt(d2.mean())), float(torch.sqrt(d2[ins].mean()))

    e0 = err()
    errors, errors_in, losses, evals = [e0[0]], [e0[1]], [], [0]
    t0 = time.perf_counter()
    for _ in range(iters):
        info = lb.step(th)
        e = err()
        errors.append(e[0])
        errors_in.append(e[1])
        losses.append(info["loss"])
        evals.append(evals[-1] + info["evals"])
        if info["status"] == 2:
            break
    secs = time.perf_counter() - t0
    lb.close()
    ctx.close()
    return {"L": L, "error": errors, "error_inside": errors_in, "loss": losses, "evals": evals,
            "seconds": secs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--history", type=int, default=50)
    args = ap.parse_args()
    n = args.n
    x = (np.arange(n) + 0.5) / n
    ref = reference(n, x)
    out = {"n": n, "runs": []}
    for frac in (0.95, 0.75, 1.0 / 3.0):
        idx, inside = rectangle_cells(n, frac)
        clean = ref.reshape(-1)[idx]
        noisy = clean + synth.rng(5).uniform(0.0, 0.05, size=idx.size)
        for data_name, vals in (("clean", clean), ("noisy", noisy)):
            for L in (6, 1):
                r = run(n, L, ref, idx, vals, inside, args.iters, args.history)
                r.update({"data": data_name, "square": frac, "points": int(idx.size)})
                out["runs"].append(r)
                e, ei = r["error"], r["error_inside"]
                k40 = min(40, len(e) - 1)
                print(f"[burgers] square {frac:.2f} {data_name} L={L}: error {e[-1]:.3f} "
                      f"(inside {ei[-1]:.3f}) after {len(e) - 1} iterations; at 40: {e[k40]:.3f} "
                      f"(inside {ei[k40]:.3f}); loss {r['loss'][-1]:.2e}; {r['seconds']:.2f} s", flush=True)
    json.dump(out, open(args.out, "w"))


if __name__ == "__main__":
    main()
