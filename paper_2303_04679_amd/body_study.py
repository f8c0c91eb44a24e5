"""Inferring a body's shape from velocity (Section 3.5) on the GPU: mODIL with
L-BFGS, six levels.

    python -m paper_2303_04679_amd.body_study --out body_study.json

Channel [0, 2] x [0, 1] x [0, 1] with inlet u = (1, 0, 0) at x = 0, outlet
p = 0 at x = 2 and free-slip walls elsewhere; steady Navier-Stokes with the
Brinkman penalisation of the body (lambda = 1, D = 0.4, Re = 60).  The grid
is cell-based, 128 x 64 x 64 cells (h = 1/64, the spacing of the paper's
129 x 65 x 65 nodes), or with --centering node the paper's 129 x 65 x 65
nodes; FP32 fields with FP64 loss sums, L = 6.  Node-based errors and volumes
are taken over the interior nodes (the boundary nodes' values are replaced by
the boundary conditions).

Bodies: the sphere of radius 0.2 centred at (0.5, 0.5, 0.5) and the
hemisphere, its part with y < 0.5.  The prescribed body fraction is the
volume fraction of each cell inside the body (4^3 sub-points per cell).

Forward problem: u, v, w, p with the body fraction fixed, from u = (1, 0, 0),
p = 0 (on the coarsest level), L-BFGS.  Its velocity at the measurement points
is the reference data.  Measurement points: a lattice of 19 x-positions
(x = 0.1, 0.2, ..., 1.9) and 6 x 6 (684 points) or 3 x 3 (171 points) evenly
spaced (y, z) positions (cell centres of a uniform partition of the unit
square), each at the cell containing it; three velocity components each, the
data term the mean over the points.

Inverse problem: u, v, w, p and the transformed body fraction chihat
(chi = 1 / (1 + exp(-(chihat - 5))), so chihat = 0 gives chi = 1/(1 + e^5)),
from u = (1, 0, 0), p = 0, chihat = 0, L-BFGS.  Reported every check: the
square root of the loss, the RMS error of the velocity against the forward
solution, and the relative L2 error of the body fraction against the
prescribed one; at the end also the inferred body volume (sum of chi h^3)
against the prescribed volume.
"""
import argparse
import json
import time

import numpy as np
import torch

from .modil import LBFGS, Context, ProblemSpec

NX, NY, NZ = 128, 64, 64
LENGTHS = (1.0, 1.0, 2.0)  # z, y, x
H = 1.0 / 64
CENTERING = "cell"   # set by --centering


def _extra():
    return 1 if CENTERING == "node" else 0


def body_fraction(kind, sub=4):
    """Volume fraction inside the body of every cell [z][y][x] or, node-based,
    of the cell of size h centred on every node."""
    e = _extra()

    def axis(n):
        c = (np.arange(n + e)[:, None] - 0.5 * e + (np.arange(sub)[None, :] + 0.5) / sub) * H
        return c.reshape(-1)
    x, y, z = axis(NX), axis(NY), axis(NZ)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    inside = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 <= 0.2 ** 2
    if kind == "hemisphere":
        inside &= Y < 0.5
    f = inside.reshape(NZ + e, sub, NY + e, sub, NX + e, sub).mean(axis=(1, 3, 5))
    return f.astype(np.float64)


def lattice_cells(m):
    """Flat indices [z][y][x] of the 19 x m x m measurement lattice: the cell
    containing each point or, node-based, its nearest node."""
    e = _extra()
    pos = (lambda v: int(round(v / H))) if e else (lambda v: int(v / H))
    xs = 0.1 * np.arange(1, 20)
    ys = (np.arange(m) + 0.5) / m
    cells = []
    for x in xs:
        for y in ys:
            for z in ys:
                i, j, k = pos(x), pos(y), pos(z)
                cells.append((k * (NY + e) + j) * (NX + e) + i)
    cells = np.array(cells, dtype=np.int32)
    assert np.unique(cells).size == cells.size
    return np.sort(cells)


def interior():
    """Values that carry equations: every cell, or the nodes off the boundary."""
    if CENTERING == "cell":
        return (slice(None),) * 3
    return (slice(1, -1),) * 3


def spec(chi_fixed, n_meas):
    return ProblemSpec("ns3d", (NZ, NY, NX), LENGTHS, 6, dtype="f32", chi_fixed=chi_fixed,
                       max_meas=3 * n_meas, re=60.0, diam=0.4, lam=1.0, chi_shift=5.0,
                       tau_coef=0.5, u_ref=1.0, w_pde=1.0, centering=CENTERING)


def initial(ctx):
    th = ctx.new_pack()
    ctx.level_views(th)[-1][0].fill_(1.0)  # u = 1 on the coarsest level
    return th


def run_lbfgs(ctx, th, iters, history, check_every, observe):
    lb = LBFGS(ctx, history=history)
    hist = [observe(th, 0, None)]
    evals = 0
    t0 = time.perf_counter()
    status = 0
    for it in range(1, iters + 1):
        info = lb.step(th)
        evals += info["evals"]
        status = info["status"]
        if it % check_every == 0 or it == iters or status == 2:
            hist.append(observe(th, it, info))
        if status == 2:
            break
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    lb.close()
    return hist, evals, secs, status


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--forward-iters", type=int, default=10000)
    ap.add_argument("--inverse-iters", type=int, default=20000)
    ap.add_argument("--history", type=int, default=50)
    ap.add_argument("--check-every", type=int, default=500)
    ap.add_argument("--bodies", default="sphere,hemisphere")
    ap.add_argument("--centering", choices=("cell", "node"), default="cell")
    args = ap.parse_args()
    global CENTERING
    CENTERING = args.centering
    e = _extra()
    out = {"grid": [NX + e, NY + e, NZ + e], "centering": CENTERING, "levels": 6, "runs": []}
    inner = interior()
    vol_cell = H ** 3
    for body in args.bodies.split(","):
        chi_ref = body_fraction(body)
        chi_t = torch.tensor(chi_ref.ravel(), dtype=torch.float32, device="cuda")
        # forward problem
        fctx = Context(spec(True, 0))
        fctx.set_field("chi", chi_t)
        th = initial(fctx)

        def observe_f(t, it, info):
            loss = float(fctx.loss(t).sum())
            print(f"[body] {body} forward it {it}: sqrt(loss) {loss ** 0.5:.3e}", flush=True)
            return {"it": it, "sqrt_loss": loss ** 0.5}

        fh, fev, fsec, _ = run_lbfgs(fctx, th, args.forward_iters, args.history, args.check_every,
                                      observe_f)
        u_ref = torch.stack(fctx.fine_views(fctx.prolong(th))[:3]).clone()
        out["runs"].append({"body": body, "problem": "forward", "history": fh, "evaluations": fev,
                            "seconds": fsec, "iterations": fh[-1]["it"]})
        fctx.close()
        for m in (6, 3):
            cells = lattice_cells(m)
            n = cells.size
            ictx = Context(spec(False, n))
            for c in range(3):
                vals = u_ref[c].reshape(-1)[torch.tensor(cells, device="cuda", dtype=torch.long)]
                ictx.set_measurements(c, cells, vals.double().cpu().numpy(), 1.0 / n)
            th = initial(ictx)
            chi_ref_d = torch.tensor(chi_ref, dtype=torch.float64, device="cuda")

            def observe_i(t, it, info):
                loss = float(ictx.loss(t).sum())
                f = ictx.fine_views(ictx.prolong(t))
                u = torch.stack(f[:3]).double()
                chi = torch.sigmoid(f[4].double() - 5.0)[inner]
                cr = chi_ref_d[inner]
                du = (u - u_ref.double())[(slice(None),) + inner]
                eu = float(torch.sqrt((du ** 2).sum(0).mean()))
                ec = float(torch.linalg.vector_norm(chi - cr) / torch.linalg.vector_norm(cr))
                vol = float(chi.sum()) * vol_cell
                print(f"[body] {body} {n} points it {it}: sqrt(loss) {loss ** 0.5:.3e} velocity error "
                      f"{eu:.3e} body fraction error {ec:.3f} volume {vol:.4f}", flush=True)
                return {"it": it, "sqrt_loss": loss ** 0.5, "velocity_error": eu,
                        "chi_error": ec, "volume": vol}

            ih, iev, isec, _ = run_lbfgs(ictx, th, args.inverse_iters, args.history,
                                          args.check_every, observe_i)
            out["runs"].append({"body": body, "problem": "inverse", "points": int(n), "history": ih,
                                "evaluations": iev, "seconds": isec, "iterations": ih[-1]["it"],
                                "volume_ref": float(chi_ref[inner].sum()) * vol_cell})
            ictx.close()
    json.dump(out, open(args.out, "w"))


if __name__ == "__main__":
    main()
