"""Oracle Spec of a benchmark workload (same constants and measurement lists)."""
from oracle import operators as ops


def oracle_spec(wl, instance=0):
    s = wl.spec
    op = "ns3d_fixed" if s.chi_fixed else s.op
    return ops.Spec(op, s.dims, s.lengths, s.n_levels,
                    params={"re": s.re, "diam": s.diam, "lam": s.lam,
                            "chi_shift": s.chi_shift, "tau_coef": s.tau_coef, "u_ref": s.u_ref},
                    weights={"pde": s.w_pde, "reg": s.w_reg, "bc": s.w_bc},
                    meas=[(f, t, idx, vals, w) for inst, f, t, idx, vals, w in wl.meas
                          if inst == instance],
                    chi=wl.chi if s.chi_fixed else None, centering=s.centering)
