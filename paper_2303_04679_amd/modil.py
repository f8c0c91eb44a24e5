"""Python face of libmodil: problem description, parameter packs, iteration calls.

torch supplies device memory and the stream; every step of the iteration
runs in the HIP kernels of libmodil.  A Context owns its workspace tensor
and keeps references to the arrays attached to it.
"""
import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _lib as L

OPS = {"poisson": L.OP_POISSON, "burgers": L.OP_BURGERS, "heat": L.OP_HEAT_KX,
       "ns3d": L.OP_NS3D, "cavity": L.OP_CAVITY}
FIELDS = {"poisson": ("u",), "burgers": ("u",), "heat": ("u", "q"),
          "ns3d": ("u", "v", "w", "p", "chihat"), "ns3d_fixed": ("u", "v", "w", "p"),
          "cavity": ("u", "v", "p")}
PDE_EQUATIONS = {"poisson": 1, "burgers": 1, "heat": 1, "ns3d": 4, "cavity": 3}
DTYPES = {"f32": (L.F32, torch.float32), "f64": (L.F64, torch.float64)}


@dataclasses.dataclass
class ProblemSpec:
    """One mODIL problem (maps onto modil_problem)."""
    op: str
    dims: Sequence[int]
    lengths: Sequence[float]
    n_levels: int
    dtype: str = "f64"
    batch: int = 1
    max_meas: int = 0
    chi_fixed: bool = False
    re: float = 100.0
    diam: float = 0.4
    lam: float = 1.0
    chi_shift: float = 5.0
    tau_coef: float = 0.5
    u_ref: float = 1.0
    w_pde: float = 1.0
    w_reg: float = 0.0
    w_bc: float = 0.0
    centering: str = "cell"   # "cell", or "node" (Poisson, cavity, channel flow)
    fused_restrict: bool = False  # MODIL_FLAG_FUSED_RESTRICT

    @property
    def torch_dtype(self):
        return DTYPES[self.dtype][1]

    @property
    def fields(self):
        if self.op == "ns3d" and self.chi_fixed:
            return FIELDS["ns3d_fixed"]
        return FIELDS[self.op]

    @property
    def ndim(self):
        return len(self.dims)

    @property
    def fine_cells(self):
        """Values of one fine field (nodes for node-based grids)."""
        n = 1
        for d in self.dims:
            n *= int(d) + (1 if self.centering == "node" else 0)
        return n

    def to_c(self):
        p = L.Problem()
        p.ndim = len(self.dims)
        for a, (n, x) in enumerate(zip(self.dims, self.lengths)):
            p.dims[a] = int(n)
            p.lengths[a] = float(x)
        p.n_levels = int(self.n_levels)
        p.centering = L.NODE if self.centering == "node" else L.CELL
        p.dtype = DTYPES[self.dtype][0]
        p.op = OPS[self.op]
        p.flags = (L.FLAG_CHI_FIXED if self.chi_fixed else 0) | \
            (L.FLAG_FUSED_RESTRICT if self.fused_restrict else 0)
        p.batch = int(self.batch)
        p.max_meas = int(self.max_meas)
        p.re, p.diam, p.lambda_ = float(self.re), float(self.diam), float(self.lam)
        p.chi_shift, p.tau_coef, p.u_ref = float(self.chi_shift), float(self.tau_coef), float(self.u_ref)
        p.w_pde, p.w_reg, p.w_bc = float(self.w_pde), float(self.w_reg), float(self.w_bc)
        return p


def layout(spec: ProblemSpec) -> L.PackLayout:
    """Validate the problem and return its pack layout (host only, no GPU)."""
    out = L.PackLayout()
    p = spec.to_c()
    L.check(L.lib().modil_layout(ctypes.byref(p), ctypes.byref(out)))
    return out


def field_shape(spec, lay, level, field):
    dims = tuple(lay.field_dims[level][field])
    if spec.op == "heat" and spec.fields[field] == "q":
        return dims[2:]
    return dims[3 - spec.ndim:]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Context:
    """A libmodil context bound to a device, a stream and a workspace."""

    def __init__(self, spec: ProblemSpec, device="cuda", stream: Optional[torch.cuda.Stream] = None):
        self.spec = spec
        self._tile = True  # MODIL_OPT_TILE
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.lay = layout(spec)
        self.dtype = spec.torch_dtype
        nbytes = int(self.lay.workspace_bytes)
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        shift = (-self._ws_raw.data_ptr()) % 256
        self._ws = self._ws_raw[shift:shift + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = {}
        p = spec.to_c()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().modil_create(ctypes.byref(p), _ptr(self._ws), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    # ---------------------------------------------------------------- memory
    def new_pack(self, fill=0.0):
        return torch.full((int(self.lay.total),), fill, dtype=self.dtype, device=self.device)

    def new_fine(self):
        return torch.zeros((int(self.lay.fine_total),), dtype=self.dtype, device=self.device)

    def level_views(self, pack, instance=0):
        """Views of one instance: list over levels of list over fields."""
        out = []
        for lvl in range(self.spec.n_levels):
            row = []
            base = int(self.lay.level_offset[lvl]) + instance * int(self.lay.level_stride[lvl])
            for f in range(len(self.spec.fields)):
                shp = field_shape(self.spec, self.lay, lvl, f)
                n = 1
                for s in shp:
                    n *= s
                o = base + int(self.lay.field_offset[lvl][f])
                row.append(pack[o:o + n].view(shp))
            out.append(row)
        return out

    def fine_views(self, fine, instance=0):
        row = []
        base = instance * int(self.lay.level_stride[0])
        for f in range(len(self.spec.fields)):
            shp = field_shape(self.spec, self.lay, 0, f)
            n = 1
            for s in shp:
                n *= s
            o = base + int(self.lay.field_offset[0][f])
            row.append(fine[o:o + n].view(shp))
        return row

    def _check_pack(self, t, name, n=None):
        n = int(self.lay.total) if n is None else n
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: expected contiguous {self.dtype} tensor of {n} elements on {self.device}")

    # ------------------------------------------------------------ problem data
    def set_measurements(self, field, idx, values, weight, term="data", instance=0):
        import numpy as np
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        vals = np.ascontiguousarray(values, dtype=np.float64)
        t = {"data": L.TERM_DATA, "ic": L.TERM_IC}[term]
        L.check(L.lib().modil_set_measurements(
            self.h, instance, field, t, idx.size, idx.ctypes.data_as(ctypes.c_void_p),
            vals.ctypes.data_as(ctypes.c_void_p), float(weight)), self.h)

    def clear_measurements(self):
        L.check(L.lib().modil_clear_measurements(self.h), self.h)

    def set_field(self, which, tensor):
        """which: 'forcing0'..'forcing3' or 'chi'; tensor [batch][cells] or None."""
        slot = {"forcing0": 0, "forcing1": 1, "forcing2": 2, "forcing3": 3, "chi": L.FIELD_CHI}[which]
        if tensor is not None:
            n = self.spec.batch * self.spec.fine_cells
            if tensor.numel() != n or tensor.dtype != self.dtype or not tensor.is_contiguous():
                raise ValueError(f"{which}: expected contiguous {self.dtype} tensor of {n} elements")
        self._keep[which] = tensor
        L.check(L.lib().modil_set_field(self.h, slot, _ptr(tensor)), self.h)

    def set_reynolds(self, instance, re):
        L.check(L.lib().modil_set_instance_scalar(self.h, instance, L.SCALAR_RE, float(re)), self.h)

    # --------------------------------------------------------------- the path
    def _terms(self, terms):
        if terms is None:
            terms = torch.empty((self.spec.batch, L.N_TERMS), dtype=torch.float64, device=self.device)
        return terms

    def prolong(self, theta, out=None):
        self._check_pack(theta, "theta")
        out = self.new_fine() if out is None else out
        self._check_pack(out, "fine", int(self.lay.fine_total))
        L.check(L.lib().modil_prolong(self.h, _ptr(theta), _ptr(out)), self.h)
        return out

    def restrict_adjoint(self, fine, out=None):
        self._check_pack(fine, "fine", int(self.lay.fine_total))
        out = self.new_pack() if out is None else out
        self._check_pack(out, "grad")
        L.check(L.lib().modil_restrict_adjoint(self.h, _ptr(fine), _ptr(out)), self.h)
        return out

    def loss(self, theta, terms=None):
        self._check_pack(theta, "theta")
        terms = self._terms(terms)
        L.check(L.lib().modil_loss(self.h, _ptr(theta), _ptr(terms)), self.h)
        return terms

    def loss_grad(self, theta, grad=None, terms=None):
        self._check_pack(theta, "theta")
        grad = self.new_pack() if grad is None else grad
        self._check_pack(grad, "grad")
        terms = self._terms(terms)
        L.check(L.lib().modil_loss_grad(self.h, _ptr(theta), _ptr(grad), _ptr(terms)), self.h)
        return terms, grad

    def adam(self, theta_in, theta_out, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        hp = L.AdamHP(lr, beta1, beta2, eps)
        for t, n in ((theta_in, "theta_in"), (theta_out, "theta_out"), (m, "m"), (v, "v"), (grad, "grad")):
            self._check_pack(t, n)
        L.check(L.lib().modil_adam(self.h, _ptr(theta_in), _ptr(theta_out), _ptr(m), _ptr(v),
                                   _ptr(grad), ctypes.byref(hp), int(step)), self.h)

    def step(self, theta_in, theta_out, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             terms=None):
        hp = L.AdamHP(lr, beta1, beta2, eps)
        for t, n in ((theta_in, "theta_in"), (theta_out, "theta_out"), (m, "m"), (v, "v")):
            self._check_pack(t, n)
        L.check(L.lib().modil_step(self.h, _ptr(theta_in), _ptr(theta_out), _ptr(m), _ptr(v),
                                   ctypes.byref(hp), int(step), _ptr(terms)), self.h)
        return terms

    def run(self, theta_a, theta_b, m, v, step0, n_steps, lr=1e-3, beta1=0.9, beta2=0.999,
            eps=1e-8, terms=None):
        """n_steps iterations (steps step0 ..) alternating theta_a -> theta_b ->
        theta_a ...; returns the pack holding the result (theta_b if n_steps
        is odd).  Loss terms of the last iteration go to terms if given."""
        hp = L.AdamHP(lr, beta1, beta2, eps)
        for t, n in ((theta_a, "theta_a"), (theta_b, "theta_b"), (m, "m"), (v, "v")):
            self._check_pack(t, n)
        L.check(L.lib().modil_run(self.h, _ptr(theta_a), _ptr(theta_b), _ptr(m), _ptr(v),
                                  ctypes.byref(hp), int(step0), int(n_steps), _ptr(terms)), self.h)
        return theta_b if n_steps % 2 else theta_a

    def residual_metric(self, theta, out=None):
        self._check_pack(theta, "theta")
        out = torch.empty((self.spec.batch,), dtype=torch.float64, device=self.device) if out is None else out
        L.check(L.lib().modil_residual_metric(self.h, _ptr(theta), _ptr(out)), self.h)
        return out

    def set_fused(self, enabled: bool):
        """Use the fused finest-level kernel where one exists (default) or the generic engine."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_FUSED, 1 if enabled else 0), self.h)

    def fused_active(self) -> bool:
        """True if the finest level runs the fused kernel (option on and the
        problem admits it), False if the generic engine."""
        r = L.lib().modil_fused_active(self.h)
        L.check(min(r, 0), self.h)
        return r == 1

    def tiled_active(self) -> bool:
        """True if the generic engine runs by LDS tiles (2-D problems, option on)."""
        return self.spec.ndim == 2 and self._tile

    def set_march(self, enabled: bool):
        """Transfer levels with the lane-shuffle kernels (marching restriction,
        block prolongation) where a level admits them (default), or with the
        per-cell kernels."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_MARCH, 1 if enabled else 0), self.h)

    def set_tail(self, enabled: bool):
        """Do the small coarse levels of each instance in one LDS launch (default)."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_TAIL, 1 if enabled else 0), self.h)

    def set_tile(self, enabled: bool):
        """Generic engine on 2-D problems: LDS tiles forming every residual
        once (default), or the per-cell kernel."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_TILE, 1 if enabled else 0), self.h)
        self._tile = bool(enabled)

    def set_two_pass(self, enabled: bool):
        """Generic engine on 3-D problems: residuals formed once per cell with
        the star sensitivities gathered in a second pass (default, where the
        workspace holds their scratch), or the per-cell kernel."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_TWO_PASS, 1 if enabled else 0), self.h)

    def set_march_tile(self, rows: int = 0, planes: int = 0):
        """Coarse rows and planes per wave of the marching kernel (0, 0: automatic)."""
        L.check(L.lib().modil_set_option(self.h, L.OPT_MARCH_TILE, 64 * rows + planes), self.h)

    def check(self):
        """Synchronise; raise ModilError on a non-finite loss or a HIP error."""
        L.check(L.lib().modil_check(self.h), self.h)

    def profile(self, enable=True):
        L.check(L.lib().modil_profile(self.h, 1 if enable else 0), self.h)

    def profile_read(self, kernel_class):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        L.check(L.lib().modil_profile_read(self.h, kernel_class, ctypes.byref(ms), ctypes.byref(cnt)), self.h)
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "h", None):
            L.lib().modil_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LBFGS:
    """Limited-memory BFGS on a context's loss (modil_lbfgs_* in include/modil.h).

    Holds the device workspace (history + 1 pair slots and four pack-sized
    vectors) and the library handle.  step(theta) does one iteration in place
    and returns the iteration's info as a dict.
    """

    def __init__(self, ctx: Context, history: int = 50, max_evals: int = 20, c1: float = 1e-4,
                 c2: float = 0.9):
        self.ctx = ctx
        nb = ctypes.c_size_t()
        L.check(L.lib().modil_lbfgs_workspace(ctx.h, history, ctypes.byref(nb)), ctx.h)
        n = int(nb.value)
        self._ws_raw = torch.empty(n + 256, dtype=torch.uint8, device=ctx.device)
        shift = (-self._ws_raw.data_ptr()) % 256
        self._ws = self._ws_raw[shift:shift + n]
        prm = L.LbfgsParams(history, max_evals, c1, c2)
        h = ctypes.c_void_p()
        L.check(L.lib().modil_lbfgs_create(ctx.h, ctypes.byref(prm), _ptr(self._ws), n, ctypes.byref(h)),
                ctx.h)
        self.h = h

    def step(self, theta):
        self.ctx._check_pack(theta, "theta")
        info = L.LbfgsInfo()
        L.check(L.lib().modil_lbfgs_step(self.h, _ptr(theta), ctypes.byref(info)), self.ctx.h)
        return {k: getattr(info, k) for k, _ in L.LbfgsInfo._fields_}

    def reset(self):
        L.check(L.lib().modil_lbfgs_reset(self.h), self.ctx.h)

    def close(self):
        if getattr(self, "h", None):
            L.lib().modil_lbfgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
