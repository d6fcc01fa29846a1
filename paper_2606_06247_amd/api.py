"""Python binding of ``libfcsph.so`` (ctypes; argument marshalling only).

Every computation runs in the library's HIP kernels.  torch supplies device
memory (tensors, the plan workspace) and the HIP stream.  The names mirror the
C ABI in ``include/fcsph.h``: fc_extend, spectral_grad, spectral_div,
spectral_lap, ppe_solve, project_step.

Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import fcpoly, fctables

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcsph.so")

OK, E_INVALID, E_UNSUPPORTED, E_WORKSPACE, E_HIP, E_NONFINITE = 0, -1, -2, -3, -4, -5
PERIODIC, WALLED = 0, 1
DIRICHLET, NEUMANN = 0, 1
VELOCITY, PRESSURE = 0, 1
FP64, FP32_MIXED = 0, 1
PPE_PHYSICAL, PPE_EXTENDED = 0, 1
EIG_SPECTRAL, EIG_FD2, EIG_SPH = 0, 1, 2
KERNEL_WENDLAND_C2 = 0
KERNELS = {"wendland_c2": 0, "g2": 2, "g4": 4, "g6": 6, "g8": 8, "g10": 10}
OPS_FFT, OPS_DIRECT, OPS_FFT_WINDOW = 0, 1, 2

EXPORTS = [
    "fcsph_ctx_create", "fcsph_ctx_destroy", "fcsph_ctx_sync", "fcsph_status_string",
    "fcsph_ctx_last_error", "fcsph_plan_workspace_bytes", "fcsph_plan_create",
    "fcsph_plan_destroy", "fcsph_plan_transform_lengths", "fcsph_fc_extend", "fcsph_spectral_grad",
    "fcsph_spectral_div",
    "fcsph_spectral_lap", "fcsph_spectral_lap_noalloc", "fcsph_ppe_solve", "fcsph_check_finite", "fcsph_project_step", "fcsph_rk3_substep", "fcsph_advect_rk3_substep", "fcsph_ctx_set_timing",
    "fcsph_ctx_read_timing", "fcsph_ctx_set_timing_only", "fcsph_batch_workspace_bytes", "fcsph_batch_create", "fcsph_batch_destroy",
    "fcsph_batch_clear", "fcsph_batch_add_step", "fcsph_batch_add_rk3_substep", "fcsph_batch_add_ppe", "fcsph_batch_launch",
    "fcsph_batch_capture", "fcsph_batch_replay", "fcsph_batch_info",
]


class Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double),
        ("axis", ctypes.c_int * 3), ("vel_bc", (ctypes.c_int * 2) * 3),
        ("prs_bc", (ctypes.c_int * 2) * 3), ("fc_d", ctypes.c_int), ("fc_C", ctypes.c_int),
        ("fc_M_dir", ctypes.POINTER(ctypes.c_double)), ("fc_M_neu", ctypes.POINTER(ctypes.c_double)),
        ("kernel", ctypes.c_int), ("h_over_dx", ctypes.c_double), ("prec", ctypes.c_int),
        ("ppe_domain", ctypes.c_int), ("eig", ctypes.c_int), ("rho", ctypes.c_double),
        ("op_eval", ctypes.c_int), ("window_len", ctypes.c_int * 3), ("lines_per_group", ctypes.c_int),
        ("batched", ctypes.c_int), ("radix_order", ctypes.c_int),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2606_06247_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    L.fcsph_ctx_create.argtypes = [i, vp, P(vp)]
    L.fcsph_ctx_destroy.argtypes = [vp]
    L.fcsph_ctx_sync.argtypes = [vp]
    L.fcsph_status_string.argtypes = [i]
    L.fcsph_status_string.restype = ctypes.c_char_p
    L.fcsph_ctx_last_error.argtypes = [vp]
    L.fcsph_ctx_last_error.restype = ctypes.c_char_p
    L.fcsph_plan_workspace_bytes.argtypes = [P(Desc), P(ctypes.c_size_t)]
    L.fcsph_plan_create.argtypes = [vp, P(Desc), vp, ctypes.c_size_t, P(vp)]
    L.fcsph_plan_destroy.argtypes = [vp]
    L.fcsph_plan_transform_lengths.argtypes = [vp, P(i)]
    L.fcsph_fc_extend.argtypes = [vp, i, vp, vp]
    L.fcsph_spectral_grad.argtypes = [vp, i, vp, P(vp)]
    L.fcsph_spectral_div.argtypes = [vp, P(vp), vp]
    L.fcsph_spectral_lap.argtypes = [vp, i, vp, vp]
    L.fcsph_spectral_lap_noalloc.argtypes = [vp, i, vp, vp]
    L.fcsph_ppe_solve.argtypes = [vp, vp, vp]
    L.fcsph_check_finite.argtypes = [vp, vp, ctypes.c_size_t, P(ctypes.c_ulonglong)]
    L.fcsph_project_step.argtypes = [vp, P(vp), vp, P(vp), P(vp), d, d]
    L.fcsph_rk3_substep.argtypes = [vp, i, P(vp), vp, P(vp), P(vp), P(vp), d, d]
    L.fcsph_advect_rk3_substep.argtypes = [vp, i, vp, vp, P(d), d, vp]
    L.fcsph_ctx_set_timing.argtypes = [vp, i]
    L.fcsph_ctx_set_timing_only.argtypes = [vp, ctypes.c_char_p]
    L.fcsph_ctx_read_timing.argtypes = [vp, i, ctypes.c_char_p, P(i), P(d), P(i)]
    L.fcsph_batch_workspace_bytes.argtypes = [i, P(ctypes.c_size_t)]
    L.fcsph_batch_create.argtypes = [vp, i, vp, ctypes.c_size_t, P(vp)]
    L.fcsph_batch_destroy.argtypes = [vp]
    L.fcsph_batch_clear.argtypes = [vp]
    L.fcsph_batch_add_step.argtypes = [vp, vp, P(vp), vp, P(vp), P(vp), d, d]
    L.fcsph_batch_add_rk3_substep.argtypes = [vp, vp, i, P(vp), vp, P(vp), P(vp), P(vp), d, d]
    L.fcsph_batch_add_ppe.argtypes = [vp, vp, vp, vp]
    L.fcsph_batch_launch.argtypes = [vp]
    L.fcsph_batch_capture.argtypes = [vp]
    L.fcsph_batch_replay.argtypes = [vp]
    L.fcsph_batch_info.argtypes = [vp, P(i), P(i), P(i)]
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is None or f.restype is ctypes.c_int:
            if name not in ("fcsph_status_string", "fcsph_ctx_last_error"):
                f.restype = i
    _lib = L
    return L


class FcsphError(RuntimeError):
    pass


def _check(status: int, ctx=None, what: str = ""):
    if status != OK:
        L = lib()
        msg = L.fcsph_status_string(status).decode()
        detail = L.fcsph_ctx_last_error(ctx).decode() if ctx else ""
        raise FcsphError(f"{what}: {msg} ({status}) {detail}")


@dataclass
class Problem:
    """Lattice and method parameters (lattice order: x, y[, z])."""

    n: tuple
    walled: tuple
    dx: float
    vel_bc: tuple = None          # per axis ('D'|'N', 'D'|'N')
    prs_bc: tuple = None
    h_over_dx: float = 1.3
    kernel: str = "wendland_c2"   # or the Gaussian family 'g2' .. 'g10' (2D, op_eval 'fft')
    precision: str = "fp64"       # 'fp64' | 'fp32'
    eig: str = "spectral"         # 'spectral' | 'fd2' | 'sph' (2D, every axis periodic)
    rho: float = 1.0
    ppe_domain: str = "physical"  # 'physical' | 'extended' (projection on the extended lattice)
    op_eval: str = "fft"          # 'fft' | 'fft_window' | 'direct'
    fc_d: int = 5
    fc_C: int = 25
    # "gram": FC(Gram) maps (fc_d = 5, fc_C = 25); "poly": the paper's own FC
    # (fc_d fit points, degree fc_p, fc_C extension points)
    fc_kind: str = "gram"
    fc_p: int = 5
    window_len: tuple = ()        # schedule hint per axis (0 = library choice)
    lines_per_group: int = 0      # schedule hint (0 = library choice)
    batched: bool = False         # plan also runs in batches (no streamed PPE radices)
    radix_order: int = 0          # schedule hint: operator stage order (0 = library order)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def ext_shape(self):
        return tuple(reversed([k + (self.fc_C if w else 0) for k, w in zip(self.n, self.walled)]))


def _bc(c):
    return {"D": DIRICHLET, "N": NEUMANN}[c]


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        L = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(L.fcsph_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
               None, "fcsph_ctx_create")
        self.handle = h

    def sync(self):
        _check(lib().fcsph_ctx_sync(self.handle), self.handle, "fcsph_ctx_sync")

    def set_timing(self, on: bool, only: str | None = None):
        """Bracket launches with events (all kinds, or only kind `only`)."""
        _check(lib().fcsph_ctx_set_timing_only(self.handle, only.encode() if only else None),
               self.handle, "set_timing_only")
        _check(lib().fcsph_ctx_set_timing(self.handle, int(bool(on))), self.handle, "set_timing")

    def read_timing(self) -> dict:
        """{kernel kind: (launches, total ms)} since the last read (waits for the stream)."""
        cap = 64
        names = ctypes.create_string_buffer(32 * cap)
        counts = (ctypes.c_int * cap)()
        tot = (ctypes.c_double * cap)()
        n = ctypes.c_int()
        _check(lib().fcsph_ctx_read_timing(self.handle, cap, names, counts, tot, ctypes.byref(n)),
               self.handle, "read_timing")
        out = {}
        for k in range(n.value):
            name = names.raw[32 * k:32 * (k + 1)].split(b"\0")[0].decode()
            out[name] = (counts[k], tot[k])
        return out

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().fcsph_ctx_destroy(self.handle)
        except Exception:
            pass


def make_desc(prob: "Problem"):
    """The C descriptor of a Problem, with the FC map arrays it points into
    (keep them alive while the descriptor is used)."""
    if prob.fc_kind == "gram":
        tabs = fctables.load(prob.fc_d, prob.fc_C)
        mdir, mneu = tabs["dirichlet"], tabs["neumann"]
    elif prob.fc_kind == "poly":
        mdir, mneu = fcpoly.build(prob.fc_d, prob.fc_p, prob.fc_C)
    else:
        raise ValueError(f"unknown fc_kind {prob.fc_kind!r}")
    mdir = np.ascontiguousarray(mdir, dtype=np.float64)
    mneu = np.ascontiguousarray(mneu, dtype=np.float64)
    d = Desc()
    d.ndim = prob.ndim
    for a in range(prob.ndim):
        d.n[a] = prob.n[a]
        d.axis[a] = WALLED if prob.walled[a] else PERIODIC
        if prob.walled[a]:
            for s in range(2):
                d.vel_bc[a][s] = _bc(prob.vel_bc[a][s])
                d.prs_bc[a][s] = _bc(prob.prs_bc[a][s])
    d.dx = prob.dx
    d.fc_d, d.fc_C = prob.fc_d, prob.fc_C
    d.fc_M_dir = mdir.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.fc_M_neu = mneu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.kernel = KERNELS[prob.kernel]
    d.h_over_dx = prob.h_over_dx
    d.prec = FP32_MIXED if prob.precision == "fp32" else FP64
    d.ppe_domain = {"physical": PPE_PHYSICAL, "extended": PPE_EXTENDED}[prob.ppe_domain]
    d.eig = {"spectral": EIG_SPECTRAL, "fd2": EIG_FD2, "sph": EIG_SPH}[prob.eig]
    d.rho = prob.rho
    d.op_eval = {"fft": OPS_FFT, "direct": OPS_DIRECT, "fft_window": OPS_FFT_WINDOW}[prob.op_eval]
    for a, L in enumerate(prob.window_len):
        d.window_len[a] = int(L)
    d.lines_per_group = int(prob.lines_per_group)
    d.batched = 1 if prob.batched else 0
    d.radix_order = int(prob.radix_order)
    return d, mdir, mneu


def workspace_bytes(prob: "Problem") -> int:
    """Device workspace bytes a plan for prob needs (host-only query)."""
    d, _m1, _m2 = make_desc(prob)
    nbytes = ctypes.c_size_t()
    _check(lib().fcsph_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)), None,
           "fcsph_plan_workspace_bytes")
    return nbytes.value


class Plan:
    """A plan for one lattice; owns its device workspace (a torch tensor)."""

    def __init__(self, ctx: Context, prob: Problem):
        import torch
        L = lib()
        self.ctx, self.prob = ctx, prob
        self.desc, self._mdir, self._mneu = make_desc(prob)
        d = self.desc
        nbytes = ctypes.c_size_t()
        _check(L.fcsph_plan_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)), None,
               "fcsph_plan_workspace_bytes")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(L.fcsph_plan_create(ctx.handle, ctypes.byref(d), ctypes.c_void_p(base + off),
                                   nbytes.value, ctypes.byref(h)), ctx.handle, "fcsph_plan_create")
        self.handle = h
        self.out_dtype = torch.float32 if prob.precision == "fp32" else torch.float64

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().fcsph_plan_destroy(self.handle)
        except Exception:
            pass

    # -- helpers
    def _t(self, x, dtype=None):
        import torch
        dtype = dtype or torch.float64
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dtype and x.is_contiguous()):
            raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
        return x

    def _phys(self, x, dtype=None):
        x = self._t(x, dtype)
        if tuple(x.shape) != self.prob.shape:
            raise ValueError(f"expected shape {self.prob.shape}, got {tuple(x.shape)}")
        return ctypes.c_void_p(x.data_ptr())

    def _new(self, dtype=None, shape=None):
        import torch
        return torch.empty(shape or self.prob.shape, dtype=dtype or torch.float64,
                           device=f"cuda:{self.ctx.device}")

    @staticmethod
    def _ptrs(ts):
        arr = (ctypes.c_void_p * 3)()
        for i, t in enumerate(ts):
            arr[i] = None if t is None else t
        return arr

    # -- entry points (same names as the C ABI)
    def transform_lengths(self) -> tuple:
        """Operator transform length per lattice axis."""
        arr = (ctypes.c_int * 3)()
        _check(lib().fcsph_plan_transform_lengths(self.handle, arr), self.ctx.handle,
               "fcsph_plan_transform_lengths")
        return tuple(arr[a] for a in range(self.prob.ndim))

    def fc_extend(self, f, field: int = VELOCITY, out=None):
        import torch
        out = self._new(torch.float64, self.prob.ext_shape) if out is None else out
        self._t(out)
        if tuple(out.shape) != self.prob.ext_shape:
            raise ValueError("bad output shape")
        _check(lib().fcsph_fc_extend(self.handle, field, self._phys(f), ctypes.c_void_p(out.data_ptr())),
               self.ctx.handle, "fcsph_fc_extend")
        return out

    def spectral_grad(self, f, field: int = VELOCITY, out=None):
        out = [self._new(self.out_dtype) for _ in range(self.prob.ndim)] if out is None else out
        ptrs = self._ptrs([self._phys(o, self.out_dtype).value for o in out])
        _check(lib().fcsph_spectral_grad(self.handle, field, self._phys(f), ptrs), self.ctx.handle,
               "fcsph_spectral_grad")
        return out

    def spectral_div(self, u, out=None):
        out = self._new(self.out_dtype) if out is None else out
        ptrs = self._ptrs([self._phys(c).value for c in u])
        _check(lib().fcsph_spectral_div(self.handle, ptrs, self._phys(out, self.out_dtype)),
               self.ctx.handle, "fcsph_spectral_div")
        return out

    def spectral_lap(self, f, field: int = VELOCITY, out=None):
        out = self._new(self.out_dtype) if out is None else out
        _check(lib().fcsph_spectral_lap(self.handle, field, self._phys(f), self._phys(out, self.out_dtype)),
               self.ctx.handle, "fcsph_spectral_lap")
        return out

    def spectral_lap_noalloc(self, f, field: int = VELOCITY, out=None):
        """fcsph_spectral_lap_noalloc: the Laplacian with its intermediates in
        the library's static device scratch (no allocation by the library)."""
        out = self._new(self.out_dtype) if out is None else out
        _check(lib().fcsph_spectral_lap_noalloc(self.handle, field, self._phys(f), self._phys(out, self.out_dtype)),
               self.ctx.handle, "fcsph_spectral_lap_noalloc")
        return out

    def nonfinite_count(self, x) -> int:
        """fcsph_check_finite: the number of NaN / infinite values of an FP64
        device tensor (counted by the library's kernel; waits for the stream)."""
        t = self._t(x)
        cnt = ctypes.c_ulonglong(0)
        st = lib().fcsph_check_finite(self.handle, ctypes.c_void_p(t.data_ptr()), t.numel(), ctypes.byref(cnt))
        if st not in (OK, E_NONFINITE):
            _check(st, self.ctx.handle, "fcsph_check_finite")
        return int(cnt.value)

    def ppe_solve(self, rhs, out=None):
        out = self._new() if out is None else out
        _check(lib().fcsph_ppe_solve(self.handle, self._phys(rhs, self.out_dtype), self._phys(out)),
               self.ctx.handle, "fcsph_ppe_solve")
        return out

    def project_step(self, u, dt: float, nu: float, p_out=None, force=None, wall=None):
        """One FOP step; u (list of tensors) is updated in place."""
        up = self._ptrs([self._phys(c).value for c in u])
        fp = self._ptrs([self._phys(c).value for c in force]) if force is not None else None
        wp = self._ptrs([self._phys(c).value for c in wall]) if wall is not None else None
        pp = self._phys(p_out) if p_out is not None else None
        _check(lib().fcsph_project_step(self.handle, up, pp, fp, wp, float(dt), float(nu)),
               self.ctx.handle, "fcsph_project_step")
        return u, p_out

    def advect_rk3_substep(self, k: int, u, F, c, dt: float, inflow=None):
        """fcsph_advect_rk3_substep: RK3 sub-step k of linear advection of the
        scalar u (in place) with velocity c; F holds F of the previous
        sub-step and receives this one's; inflow: wall values of the inflow walls."""
        cc = (ctypes.c_double * 2)(*[float(x) for x in c])
        _check(lib().fcsph_advect_rk3_substep(self.handle, int(k), self._phys(u), self._phys(F), cc, float(dt),
                                              self._phys(inflow) if inflow is not None else None),
               self.ctx.handle, "fcsph_advect_rk3_substep")
        return u

    def rk3_substep(self, k: int, u, F, dt: float, nu: float, p_out=None, force=None, wall=None):
        """RK3 sub-step k (0, 1, 2) of the whole step dt; u (list of tensors) is
        updated in place, F (list of FP64 tensors, one per component) carries
        F of the previous sub-step in and this sub-step's F out."""
        up = self._ptrs([self._phys(c).value for c in u])
        Fp = self._ptrs([self._phys(c).value for c in F])
        fp = self._ptrs([self._phys(c).value for c in force]) if force is not None else None
        wp = self._ptrs([self._phys(c).value for c in wall]) if wall is not None else None
        pp = self._phys(p_out) if p_out is not None else None
        _check(lib().fcsph_rk3_substep(self.handle, int(k), up, pp, fp, wp, Fp, float(dt), float(nu)),
               self.ctx.handle, "fcsph_rk3_substep")
        return u, p_out


class Batch:
    """Many plans' steps / PPE solves issued as grouped launches (fcsph_batch_*).

    add_step / add_ppe record a call (buffers are read when the batch runs;
    the batch keeps references to the tensors until clear()); launch() runs
    every recorded call; capture() / replay() turn the last launch into a HIP
    graph and run it again on the same buffers."""

    def __init__(self, ctx: Context, max_items: int):
        import torch
        L = lib()
        self.ctx = ctx
        nb = ctypes.c_size_t()
        _check(L.fcsph_batch_workspace_bytes(int(max_items), ctypes.byref(nb)), None,
               "fcsph_batch_workspace_bytes")
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(L.fcsph_batch_create(ctx.handle, int(max_items), ctypes.c_void_p(base + off), nb.value,
                                    ctypes.byref(h)), ctx.handle, "fcsph_batch_create")
        self.handle = h
        self._keep = []

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.fcsph_batch_destroy(h)
            self.handle = None

    def add_step(self, plan: "Plan", u, dt: float, nu: float, p_out=None, force=None, wall=None):
        up = plan._ptrs([plan._phys(c).value for c in u])
        fp = plan._ptrs([plan._phys(c).value for c in force]) if force is not None else None
        wp = plan._ptrs([plan._phys(c).value for c in wall]) if wall is not None else None
        pp = plan._phys(p_out) if p_out is not None else None
        _check(lib().fcsph_batch_add_step(self.handle, plan.handle, up, pp, fp, wp, float(dt), float(nu)),
               self.ctx.handle, "fcsph_batch_add_step")
        self._keep.append((plan, u, p_out, force, wall))

    def add_rk3_substep(self, plan: "Plan", k: int, u, F, dt: float, nu: float, p_out=None, force=None,
                        wall=None):
        up = plan._ptrs([plan._phys(c).value for c in u])
        Fp = plan._ptrs([plan._phys(c).value for c in F])
        fp = plan._ptrs([plan._phys(c).value for c in force]) if force is not None else None
        wp = plan._ptrs([plan._phys(c).value for c in wall]) if wall is not None else None
        pp = plan._phys(p_out) if p_out is not None else None
        _check(lib().fcsph_batch_add_rk3_substep(self.handle, plan.handle, int(k), up, pp, fp, wp, Fp,
                                                 float(dt), float(nu)),
               self.ctx.handle, "fcsph_batch_add_rk3_substep")
        self._keep.append((plan, u, F, p_out, force, wall))

    def add_ppe(self, plan: "Plan", rhs, out=None):
        out = plan._new() if out is None else out
        _check(lib().fcsph_batch_add_ppe(self.handle, plan.handle, plan._phys(rhs, plan.out_dtype),
                                         plan._phys(out)), self.ctx.handle, "fcsph_batch_add_ppe")
        self._keep.append((plan, rhs, out))
        return out

    def launch(self):
        _check(lib().fcsph_batch_launch(self.handle), self.ctx.handle, "fcsph_batch_launch")

    def capture(self):
        _check(lib().fcsph_batch_capture(self.handle), self.ctx.handle, "fcsph_batch_capture")

    def replay(self):
        _check(lib().fcsph_batch_replay(self.handle), self.ctx.handle, "fcsph_batch_replay")

    def clear(self):
        _check(lib().fcsph_batch_clear(self.handle), self.ctx.handle, "fcsph_batch_clear")
        self._keep = []

    def info(self) -> tuple:
        """(items, groups, grouped launches) of the last launch."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().fcsph_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               self.ctx.handle, "fcsph_batch_info")
        return a.value, b.value, c.value


# module-level aliases with the C ABI names
def fc_extend(plan: Plan, f, field=VELOCITY, out=None):
    return plan.fc_extend(f, field, out)


def spectral_grad(plan: Plan, f, field=VELOCITY, out=None):
    return plan.spectral_grad(f, field, out)


def spectral_div(plan: Plan, u, out=None):
    return plan.spectral_div(u, out)


def spectral_lap(plan: Plan, f, field=VELOCITY, out=None):
    return plan.spectral_lap(f, field, out)


def ppe_solve(plan: Plan, rhs, out=None):
    return plan.ppe_solve(rhs, out)


def project_step(plan: Plan, u, dt, nu, p_out=None, force=None, wall=None):
    return plan.project_step(u, dt, nu, p_out, force, wall)
