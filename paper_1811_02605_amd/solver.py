"""PyTorch-facing layer over the C ABI.

PyTorch provides device memory (operator storage, workspace, vectors) and
the current HIP stream; every step of the solve runs in the HIP library.
Nothing here computes on tensors.

    grid = Grid(r_faces, t_faces, np)
    op = Operator(grid, nu, dt, precision="fp64")        # mas_op_build
    x, info = op.solve(rhs)                              # mas_pcg_solve
    x, info = op.solve_noalloc(rhs)                      # mas_pcg_solve_noalloc (no allocation)
    lam, g_nu, g_rhs, info = op.adjoint(x, gx)           # mas_pcg_solve_adjoint
    u1, info = op.sts_step(u0)                           # mas_sts_step (explicit RKL2)
    X, infos = op.solve_multi(RHS)                       # mas_pcg_solve_multi (RHS: (m, nr, nt, np))
    x = solve(nu, rhs, grid, dt)                          # differentiable (MasSolve)
"""
from __future__ import annotations

import ctypes
import warnings

import numpy as np
import torch

from . import _abi as abi

PRECISIONS = {"fp64": abi.MAS_FP64, "fp32_refined": abi.MAS_FP32_REFINED}


class Grid:
    """Radial and colatitude faces (host, float64) and the phi cell count."""

    def __init__(self, r_faces, t_faces, np_, bc_inner=abi.MAS_BC_DIRICHLET0,
                 bc_outer=abi.MAS_BC_DIRICHLET0):
        self.r_faces = np.ascontiguousarray(r_faces, dtype=np.float64)
        self.t_faces = np.ascontiguousarray(t_faces, dtype=np.float64)
        self.nr = self.r_faces.size - 1
        self.nt = self.t_faces.size - 1
        self.np = int(np_)
        self.bc_inner = int(bc_inner)
        self.bc_outer = int(bc_outer)

    @property
    def shape(self):
        return (self.nr, self.nt, self.np)

    @property
    def n(self):
        return self.nr * self.nt * self.np

    def c_struct(self) -> abi.mas_grid:
        dp = ctypes.POINTER(ctypes.c_double)
        return abi.mas_grid(self.nr, self.nt, self.np, self.r_faces.ctypes.data_as(dp),
                            self.t_faces.ctypes.data_as(dp), self.bc_inner, self.bc_outer)

    @classmethod
    def from_problem(cls, p):
        return cls(p.r_faces, p.t_faces, p.cfg.np_, p.bc_inner, p.bc_outer)


REFINES = {"restart": abi.MAS_REFINE_RESTART, "reliable": abi.MAS_REFINE_RELIABLE}
PRECONDS = {"pc1": abi.MAS_PC1, "pc2": abi.MAS_PC2}
LAUNCHES = {"auto": abi.MAS_LAUNCH_AUTO, "per_iteration": abi.MAS_LAUNCH_PER_ITERATION,
            "persistent": abi.MAS_LAUNCH_PERSISTENT}


def make_opts(rtol=None, max_iters=None, precision=None, inner_rtol=None, max_outer=None,
              check_every=None, use_x0=None, max_restarts=None, sample_timing=None, refine=None,
              precond=None, chunk_planes=None, launch=None):
    o = abi.default_opts()
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    if isinstance(launch, str):
        launch = LAUNCHES[launch]
    if isinstance(refine, str):
        refine = REFINES[refine]
    if isinstance(precond, str):
        precond = PRECONDS[precond]
    for name, v in dict(rtol=rtol, max_iters=max_iters, precision=precision,
                        inner_rtol=inner_rtol, max_outer=max_outer, check_every=check_every,
                        use_x0=use_x0, max_restarts=max_restarts,
                        sample_timing=sample_timing, refine=refine, precond=precond,
                        chunk_planes=chunk_planes, launch=launch).items():
        if v is not None:
            setattr(o, name, type(getattr(o, name))(v))
    return o


def _copy_opts(opts, **overrides):
    """A private copy of an options struct (the caller's object is never
    modified), with the given fields replaced."""
    o = abi.mas_pcg_opts()
    ctypes.pointer(o)[0] = opts if opts is not None else make_opts()
    for name, v in overrides.items():
        setattr(o, name, type(getattr(o, name))(v))
    return o


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_vec(t: torch.Tensor, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA/HIP tensor")
    # the arrays are read phi-fastest as (.., nr, nt, np): accept exactly that
    # shape or a flat vector of the same length, nothing else
    flat = (int(np.prod(shape)),)
    if tuple(t.shape) != tuple(shape) and tuple(t.shape) != flat:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)} or {flat}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _device_bytes(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if buf.data_ptr() % 256:
        raise RuntimeError("device allocation is not 256-byte aligned")
    return buf


class Operator:
    """A(nu, dt) built by mas_op_build into torch-owned device storage."""

    def __init__(self, grid: Grid, nu: torch.Tensor, dt: float, precision="fp64"):
        lib = abi.load()
        _check_vec(nu, grid.shape, "nu")
        self.grid = grid
        self.device = nu.device
        self.dt = float(dt)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        g = grid.c_struct()
        nbytes = lib.mas_op_storage_bytes(ctypes.byref(g), self.precision)
        abi.check(int(nbytes) if nbytes < 0 else 0, "mas_op_storage_bytes")
        self.storage = _device_bytes(nbytes, self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.mas_op_build(ctypes.byref(g), nu.data_ptr(), self.dt, self.precision,
                                  self.storage.data_ptr(), nbytes, _stream(self.device),
                                  ctypes.byref(h))
        abi.check(st, "mas_op_build")
        self._h = h
        self._work = {}
        # bound now: at interpreter exit the module's globals may be gone
        # before the last operator is collected
        self._destroy = lib.mas_op_destroy

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        _check_vec(x, self.grid.shape, "x")
        y = torch.empty_like(x)
        with torch.cuda.device(self.device):
            abi.check(abi.load().mas_op_apply(self._h, x.data_ptr(), y.data_ptr(),
                                              _stream(self.device)), "mas_op_apply")
        return y

    def export(self):
        """(cr, ct, cp, diag): couplings to the +r/+theta/+phi neighbours and diag(A)."""
        outs = [torch.empty(self.grid.shape, dtype=torch.float64, device=self.device)
                for _ in range(4)]
        with torch.cuda.device(self.device):
            abi.check(abi.load().mas_op_export(self._h, *[o.data_ptr() for o in outs],
                                               _stream(self.device)), "mas_op_export")
        return tuple(outs)

    def workspace(self, opts) -> tuple[torch.Tensor, int]:
        nbytes = int(abi.load().mas_pcg_workspace_bytes(self._h, ctypes.byref(opts)))
        abi.check(nbytes if nbytes < 0 else 0, "mas_pcg_workspace_bytes")
        buf = self._work.get(opts.precision)
        if buf is None or buf.numel() < nbytes:
            buf = _device_bytes(nbytes, self.device)
            self._work[opts.precision] = buf
        return buf, nbytes

    def solve(self, rhs: torch.Tensor, opts=None, x0: torch.Tensor | None = None,
              out: torch.Tensor | None = None, allow_notconv=True):
        """x = A^-1 (V .* rhs).  Returns (x, info dict)."""
        _check_vec(rhs, self.grid.shape, "rhs")
        x = out if out is not None else torch.empty_like(rhs)
        # the solution buffer is the starting guess only when x0 is given
        if x0 is not None:
            _check_vec(x0, self.grid.shape, "x0")
            x.copy_(x0)
        opts = _copy_opts(opts, use_x0=int(x0 is not None))
        work, nbytes = self.workspace(opts)
        info = abi.mas_pcg_info()
        with torch.cuda.device(self.device):
            st = abi.load().mas_pcg_solve(self._h, rhs.data_ptr(), x.data_ptr(), ctypes.byref(opts),
                                          work.data_ptr(), nbytes, _stream(self.device),
                                          ctypes.byref(info))
        abi.check(st, "mas_pcg_solve", allow_notconv=allow_notconv)
        if st == abi.MAS_ENOTCONV:
            warnings.warn(f"mas_pcg_solve did not converge: {info.as_dict()}")
        return x, info.as_dict()

    def solve_noalloc(self, rhs: torch.Tensor, opts=None, x0: torch.Tensor | None = None,
                      out: torch.Tensor | None = None, allow_notconv=True):
        """The same solve as solve(), through mas_pcg_solve_noalloc: the
        library takes the workspace from its static device array and
        allocates nothing during the call (out, when given, must be a
        preallocated float64 tensor of the grid's shape)."""
        _check_vec(rhs, self.grid.shape, "rhs")
        x = out if out is not None else torch.empty_like(rhs)
        _check_vec(x, self.grid.shape, "out")
        if x0 is not None:
            _check_vec(x0, self.grid.shape, "x0")
            x.copy_(x0)
        opts = _copy_opts(opts, use_x0=int(x0 is not None))
        info = abi.mas_pcg_info()
        with torch.cuda.device(self.device):
            st = abi.load().mas_pcg_solve_noalloc(self._h, rhs.data_ptr(), x.data_ptr(),
                                                  ctypes.byref(opts), _stream(self.device),
                                                  ctypes.byref(info))
        abi.check(st, "mas_pcg_solve_noalloc", allow_notconv=allow_notconv)
        if st == abi.MAS_ENOTCONV:
            warnings.warn(f"mas_pcg_solve_noalloc did not converge: {info.as_dict()}")
        return x, info.as_dict()

    def solve_multi(self, rhs: torch.Tensor, opts=None, x0: torch.Tensor | None = None,
                    out: torch.Tensor | None = None, allow_notconv=True):
        """X[h] = A^-1 (V .* rhs[h]) for the m = rhs.shape[0] right-hand sides
        (1..4) in one double-precision solve.  Returns (X, [info dict per h])."""
        m = int(rhs.shape[0])
        shape = (m,) + tuple(self.grid.shape)
        _check_vec(rhs, shape, "rhs")
        x = out if out is not None else torch.empty_like(rhs)
        _check_vec(x, shape, "out")
        if x0 is not None:
            _check_vec(x0, shape, "x0")
            x.copy_(x0)
        opts = _copy_opts(opts, use_x0=int(x0 is not None))
        lib = abi.load()
        nbytes = int(lib.mas_pcg_multi_workspace_bytes(self._h, m))
        abi.check(nbytes if nbytes < 0 else 0, "mas_pcg_multi_workspace_bytes")
        key = ("multi", m)
        buf = self._work.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = _device_bytes(nbytes, self.device)
            self._work[key] = buf
        infos = (abi.mas_pcg_info * m)()
        with torch.cuda.device(self.device):
            st = lib.mas_pcg_solve_multi(self._h, m, rhs.data_ptr(), x.data_ptr(), ctypes.byref(opts),
                                         buf.data_ptr(), nbytes, _stream(self.device), infos)
        abi.check(st, "mas_pcg_solve_multi", allow_notconv=allow_notconv)
        if st == abi.MAS_ENOTCONV:
            warnings.warn("mas_pcg_solve_multi: a right-hand side did not converge")
        return x, [i.as_dict() for i in infos]

    def adjoint(self, x: torch.Tensor, gx: torch.Tensor, opts=None, allow_notconv=True):
        """(lambda, dL/dnu, dL/drhs, info) for dL/dx = gx at the solution x."""
        _check_vec(x, self.grid.shape, "x")
        _check_vec(gx, self.grid.shape, "gx")
        # lambda starts from zero: its buffer is fresh memory
        opts = _copy_opts(opts, use_x0=0)
        lam = torch.empty_like(x)
        gnu = torch.empty_like(x)
        grhs = torch.empty_like(x)
        work, nbytes = self.workspace(opts)
        info = abi.mas_pcg_info()
        with torch.cuda.device(self.device):
            st = abi.load().mas_pcg_solve_adjoint(
                self._h, x.data_ptr(), gx.data_ptr(), lam.data_ptr(), gnu.data_ptr(),
                grhs.data_ptr(), ctypes.byref(opts), work.data_ptr(), nbytes,
                _stream(self.device), ctypes.byref(info))
        abi.check(st, "mas_pcg_solve_adjoint", allow_notconv=allow_notconv)
        return lam, gnu, grhs, info.as_dict()

    def sts_stages(self) -> int:
        """Automatic RKL2 stage count for this operator's dt."""
        s = int(abi.load().mas_sts_stages(self._h))
        abi.check(s if s < 0 else 0, "mas_sts_stages")
        return s

    def sts_step(self, u0: torch.Tensor, stages: int = 0, out: torch.Tensor | None = None,
                 sample_timing: bool = False, stage_pairs: bool = True):
        """One RKL2 super time-step of du/dt = L u over dt.  Returns (u1, info).
        out may be u0 itself (in-place step).  stage_pairs=False runs one stage
        per kernel (the two-stage kernel's result is the same bit for bit)."""
        _check_vec(u0, self.grid.shape, "u0")
        u1 = out if out is not None else torch.empty_like(u0)
        _check_vec(u1, self.grid.shape, "out")
        lib = abi.load()
        nbytes = int(lib.mas_sts_workspace_bytes(self._h))
        abi.check(nbytes if nbytes < 0 else 0, "mas_sts_workspace_bytes")
        buf = self._work.get("sts")
        if buf is None or buf.numel() < nbytes:
            buf = _device_bytes(nbytes, self.device)
            self._work["sts"] = buf
        o = abi.mas_sts_opts()
        lib.mas_sts_default_opts(ctypes.byref(o))
        o.stages = int(stages)
        o.sample_timing = int(bool(sample_timing))
        o.single_stage_kernels = int(not stage_pairs)
        info = abi.mas_sts_info()
        with torch.cuda.device(self.device):
            st = lib.mas_sts_step(self._h, u0.data_ptr(), u1.data_ptr(), ctypes.byref(o),
                                  buf.data_ptr(), nbytes, _stream(self.device), ctypes.byref(info))
        abi.check(st, "mas_sts_step")
        return u1, info.as_dict()


def probe_copy(src: torch.Tensor, dst: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    with torch.cuda.device(src.device):
        abi.check(abi.load().mas_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes,
                                            _stream(src.device)), "mas_probe_copy")


def probe_stream(n: int, nin: int, nout: int, device="cuda", reps: int = 10) -> float:
    """GB/s of the streaming probe with nin arrays read and nout written per
    cell (n cells each), from HIP events around reps back-to-back launches
    after one warm-up launch."""
    lib = abi.load()
    nbytes = int(lib.mas_probe_stream_bytes(int(n), int(nin), int(nout)))
    abi.check(nbytes if nbytes < 0 else 0, "mas_probe_stream_bytes")
    buf = _device_bytes(nbytes, device)
    buf.zero_()
    with torch.cuda.device(buf.device):
        s = _stream(buf.device)
        abi.check(lib.mas_probe_stream(buf.data_ptr(), nbytes, int(n), int(nin), int(nout), s),
                  "mas_probe_stream")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            abi.check(lib.mas_probe_stream(buf.data_ptr(), nbytes, int(n), int(nin), int(nout), s),
                      "mas_probe_stream")
        e1.record()
        torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    return (nin + nout) * 8 * int(n) / sec / 1e9


class MasSolve(torch.autograd.Function):
    """x = A(nu)^-1 (V .* rhs); backward runs the adjoint solve and the fused
    dL/dnu, dL/drhs kernel in the HIP library."""

    @staticmethod
    def forward(ctx, nu, rhs, grid, dt, opts_kw):
        opts_kw = dict(opts_kw or {})
        opts_kw.pop("use_x0", None)  # the solution buffer is fresh memory: start from zero
        op = Operator(grid, nu.detach().contiguous(), dt,
                      precision=opts_kw.get("precision", "fp64"))
        x, info = op.solve(rhs.detach().contiguous(), make_opts(**opts_kw), allow_notconv=False)
        ctx.op = op
        ctx.opts_kw = opts_kw
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        opts = make_opts(**ctx.opts_kw)
        _, gnu, grhs, _ = ctx.op.adjoint(x, gx.contiguous(), opts, allow_notconv=False)
        return gnu, grhs, None, None, None


def solve(nu: torch.Tensor, rhs: torch.Tensor, grid: Grid, dt: float, **opts) -> torch.Tensor:
    """Differentiable implicit viscous step: gradients flow to nu and rhs."""
    return MasSolve.apply(nu, rhs, grid, dt, opts)
