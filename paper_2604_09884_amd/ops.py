"""Python surface of libinrct: handles, the five named calls and the
autograd wrapper of the INR VJP.

Argument marshalling only: tensors are allocated with torch on the current
device, their data pointers and torch's current HIP stream are passed to the
C ABI, and every step runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import lib as L
from .configs import INRArch, Problem


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, numel=None, name="tensor"):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


def view_angles(problem: Problem) -> np.ndarray:
    return np.arange(problem.n_views, dtype=np.float64) * (problem.view_span / problem.n_views)


def _geometry_struct(problem: Problem, angles: np.ndarray):
    g = L.CtGeometry()
    kinds = {"par2d": L.INRCT_PAR2D, "fan2d": L.INRCT_FAN2D, "cone3d": L.INRCT_CONE3D}
    if problem.geometry not in kinds:
        raise ValueError("unknown geometry %r" % problem.geometry)
    g.kind = kinds[problem.geometry]
    g.n_views, g.n_u, g.n_v = len(angles), problem.n_u, problem.n_v
    g.du, g.dv, g.sid, g.idd = problem.du, problem.dv, problem.dso, problem.dod
    g.angles = angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g


def _step_cfg(k, lr, seed=0, loss=L.INRCT_LS, v_mode=L.INRCT_V_FULL, beta1=0.9, beta2=0.999,
              eps=1e-8):
    return L.StepCfg(loss, int(k), seed, lr, beta1, beta2, eps, v_mode)


def workspace_bytes(which, arch: INRArch | None = None, mlp_dtype: str = "fp32",
                    problem: Problem | None = None, angles=None, dim=None, N=None, max_k=0,
                    cfg=None) -> int:
    """Device bytes of a handle's workspace (inrct_workspace_bytes): the
    library's own arithmetic, run on the host."""
    lib = L.load()
    a = arch_struct(arch, mlp_dtype) if arch is not None else None
    g = None
    if problem is not None:
        ang = np.ascontiguousarray(view_angles(problem) if angles is None
                                   else np.asarray(angles, np.float64))
        g = _geometry_struct(problem, ang)
        dim = problem.dim if dim is None else dim
        N = problem.N if N is None else N
    grid = L.InrGrid(dim, N) if dim is not None else None
    ref = ctypes.byref
    nb = lib.inrct_workspace_bytes(which, ref(a) if a is not None else None,
                                   ref(g) if g is not None else None,
                                   ref(grid) if grid is not None else None, int(max_k),
                                   ref(cfg) if cfg is not None else None)
    if nb < 0:
        L.check(int(nb))
    return int(nb)


def request_device_bytes(problem: Problem, mlp_dtype: str | None = None,
                         v_mode=L.INRCT_V_FULL) -> int:
    """Device bytes one reconstruction holds while resident: the three
    workspaces (geometry, model, context) plus the caller's buffers theta,
    its two Adam moments, B and y."""
    dtype = mlp_dtype or problem.mlp_dtype
    k = problem.k()
    ws = (workspace_bytes(L.INRCT_WS_GEOM, problem=problem)
          + workspace_bytes(L.INRCT_WS_MODEL, problem.arch, dtype, dim=problem.dim,
                            N=problem.N, max_k=k)
          + workspace_bytes(L.INRCT_WS_CTX, problem.arch, dtype, problem=problem, max_k=k,
                            cfg=_step_cfg(k, problem.lr, v_mode=v_mode)))
    own = 4 * (3 * problem.arch.n_params + problem.n_rays
               + max(1, problem.arch.n_freq * problem.arch.in_dim))
    return ws + own


def _workspace(nbytes, device):
    """A caller-owned device workspace (torch), 256-byte aligned."""
    t = torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise L.InrctError("torch returned a workspace that is not 256-byte aligned")
    return t


def _device():
    return torch.device("cuda", torch.cuda.current_device())


class Geometry:
    """A scan geometry on a grid (inrct_geom); its tables and scratch live
    in a torch-owned workspace."""

    def __init__(self, problem: Problem, angles=None):
        lib = L.load()
        self.problem = problem
        self.angles = np.ascontiguousarray(
            view_angles(problem) if angles is None else np.asarray(angles, np.float64))
        g = _geometry_struct(problem, self.angles)
        grid = L.InrGrid(problem.dim, problem.N)
        self.ws_bytes = workspace_bytes(L.INRCT_WS_GEOM, problem=problem, angles=self.angles)
        self.ws = _workspace(self.ws_bytes, _device())
        h = ctypes.c_void_p()
        L.check(lib.inrct_geom_create(ctypes.byref(g), ctypes.byref(grid), _ptr(self.ws),
                                      self.ws_bytes, _stream(), ctypes.byref(h)))
        self.handle = h
        self.n_rays = lib.inrct_geom_n_rays(h)
        self.adjoint_kind = lib.inrct_geom_adjoint_kind(h)  # INRCT_ADJ_*
        self.grid_shape = (problem.N,) * problem.dim
        self.proj_shape = ((len(self.angles), problem.n_u) if problem.dim == 2 else
                           (len(self.angles), problem.n_v, problem.n_u))

    def close(self):
        if getattr(self, "handle", None):
            L.load().inrct_geom_destroy(self.handle)
            self.handle = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ct_project(geom: Geometry, u, out=None):
    """z = P u (Sec. III)."""
    _need(u, torch.float32, math.prod(geom.grid_shape), "u")
    z = torch.empty(geom.proj_shape, device=u.device) if out is None else out
    L.check(L.load().ct_project(geom.handle, _ptr(u), _ptr(z), _stream()))
    return z


def ct_backproject(geom: Geometry, r, out=None):
    """v = P^T r, exact transpose of ct_project."""
    _need(r, torch.float32, geom.n_rays, "r")
    v = torch.empty(geom.grid_shape, device=r.device) if out is None else out
    L.check(L.load().ct_backproject(geom.handle, _ptr(r), _ptr(v), _stream()))
    return v


def ct_backproject_at(geom: Geometry, r, idx):
    _need(r, torch.float32, geom.n_rays, "r")
    _need(idx, torch.int32, None, "idx")
    out = torch.empty(idx.numel(), device=r.device)
    L.check(L.load().ct_backproject_at(geom.handle, _ptr(r), _ptr(idx), idx.numel(),
                                       _ptr(out), _stream()))
    return out


def residual_loss(geom: Geometry, z, y, loss=L.INRCT_LS, r=None):
    """(r, L) with r = dL/dz and L as a float64 device scalar (Sec. II)."""
    _need(z, torch.float32, geom.n_rays, "z")
    _need(y, torch.float32, geom.n_rays, "y")
    r = torch.empty_like(z) if r is None else r
    lo = torch.empty((), dtype=torch.float64, device=z.device)
    L.check(L.load().inrct_residual_loss(geom.handle, loss, _ptr(z), _ptr(y), _ptr(r),
                                         _ptr(lo), _stream()))
    return r, lo


def arch_struct(arch: INRArch, mlp_dtype: str):
    a = L.InrArch()
    kinds = {"ffn": L.INRCT_FFN, "siren": L.INRCT_SIREN, "hash": L.INRCT_HASH}
    a.kind = kinds[arch.kind]
    if arch.kind == "hash":
        if arch.hash_feats != 2:
            raise ValueError("the hash encoding runs with 2 features per level")
        a.hash_levels, a.hash_log2_size = arch.hash_levels, arch.hash_log2_size
        a.hash_base_res, a.hash_max_res = arch.hash_base_res, arch.hash_max_res
    a.in_dim, a.n_freq, a.width, a.depth = arch.in_dim, arch.n_freq, arch.width, arch.depth
    a.omega0 = arch.omega0
    a.mlp_dtype = L.INRCT_BF16 if mlp_dtype == "bf16" else L.INRCT_FP32
    return a


class Model:
    """An INR architecture on a grid (inrct_model)."""

    def __init__(self, arch: INRArch, dim: int, N: int, mlp_dtype: str = "fp32",
                 max_k: int | None = None):
        lib = L.load()
        self.arch, self.dim, self.N, self.mlp_dtype = arch, dim, N, mlp_dtype
        a = arch_struct(arch, mlp_dtype)
        grid = L.InrGrid(dim, N)
        h = ctypes.c_void_p()
        max_k = N ** dim if max_k is None else max_k
        self.ws_bytes = workspace_bytes(L.INRCT_WS_MODEL, arch, mlp_dtype, dim=dim, N=N,
                                        max_k=max_k)
        self.ws = _workspace(self.ws_bytes, _device())
        L.check(lib.inrct_model_create(ctypes.byref(a), ctypes.byref(grid), int(max_k),
                                       _ptr(self.ws), self.ws_bytes, _stream(),
                                       ctypes.byref(h)))
        self.handle = h
        self.max_k = int(max_k)
        self.n_params = lib.inrct_model_n_params(h)
        self.n_fov = lib.inrct_model_n_fov(h)
        self.grid_shape = (N,) * dim

    @classmethod
    def for_problem(cls, p: Problem, mlp_dtype: str | None = None, max_k=None):
        return cls(p.arch, p.dim, p.N, mlp_dtype or p.mlp_dtype,
                   p.k() if max_k is None else max_k)

    def close(self):
        if getattr(self, "handle", None):
            L.load().inrct_model_destroy(self.handle)
            self.handle = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_params(self, theta, B):
        _need(theta, torch.float32, self.n_params, "theta")
        if self.arch.kind == "ffn":
            _need(B, torch.float32, self.arch.n_freq * self.arch.in_dim, "B")


def inr_eval_grid(model: Model, theta, B, out=None):
    """u = E{f_theta} on the full grid (0 outside the FOV)."""
    model._check_params(theta, B)
    u = torch.empty(model.grid_shape, device=theta.device) if out is None else out
    L.check(L.load().inr_eval_grid(model.handle, _ptr(theta), _ptr(B), _ptr(u), _stream()))
    return u


def inr_eval_points(model: Model, theta, B, idx):
    model._check_params(theta, B)
    _need(idx, torch.int32, None, "idx")
    f = torch.empty(idx.numel(), device=theta.device)
    L.check(L.load().inr_eval_points(model.handle, _ptr(theta), _ptr(B), _ptr(idx),
                                     idx.numel(), _ptr(f), _stream()))
    return f


def inr_vjp_subsampled(model: Model, theta, B, idx, v, scale, v_compact=None, out=None):
    """g = scale * sum_j v_j grad f(x_{idx_j})  (Eq. (2))."""
    model._check_params(theta, B)
    _need(idx, torch.int32, None, "idx")
    if v_compact is None:
        v_compact = v.numel() == idx.numel() and v.numel() != math.prod(model.grid_shape)
    _need(v, torch.float32, idx.numel() if v_compact else math.prod(model.grid_shape), "v")
    g = torch.empty(model.n_params, device=theta.device) if out is None else out
    L.check(L.load().inr_vjp_subsampled(model.handle, _ptr(theta), _ptr(B), _ptr(idx),
                                        idx.numel(), _ptr(v), 1 if v_compact else 0,
                                        float(scale), _ptr(g), _stream()))
    return g


def sample(model: Model, seed: int, step: int, k: int, device="cuda"):
    idx = torch.empty(k, dtype=torch.int32, device=device)
    L.check(L.load().inrct_sample(model.handle, seed, step, k, _ptr(idx), _stream()))
    return idx


def adam(model: Model, theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    gn = torch.empty((), dtype=torch.float64, device=theta.device)
    L.check(L.load().inrct_adam(model.handle, _ptr(theta), _ptr(m), _ptr(v), _ptr(g), t, lr,
                                beta1, beta2, eps, _ptr(gn), _stream()))
    return gn


class GradStepper:
    """Algorithm 1 + Adam on caller-owned theta / Adam state / data
    (inr_ctx)."""

    def __init__(self, model: Model, geom: Geometry, theta, B, y, k, lr, seed=0,
                 loss=L.INRCT_LS, v_mode=L.INRCT_V_FULL, beta1=0.9, beta2=0.999,
                 eps=1e-8):
        lib = L.load()
        model._check_params(theta, B)
        _need(y, torch.float32, geom.n_rays, "y")
        self.model, self.geom = model, geom
        self.theta, self.B, self.y = theta, B, y
        self.m = torch.zeros_like(theta)
        self.v = torch.zeros_like(theta)
        self.k = int(k)
        cfg = _step_cfg(self.k, lr, seed, loss, v_mode, beta1, beta2, eps)
        p = geom.problem
        self.ws_bytes = workspace_bytes(L.INRCT_WS_CTX, model.arch, model.mlp_dtype,
                                        problem=p, angles=geom.angles, dim=model.dim,
                                        N=model.N, max_k=model.max_k, cfg=cfg)
        self.ws = _workspace(self.ws_bytes, theta.device)
        h = ctypes.c_void_p()
        L.check(lib.inr_ctx_create(model.handle, geom.handle, ctypes.byref(cfg), _ptr(theta),
                                   _ptr(self.m), _ptr(self.v), _ptr(B), _ptr(y),
                                   _ptr(self.ws), self.ws_bytes, _stream(), ctypes.byref(h)))
        self.handle = h
        dev = theta.device
        # the step's loss and ||g||^2 side by side, so one copy reads both
        self.stats = torch.zeros(2, dtype=torch.float64, device=dev)
        self.loss, self.gnorm2 = self.stats[0], self.stats[1]

    def step(self, t: int):
        """Runs step t (0-based); loss and ||g||^2 land in self.loss /
        self.gnorm2 (device) without a host sync."""
        L.check(L.load().inr_grad_step(self.handle, t, _ptr(self.loss), _ptr(self.gnorm2),
                                       _stream()))

    def step_views(self, t: int, geom: "Geometry", y):
        """Step t with the loss over the views of `geom` (data `y` in its ray
        order) in place of the context's geometry and data."""
        _need(y, torch.float32, geom.n_rays, "y")
        L.check(L.load().inr_grad_step_views(self.handle, t, geom.handle, _ptr(y),
                                             _ptr(self.loss), _ptr(self.gnorm2), _stream()))

    STAGES = ("eval_grid", "project", "residual", "sample", "backproject", "vjp", "adam",
              "step")

    def enable_timing(self, max_steps):
        L.check(L.load().inr_ctx_enable_timing(self.handle, int(max_steps)))

    def stage_ms(self):
        """Summed per-stage milliseconds of the steps recorded since
        enable_timing (or the previous call), from HIP events on the step's
        stream."""
        out = (ctypes.c_double * 8)()
        L.check(L.load().inr_ctx_stage_ms(self.handle, 8, out))
        return dict(zip(self.STAGES, list(out)))

    def buffer(self, which, numel, dtype=torch.float32):
        """A context buffer as a tensor view (0 u, 1 r, 2 v, 3 g, 4 I)."""
        p = L.load().inr_ctx_buffer(self.handle, which)
        return _wrap_device(p, numel, dtype, self.theta.device)

    def close(self):
        if getattr(self, "handle", None):
            L.load().inr_ctx_destroy(self.handle)
            self.handle = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def subset_views(n_views: int, n_subsets: int, s: int) -> np.ndarray:
    """Views of ordered subset s: j with j mod n_subsets == s, ascending."""
    if not 1 <= n_subsets <= n_views or not 0 <= s < n_subsets:
        raise ValueError("need 1 <= n_subsets <= n_views and 0 <= s < n_subsets")
    return np.arange(s, n_views, n_subsets)


class OrderedSubsets:
    """Ordered-subsets stepping (the view-subset use of Algorithm 1): step
    t takes the loss over subset t mod S of the views, i.e. views j with
    j mod S == t mod S, with its own geometry and slice of the data, all
    resident on the device."""

    def __init__(self, stepper: GradStepper, n_subsets: int):
        p = stepper.geom.problem
        angles = stepper.geom.angles
        V = len(angles)
        y = stepper.y.reshape(V, -1)
        self.stepper, self.S = stepper, int(n_subsets)
        self.geoms, self.ys = [], []
        for s in range(self.S):
            views = subset_views(V, self.S, s)
            self.geoms.append(Geometry(p, angles=angles[views]))
            self.ys.append(y[torch.as_tensor(views, device=y.device)].reshape(-1).contiguous())

    def step(self, t: int):
        s = t % self.S
        self.stepper.step_views(t, self.geoms[s], self.ys[s])

    def close(self):
        for g in self.geoms:
            g.close()
        self.geoms, self.ys = [], []


def _wrap_device(ptr, numel, dtype, device):
    """Copies `numel` elements at a library-owned device pointer into a new
    tensor (the library keeps ownership)."""
    out = torch.empty(numel, dtype=dtype, device=device)
    nbytes = numel * out.element_size()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.restype = ctypes.c_int
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int, ctypes.c_void_p]
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr),
                            nbytes, 3, _stream())
    if rc != 0:
        raise L.InrctError("hipMemcpyAsync failed: %d" % rc)
    return out


class INRFunction(torch.autograd.Function):
    """f_theta at listed grid points, differentiable in theta.

    forward evaluates f on the matrix cores and saves only (theta, idx);
    backward receives dL/df (for the virtual loss of Eq. (3) this is
    (n/|I|) v_I) and runs the hand-written VJP, which recomputes the
    activations per tile instead of keeping them."""

    @staticmethod
    def forward(ctx, theta, B, idx, model):
        ctx.model = model
        ctx.save_for_backward(theta, B, idx)
        return inr_eval_points(model, theta.detach(), B, idx)

    @staticmethod
    def backward(ctx, grad_out):
        theta, B, idx = ctx.saved_tensors
        g = inr_vjp_subsampled(ctx.model, theta.detach(), B, idx,
                               grad_out.contiguous().float(), 1.0, v_compact=True)
        return g, None, None, None
