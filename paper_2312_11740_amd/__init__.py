"""MI355X (gfx950) multiphase pressure-projection solver.

Python binding of libmpp.so (include/mpp.h).  This layer only marshals arguments:
PyTorch supplies device memory (the operator workspace and every field) and the HIP
stream; every step of the computation runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing or no GPU is visible, calls raise.

Fields are float64 CUDA tensors of shape (n, n, n) or (batch, n, n, n), contiguous,
indexed [k, j, i] (x fastest), cell centres at ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpp.so")
# parameters of the learned-guess network trained on 64^3 problems (train.py)
TRAINED_WEIGHTS = os.path.join(HERE, "weights", "unet64.f32")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONVERGED, EBREAKDOWN = 0, -1, -2, -3, -4, -5
MODE_FP64, MODE_MIXED = 0, 1
GUESS_ZERO, GUESS_GIVEN = 0, 1

EXPORTS = (
    "mpp_default_opts", "mpp_workspace_bytes", "mpp_build_operator", "mpp_apply_stencil",
    "mpp_solve", "mpp_rhs", "mpp_vcycle", "mpp_operator_fields", "mpp_levels",
    "mpp_destroy_operator", "mpp_strerror", "mpp_profile_start", "mpp_profile_stop",
    "mpp_update_operator", "mpp_net_param_count", "mpp_net_workspace_bytes", "mpp_net_create",
    "mpp_net_destroy", "mpp_net_set_params", "mpp_net_get_params", "mpp_net_forward",
    "mpp_net_loss", "mpp_net_backward", "mpp_net_get_grads", "mpp_net_adam",
    "mpp_net_features", "mpp_learned_guess", "mpp_divergence", "mpp_project",
    "mpp_ls_advect", "mpp_ls_reinit", "mpp_heat_solve", "mpp_blocks_scatter",
    "mpp_blocks_gather", "mpp_blocks_fill_guards", "mpp_blocks_apply",
    "mpp_amr_workspace_bytes", "mpp_amr_create", "mpp_amr_destroy", "mpp_amr_level1_blocks",
    "mpp_amr_fill_guards", "mpp_amr_apply", "mpp_amr_solve_work_bytes", "mpp_amr_solve",
    "mpp_amr_coarse_operator", "mpp_net_train", "mpp_ls_reinit_noalloc", "mpp_deflation_info",
)
FLAG_NO_GRAPHS = 1


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("batch", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("guess", ctypes.c_int32), ("nu", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("nu_coarse", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("deflate", ctypes.c_int32), ("reuse_rhs", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("removed_mean", ctypes.c_double),
                ("bnorm", ctypes.c_double)]


class NetTrainOpts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("first_step", ctypes.c_int64), ("total_steps", ctypes.c_int64),
                ("lr0", ctypes.c_float), ("lr1", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class MppError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, strerror(status), status))


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libmpp.so and declares its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmpp.so is not built: run `python -m paper_2312_11740_amd.build` "
                           "(hipcc --offload-arch=gfx950)")
    # torch first: its HIP runtime must be the one the library's calls resolve to, so
    # that device pointers and streams from torch are valid in the library
    _torch()
    L = ctypes.CDLL(path)
    P, i32, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.mpp_default_opts.argtypes = [ctypes.POINTER(SolveOpts)]
    L.mpp_default_opts.restype = None
    L.mpp_workspace_bytes.argtypes = [ctypes.POINTER(Desc)]
    L.mpp_workspace_bytes.restype = ctypes.c_size_t
    L.mpp_build_operator.argtypes = [ctypes.POINTER(Desc), P, P, P, P, P, ctypes.c_size_t, P,
                                     ctypes.POINTER(P)]
    L.mpp_update_operator.argtypes = [P, P, P, P, P, P]
    L.mpp_apply_stencil.argtypes = [P, P, P, P]
    L.mpp_solve.argtypes = [P, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P]
    L.mpp_rhs.argtypes = [P, P, P, P, P]
    L.mpp_vcycle.argtypes = [P, P, P, i32, P]
    L.mpp_operator_fields.argtypes = [P, P, P, P, P, P, P]
    L.mpp_levels.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.mpp_deflation_info.argtypes = [P, P, P, P, P]
    L.mpp_destroy_operator.argtypes = [P]
    L.mpp_destroy_operator.restype = None
    L.mpp_profile_start.argtypes = [P]
    L.mpp_profile_stop.argtypes = [P, ctypes.POINTER(KernelStat), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    L.mpp_strerror.argtypes = [i32]
    L.mpp_strerror.restype = ctypes.c_char_p
    L.mpp_net_param_count.argtypes = []
    L.mpp_net_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.mpp_net_workspace_bytes.restype = ctypes.c_size_t
    L.mpp_net_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P,
                                 ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.mpp_net_destroy.argtypes = [P]
    L.mpp_net_destroy.restype = None
    L.mpp_net_set_params.argtypes = [P, P, P]
    L.mpp_net_get_params.argtypes = [P, P, P]
    L.mpp_net_forward.argtypes = [P, P, P, ctypes.c_int32, P]
    L.mpp_net_loss.argtypes = [P, P, P, P, P, ctypes.c_int32, P]
    L.mpp_net_backward.argtypes = [P, P, ctypes.c_int32, P]
    L.mpp_net_get_grads.argtypes = [P, P, P]
    L.mpp_net_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, P]
    L.mpp_net_train.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(NetTrainOpts), P, P]
    L.mpp_net_features.argtypes = [P, P, P, P, P, P, P, P]
    L.mpp_learned_guess.argtypes = [P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32),
                                    P]
    L.mpp_divergence.argtypes = [P, P, P, P, d, P, P]
    L.mpp_project.argtypes = [P, P, P, d, P, P, P, P]
    L.mpp_ls_advect.argtypes = [i32, i32, P, P, P, P, d, P, P]
    L.mpp_ls_reinit.argtypes = [i32, i32, P, P, P, i32, d, P]
    L.mpp_ls_reinit_noalloc.argtypes = [i32, i32, P, P, i32, d, P]
    for nm in ("mpp_blocks_scatter", "mpp_blocks_gather"):
        getattr(L, nm).argtypes = [i32, i32, i32, i32, P, P, P]
    L.mpp_blocks_fill_guards.argtypes = [i32, i32, i32, i32, P, P]
    L.mpp_blocks_apply.argtypes = [P, i32, i32, P, P, P]
    L.mpp_amr_workspace_bytes.argtypes = [i32, i32]
    L.mpp_amr_workspace_bytes.restype = ctypes.c_size_t
    L.mpp_amr_create.argtypes = [i32, i32, i32, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.mpp_amr_destroy.argtypes = [P]
    L.mpp_amr_destroy.restype = None
    L.mpp_amr_level1_blocks.argtypes = [P, ctypes.POINTER(ctypes.c_int32), P]
    L.mpp_amr_fill_guards.argtypes = [P, P, P, P]
    L.mpp_amr_apply.argtypes = [P, P, P, P, P, d, d, P, P, P]
    L.mpp_amr_coarse_operator.argtypes = [P, P, P, P, d, d, P]
    L.mpp_amr_solve_work_bytes.argtypes = [P]
    L.mpp_amr_solve_work_bytes.restype = ctypes.c_size_t
    L.mpp_amr_solve.argtypes = [P, P, P, P, d, d, P, P, P, P, d, i32, P, ctypes.c_size_t,
                                ctypes.POINTER(i32), ctypes.POINTER(d), P]
    L.mpp_heat_solve.argtypes = [P, P, P, d, P, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(SolveInfo), P]
    for name in (n for n in EXPORTS if n not in ("mpp_default_opts", "mpp_destroy_operator",
                                                 "mpp_strerror", "mpp_workspace_bytes",
                                                 "mpp_net_workspace_bytes",
                                                 "mpp_net_destroy", "mpp_amr_workspace_bytes",
                                                 "mpp_amr_destroy", "mpp_amr_solve_work_bytes")):
        getattr(L, name).restype = i32
    _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return load_library().mpp_strerror(int(status)).decode()
    except RuntimeError:
        return "status %d" % status


def workspace_bytes(n: int, batch: int = 1) -> int:
    d = Desc(n, batch, 0)
    return int(load_library().mpp_workspace_bytes(ctypes.byref(d)))


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_field(t, shape, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % what)
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be contiguous with shape %s, got %s" % (what, tuple(shape),
                                                                          tuple(t.shape)))


@dataclass
class Info:
    status: int
    iters: int
    outer_iters: int
    rel_resid: float
    removed_mean: float
    bnorm: float


class Operator:
    """A built operator: ghost-fluid faces, curvature, jump term, multigrid hierarchy.

    phi: (n,n,n) or (B,n,n,n) float64 CUDA tensor; rho_neg, rho_pos, sigma: scalars or
    length-B sequences (density where phi <= 0, where phi > 0, surface tension)."""

    def __init__(self, phi, rho_neg, rho_pos, sigma, workspace=None, graphs=True):
        torch = _torch()
        L = load_library()
        self.batched = phi.dim() == 4
        if phi.dim() not in (3, 4):
            raise ValueError("phi must be (n,n,n) or (B,n,n,n)")
        B = phi.shape[0] if self.batched else 1
        n = phi.shape[-1]
        self.n, self.batch = int(n), int(B)
        self.shape = tuple(phi.shape)
        _check_field(phi, self.shape, "phi")
        self.device = phi.device

        def arr(v):
            vals = list(v) if hasattr(v, "__len__") else [v] * B
            if len(vals) != B:
                raise ValueError("need %d values" % B)
            return (ctypes.c_double * B)(*[float(x) for x in vals])

        self._rn, self._rp, self._sg = arr(rho_neg), arr(rho_pos), arr(sigma)
        self._desc = Desc(self.n, self.batch, 0 if graphs else FLAG_NO_GRAPHS)
        nbytes = int(L.mpp_workspace_bytes(ctypes.byref(self._desc)))
        if nbytes == 0:
            raise MppError(EINVAL, "unsupported shape n=%d batch=%d" % (n, B))
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif workspace.dtype != torch.uint8 or workspace.numel() < nbytes or not workspace.is_cuda:
            raise ValueError("workspace must be a CUDA uint8 tensor of >= %d bytes" % nbytes)
        self.workspace = workspace
        h = ctypes.c_void_p()
        st = L.mpp_build_operator(ctypes.byref(self._desc), ctypes.c_void_p(phi.data_ptr()),
                                  self._rn, self._rp, self._sg,
                                  ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  _stream_handle(self.device), ctypes.byref(h))
        if st != OK:
            raise MppError(st, "mpp_build_operator")
        self._h = h

    def update(self, phi, rho_neg, rho_pos, sigma):
        """Rebuilds the operator in place for a new level set and constants."""
        _check_field(phi, self.shape, "phi")
        B = self.batch

        def arr(v):
            vals = list(v) if hasattr(v, "__len__") else [v] * B
            return (ctypes.c_double * B)(*[float(x) for x in vals])

        self._rn, self._rp, self._sg = arr(rho_neg), arr(rho_pos), arr(sigma)
        st = load_library().mpp_update_operator(self._h, ctypes.c_void_p(phi.data_ptr()),
                                                self._rn, self._rp, self._sg,
                                                _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_update_operator")

    # -- calls --------------------------------------------------------------------
    def _new(self):
        return _torch().empty(self.shape, dtype=_torch().float64, device=self.device)

    def apply(self, x, out=None):
        _check_field(x, self.shape, "x")
        y = self._new() if out is None else out
        _check_field(y, self.shape, "out")
        st = load_library().mpp_apply_stencil(self._h, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(y.data_ptr()),
                                              _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_apply_stencil")
        return y

    def rhs(self, f):
        _check_field(f, self.shape, "f")
        b = self._new()
        means = (ctypes.c_double * self.batch)()
        st = load_library().mpp_rhs(self._h, ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(b.data_ptr()), means,
                                    _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_rhs")
        return b, list(means)

    def vcycle(self, r, nu=2):
        _check_field(r, self.shape, "r")
        z = self._new()
        st = load_library().mpp_vcycle(self._h, ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(z.data_ptr()), int(nu),
                                       _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_vcycle")
        return z

    def fields(self):
        out = {k: self._new() for k in ("beta_x", "beta_y", "beta_z", "kappa", "jterm")}
        st = load_library().mpp_operator_fields(
            self._h, *[ctypes.c_void_p(out[k].data_ptr())
                       for k in ("beta_x", "beta_y", "beta_z", "kappa", "jterm")],
            _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_operator_fields")
        return out

    def deflation_info(self):
        """(labels uint8 CUDA tensor of the operator's shape, k per problem, E as a float64
        numpy array [batch][32][32]) of the deflation regions."""
        import numpy as np
        torch = _torch()
        lab = torch.empty(self.shape, dtype=torch.uint8, device=self.device)
        k = (ctypes.c_int32 * self.batch)()
        E = np.empty((self.batch, 32, 32))
        st = load_library().mpp_deflation_info(self._h, ctypes.c_void_p(lab.data_ptr()), k,
                                               E.ctypes.data_as(ctypes.c_void_p),
                                               _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_deflation_info")
        return lab, [int(v) for v in k], E

    def levels(self):
        nl = ctypes.c_int32(0)
        sizes = (ctypes.c_int32 * 16)()
        st = load_library().mpp_levels(self._h, ctypes.byref(nl), sizes)
        if st != OK:
            raise MppError(st, "mpp_levels")
        return [sizes[i] for i in range(nl.value)]

    def solve(self, f, p=None, rtol=1e-10, mode="fp64", max_iter=500, nu=2, check_every=2,
              inner_rtol=1e-5, raise_on_error=True, nu_coarse=0, deflate=True, zero=False,
              reuse_rhs=False):
        """Returns (p, [Info per problem]).  p: optional initial guess (overwritten); with
        zero=True p is only the output array and the solve starts from zero.  deflate:
        deflate the lighter phase's regions (mpp_solve_opts.deflate).  reuse_rhs: take the
        right-hand side the preceding learned_guess with this f assembled
        (mpp_solve_opts.reuse_rhs)."""
        _check_field(f, self.shape, "f")
        opts = SolveOpts()
        load_library().mpp_default_opts(ctypes.byref(opts))
        opts.deflate = 1 if deflate else 0
        opts.reuse_rhs = 1 if reuse_rhs else 0
        opts.rtol, opts.max_iter, opts.nu = float(rtol), int(max_iter), int(nu)
        opts.check_every, opts.inner_rtol = int(check_every), float(inner_rtol)
        opts.nu_coarse = int(nu_coarse)
        opts.mode = {"fp64": MODE_FP64, "mixed": MODE_MIXED}[mode]
        if p is None:
            p = self._new()
            opts.guess = GUESS_ZERO
        else:
            _check_field(p, self.shape, "p")
            opts.guess = GUESS_ZERO if zero else GUESS_GIVEN
        infos = (SolveInfo * self.batch)()
        st = load_library().mpp_solve(self._h, ctypes.c_void_p(f.data_ptr()),
                                      ctypes.c_void_p(p.data_ptr()), ctypes.byref(opts), infos,
                                      _stream_handle(self.device))
        out = [Info(q.status, q.iters, q.outer_iters, q.rel_resid, q.removed_mean, q.bnorm)
               for q in infos]
        if st != OK and raise_on_error:
            raise MppError(st, "mpp_solve")
        return p, out

    def heat_solve(self, t_old, dt, src=None, t=None, rtol=1e-10, precond="mg", mode="fp64",
                   nu=2, max_iter=2000, check_every=2, inner_rtol=1e-5, raise_on_error=True):
        """One backward-Euler diffusion step (I - dt div(K grad)) T = t_old + dt src on
        this operator's face coefficients, read as conductivities K (build the operator
        with rho_neg = 1/K_neg, rho_pos = 1/K_pos; sigma plays no part).  precond "mg":
        the pressure solve's MG-PCG on the shifted operator (mode "fp64" or "mixed");
        "jacobi": CG with the inverse diagonal (FP64).  t: optional initial guess,
        overwritten with T (may be t_old).  Returns (T, [Info])."""
        _check_field(t_old, self.shape, "t_old")
        if src is not None:
            _check_field(src, self.shape, "src")
        opts = SolveOpts()
        load_library().mpp_default_opts(ctypes.byref(opts))
        opts.rtol, opts.max_iter, opts.check_every = float(rtol), int(max_iter), int(check_every)
        opts.nu = {"mg": int(nu), "jacobi": 0}[precond]
        opts.mode = {"fp64": MODE_FP64, "mixed": MODE_MIXED}[mode]
        opts.inner_rtol = float(inner_rtol)
        if t is None:
            t = self._new()
            opts.guess = GUESS_ZERO
        else:
            _check_field(t, self.shape, "t")
            opts.guess = GUESS_GIVEN
        infos = (SolveInfo * self.batch)()
        st = load_library().mpp_heat_solve(
            self._h, ctypes.c_void_p(t_old.data_ptr()),
            ctypes.c_void_p(src.data_ptr() if src is not None else None), float(dt),
            ctypes.c_void_p(t.data_ptr()), ctypes.byref(opts), infos, _stream_handle(self.device))
        out = [Info(q.status, q.iters, q.outer_iters, q.rel_resid, q.removed_mean, q.bnorm)
               for q in infos]
        if st != OK and raise_on_error:
            raise MppError(st, "mpp_heat_solve")
        return t, out

    def blocks_apply(self, x_blocks, nb, g, out=None):
        """y = A x on the block layout (guards of x filled); y's guards are 0."""
        shape = _blocks_dims(self.n, nb, g, self.batch if self.batched else None)
        _check_field(x_blocks, shape, "x_blocks")
        y = _torch().empty_like(x_blocks) if out is None else out
        _check_field(y, shape, "y_blocks")
        st = load_library().mpp_blocks_apply(self._h, nb, g, ctypes.c_void_p(x_blocks.data_ptr()),
                                             ctypes.c_void_p(y.data_ptr()),
                                             _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_blocks_apply")
        return y

    def divergence(self, u, dt, out=None):
        """f = div(u)/dt of the low-face velocities u = (ux, uy, uz)."""
        for name, a in zip(("ux", "uy", "uz"), u):
            _check_field(a, self.shape, name)
        f = self._new() if out is None else out
        _check_field(f, self.shape, "out")
        st = load_library().mpp_divergence(self._h, *[ctypes.c_void_p(a.data_ptr()) for a in u],
                                           float(dt), ctypes.c_void_p(f.data_ptr()),
                                           _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_divergence")
        return f

    def project(self, phi, p, dt, u):
        """u -= dt beta grad p (jump-corrected), in place; returns u."""
        _check_field(phi, self.shape, "phi")
        _check_field(p, self.shape, "p")
        for name, a in zip(("ux", "uy", "uz"), u):
            _check_field(a, self.shape, name)
        st = load_library().mpp_project(self._h, ctypes.c_void_p(phi.data_ptr()),
                                        ctypes.c_void_p(p.data_ptr()), float(dt),
                                        *[ctypes.c_void_p(a.data_ptr()) for a in u],
                                        _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_project")
        return u

    def learned_guess(self, net, f, sweeps=2, out=None, judge="plain"):
        """Initial guess from the network (device float64, the operator's shape) and the
        per-problem fallback flags (1 where the guess was replaced by zero).  judge:
        "plain" (for a solve without deflation) or "deflated" (for a deflated one)."""
        _check_field(f, self.shape, "f")
        p = self._new() if out is None else out
        _check_field(p, self.shape, "out")
        flags = (ctypes.c_int32 * self.batch)()
        jd = {"plain": 0, "deflated": 1}[judge]
        st = load_library().mpp_learned_guess(self._h, net._h, ctypes.c_void_p(f.data_ptr()),
                                              ctypes.c_void_p(p.data_ptr()), int(sweeps), jd,
                                              flags, _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_learned_guess")
        return p, [int(v) for v in flags]

    def profile_start(self):
        st = load_library().mpp_profile_start(self._h)
        if st != OK:
            raise MppError(st, "mpp_profile_start")

    def profile_stop(self):
        """Per-kernel launches, event time (ms) and algorithmic bytes since profile_start."""
        stats = (KernelStat * 32)()
        cnt = ctypes.c_int32(0)
        st = load_library().mpp_profile_stop(self._h, stats, 32, ctypes.byref(cnt))
        if st != OK:
            raise MppError(st, "mpp_profile_stop")
        return {stats[i].name.decode(): dict(launches=stats[i].launches, ms=stats[i].total_ms,
                                             bytes=stats[i].bytes)
                for i in range(cnt.value)}

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            load_library().mpp_destroy_operator(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _grid_shape(phi):
    """(n, batch) of a device float64 cell field [n,n,n] or [batch,n,n,n]."""
    torch = _torch()
    if not isinstance(phi, torch.Tensor) or not phi.is_cuda or phi.dtype != torch.float64:
        raise TypeError("phi must be a float64 CUDA (HIP) tensor")
    if phi.dim() == 3:
        batch, n = 1, phi.shape[0]
    elif phi.dim() == 4:
        batch, n = phi.shape[0], phi.shape[1]
    else:
        raise ValueError("phi must have shape [n,n,n] or [batch,n,n,n]")
    if tuple(phi.shape[-3:]) != (n, n, n) or not phi.is_contiguous():
        raise ValueError("phi must be contiguous and cubic")
    return n, batch


def ls_advect(phi, u, dt, out=None):
    """One upwind advection step of the level set phi by the low-face velocities
    u = (ux, uy, uz) (same shape as phi); returns the new level set."""
    n, batch = _grid_shape(phi)
    for name, a in zip(("ux", "uy", "uz"), u):
        _check_field(a, phi.shape, name)
    out = _torch().empty_like(phi) if out is None else out
    _check_field(out, phi.shape, "out")
    st = load_library().mpp_ls_advect(n, batch, ctypes.c_void_p(phi.data_ptr()),
                                      *[ctypes.c_void_p(a.data_ptr()) for a in u], float(dt),
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(phi.device))
    if st != OK:
        raise MppError(st, "mpp_ls_advect")
    return out


def ls_reinit(phi, iters, dtau=None, phi0=None, work=None):
    """iters re-distancing steps of phi in place (signs from phi0, default a copy of phi;
    dtau default h/2); returns phi."""
    torch = _torch()
    n, batch = _grid_shape(phi)
    phi0 = phi.clone() if phi0 is None else phi0
    work = torch.empty_like(phi) if work is None else work
    _check_field(phi0, phi.shape, "phi0")
    _check_field(work, phi.shape, "work")
    dtau = 0.5 / n if dtau is None else dtau
    st = load_library().mpp_ls_reinit(n, batch, ctypes.c_void_p(phi0.data_ptr()),
                                      ctypes.c_void_p(phi.data_ptr()),
                                      ctypes.c_void_p(work.data_ptr()), int(iters), float(dtau),
                                      _stream_handle(phi.device))
    if st != OK:
        raise MppError(st, "mpp_ls_reinit")
    return phi


REINIT_NOALLOC_MAX_CELLS = 1 << 24


def ls_reinit_noalloc(phi, phi0, iters, dtau=None):
    """ls_reinit through mpp_ls_reinit_noalloc: no work array, nothing allocated (phi0 is
    required, so the call makes no copy either); at most 2^24 cells over the batch."""
    n, batch = _grid_shape(phi)
    _check_field(phi0, phi.shape, "phi0")
    dtau = 0.5 / n if dtau is None else dtau
    st = load_library().mpp_ls_reinit_noalloc(n, batch, ctypes.c_void_p(phi0.data_ptr()),
                                              ctypes.c_void_p(phi.data_ptr()), int(iters),
                                              float(dtau), _stream_handle(phi.device))
    if st != OK:
        raise MppError(st, "mpp_ls_reinit_noalloc")
    return phi


def _blocks_dims(n, nb, g, batch):
    nbx = n // nb
    shape = (nbx ** 3, nb + 2 * g, nb + 2 * g, nb + 2 * g)
    return shape if batch is None else (batch,) + shape


def blocks_scatter(grid, nb, g, out=None):
    """Grid (n,n,n) or (B,n,n,n) -> block layout (nblk,P,P,P) or (B,nblk,P,P,P); guards
    of a new `out` are 0."""
    torch = _torch()
    batched = grid.dim() == 4
    n = grid.shape[-1]
    _check_field(grid, tuple(grid.shape), "grid")
    shape = _blocks_dims(n, nb, g, grid.shape[0] if batched else None)
    if out is None:
        out = torch.zeros(shape, dtype=torch.float64, device=grid.device)
    _check_field(out, shape, "blocks")
    st = load_library().mpp_blocks_scatter(n, grid.shape[0] if batched else 1, nb, g,
                                           ctypes.c_void_p(grid.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(grid.device))
    if st != OK:
        raise MppError(st, "mpp_blocks_scatter")
    return out


def blocks_gather(blocks, n, nb, g, out=None):
    """Block layout -> grid (n,n,n) or (B,n,n,n)."""
    torch = _torch()
    batched = blocks.dim() == 5
    B = blocks.shape[0] if batched else 1
    _check_field(blocks, _blocks_dims(n, nb, g, B if batched else None), "blocks")
    shape = (B, n, n, n) if batched else (n, n, n)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=blocks.device)
    _check_field(out, shape, "grid")
    st = load_library().mpp_blocks_gather(n, B, nb, g, ctypes.c_void_p(blocks.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()),
                                          _stream_handle(blocks.device))
    if st != OK:
        raise MppError(st, "mpp_blocks_gather")
    return out


def blocks_fill_guards(blocks, n, nb, g):
    """Fills the guard cells of a block layout in place; returns it."""
    batched = blocks.dim() == 5
    B = blocks.shape[0] if batched else 1
    _check_field(blocks, _blocks_dims(n, nb, g, B if batched else None), "blocks")
    st = load_library().mpp_blocks_fill_guards(n, B, nb, g, ctypes.c_void_p(blocks.data_ptr()),
                                               _stream_handle(blocks.device))
    if st != OK:
        raise MppError(st, "mpp_blocks_fill_guards")
    return blocks


class AmrGrid:
    """Two-level composite grid (include/mpp.h): level 0 of n0^3 cells in blocks of nb^3
    with g guard layers, the blocks flagged in `refined0` ((n0/nb)^3 uint8, [bk, bj, bi])
    covered by level 1 at half the spacing.  Fields are float64 CUDA tensors in the block
    layout: level 0 (nblk0, P, P, P), level 1 (nblk1, P, P, P); `list1` holds the
    position of each stored level-1 block."""

    def __init__(self, n0, nb, g, refined0, device="cuda"):
        torch = _torch()
        L = load_library()
        import numpy as np
        flags = np.ascontiguousarray(np.asarray(refined0), dtype=np.uint8).reshape(-1)
        self.n0, self.nb, self.g, self.P = int(n0), int(nb), int(g), int(nb) + 2 * int(g)
        self.device = torch.device(device)
        self.nblk0 = (self.n0 // self.nb) ** 3 if self.nb > 0 else 0
        if flags.size != self.nblk0:
            raise ValueError("refined0 must hold (n0/nb)^3 = %d flags" % self.nblk0)
        nbytes = int(L.mpp_amr_workspace_bytes(self.n0, self.nb))
        if nbytes == 0:
            raise MppError(-1, "mpp_amr_workspace_bytes")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = L.mpp_amr_create(self.n0, self.nb, self.g, flags.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_void_p(self._ws.data_ptr()), nbytes,
                              _stream_handle(self.device), ctypes.byref(h))
        if st != OK:
            raise MppError(st, "mpp_amr_create")
        self._h = h
        cnt = ctypes.c_int32(0)
        L.mpp_amr_level1_blocks(self._h, ctypes.byref(cnt), None)
        self.nblk1 = int(cnt.value)
        self.list1 = np.zeros(max(self.nblk1, 1), dtype=np.int32)
        L.mpp_amr_level1_blocks(self._h, ctypes.byref(cnt), self.list1.ctypes.data_as(ctypes.c_void_p))
        self.list1 = self.list1[:self.nblk1]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            load_library().mpp_amr_destroy(h)
            self._h = None

    def shapes(self):
        P = self.P
        return (self.nblk0, P, P, P), (self.nblk1, P, P, P)

    def empty(self):
        torch = _torch()
        s0, s1 = self.shapes()
        return (torch.zeros(s0, dtype=torch.float64, device=self.device),
                torch.zeros(s1, dtype=torch.float64, device=self.device))

    def _fields(self, pairs):
        s0, s1 = self.shapes()
        out = []
        for (a0, a1), what in pairs:
            _check_field(a0, s0, what + "0")
            if self.nblk1:
                _check_field(a1, s1, what + "1")
            out += [ctypes.c_void_p(a0.data_ptr()),
                    ctypes.c_void_p(a1.data_ptr()) if self.nblk1 else None]
        return out

    def fill_guards(self, b0, b1):
        """Guard cells of both levels in place; returns (b0, b1)."""
        p = self._fields([((b0, b1), "blocks")])
        st = load_library().mpp_amr_fill_guards(self._h, p[0], p[1], _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_amr_fill_guards")
        return b0, b1

    def coarse_operator(self, phi0, phi, rho_neg, rho_pos):
        """The level-0 Operator of the two-level cycle, built from phi0 ((n0,)*3 float64
        CUDA tensor) with its faces next to refined blocks averaged from the fine level
        (phi: (level0, level1) blocks with filled guards)."""
        op = Operator(phi0, rho_neg, rho_pos, 0.0)
        p = self._fields([(phi, "phi")])
        st = load_library().mpp_amr_coarse_operator(self._h, op._h,
                                                    ctypes.c_void_p(phi0.data_ptr()), p[1],
                                                    float(rho_neg), float(rho_pos),
                                                    _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_amr_coarse_operator")
        return op

    def solve(self, phi, b, rho_neg, rho_pos, x=None, rtol=1e-10, max_iter=100000, coarse=None):
        """x with A x = b - mean(b) on the leaves (preconditioned CG, zero weighted mean);
        phi: (level0, level1) blocks with filled guards; b: (level0, level1) blocks; x:
        initial guess, updated in place (zeros if None); coarse: None (the inverse
        diagonal) or an Operator on the level-0 grid (a two-level multigrid cycle).
        Returns (x, Info)."""
        torch = _torch()
        if x is None:
            x = self.empty()
        p = self._fields([(phi, "phi"), (b, "b"), (x, "x")])
        L = load_library()
        nbytes = int(L.mpp_amr_solve_work_bytes(self._h))
        if getattr(self, "_work", None) is None or self._work.numel() < nbytes:
            self._work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = L.mpp_amr_solve(self._h, coarse._h if coarse is not None else None, p[0], p[1],
                             float(rho_neg), float(rho_pos), p[2], p[3],
                             p[4], p[5], float(rtol), int(max_iter),
                             ctypes.c_void_p(self._work.data_ptr()), nbytes, ctypes.byref(it),
                             ctypes.byref(rel), _stream_handle(self.device))
        if st not in (OK, ENOTCONVERGED):
            raise MppError(st, "mpp_amr_solve")
        return x, Info(st, int(it.value), 0, float(rel.value), 0.0, 0.0)

    def apply(self, phi, x, rho_neg, rho_pos, y=None):
        """y = A x on the leaves; phi, x: (level0, level1) pairs with filled guards."""
        if y is None:
            y = self.empty()
        p = self._fields([(phi, "phi"), (x, "x"), (y, "y")])
        st = load_library().mpp_amr_apply(self._h, p[0], p[1], p[2], p[3], float(rho_neg),
                                          float(rho_pos), p[4], p[5], _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_amr_apply")
        return y


def net_param_count() -> int:
    return int(load_library().mpp_net_param_count())


def net_workspace_bytes(n: int, batch_max: int) -> int:
    return int(load_library().mpp_net_workspace_bytes(int(n), int(batch_max)))


class Net:
    """The learned-guess U-Net (include/mpp.h) at resolution n for batches of up to
    batch_max samples.  Inputs x: bfloat16 CUDA tensors (B, n, n, n, 4); predictions,
    targets and gradients: float32 CUDA tensors (B, n, n, n)."""

    def __init__(self, n, batch_max=1, seed=0, device="cuda", workspace=None):
        torch = _torch()
        L = load_library()
        self.n, self.batch_max = int(n), int(batch_max)
        self.device = torch.device(device)
        nbytes = net_workspace_bytes(self.n, self.batch_max)
        if nbytes == 0:
            raise MppError(EINVAL, "unsupported network shape n=%d batch_max=%d" % (n, batch_max))
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        elif workspace.dtype != torch.uint8 or workspace.numel() < nbytes or not workspace.is_cuda:
            raise ValueError("workspace must be a CUDA uint8 tensor of >= %d bytes" % nbytes)
        self.workspace = workspace
        h = ctypes.c_void_p()
        st = L.mpp_net_create(self.n, self.batch_max, int(seed) & (2**64 - 1),
                              ctypes.c_void_p(workspace.data_ptr()), nbytes,
                              _stream_handle(self.device), ctypes.byref(h))
        if st != OK:
            raise MppError(st, "mpp_net_create")
        self._h = h
        self.nparams = net_param_count()

    def _stream(self):
        return _stream_handle(self.device)

    def _check(self, t, dtype, shape, what):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
            raise TypeError("%s must be a CUDA %s tensor" % (what, dtype))
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("%s must be contiguous with shape %s, got %s"
                             % (what, tuple(shape), tuple(t.shape)))

    def get_params(self):
        import numpy as np
        out = np.empty(self.nparams, dtype=np.float32)
        st = load_library().mpp_net_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                               self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_get_params")
        return out

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.nparams:
            raise ValueError("need %d parameters" % self.nparams)
        st = load_library().mpp_net_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p),
                                               self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_set_params")

    def load(self, path):
        """Parameters from a raw little-endian FP32 file (as train.py writes them)."""
        import numpy as np
        self.set_params(np.fromfile(path, dtype="<f4"))

    def save(self, path):
        self.get_params().astype("<f4").tofile(path)

    def get_grads(self):
        import numpy as np
        out = np.empty(self.nparams, dtype=np.float32)
        st = load_library().mpp_net_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                              self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_get_grads")
        return out

    def forward(self, x, out=None):
        torch = _torch()
        B = x.shape[0]
        self._check(x, torch.bfloat16, (B, self.n, self.n, self.n, 4), "x")
        y = torch.empty((B, self.n, self.n, self.n), dtype=torch.float32, device=self.device) \
            if out is None else out
        self._check(y, torch.float32, (B, self.n, self.n, self.n), "y")
        st = load_library().mpp_net_forward(self._h, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()), int(B), self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_forward")
        return y

    def loss(self, y, t):
        """Per-sample losses (float32 CUDA tensor) and dloss/dy of their mean."""
        torch = _torch()
        B = y.shape[0]
        shp = (B, self.n, self.n, self.n)
        self._check(y, torch.float32, shp, "y")
        self._check(t, torch.float32, shp, "t")
        dy = torch.empty(shp, dtype=torch.float32, device=self.device)
        lo = torch.empty(B, dtype=torch.float32, device=self.device)
        st = load_library().mpp_net_loss(self._h, ctypes.c_void_p(y.data_ptr()),
                                         ctypes.c_void_p(t.data_ptr()),
                                         ctypes.c_void_p(dy.data_ptr()),
                                         ctypes.c_void_p(lo.data_ptr()), int(B), self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_loss")
        return lo, dy

    def backward(self, dy):
        torch = _torch()
        B = dy.shape[0]
        self._check(dy, torch.float32, (B, self.n, self.n, self.n), "dy")
        st = load_library().mpp_net_backward(self._h, ctypes.c_void_p(dy.data_ptr()), int(B),
                                             self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_backward")

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        st = load_library().mpp_net_adam(self._h, float(lr), float(beta1), float(beta2),
                                         float(eps), self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_adam")

    def train(self, x, t, steps, batch, lr=1e-3, lr_final=None, seed=0, first_step=0,
              total_steps=None, beta1=0.9, beta2=0.999, eps=1e-8, losses=True):
        """`steps` training steps of `batch` samples drawn from the stored samples x
        (bfloat16 (count, n, n, n, 4)) and targets t (float32 (count, n, n, n)), in one
        call of mpp_net_train: step g = first_step + s draws its samples from `seed` (0: in
        order) and takes the learning rate lr * (lr_final / lr)^(g / (total_steps - 1)).
        Returns the per-sample losses (float32 (steps, batch), device) or None."""
        torch = _torch()
        count = x.shape[0]
        self._check(x, torch.bfloat16, (count, self.n, self.n, self.n, 4), "x")
        self._check(t, torch.float32, (count, self.n, self.n, self.n), "t")
        o = NetTrainOpts(batch=int(batch), steps=int(steps), first_step=int(first_step),
                         total_steps=int(steps if total_steps is None else total_steps),
                         lr0=float(lr), lr1=float(lr if lr_final is None else lr_final),
                         beta1=float(beta1), beta2=float(beta2), eps=float(eps), reserved=0,
                         seed=int(seed) & (2**64 - 1))
        lo = torch.empty((max(int(steps), 1), int(batch)), dtype=torch.float32,
                         device=self.device) if losses else None
        st = load_library().mpp_net_train(self._h, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(t.data_ptr()), int(count),
                                          ctypes.byref(o),
                                          ctypes.c_void_p(lo.data_ptr() if lo is not None else 0),
                                          self._stream())
        if st != OK:
            raise MppError(st, "mpp_net_train")
        return lo

    def train_step(self, x, t, lr=1e-3):
        """One training step on exactly the samples given (forward, loss, backward, Adam,
        through mpp_net_train in order); returns the per-sample losses (device)."""
        return self.train(x, t, 1, x.shape[0], lr=lr)[0]

    def features(self, op, f, p=None):
        """Network inputs x (bf16) of the operator's problems, targets t (float32, when p
        is given) and rms of the coarse right-hand side per problem."""
        torch = _torch()
        _check_field(f, op.shape, "f")
        if p is not None:
            _check_field(p, op.shape, "p")
        B = op.batch
        x = torch.empty((B, self.n, self.n, self.n, 4), dtype=torch.bfloat16, device=self.device)
        t = torch.empty((B, self.n, self.n, self.n), dtype=torch.float32, device=self.device) \
            if p is not None else None
        rms = torch.empty(B, dtype=torch.float32, device=self.device)
        st = load_library().mpp_net_features(
            self._h, op._h, ctypes.c_void_p(f.data_ptr()),
            ctypes.c_void_p(p.data_ptr() if p is not None else 0),
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr() if t is not None else 0),
            ctypes.c_void_p(rms.data_ptr()), _stream_handle(self.device))
        if st != OK:
            raise MppError(st, "mpp_net_features")
        return x, t, rms

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            load_library().mpp_net_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
