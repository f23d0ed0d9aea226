"""ctypes front end of the FP64 CPU oracle (liboracle: mpp_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library and its Python binding never
import this package.

All arrays are float64, C-contiguous, shape (n, n, n) indexed [k, j, i].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpp_oracle.c")
_LIB = os.path.join(_HERE, "libmpp_oracle.so")

OK, EINVAL, ENOMEM, ENOTCONVERGED, EBREAKDOWN = 0, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-shared",
               "-fPIC", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.orc_faces.argtypes = [i, P, d, d, P, P, P]
        L.orc_curvature.argtypes = [i, P, P]
        L.orc_jump.argtypes = [i, P, P, d, d, d, P]
        L.orc_rhs.argtypes = [i, P, P, P, P]
        L.orc_apply.argtypes = [i, P, P, P, P, P]
        L.orc_apply.restype = None
        L.orc_rel_residual.argtypes = [i, P, P, P, P, P]
        L.orc_rel_residual.restype = d
        L.orc_solve_dense.argtypes = [i, P, P, P, P, P]
        L.orc_solve_jacobi_pcg.argtypes = [i, P, P, P, P, P, d, i, P, P]
        L.orc_solve_mg_pcg.argtypes = [i, P, P, P, P, P, d, i, i, P, P]
        L.orc_pipeline.argtypes = [i, P, P, d, d, d, P, P, P, P, P, P, P, P]
        L.orc_divergence.argtypes = [i, P, P, P, d, P]
        L.orc_project.argtypes = [i, P, P, P, d, d, d, d, P, P, P]
        L.orc_ls_advect.argtypes = [i, P, P, P, P, d, P]
        L.orc_ls_reinit.argtypes = [i, P, P, i, d, P]
        L.orc_heat_apply.argtypes = [i, P, P, P, d, P, P]
        L.orc_heat_apply.restype = None
        L.orc_heat_solve.argtypes = [i, P, P, P, d, P, P, d, i, P, P]
        for nm in ("orc_blocks_scatter", "orc_blocks_gather"):
            getattr(L, nm).argtypes = [i, i, i, P, P]
        L.orc_blocks_fill_guards.argtypes = [i, i, i, P]
        L.orc_blocks_apply.argtypes = [i, i, i, P, P, P, P, P]
        L.orc_amr_apply.argtypes = [i, i, P, P, P, P, P, d, d, P, P]
        L.orc_amr_fill.argtypes = [i, i, i, P, P, P, P, P]
        L.orc_amr_solve.argtypes = [i, i, P, P, P, d, d, P, P, P, P, d, i,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.orc_gs_colour.argtypes = [i, P, P, P, P, P, i]
        L.orc_gs_colour.restype = None
        L.orc_restrict.argtypes = [i, P, P]
        L.orc_restrict.restype = None
        L.orc_prolong_add.argtypes = [i, P, P]
        L.orc_prolong_add.restype = None
        L.orc_coarsen_faces.argtypes = [i, P, P, P, P, P, P]
        L.orc_coarsen_faces.restype = None
        L.orc_mg_create.argtypes = [i, P, P, P, i]
        L.orc_mg_create.restype = P
        L.orc_mg_destroy.argtypes = [P]
        L.orc_mg_destroy.restype = None
        L.orc_mg_vcycle.argtypes = [P, P, P]
        L.orc_mg_vcycle.restype = None
        L.orc_mg_levels.argtypes = [P]
        _lib = L
    return _lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _n(a):
    n = a.shape[0]
    assert a.shape == (n, n, n), a.shape
    return n


class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st != OK:
        raise OracleError("%s failed with status %d" % (what, st))


def faces(phi, rho_neg, rho_pos):
    """Ghost-fluid face coefficients (bx, by, bz), low-face convention."""
    phi = _c(phi)
    n = _n(phi)
    bx, by, bz = (np.empty_like(phi) for _ in range(3))
    _check(lib().orc_faces(n, _p(phi), rho_neg, rho_pos, _p(bx), _p(by), _p(bz)), "faces")
    return bx, by, bz


def curvature(phi):
    phi = _c(phi)
    k = np.empty_like(phi)
    _check(lib().orc_curvature(_n(phi), _p(phi), _p(k)), "curvature")
    return k


def jump(phi, kappa, rho_neg, rho_pos, sigma):
    phi, kappa = _c(phi), _c(kappa)
    j = np.empty_like(phi)
    _check(lib().orc_jump(_n(phi), _p(phi), _p(kappa), rho_neg, rho_pos, sigma, _p(j)), "jump")
    return j


def rhs(f, jterm=None):
    """b = f + jterm, mean-removed; returns (b, removed_mean)."""
    f = _c(f)
    b = np.empty_like(f)
    m = ctypes.c_double(0.0)
    jt = _c(jterm) if jterm is not None else None
    _check(lib().orc_rhs(_n(f), _p(f), _p(jt) if jt is not None else None, _p(b),
                         ctypes.byref(m)), "rhs")
    return b, m.value


def apply(fc, x):
    bx, by, bz = (_c(a) for a in fc)
    x = _c(x)
    y = np.empty_like(x)
    lib().orc_apply(_n(x), _p(bx), _p(by), _p(bz), _p(x), _p(y))
    return y


def rel_residual(fc, b, x):
    bx, by, bz = (_c(a) for a in fc)
    b, x = _c(b), _c(x)
    return lib().orc_rel_residual(_n(b), _p(bx), _p(by), _p(bz), _p(b), _p(x))


def solve_dense(fc, b):
    bx, by, bz = (_c(a) for a in fc)
    b = _c(b)
    p = np.empty_like(b)
    _check(lib().orc_solve_dense(_n(b), _p(bx), _p(by), _p(bz), _p(b), _p(p)), "solve_dense")
    return p


def solve_jacobi_pcg(fc, b, tol=1e-13, max_iter=200000, x0=None):
    bx, by, bz = (_c(a) for a in fc)
    b = _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = lib().orc_solve_jacobi_pcg(_n(b), _p(bx), _p(by), _p(bz), _p(b), _p(x), tol, max_iter,
                                    ctypes.byref(it), ctypes.byref(rr))
    return x, dict(status=st, iters=it.value, rel_residual=rr.value)


def solve_mg_pcg(fc, b, tol=1e-13, max_iter=1000, nu=2, x0=None):
    bx, by, bz = (_c(a) for a in fc)
    b = _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = lib().orc_solve_mg_pcg(_n(b), _p(bx), _p(by), _p(bz), _p(b), _p(x), tol, max_iter, nu,
                                ctypes.byref(it), ctypes.byref(rr))
    return x, dict(status=st, iters=it.value, rel_residual=rr.value)


def divergence(u, dt):
    """u = (ux, uy, uz) low-face velocities -> f = div(u)/dt at the cell centres."""
    ux, uy, uz = (_c(a) for a in u)
    f = np.empty_like(ux)
    _check(lib().orc_divergence(_n(ux), _p(ux), _p(uy), _p(uz), float(dt), _p(f)), "divergence")
    return f


def project(phi, kappa, p, rho_neg, rho_pos, sigma, dt, u):
    """u - dt beta grad p with the jump-corrected gradient (returns new arrays)."""
    phi, kappa, p = _c(phi), _c(kappa), _c(p)
    ux, uy, uz = (_c(a).copy() for a in u)
    _check(lib().orc_project(_n(phi), _p(phi), _p(kappa), _p(p), float(rho_neg), float(rho_pos),
                             float(sigma), float(dt), _p(ux), _p(uy), _p(uz)), "project")
    return ux, uy, uz


def ls_advect(phi, u, dt):
    """One upwind advection step of the level set by the face velocities u = (ux, uy, uz)."""
    phi = _c(phi)
    ux, uy, uz = (_c(a) for a in u)
    out = np.empty_like(phi)
    _check(lib().orc_ls_advect(_n(phi), _p(phi), _p(ux), _p(uy), _p(uz), float(dt), _p(out)),
           "ls_advect")
    return out


def ls_reinit(phi0, phi, iters, dtau):
    """iters re-distancing steps of size dtau from phi, signs from phi0."""
    phi0, phi = _c(phi0), _c(phi)
    out = np.empty_like(phi)
    _check(lib().orc_ls_reinit(_n(phi), _p(phi0), _p(phi), int(iters), float(dtau), _p(out)),
           "ls_reinit")
    return out


def heat_faces(phi, k_neg, k_pos):
    """Conductivity on the faces: the ghost-fluid face rule with rho = 1/K of each phase
    (K_neg where phi <= 0, K_pos where phi > 0; the two in series on a crossed face)."""
    return faces(phi, 1.0 / k_neg, 1.0 / k_pos)


def heat_apply(fc, dt, x):
    """y = x - dt div(K grad x), insulated walls."""
    bx, by, bz = (_c(a) for a in fc)
    x = _c(x)
    y = np.empty_like(x)
    lib().orc_heat_apply(_n(x), _p(bx), _p(by), _p(bz), float(dt), _p(x), _p(y))
    return y


def heat_step(fc, t_old, dt, src=None, tol=1e-13, max_iter=100000, x0=None):
    """One backward-Euler diffusion step: solves (I - dt div(K grad)) T = t_old + dt src
    by conjugate gradients; returns (T, iterations, relative residual)."""
    bx, by, bz = (_c(a) for a in fc)
    rhs = _c(t_old).copy() if src is None else _c(t_old) + float(dt) * _c(src)
    x = np.zeros_like(rhs) if x0 is None else _c(x0).copy()
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    _check(lib().orc_heat_solve(_n(rhs), _p(bx), _p(by), _p(bz), float(dt), _p(rhs), _p(x),
                                float(tol), int(max_iter), ctypes.byref(it), ctypes.byref(rr)),
           "heat_solve")
    return x, it.value, rr.value


def blocks_shape(n, nb, g):
    """(blocks, padded edge) of the block layout: (n/nb)^3 blocks of (nb + 2g)^3 values."""
    return (n // nb) ** 3, nb + 2 * g


def blocks_scatter(grid, nb, g, blocks=None):
    """Grid (n, n, n) -> block layout (nblk, P, P, P); guards zero unless `blocks` given."""
    grid = _c(grid)
    n = _n(grid)
    nblk, P = blocks_shape(n, nb, g)
    out = np.zeros((nblk, P, P, P)) if blocks is None else _c(blocks).copy()
    _check(lib().orc_blocks_scatter(n, nb, g, _p(grid), _p(out)), "blocks_scatter")
    return out


def blocks_gather(blocks, n, nb, g):
    blocks = _c(blocks)
    out = np.empty((n, n, n))
    _check(lib().orc_blocks_gather(n, nb, g, _p(blocks), _p(out)), "blocks_gather")
    return out


def blocks_fill_guards(blocks, n, nb, g):
    out = _c(blocks).copy()
    _check(lib().orc_blocks_fill_guards(n, nb, g, _p(out)), "blocks_fill_guards")
    return out


def blocks_apply(fc, xblk, nb, g):
    bx, by, bz = (_c(a) for a in fc)
    n = _n(bx)
    xblk = _c(xblk)
    y = np.empty_like(xblk)
    _check(lib().orc_blocks_apply(n, nb, g, _p(bx), _p(by), _p(bz), _p(xblk), _p(y)),
           "blocks_apply")
    return y


def amr_apply(refined0, nb, phi0, phi1, x0, x1, rho_neg, rho_pos):
    """Composite operator of a two-level grid: refined0 (nbx^3 uint8) marks the level-0
    blocks covered by level 1; phi0, x0 (n0^3) and phi1, x1 ((2 n0)^3) hold the two
    levels (only leaf cells matter).  Returns (y0, y1), zero off the leaves."""
    refined0 = np.ascontiguousarray(refined0, dtype=np.uint8)
    phi0, phi1, x0, x1 = (_c(a) for a in (phi0, phi1, x0, x1))
    n0 = _n(phi0)
    y0, y1 = np.empty_like(x0), np.empty_like(x1)
    _check(lib().orc_amr_apply(n0, nb, _p(refined0), _p(phi0), _p(phi1), _p(x0), _p(x1),
                               float(rho_neg), float(rho_pos), _p(y0), _p(y1)), "amr_apply")
    return y0, y1


def amr_fill(refined0, nb, g, v0, v1):
    """Padded blocks of both levels of a composite field with their guard cells:
    ((n0/nb)^3, P, P, P) and ((2 n0/nb)^3, P, P, P)."""
    refined0 = np.ascontiguousarray(refined0, dtype=np.uint8)
    v0, v1 = _c(v0), _c(v1)
    n0 = _n(v0)
    P = nb + 2 * g
    b0 = np.empty(((n0 // nb) ** 3, P, P, P))
    b1 = np.empty(((2 * n0 // nb) ** 3, P, P, P))
    _check(lib().orc_amr_fill(n0, nb, g, _p(refined0), _p(v0), _p(v1), _p(b0), _p(b1)),
           "amr_fill")
    return b0, b1


def amr_solve(refined0, nb, phi0, phi1, b0, b1, rho_neg, rho_pos, rtol=1e-10, max_iter=100000,
              x0=None, x1=None):
    """A x = b on the leaves of the composite grid (b's weighted mean removed), Jacobi-
    preconditioned CG in the volume-weighted inner product; returns (x0, x1, iters,
    rel_residual), x of zero weighted mean and zero off the leaves."""
    refined0 = np.ascontiguousarray(refined0, dtype=np.uint8)
    phi0, phi1, b0, b1 = (_c(a) for a in (phi0, phi1, b0, b1))
    n0 = _n(phi0)
    x0 = np.zeros_like(b0) if x0 is None else _c(x0).copy()
    x1 = np.zeros_like(b1) if x1 is None else _c(x1).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    _check(lib().orc_amr_solve(n0, nb, _p(refined0), _p(phi0), _p(phi1), float(rho_neg),
                               float(rho_pos), _p(b0), _p(b1), _p(x0), _p(x1), float(rtol),
                               int(max_iter), ctypes.byref(it), ctypes.byref(rel)), "amr_solve")
    return x0, x1, it.value, rel.value


def pipeline(phi, f, rho_neg, rho_pos, sigma, kappa_override=None):
    """phi, f -> dict(faces, kappa, jterm, b, mean)."""
    phi, f = _c(phi), _c(f)
    n = _n(phi)
    bx, by, bz, kap, jt, b = (np.empty_like(phi) for _ in range(6))
    m = ctypes.c_double(0.0)
    ko = _c(kappa_override) if kappa_override is not None else None
    _check(lib().orc_pipeline(n, _p(phi), _p(f), rho_neg, rho_pos, sigma,
                              _p(ko) if ko is not None else None, _p(bx), _p(by), _p(bz),
                              _p(kap), _p(jt), _p(b), ctypes.byref(m)), "pipeline")
    return dict(faces=(bx, by, bz), kappa=kap, jterm=jt, b=b, mean=m.value)


def solve(phi, f, rho_neg, rho_pos, sigma, tol=1e-13, nu=2, kappa_override=None):
    """The full oracle: assemble and solve to tol; returns (p, pipeline dict, info)."""
    d = pipeline(phi, f, rho_neg, rho_pos, sigma, kappa_override)
    n = phi.shape[0]
    if n <= 12:
        p = solve_dense(d["faces"], d["b"])
        p -= p.mean()
        info = dict(status=OK, iters=0, rel_residual=rel_residual(d["faces"], d["b"], p))
    else:
        p, info = solve_mg_pcg(d["faces"], d["b"], tol=tol, nu=nu)
    return p, d, info


# --- reference semantics of the multigrid pieces (one call = one definition) ---------

def gs_colour(fc, b, x, colour):
    """One red (colour 0) or black (colour 1) Gauss-Seidel half-sweep, returns new x."""
    bx, by, bz = (_c(a) for a in fc)
    b = _c(b)
    x = _c(x).copy()
    lib().orc_gs_colour(_n(b), _p(bx), _p(by), _p(bz), _p(b), _p(x), colour)
    return x


def restrict(r):
    r = _c(r)
    n = _n(r)
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict(n, _p(r), _p(out))
    return out


def prolong_add(ec, xf):
    ec = _c(ec)
    xf = _c(xf).copy()
    lib().orc_prolong_add(_n(xf), _p(ec), _p(xf))
    return xf


def coarsen_faces(fc):
    bx, by, bz = (_c(a) for a in fc)
    n = _n(bx)
    out = [np.empty((n // 2,) * 3) for _ in range(3)]
    lib().orc_coarsen_faces(n, _p(bx), _p(by), _p(bz), *[_p(o) for o in out])
    return tuple(out)


class MG:
    """The oracle's V-cycle preconditioner z = V(r)."""

    def __init__(self, fc, nu=1):
        self._fc = tuple(_c(a) for a in fc)
        self.n = _n(self._fc[0])
        self._h = lib().orc_mg_create(self.n, *[_p(a) for a in self._fc], nu)
        if not self._h:
            raise OracleError("mg_create failed")

    @property
    def levels(self):
        return lib().orc_mg_levels(self._h)

    def vcycle(self, r):
        r = _c(r)
        z = np.empty_like(r)
        lib().orc_mg_vcycle(self._h, _p(r), _p(z))
        return z

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_mg_destroy(h)
            self._h = None
