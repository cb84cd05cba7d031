"""FP64 CPU oracle of the electrostatic PIC hot path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never imports,
links or executes anything here, and nothing here imports the product.

The arithmetic lives in ``pic_oracle.c`` (plain C, FP64, compiled with
``-ffp-contract=off``); this module only marshals NumPy arrays into it and
composes whole PIC steps from its pieces in the order of the paper's PIC loop
(Sec. 2, Fig. pic-loop: scatter -> solve -> gather -> push).  The network
pieces of the learned preconditioner are in ``oracle.unet`` (NumPy, FP64).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")

PRECOND_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        c_int, c_i64, c_dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.or_abi_version.restype = c_int
        L.or_num_threads.restype = c_int
        L.or_cell_keys.argtypes = [c_i64, c_int, c_dbl, _dp, _dp, _dp, _u32p]
        L.or_sort_by_key.argtypes = [c_i64, c_i64, _u32p, _i64p, _i64p]
        L.or_sort_by_key.restype = c_int
        L.or_deposit.argtypes = [c_i64, c_int, c_dbl, c_dbl, c_dbl, _dp, _dp, _dp,
                                 ctypes.c_void_p, _dp]
        L.or_deposit.restype = c_dbl
        L.or_apply_A.argtypes = [c_int, c_dbl, _dp, _dp]
        L.or_apply_A_bc.argtypes = [c_int, c_dbl, c_int, _dp, _dp]
        L.or_residual_norm.argtypes = [c_int, c_dbl, _dp, _dp]
        L.or_residual_norm.restype = c_dbl
        L.or_residual_norm_bc.argtypes = [c_int, c_dbl, c_int, _dp, _dp]
        L.or_residual_norm_bc.restype = c_dbl
        L.or_pcg.argtypes = [c_int, c_dbl, _dp, _dp, c_dbl, c_i64, _dp]
        L.or_pcg_bc.argtypes = [c_int, c_dbl, c_int, _dp, _dp, c_dbl, c_i64, _dp]
        L.or_efield.argtypes = [c_int, c_dbl, _dp, _dp, _dp, _dp]
        L.or_efield.restype = c_dbl
        L.or_efield_bc.argtypes = [c_int, c_dbl, c_int, _dp, _dp, _dp, _dp]
        L.or_efield_bc.restype = c_dbl
        L.or_gather_push.argtypes = [c_i64, c_int, c_dbl, c_dbl, c_dbl, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_void_p]
        L.or_half_kick.argtypes = [c_i64, c_int, c_dbl, c_dbl, c_dbl, _dp, _dp, _dp,
                                   _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_gather_scalar.argtypes = [c_i64, c_int, c_dbl, _dp, _dp, _dp, _dp, _dp]
        L.or_mixed_pcg.argtypes = [c_int, c_dbl, _dp, _dp, c_dbl, c_i64, c_dbl, c_i64, _dp]
        L.or_ssor_apply.argtypes = [c_int, c_dbl, c_dbl, c_int, c_int, _dp, _dp]
        L.or_ssor_apply.restype = c_int
        L.or_pcg_ssor.argtypes = [c_int, c_dbl, _dp, _dp, c_dbl, c_i64, c_dbl, c_int, c_int, _dp]
        L.or_ssor_apply_bc.argtypes = [c_int, c_dbl, c_int, c_dbl, c_int, c_int, _dp, _dp]
        L.or_ssor_apply_bc.restype = c_int
        L.or_pcg_ssor_bc.argtypes = [c_int, c_dbl, c_int, _dp, _dp, c_dbl, c_i64, c_dbl, c_int,
                                     c_int, _dp]
        L.or_mixed_pcg_ex.argtypes = [c_int, c_dbl, _dp, _dp, c_dbl, c_i64, c_dbl, c_i64,
                                      ctypes.c_int, c_i64, _dp]
        L.or_deposit_vertices.argtypes = [c_i64, c_int, c_dbl, c_dbl, _dp, _dp, _dp, c_i64, _i64p, _dp]
        L.or_fcg.argtypes = [c_int, c_dbl, _dp, _dp, c_dbl, c_i64, c_int, PRECOND_FN,
                             ctypes.c_void_p, _dp]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Pieces of the step
# --------------------------------------------------------------------------

def cell_keys(N: int, L: float, x, y, z) -> np.ndarray:
    """Cell key (iz*N+iy)*N+ix of each particle (uint32)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    key = np.empty(x.shape[0], dtype=np.uint32)
    lib().or_cell_keys(x.shape[0], N, L, x, y, z, key)
    return key


def sort_by_key(key, ncell: int):
    """Stable counting sort: (perm, cell_start) with cell_start of ncell+1."""
    key = np.ascontiguousarray(key, dtype=np.uint32)
    perm = np.empty(key.shape[0], dtype=np.int64)
    cs = np.empty(ncell + 1, dtype=np.int64)
    rc = lib().or_sort_by_key(key.shape[0], ncell, key, perm, cs)
    if rc != 0:
        raise ValueError("or_sort_by_key failed (%d)" % rc)
    return perm, cs


def deposit(N: int, L: float, q: float, rho_bg: float, x, y, z, want_rho_e=False):
    """CIC deposit + background + zero-mean projection -> (b, ||b||[, rho_e])."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    b = np.empty(N * N * N, dtype=np.float64)
    rho_e = np.empty(N * N * N, dtype=np.float64) if want_rho_e else None
    ptr = rho_e.ctypes.data_as(ctypes.c_void_p) if want_rho_e else None
    nb = lib().or_deposit(x.shape[0], N, L, q, rho_bg, x, y, z, ptr, b)
    if want_rho_e:
        return b, nb, rho_e
    return b, nb


def deposit_vertices(N: int, L: float, q: float, x, y, z, vid) -> np.ndarray:
    """rho_e at the listed vertices from the listed particles (no background)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    vid = np.ascontiguousarray(vid, dtype=np.int64)
    out = np.empty(vid.size)
    lib().or_deposit_vertices(x.shape[0], N, L, q, x, y, z, vid.size, vid, out)
    return out


# Boundary kinds of the PCG solve (Sec. 3.2): the periodic box of the PIC
# loop, and the bounded boxes (homogeneous, all six faces) of or_apply_A_bc.
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2


def grid_h(N: int, L: float, bc: int = 0) -> float:
    """Grid spacing: L/(N+1) for Dirichlet (interior vertices), else L/N."""
    return L / (N + 1) if bc == BC_DIRICHLET else L / N


def apply_A(N: int, L: float, u, bc: int = 0) -> np.ndarray:
    u = _f64(u).reshape(-1)
    out = np.empty_like(u)
    lib().or_apply_A_bc(N, L, bc, u, out)
    return out


def residual_norm(N: int, L: float, b, x, bc: int = 0) -> float:
    return lib().or_residual_norm_bc(N, L, bc, _f64(b).reshape(-1), _f64(x).reshape(-1))


def pcg(N: int, L: float, b, x0, rtol: float, max_iter: int, bc: int = 0):
    """Jacobi-PCG; returns (x, info dict)."""
    b = _f64(b).reshape(-1)
    x = _f64(x0).reshape(-1).copy()
    info = np.zeros(5)
    lib().or_pcg_bc(N, L, bc, b, x, rtol, max_iter, info)
    return x, dict(iters=int(info[0]), rel_res=info[1], true_rel_res=info[2],
                   converged=bool(info[3]), replacements=int(info[4]))


SSOR_OMEGA = math.pi / 2  # the damping factor of the paper's PCG runs (Sec. 4.1)


def ssor_apply(N, L, r, omega=SSOR_OMEGA, inner=4, outer=2, bc=0):
    """z = SSOR preconditioner applied to r (see or_ssor_apply)."""
    r = _f64(r).reshape(-1)
    z = np.empty_like(r)
    if lib().or_ssor_apply_bc(N, L, bc, omega, inner, outer, r, z) != 0:
        raise MemoryError("or_ssor_apply")
    return z


def pcg_ssor(N, L, b, x0, rtol, max_iter, omega=SSOR_OMEGA, inner=4, outer=2, bc=0):
    """PCG with the SSOR preconditioner; returns (x, info dict) as pcg()."""
    b = _f64(b).reshape(-1)
    x = _f64(x0).reshape(-1).copy()
    info = np.zeros(5)
    lib().or_pcg_ssor_bc(N, L, bc, b, x, rtol, max_iter, omega, inner, outer, info)
    return x, dict(iters=int(info[0]), rel_res=info[1], true_rel_res=info[2],
                   converged=bool(info[3]), replacements=int(info[4]))


def efield(N: int, L: float, phi, bc: int = 0):
    """Gauge-fix phi (returned copy; not for Dirichlet) and E = -grad phi;
    returns (phi, ex, ey, ez, Wx)."""
    phi = _f64(phi).reshape(-1).copy()
    ex, ey, ez = (np.empty_like(phi) for _ in range(3))
    wx = lib().or_efield_bc(N, L, bc, phi, ex, ey, ez)
    return phi, ex, ey, ez, wx


def gather_push(N, L, dt, qm, x, y, z, vx, vy, vz, ex, ey, ez, want_key=True):
    """In-place push of copies; returns (x, y, z, vx, vy, vz, key)."""
    arrs = [_f64(a).copy() for a in (x, y, z, vx, vy, vz)]
    key = np.empty(arrs[0].shape[0], dtype=np.uint32) if want_key else None
    kp = key.ctypes.data_as(ctypes.c_void_p) if want_key else None
    lib().or_gather_push(arrs[0].shape[0], N, L, dt, qm, *arrs, _f64(ex), _f64(ey), _f64(ez), kp)
    return (*arrs, key)


def half_kick(N, L, dt, qm, x, y, z, vx, vy, vz, ex, ey, ez):
    v = [_f64(a).copy() for a in (vx, vy, vz)]
    lib().or_half_kick(v[0].shape[0], N, L, dt, qm, _f64(x), _f64(y), _f64(z), *v,
                       _f64(ex), _f64(ey), _f64(ez))
    return tuple(v)


def gather_scalar(N, L, x, y, z, F) -> np.ndarray:
    x = _f64(x)
    out = np.empty(x.shape[0])
    lib().or_gather_scalar(x.shape[0], N, L, x, _f64(y), _f64(z), _f64(F).reshape(-1), out)
    return out


def mixed_pcg(N, L, b, x0, rtol, max_outer=50, inner_rtol=1e-3, max_inner=20000,
              reliable=False, max_iter=20000):
    """FP32-inner / FP64-outer refinement; `reliable` keeps the inner
    direction across refinements (reliable updates) instead of restarting.
    `refused`: refinements whose carried direction the residual-gap test
    refused; `switched`: the progress stop handed the solve to FP64 PCG,
    which took `fp64_iters` iterations (at most max_iter)."""
    b = _f64(b).reshape(-1)
    x = _f64(x0).reshape(-1).copy()
    info = np.zeros(7)
    lib().or_mixed_pcg_ex(N, L, b, x, rtol, max_outer, inner_rtol, max_inner,
                          1 if reliable else 0, max_iter, info)
    return x, dict(outer=int(info[0]), inner=int(info[1]), true_rel_res=info[2],
                   converged=bool(info[3]), refused=int(info[4]), switched=bool(info[5]),
                   fp64_iters=int(info[6]))


def fcg(N, L, b, x0, rtol, max_iter, precond, window=10):
    """Flexible PCG with a Python preconditioner ``precond(r) -> z`` (FP64)."""
    b = _f64(b).reshape(-1)
    x = _f64(x0).reshape(-1).copy()
    n3 = N * N * N

    def _cb(rp, zp, _user):
        r = np.ctypeslib.as_array(rp, shape=(n3,))
        z = np.ctypeslib.as_array(zp, shape=(n3,))
        z[:] = np.asarray(precond(r.copy()), dtype=np.float64).reshape(-1)

    cb = PRECOND_FN(_cb)
    info = np.zeros(5)
    lib().or_fcg(N, L, b, x, rtol, max_iter, window, cb, None, info)
    return x, dict(iters=int(info[0]), flex_iters=int(info[1]), true_rel_res=info[2],
                   converged=bool(info[3]), fell_back=bool(info[4]))


# --------------------------------------------------------------------------
# Whole steps, composed in the order of the PIC loop (Fig. pic-loop)
# --------------------------------------------------------------------------

class State:
    """Particles (SoA, FP64), fields and the step's diagnostics."""

    def __init__(self, N, L, q, qm, dt, x, y, z, vx, vy, vz):
        self.N, self.L, self.q, self.qm, self.dt = N, L, float(q), float(qm), float(dt)
        self.x, self.y, self.z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
        self.vx, self.vy, self.vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
        self.np = self.x.shape[0]
        self.rho_bg = -(self.q * self.np) / (L ** 3)
        n3 = N ** 3
        self.phi = np.zeros(n3)
        self.ex = self.ey = self.ez = None
        self.b = None
        self.wx = None
        self.last_solve = None

    def sort(self):
        key = cell_keys(self.N, self.L, self.x, self.y, self.z)
        perm, cs = sort_by_key(key, self.N ** 3)
        for nm in ("x", "y", "z", "vx", "vy", "vz"):
            setattr(self, nm, getattr(self, nm)[perm].copy())
        self.cell_start = cs
        return perm

    def solve(self, rtol, max_iter):
        self.b, self.nb = deposit(self.N, self.L, self.q, self.rho_bg, self.x, self.y, self.z)
        self.phi, info = pcg(self.N, self.L, self.b, self.phi, rtol, max_iter)
        self.phi, self.ex, self.ey, self.ez, self.wx = efield(self.N, self.L, self.phi)
        self.last_solve = info
        return info

    def init(self, rtol, max_iter):
        """Initial sort, t=0 deposit/solve/field, then the leapfrog half kick."""
        self.sort()
        info = self.solve(rtol, max_iter)
        self.vx, self.vy, self.vz = half_kick(self.N, self.L, self.dt, self.qm, self.x,
                                              self.y, self.z, self.vx, self.vy, self.vz,
                                              self.ex, self.ey, self.ez)
        return info

    def step(self, rtol, max_iter):
        """gather+push -> stable cell sort -> deposit -> PCG -> E."""
        (self.x, self.y, self.z, self.vx, self.vy, self.vz, key) = gather_push(
            self.N, self.L, self.dt, self.qm, self.x, self.y, self.z, self.vx, self.vy,
            self.vz, self.ex, self.ey, self.ez)
        perm, cs = sort_by_key(key, self.N ** 3)
        for nm in ("x", "y", "z", "vx", "vy", "vz"):
            setattr(self, nm, getattr(self, nm)[perm].copy())
        self.cell_start = cs
        return self.solve(rtol, max_iter)
