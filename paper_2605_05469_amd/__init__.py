"""Python binding of libpic.so -- the MI355X electrostatic PIC hot path.

Argument marshalling only: every step runs in the library's HIP kernels
(include/pic.h documents each entry point).  PyTorch provides device memory
(tensors are passed by ``data_ptr()``) and the stream.  If the library has not
been built the import of the binding's functions fails loudly; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_NOT_CONVERGED = 0, 1
PIC_ERR_INVALID, PIC_ERR_HIP, PIC_ERR_NOMEM, PIC_ERR_STATE = -1, -2, -3, -4
SOLVERS = {"pcg_fp64": 0, "pcg_mixed": 1, "fcg_learned": 2, "pcg_ssor": 3, "fft": 4, "pif": 5}
FLAG_NO_WARM_START = 1
FLAG_WARM_START_ONLY = 2
FLAG_MIXED_RELIABLE = 4
FLAG_LEARNED_MIXED = 8
FLAG_FFT_SPECTRAL = 16
FLAG_SSOR_UNFUSED = 32
FLAG_PCG_TWO_SWEEP = 64
FLAG_PCG_SINGLE_SWEEP = 128

# pic_params.bc: the box's boundary kind (the particle phases need PERIODIC)
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pic error %d: %s" % (code, msg))
        self.code = code


class pic_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ppc", ctypes.c_int32), ("np_max", ctypes.c_int64),
                ("length", ctypes.c_double), ("charge", ctypes.c_double),
                ("qm", ctypes.c_double), ("rho_bg", ctypes.c_double), ("dt", ctypes.c_double),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("solver", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("max_inner", ctypes.c_int64),
                ("max_outer", ctypes.c_int64), ("fcg_window", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("ssor_omega", ctypes.c_double),
                ("ssor_inner", ctypes.c_int32), ("ssor_outer", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("pif_tol", ctypes.c_double)]


class pic_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("outer_iterations", ctypes.c_int64),
                ("flex_iterations", ctypes.c_int64), ("rel_res", ctypes.c_double),
                ("norm_b", ctypes.c_double), ("wx", ctypes.c_double),
                ("converged", ctypes.c_int32), ("replacements", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("warm_start_used", ctypes.c_int32),
                ("gap_restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fp64_iterations", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pic_particle_arrays(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "y", "z", "vx", "vy", "vz")]


class pic_particles(ctypes.Structure):
    _fields_ = [("cur", pic_particle_arrays), ("alt", pic_particle_arrays),
                ("np", ctypes.c_int64), ("key", ctypes.c_void_p),
                ("cell_start", ctypes.c_void_p)]


class pic_fields(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("rho", "phi", "ex", "ey", "ez")]


class pic_step_info(ctypes.Structure):
    _fields_ = [("solve", pic_solve_info), ("ms_push", ctypes.c_double),
                ("ms_sort", ctypes.c_double), ("ms_deposit", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("ms_field", ctypes.c_double)]

    def as_dict(self):
        d = self.solve.as_dict()
        for f in ("ms_push", "ms_sort", "ms_deposit", "ms_solve", "ms_field"):
            d[f] = getattr(self, f)
        return d


_lib = None

# every entry point declared in include/pic.h
EXPORTS = ["pic_create", "pic_destroy", "pic_workspace_bytes", "pic_last_error",
           "pic_set_solver", "pic_set_flags", "pic_abi_version", "pic_cell_keys", "pic_sort_cells",
           "pic_deposit_cic", "pic_poisson_pcg", "pic_gather_push", "pic_half_kick",
           "pic_efield", "pic_init", "pic_step", "pic_set_kernel_timing", "pic_kernel_time",
           "pic_unet_param_count", "pic_set_unet", "pic_unet_precondition", "pic_net_create",
           "pic_net_destroy", "pic_net_set_params", "pic_net_get_params", "pic_net_forward",
           "pic_net_backward", "pic_net_train_step", "pic_net_precondition",
           "pic_conv3d_frag_elems", "pic_conv3d_pack", "pic_conv3d_fwd", "pic_conv3d_bwd_data",
           "pic_conv3d_wgrad_scratch_elems", "pic_conv3d_bwd_weight", "pic_adam_step",
           "pic_pif_field", "pic_deposit_cic_noalloc", "pic_stream_triad", "pic_net_loss",
           "pic_net_make_pair"]


def lib():
    """Load libpic.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library must share)

    if not os.path.exists(LIB_PATH):
        raise ImportError("libpic.so is not built (run paper_2605_05469_amd/build.py); "
                          "there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.pic_create.argtypes = [ctypes.POINTER(pic_params), ctypes.POINTER(vp)]
    L.pic_destroy.argtypes = [vp]
    L.pic_workspace_bytes.argtypes = [ctypes.POINTER(pic_params)]
    L.pic_workspace_bytes.restype = ctypes.c_size_t
    L.pic_last_error.restype = ctypes.c_char_p
    L.pic_set_solver.argtypes = [vp, i32]
    L.pic_set_flags.argtypes = [vp, i32]
    L.pic_cell_keys.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.pic_sort_cells.argtypes = [vp, i64, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, vp]
    L.pic_deposit_cic.argtypes = [vp, i64, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.pic_deposit_cic_noalloc.argtypes = [ctypes.POINTER(pic_params), i64, vp, vp, vp, vp, vp,
                                          ctypes.POINTER(dbl), vp]
    L.pic_poisson_pcg.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(pic_solve_info), vp]
    L.pic_gather_push.argtypes = [vp, i64] + [vp] * 10 + [vp]
    L.pic_half_kick.argtypes = [vp, i64] + [vp] * 9 + [vp]
    L.pic_efield.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.pic_pif_field.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.pic_init.argtypes = [vp, ctypes.POINTER(pic_particles), ctypes.POINTER(pic_fields),
                           ctypes.POINTER(pic_step_info), vp]
    L.pic_step.argtypes = L.pic_init.argtypes
    L.pic_set_kernel_timing.argtypes = [vp, i32]
    L.pic_kernel_time.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.pic_stream_triad.argtypes = [i64, vp, vp, vp, dbl, i32, ctypes.POINTER(dbl), vp]
    L.pic_unet_param_count.restype = i64
    L.pic_set_unet.argtypes = [vp, vp, vp]
    L.pic_unet_precondition.argtypes = [vp, vp, vp, vp]
    L.pic_net_create.argtypes = [i32, i32, ctypes.POINTER(vp)]
    L.pic_net_destroy.argtypes = [vp]
    L.pic_net_set_params.argtypes = [vp, vp, vp]
    L.pic_net_get_params.argtypes = [vp, vp, vp]
    L.pic_net_forward.argtypes = [vp, vp, vp, vp]
    L.pic_net_backward.argtypes = [vp, vp, vp, vp]
    L.pic_net_train_step.argtypes = [vp, vp, vp, dbl, dbl, ctypes.POINTER(dbl), vp]
    L.pic_net_precondition.argtypes = [vp, vp, dbl, vp, vp]
    L.pic_net_loss.argtypes = [vp, vp, vp, dbl, ctypes.POINTER(dbl), vp]
    L.pic_net_make_pair.argtypes = [vp, vp, vp, vp, vp, dbl, vp, vp, ctypes.POINTER(dbl), vp]
    L.pic_conv3d_frag_elems.argtypes = [i32, i32]
    L.pic_conv3d_frag_elems.restype = ctypes.c_size_t
    L.pic_conv3d_pack.argtypes = [i32, i32, vp, vp, vp, vp]
    L.pic_conv3d_fwd.argtypes = [i32, i32, i32, vp, vp, vp, vp, i32, vp, vp]
    L.pic_conv3d_bwd_data.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp]
    L.pic_conv3d_wgrad_scratch_elems.argtypes = [i32, i32, i32]
    L.pic_conv3d_wgrad_scratch_elems.restype = ctypes.c_size_t
    L.pic_conv3d_bwd_weight.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp]
    L.pic_adam_step.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, i32, vp]
    _lib = L
    return L


def _check(rc, allow_not_converged=True):
    if rc < 0 or (rc == PIC_NOT_CONVERGED and not allow_not_converged):
        raise PicError(rc, lib().pic_last_error().decode())
    return rc


def _ptr(t, dtype=None, name="array"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def landau_params(N, ppc, k=0.5, dt=0.05, qm=-1.0, rtol=1e-10, max_iter=20000,
                  solver="pcg_fp64", np_max=None, check_every=16, inner_rtol=1e-3,
                  max_inner=20000, max_outer=50, fcg_window=10, ssor_omega=math.pi / 2,
                  ssor_inner=4, ssor_outer=2, flags=0, bc=BC_PERIODIC, pif_tol=0.0):
    """Parameters of the Landau-damping box (Sec. 2.1): L = 2 pi / k, unit
    mean density, q = -L^3/Np, background +1."""
    L = 2.0 * math.pi / k
    npart = ppc * N ** 3
    q = -(L ** 3) / npart
    p = pic_params()
    p.n, p.ppc = N, ppc
    p.np_max = npart if np_max is None else np_max
    p.length, p.charge, p.qm = L, q, qm
    p.rho_bg = -(q * npart) / L ** 3
    p.dt, p.rtol, p.max_iter = dt, rtol, max_iter
    p.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    p.check_every = check_every
    p.inner_rtol, p.max_inner, p.max_outer = inner_rtol, max_inner, max_outer
    p.fcg_window = fcg_window
    p.ssor_omega, p.ssor_inner, p.ssor_outer = ssor_omega, ssor_inner, ssor_outer
    p.flags = flags
    p.bc = bc
    p.pif_tol = pif_tol
    return p


class Context:
    """Owns a pic_ctx (scratch on the current device)."""

    def __init__(self, params: pic_params):
        self.params = params
        self._h = ctypes.c_void_p()
        _check(lib().pic_create(ctypes.byref(params), ctypes.byref(self._h)))
        self.N = params.n

    def close(self):
        if self._h:
            lib().pic_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ pieces --
    def set_solver(self, solver):
        s = SOLVERS[solver] if isinstance(solver, str) else int(solver)
        _check(lib().pic_set_solver(self._h, s))

    def set_flags(self, flags: int):
        """FLAG_NO_WARM_START | FLAG_WARM_START_ONLY (learned form),
        FLAG_MIXED_RELIABLE (mixed form), FLAG_LEARNED_MIXED (learned form),
        FLAG_FFT_SPECTRAL (FFT form), FLAG_SSOR_UNFUSED (SSOR form),
        FLAG_PCG_TWO_SWEEP (FP64 Jacobi-PCG as two sweeps per iteration)."""
        _check(lib().pic_set_flags(self._h, int(flags)))

    def cell_keys(self, x, y, z, key, stream=None):
        import torch
        _check(lib().pic_cell_keys(self._h, x.numel(), _ptr(x, torch.float64), _ptr(y, torch.float64),
                                   _ptr(z, torch.float64), _ptr(key, torch.int32 if key.dtype == torch.int32 else torch.uint32),
                                   _stream(stream)))

    def sort_cells(self, key, src, dst, cell_start, perm=None, stream=None):
        sp = (ctypes.c_void_p * 6)(*[_ptr(a) for a in src])
        dp = (ctypes.c_void_p * 6)(*[_ptr(a) for a in dst])
        _check(lib().pic_sort_cells(self._h, src[0].numel(), _ptr(key), sp, dp, _ptr(cell_start),
                                    _ptr(perm), _stream(stream)))

    def deposit(self, x, y, z, cell_start, rho, stream=None, want_norm=False):
        nb = ctypes.c_double(0.0)
        _check(lib().pic_deposit_cic(self._h, 0 if x is None else x.numel(), _ptr(x), _ptr(y),
                                     _ptr(z), _ptr(cell_start), _ptr(rho),
                                     ctypes.byref(nb) if want_norm else None, _stream(stream)))
        return nb.value if want_norm else None

    def poisson(self, rho, phi, ex=None, ey=None, ez=None, stream=None):
        info = pic_solve_info()
        rc = _check(lib().pic_poisson_pcg(self._h, _ptr(rho), _ptr(phi), _ptr(ex), _ptr(ey),
                                          _ptr(ez), ctypes.byref(info), _stream(stream)))
        d = info.as_dict()
        d["status"] = rc
        return d

    def efield(self, phi, ex, ey, ez, stream=None):
        wx = ctypes.c_double(0.0)
        _check(lib().pic_efield(self._h, _ptr(phi), _ptr(ex), _ptr(ey), _ptr(ez),
                                ctypes.byref(wx), _stream(stream)))
        return wx.value

    def pif_field(self, x, y, z, cell_start, ex, ey, ez, stream=None):
        """PIF field at cell-sorted particles (solver "pif"); returns W_x."""
        wx = ctypes.c_double(0.0)
        _check(lib().pic_pif_field(self._h, 0 if x is None else x.numel(), _ptr(x), _ptr(y),
                                   _ptr(z), _ptr(cell_start), _ptr(ex), _ptr(ey), _ptr(ez),
                                   ctypes.byref(wx), _stream(stream)))
        return wx.value

    def gather_push(self, x, y, z, vx, vy, vz, ex, ey, ez, key=None, stream=None):
        _check(lib().pic_gather_push(self._h, x.numel(), *[_ptr(a) for a in (x, y, z, vx, vy, vz,
                                                                              ex, ey, ez)],
                                     _ptr(key), _stream(stream)))

    def half_kick(self, x, y, z, vx, vy, vz, ex, ey, ez, stream=None):
        _check(lib().pic_half_kick(self._h, x.numel(), *[_ptr(a) for a in (x, y, z, vx, vy, vz,
                                                                            ex, ey, ez)],
                                   _stream(stream)))

    def set_unet(self, params, stream=None):
        """Load the network's FP32 parameters (device tensor, canonical order)."""
        import torch
        _check(lib().pic_set_unet(self._h, _ptr(params, torch.float32, "params"), _stream(stream)))

    def precondition(self, r, z, stream=None):
        _check(lib().pic_unet_precondition(self._h, _ptr(r), _ptr(z), _stream(stream)))

    def set_kernel_timing(self, on=True):
        _check(lib().pic_set_kernel_timing(self._h, 1 if on else 0))

    def kernel_time(self, kid):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        _check(lib().pic_kernel_time(self._h, kid, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


class Simulation:
    """Device-resident PIC state driven through pic_init / pic_step."""

    def __init__(self, ctx: Context, x, y, z, vx, vy, vz):
        import torch
        self.ctx = ctx
        N = ctx.N
        dev = x.device
        n = x.numel()
        self._cur = [x, y, z, vx, vy, vz]
        self._alt = [torch.empty_like(a) for a in self._cur]
        self.key = torch.empty(n, dtype=torch.int32, device=dev)
        self.cell_start = torch.empty(N ** 3 + 1, dtype=torch.int32, device=dev)
        self.rho = torch.zeros(N ** 3, dtype=torch.float64, device=dev)
        self.phi = torch.zeros(N ** 3, dtype=torch.float64, device=dev)
        self.ex = torch.zeros(N ** 3, dtype=torch.float64, device=dev)
        self.ey = torch.zeros_like(self.ex)
        self.ez = torch.zeros_like(self.ex)
        self._P = pic_particles()
        self._P.np = n
        self._set(self._P.cur, self._cur)
        self._set(self._P.alt, self._alt)
        self._P.key = self.key.data_ptr()
        self._P.cell_start = self.cell_start.data_ptr()
        self._F = pic_fields(self.rho.data_ptr(), self.phi.data_ptr(), self.ex.data_ptr(),
                             self.ey.data_ptr(), self.ez.data_ptr())

    @staticmethod
    def _set(arr, ts):
        for nm, t in zip(("x", "y", "z", "vx", "vy", "vz"), ts):
            setattr(arr, nm, t.data_ptr())

    def _sync_views(self):
        # the library swaps cur/alt after the sort; follow it
        if self._P.cur.x != self._cur[0].data_ptr():
            self._cur, self._alt = self._alt, self._cur

    @property
    def particles(self):
        return self._cur

    def init(self, stream=None):
        info = pic_step_info()
        rc = _check(lib().pic_init(self.ctx._h, ctypes.byref(self._P), ctypes.byref(self._F),
                                   ctypes.byref(info), _stream(stream)))
        self._sync_views()
        d = info.as_dict()
        d["status"] = rc
        return d

    def step(self, stream=None, timed=True):
        info = pic_step_info()
        rc = _check(lib().pic_step(self.ctx._h, ctypes.byref(self._P), ctypes.byref(self._F),
                                   ctypes.byref(info) if timed else None, _stream(stream)))
        self._sync_views()
        d = info.as_dict()
        d["status"] = rc
        return d


def stream_triad(b, c, a, scalar=3.0, reps=10, stream=None):
    """pic_stream_triad: a = b + scalar c; returns the average ms per launch."""
    ms = ctypes.c_double(0.0)
    _check(lib().pic_stream_triad(a.numel(), _ptr(b), _ptr(c), _ptr(a), scalar, reps,
                                  ctypes.byref(ms), _stream(stream)))
    return ms.value


NOALLOC_MAX_N = 64  # PIC_NOALLOC_MAX_N


def deposit_cic_noalloc(params, x, y, z, cell_start, rho, want_norm=False, stream=None):
    """pic_deposit_cic_noalloc: the deposit without a context (static scratch,
    n <= NOALLOC_MAX_N); returns ||rho|| when want_norm."""
    nb = ctypes.c_double(0.0)
    _check(lib().pic_deposit_cic_noalloc(ctypes.byref(params), 0 if x is None else x.numel(),
                                         _ptr(x), _ptr(y), _ptr(z), _ptr(cell_start), _ptr(rho),
                                         ctypes.byref(nb) if want_norm else None,
                                         _stream(stream)))
    return nb.value if want_norm else None


def unet_param_count() -> int:
    return int(lib().pic_unet_param_count())


class Net:
    """A standalone network on an n^3 grid (training adds gradient buffers)."""

    def __init__(self, n: int, training: bool = False):
        self._h = ctypes.c_void_p()
        _check(lib().pic_net_create(n, 1 if training else 0, ctypes.byref(self._h)))
        self.n = n

    def close(self):
        if self._h:
            lib().pic_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        import torch
        _check(lib().pic_net_set_params(self._h, _ptr(params, torch.float32, "params"), _stream(stream)))

    def get_params(self, out, stream=None):
        import torch
        _check(lib().pic_net_get_params(self._h, _ptr(out, torch.float32, "params"), _stream(stream)))
        return out

    def forward(self, x, out, stream=None):
        _check(lib().pic_net_forward(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def backward(self, dout, grads, stream=None):
        _check(lib().pic_net_backward(self._h, _ptr(dout), _ptr(grads), _stream(stream)))
        return grads

    def train_step(self, rhs, target, lam=1.0, lr=1e-3, want_loss=True, stream=None):
        loss = ctypes.c_double(0.0)
        _check(lib().pic_net_train_step(self._h, _ptr(rhs), _ptr(target), lam, lr,
                                        ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def precondition(self, r, h, z, stream=None):
        _check(lib().pic_net_precondition(self._h, _ptr(r), h, _ptr(z), _stream(stream)))
        return z

    def loss(self, rhs, target, lam=1.0, stream=None):
        """The training loss at one pair, no update (pic_net_loss)."""
        L = ctypes.c_double(0.0)
        _check(lib().pic_net_loss(self._h, _ptr(rhs), _ptr(target), lam, ctypes.byref(L),
                                  _stream(stream)))
        return L.value

    def make_pair(self, rho, phi, h, rhs, target, rho_prev=None, phi_prev=None, stream=None):
        """Scale-free training pair (pic_net_make_pair); returns the scale s."""
        sc = ctypes.c_double(0.0)
        _check(lib().pic_net_make_pair(self._h, _ptr(rho), _ptr(phi), _ptr(rho_prev),
                                       _ptr(phi_prev), h, _ptr(rhs), _ptr(target),
                                       ctypes.byref(sc), _stream(stream)))
        return sc.value


def conv3d_frag_elems(ci, co):
    return int(lib().pic_conv3d_frag_elems(ci, co))


def conv3d_pack(ci, co, w, frag_fwd=None, frag_bwd=None, stream=None):
    _check(lib().pic_conv3d_pack(ci, co, _ptr(w), _ptr(frag_fwd), _ptr(frag_bwd), _stream(stream)))


def conv3d_fwd(n, ci, co, x, frag_fwd, bias, y, skip=None, relu=True, stream=None):
    _check(lib().pic_conv3d_fwd(n, ci, co, _ptr(x), _ptr(frag_fwd), _ptr(bias), _ptr(skip),
                                1 if relu else 0, _ptr(y), _stream(stream)))


def conv3d_bwd_data(n, ci, co, gy, frag_bwd, gx, accumulate=False, stream=None):
    _check(lib().pic_conv3d_bwd_data(n, ci, co, _ptr(gy), _ptr(frag_bwd), _ptr(gx),
                                     1 if accumulate else 0, _stream(stream)))


def conv3d_wgrad_scratch_elems(n, ci, co):
    return int(lib().pic_conv3d_wgrad_scratch_elems(n, ci, co))


def conv3d_bwd_weight(n, ci, co, x, gy, scratch, grad, stream=None):
    _check(lib().pic_conv3d_bwd_weight(n, ci, co, _ptr(x), _ptr(gy), _ptr(scratch), _ptr(grad),
                                       _stream(stream)))


def adam_step(theta, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().pic_adam_step(theta.numel(), _ptr(theta), _ptr(m), _ptr(v), _ptr(g), lr, beta1,
                               beta2, eps, step, _stream(stream)))
