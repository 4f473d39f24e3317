"""Python binding of ``libib.so`` (include/ib.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module
checks tensor shapes, dtypes and devices, passes raw device pointers and
turns error codes into exceptions.  There is no fallback: if the library is
not built, importing this module raises.

Tensors: markers (3, M) float64 on the GPU; grid fields (3, Nz, N, N) in the
fluid precision (float32 for ``precision="fp32"``, float64 for ``"fp64"``),
indexed [component, z, y, x] (Nz = N for the cube, N / 2 for the half-cube).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libib.so")

IB_OK, IB_EINVAL, IB_ENOMEM, IB_EDEVICE, IB_ENOTSUP, IB_ENONFINITE = 0, -1, -2, -3, -4, -5
IB_FLUID_FP64, IB_FLUID_FP32 = 0, 1
_CODES = {IB_EINVAL: "IB_EINVAL", IB_ENOMEM: "IB_ENOMEM", IB_EDEVICE: "IB_EDEVICE",
          IB_ENOTSUP: "IB_ENOTSUP", IB_ENONFINITE: "IB_ENONFINITE"}


class IBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class ib_params(C.Structure):
    _fields_ = [("n", C.c_int32), ("L", C.c_double), ("rho", C.c_double), ("mu", C.c_double),
                ("dt", C.c_double), ("fluid_precision", C.c_int32), ("convect", C.c_int32),
                ("n_markers", C.c_int64), ("stream", C.c_void_p), ("nz", C.c_int32),
                ("displacement", C.c_int32)]


class ib_lattice(C.Structure):
    _fields_ = [("first", C.c_int64), ("n1", C.c_int32), ("n2", C.c_int32), ("periodic2", C.c_int32),
                ("Ks", C.c_double), ("Kb", C.c_double)]


class ib_elastic(C.Structure):
    _fields_ = [("w", C.c_void_p), ("k", C.c_void_p), ("X_ref", C.c_void_p), ("kappa", C.c_void_p),
                ("n_lattices", C.c_int32), ("lattices", C.POINTER(ib_lattice)),
                ("n_springs", C.c_int64), ("spring_ab", C.c_void_p), ("spring_rest", C.c_void_p),
                ("K_spring", C.c_double),
                ("n_drive", C.c_int64), ("drive_idx", C.c_void_p), ("drive_dir", C.c_void_p),
                ("drive_A", C.c_double), ("drive_freq", C.c_double)]


EXPORTS = ["ib_create", "ib_destroy", "ib_set_material", "ib_set_stream", "ib_step", "ib_force",
           "ib_spread", "ib_interp", "ib_fluid", "ib_bin", "ib_adjoint_step", "ib_adjoint_step_u", "ib_probe", "ib_last_error",
           "ib_workspace_bytes", "ib_timers_enable", "ib_timers_select", "ib_timers_read", "ib_timer_name",
           "ib_graph_enable", "ib_graph_stats", "ib_fluid_noalloc", "ib_bin_reuse"]
IB_N_TIMERS = 32

_lib = None


def load_library():
    """Load libib.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_math_0301321_amd.build` "
                          "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.c_double
    lib.ib_create.argtypes = [C.POINTER(ib_params), C.POINTER(ib_elastic), C.POINTER(vp)]
    lib.ib_destroy.argtypes = [vp]
    lib.ib_destroy.restype = None
    lib.ib_set_material.argtypes = [vp, vp, vp, vp, vp]
    lib.ib_set_stream.argtypes = [vp, vp]
    lib.ib_step.argtypes = [vp, vp, vp, dp, vp]
    lib.ib_force.argtypes = [vp, vp, dp, vp]
    lib.ib_spread.argtypes = [vp, vp, vp, vp]
    lib.ib_interp.argtypes = [vp, vp, vp, vp]
    lib.ib_fluid.argtypes = [vp, vp, vp]
    lib.ib_bin.argtypes = [vp, vp, vp, vp]
    lib.ib_adjoint_step.argtypes = [vp, vp, vp, dp, vp, vp, vp]
    lib.ib_adjoint_step_u.argtypes = [vp, vp, vp, vp, dp, vp, vp, vp]
    lib.ib_probe.argtypes = [vp, vp, vp, vp, vp, C.c_int64, vp, vp]
    lib.ib_last_error.argtypes = [vp]
    lib.ib_last_error.restype = C.c_char_p
    lib.ib_workspace_bytes.argtypes = [vp]
    lib.ib_workspace_bytes.restype = C.c_int64
    lib.ib_timers_enable.argtypes = [vp, C.c_int]
    lib.ib_timers_select.argtypes = [vp, C.c_uint32]
    lib.ib_timers_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    lib.ib_fluid_noalloc.argtypes = [C.POINTER(ib_params), vp, vp]
    lib.ib_graph_enable.argtypes = [vp, C.c_int]
    lib.ib_bin_reuse.argtypes = [vp, C.c_int]
    lib.ib_graph_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.ib_timer_name.argtypes = [C.c_int]
    lib.ib_timer_name.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("ib_destroy", "ib_last_error", "ib_workspace_bytes", "ib_timer_name"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def fluid_noalloc(u, F=None, *, L=1.0, rho=1.0, mu=0.01, dt=1e-3, convect=1, stream=None):
    """ib_fluid_noalloc: u^n -> u^{n+1} in place without a context (no device
    allocation; the library's static scratch).  u, F: contiguous cuda tensors of
    shape (3, nz, n, n), float32 or float64 (the fluid precision)."""
    lib = load_library()
    if u.device.type != "cuda" or u.dtype not in (torch.float32, torch.float64) or not u.is_contiguous() \
            or u.dim() != 4 or u.shape[0] != 3 or u.shape[2] != u.shape[3]:
        raise ValueError("u must be a contiguous cuda float32/float64 tensor of shape (3, nz, n, n)")
    if F is not None and (F.device != u.device or F.dtype != u.dtype or not F.is_contiguous()
                          or F.shape != u.shape):
        raise ValueError("F must be a contiguous tensor like u")
    n, nz = int(u.shape[3]), int(u.shape[1])
    if stream is None:
        stream = torch.cuda.current_stream(u.device).cuda_stream
    p = ib_params(n, float(L), float(rho), float(mu), float(dt),
                  IB_FLUID_FP32 if u.dtype == torch.float32 else IB_FLUID_FP64, int(convect), 0,
                  C.c_void_p(stream), nz, 0)
    rc = lib.ib_fluid_noalloc(C.byref(p), _ptr(u), _ptr(F))
    if rc != IB_OK:
        raise IBError(rc, lib.ib_last_error(None).decode())


class Context:
    """An ``ib_ctx`` for one workload on the current GPU.

    ``wl`` is a :class:`paper_math_0301321_amd.workloads.Workload`.  The
    material arrays are copied to the GPU once and read by every call;
    ``set_stiffness`` swaps the stiffness array (used by the adjoint).  With
    ``displacement=True`` every marker-state tensor holds D = X - X_ref.
    """

    def __init__(self, wl, precision: str = "fp32", N: int | None = None, convect: int | None = None,
                 device: str | torch.device = "cuda", stream=None, displacement: bool = False):
        self.lib = load_library()
        self.wl = wl
        self.N = int(wl.N if N is None else N)
        self.Nz = int(wl.nz) * self.N // int(wl.N)     # z nodes: N (cube) or N / 2 (half-cube)
        self.M = int(wl.M)
        self.precision = precision
        if precision not in ("fp32", "fp64"):
            raise ValueError("precision must be 'fp32' or 'fp64'")
        self.fluid_dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device(device)
        self.convect = int(wl.convect if convect is None else convect)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.w = torch.as_tensor(np.asarray(wl.w), **f64).contiguous()
        self.k = torch.as_tensor(np.asarray(wl.k), **f64).contiguous()
        self.X_ref = torch.as_tensor(np.asarray(wl.X_ref), **f64).contiguous()
        self.kappa = torch.as_tensor(np.asarray(wl.kappa), **f64).contiguous()
        lats = wl.lattices
        lat_arr = (ib_lattice * max(1, len(lats)))()
        for i, l in enumerate(lats):
            lat_arr[i] = ib_lattice(l.first, l.n1, l.n2, int(l.periodic2), l.Ks, l.Kb)
        sab = np.ascontiguousarray(wl.spring_ab if wl.spring_ab is not None else np.zeros((2, 0)), dtype=np.int32)
        srest = np.ascontiguousarray(wl.spring_rest if wl.spring_rest is not None else np.zeros(0), dtype=np.float64)
        didx = np.ascontiguousarray(wl.drive_idx if wl.drive_idx is not None else np.zeros(0), dtype=np.int32)
        ddir = np.ascontiguousarray(wl.drive_dir if wl.drive_dir is not None else np.zeros((3, 0)), dtype=np.float64)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self.stream = stream
        self.displacement = bool(displacement)
        p = ib_params(self.N, float(wl.L), float(wl.rho), float(wl.mu), float(wl.dt),
                      IB_FLUID_FP32 if precision == "fp32" else IB_FLUID_FP64, self.convect, self.M,
                      C.c_void_p(stream), self.Nz, int(self.displacement))
        e = ib_elastic(_ptr(self.w), _ptr(self.k), _ptr(self.X_ref), _ptr(self.kappa),
                       len(lats), lat_arr,
                       sab.shape[1] if sab.ndim == 2 else 0, sab.ctypes.data_as(C.c_void_p),
                       srest.ctypes.data_as(C.c_void_p), float(wl.K_spring),
                       didx.shape[0], didx.ctypes.data_as(C.c_void_p), ddir.ctypes.data_as(C.c_void_p),
                       float(wl.drive_A), float(wl.drive_freq))
        h = C.c_void_p()
        rc = self.lib.ib_create(C.byref(p), C.byref(e), C.byref(h))
        if rc != IB_OK:
            raise IBError(rc, self.lib.ib_last_error(None).decode())
        self._h = h

    # ---------------------------------------------------------------- utils
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ib_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != IB_OK:
            raise IBError(rc, self.lib.ib_last_error(self._h).decode())

    def _markers(self, t, name):
        if (t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous()
                or tuple(t.shape) != (3, self.M)):
            raise ValueError(f"{name} must be a contiguous cuda float64 tensor of shape (3, {self.M})")
        return _ptr(t)

    @property
    def grid_shape(self) -> tuple:
        """Shape of a grid field: (3, Nz, N, N), [component, z, y, x]."""
        return (3, self.Nz, self.N, self.N)

    def _grid(self, t, name):
        if (t.device.type != "cuda" or t.dtype != self.fluid_dtype or not t.is_contiguous()
                or tuple(t.shape) != self.grid_shape):
            raise ValueError(f"{name} must be a contiguous cuda {self.fluid_dtype} tensor of shape {self.grid_shape}")
        return _ptr(t)

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.ib_workspace_bytes(self._h))

    def new_grid(self):
        return torch.zeros(self.grid_shape, dtype=self.fluid_dtype, device=self.device)

    def set_stiffness(self, k: torch.Tensor):
        if k.device.type != "cuda" or k.dtype != torch.float64 or not k.is_contiguous() or k.numel() != self.M:
            raise ValueError("k must be a contiguous cuda float64 tensor with M entries")
        self.k = k
        self._check(self.lib.ib_set_material(self._h, None, _ptr(k), None, None))

    def timers_enable(self, on: bool = True):
        """Start (and reset) or stop the per-phase HIP-event timers."""
        self._check(self.lib.ib_timers_enable(self._h, 1 if on else 0))

    def timers_select(self, phases=None):
        """Time only the named phases (None: all)."""
        if phases is None:
            mask = 0xFFFFFFFF
        else:
            names = [self.lib.ib_timer_name(i) for i in range(IB_N_TIMERS)]
            names = [n.decode() if n else None for n in names]
            mask = 0
            for p in phases:
                if p not in names:
                    raise ValueError(f"unknown phase {p!r}")
                mask |= 1 << names.index(p)
        self._check(self.lib.ib_timers_select(self._h, mask))

    def timers_read(self) -> dict:
        """{phase: (total_ms, launches)} since the timers were enabled (synchronises the stream)."""
        ms = (C.c_double * IB_N_TIMERS)()
        calls = (C.c_int64 * IB_N_TIMERS)()
        self._check(self.lib.ib_timers_read(self._h, ms, calls, IB_N_TIMERS))
        out = {}
        for i in range(IB_N_TIMERS):
            name = self.lib.ib_timer_name(i)
            if name is None:
                break
            if calls[i]:
                out[name.decode()] = (ms[i], int(calls[i]))
        return out

    def graph_enable(self, on: bool = True):
        """Replay the step as a HIP graph (captured per (X, u, F_out) pointers)."""
        self._check(self.lib.ib_graph_enable(self._h, 1 if on else 0))

    def bin_reuse(self, on: bool = True):
        """Keep the last marker partition when no marker changed cell (default on);
        off rebuilds it at every binning.  Results are bitwise the same."""
        self._check(self.lib.ib_bin_reuse(self._h, 1 if on else 0))

    def graph_stats(self) -> tuple:
        """(graphs captured, graph launches) on this context."""
        cap, lau = C.c_int64(), C.c_int64()
        self._check(self.lib.ib_graph_stats(self._h, C.byref(cap), C.byref(lau)))
        return int(cap.value), int(lau.value)

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.ib_set_stream(self._h, C.c_void_p(stream)))

    # ------------------------------------------------------- entry points
    def step(self, X, u, t: float, F_out=None):
        """One time step in place: X^n -> X^{n+1}, u^n -> u^{n+1}."""
        self._check(self.lib.ib_step(self._h, self._markers(X, "X"), self._grid(u, "u"), float(t),
                                     None if F_out is None else self._markers(F_out, "F_out")))

    def force(self, X, t: float, F_out=None):
        F = torch.empty_like(X) if F_out is None else F_out
        self._check(self.lib.ib_force(self._h, self._markers(X, "X"), float(t), self._markers(F, "F")))
        return F

    def spread(self, X, F_lag, F_grid=None):
        Fg = self.new_grid() if F_grid is None else F_grid
        self._check(self.lib.ib_spread(self._h, self._markers(X, "X"), self._markers(F_lag, "F_lag"),
                                       self._grid(Fg, "F_grid")))
        return Fg

    def interp(self, X, u, U_out=None):
        U = torch.empty_like(X) if U_out is None else U_out
        self._check(self.lib.ib_interp(self._h, self._markers(X, "X"), self._grid(u, "u"), self._markers(U, "U")))
        return U

    def fluid(self, u, F_grid=None):
        """NS update in place: u^n -> u^{n+1} given the grid force density."""
        self._check(self.lib.ib_fluid(self._h, self._grid(u, "u"),
                                      None if F_grid is None else self._grid(F_grid, "F_grid")))

    def bin(self, X):
        keys = torch.empty(self.M, dtype=torch.int32, device=X.device)
        perm = torch.empty(self.M, dtype=torch.int32, device=X.device)
        self._check(self.lib.ib_bin(self._h, self._markers(X, "X"), _ptr(keys), _ptr(perm)))
        return keys, perm

    def probe(self, X, X0, idx, dirs, disp=None, env=None):
        """disp[i] = (X[:, idx[i]] - X0[:, idx[i]]) . dirs[:, i] (returned; written into
        `disp` when given) and env[i] = max(env[i], |disp[i]|) when `env` is given."""
        n = int(idx.numel())
        if idx.device.type != "cuda" or idx.dtype != torch.int32 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous cuda int32 tensor")
        if (dirs.device.type != "cuda" or dirs.dtype != torch.float64 or not dirs.is_contiguous()
                or tuple(dirs.shape) != (3, n)):
            raise ValueError(f"dirs must be a contiguous cuda float64 tensor of shape (3, {n})")
        d = torch.empty(n, dtype=torch.float64, device=idx.device) if disp is None else disp
        for t_, nm in ((d, "disp"), (env, "env")):
            if t_ is not None and (t_.device.type != "cuda" or t_.dtype != torch.float64
                                   or not t_.is_contiguous() or t_.numel() != n):
                raise ValueError(f"{nm} must be a contiguous cuda float64 tensor with {n} entries")
        self._check(self.lib.ib_probe(self._h, self._markers(X, "X"), self._markers(X0, "X0"), _ptr(idx),
                                      _ptr(dirs), n, _ptr(d), None if env is None else _ptr(env)))
        return d

    def adjoint_step(self, X_n, u_np1, t: float, Xbar, ubar, kbar, u_n=None):
        """Adjoint of one step: Xbar, ubar (n+1 -> n) in place, kbar accumulated.  With
        convect = 1, u_n (the velocity the step started from) is required."""
        if (kbar.device.type != "cuda" or kbar.dtype != torch.float64 or not kbar.is_contiguous()
                or kbar.numel() != self.M):
            raise ValueError("kbar must be a contiguous cuda float64 tensor with M entries")
        un = None if u_n is None else self._grid(u_n, "u_n")
        self._check(self.lib.ib_adjoint_step_u(self._h, self._markers(X_n, "X_n"), un,
                                               self._grid(u_np1, "u_np1"), float(t), self._markers(Xbar, "Xbar"),
                                               self._grid(ubar, "ubar"), _ptr(kbar)))
