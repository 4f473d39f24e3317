"""ORACLE for the immersed-boundary time step -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation (``ibo.c``) of the method of Givelberg & Bunn,
Sec. 3, wrapped with ctypes and numpy.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package; the product
(``paper_math_0301321_amd``) never does, and this package never imports the
product.  Inputs come from ``paper_math_0301321_amd.workloads`` (the seeded
model generator, which holds none of the step's arithmetic) or from the
tests themselves.

Arrays: markers (3, M) float64; grid fields (3, Nz, N, N) float64 indexed
[component, z, y, x] (x fastest), Nz = N for the cube and N/2 for the
half-cube of Sec. 4 (one mesh width h = L/N in every direction).  Functions
that take a grid field read Nz from its shape; the others take ``Nz``
(default N).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libibo_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)


class _Model(C.Structure):
    _fields_ = [("M", C.c_int64),
                ("w", _dp), ("k", _dp), ("X_ref", _dp), ("kappa", _dp),
                ("n_lat", C.c_int32),
                ("lat_first", _i64p),
                ("lat_n1", _i32p), ("lat_n2", _i32p), ("lat_periodic2", _i32p),
                ("lat_Ks", _dp), ("lat_Kb", _dp),
                ("n_springs", C.c_int64),
                ("spring_ab", _i32p), ("spring_rest", _dp), ("K_spring", C.c_double),
                ("n_drive", C.c_int64),
                ("drive_idx", _i32p), ("drive_dir", _dp),
                ("drive_A", C.c_double), ("drive_freq", C.c_double),
                ("disp", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _lib.ibo_phi.restype = C.c_double
        _lib.ibo_phi.argtypes = [C.c_double]
        _lib.ibo_energy.restype = C.c_double
        _lib.ibo_fluid.restype = C.c_double
        _lib.ibo_num_threads.restype = C.c_int
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class Model:
    """Holds contiguous copies of a workload's material arrays for the C oracle.

    ``displacement=True``: every marker array passed with this model holds
    displacements D = X - X_ref instead of positions (the elastic terms are
    then formed from D, positions as X_ref + D)."""

    def __init__(self, wl, k=None, displacement=False):
        self.M = wl.M
        self.disp = bool(displacement)
        self.w = _f64(wl.w)
        self.k = _f64(wl.k if k is None else k)
        self.X_ref = _f64(wl.X_ref)
        self.kappa = _f64(wl.kappa)
        lats = wl.lattices
        self.lat_first = np.array([l.first for l in lats] or [0], np.int64)
        self.lat_n1 = np.array([l.n1 for l in lats] or [0], np.int32)
        self.lat_n2 = np.array([l.n2 for l in lats] or [0], np.int32)
        self.lat_per = np.array([int(l.periodic2) for l in lats] or [0], np.int32)
        self.lat_Ks = np.array([l.Ks for l in lats] or [0.0], np.float64)
        self.lat_Kb = np.array([l.Kb for l in lats] or [0.0], np.float64)
        ab = wl.spring_ab if wl.spring_ab is not None else np.zeros((2, 0), np.int32)
        self.sab = np.ascontiguousarray(ab, dtype=np.int32).reshape(2, -1)
        self.srest = _f64(wl.spring_rest if wl.spring_rest is not None else np.zeros(0))
        di = wl.drive_idx if wl.drive_idx is not None else np.zeros(0, np.int32)
        self.didx = np.ascontiguousarray(di, dtype=np.int32)
        self.ddir = _f64(wl.drive_dir if wl.drive_dir is not None else np.zeros((3, 0))).reshape(3, -1)
        self.s = _Model(
            M=self.M, w=_ptr(self.w), k=_ptr(self.k), X_ref=_ptr(self.X_ref), kappa=_ptr(self.kappa),
            n_lat=len(lats), lat_first=_ptr(self.lat_first, _i64p),
            lat_n1=_ptr(self.lat_n1, _i32p), lat_n2=_ptr(self.lat_n2, _i32p),
            lat_periodic2=_ptr(self.lat_per, _i32p), lat_Ks=_ptr(self.lat_Ks), lat_Kb=_ptr(self.lat_Kb),
            n_springs=self.sab.shape[1], spring_ab=_ptr(self.sab, _i32p),
            spring_rest=_ptr(self.srest), K_spring=float(wl.K_spring),
            n_drive=self.didx.shape[0], drive_idx=_ptr(self.didx, _i32p), drive_dir=_ptr(self.ddir),
            drive_A=float(wl.drive_A), drive_freq=float(wl.drive_freq), disp=int(self.disp))

    def ref(self):
        return C.byref(self.s)


def num_threads() -> int:
    return lib().ibo_num_threads()


def set_num_threads(nt: int) -> None:
    """Threads of the oracle's parallel loops from here on (results do not depend on it)."""
    lib().ibo_set_num_threads(C.c_int(int(nt)))


def phi(r):
    r = np.asarray(r, dtype=np.float64)
    f = lib().ibo_phi
    return np.vectorize(f, otypes=[np.float64])(r)


def _nz(N, Nz):
    return N if Nz is None else int(Nz)


def _grid_nz(N, u):
    if u.ndim != 4 or u.shape[2] != N or u.shape[3] != N:
        raise ValueError(f"grid field of shape (c, Nz, {N}, {N}) expected, got {u.shape}")
    return u.shape[1]


def bin_markers(N, L, X, Nz=None):
    """Cell-key binning of Sec. 3.3 (cells grouped in 8^3 blocks); N, Nz multiples of 8."""
    Nz = _nz(N, Nz)
    if N % 8 != 0 or Nz % 8 != 0:
        raise ValueError("bin_markers: N and Nz must be multiples of 8")
    X = _f64(X)
    M = X.shape[1]
    keys = np.zeros(M, np.uint32)
    perm = np.zeros(M, np.int32)
    lib().ibo_bin(C.c_int(N), C.c_int(Nz), C.c_double(L), C.c_int64(M), _ptr(X), _ptr(keys, _u32p), _ptr(perm, _i32p))
    return keys, perm


def force(model: Model, X, t):
    X = _f64(X)
    F = np.zeros_like(X)
    lib().ibo_force(model.ref(), _ptr(X), C.c_double(t), _ptr(F))
    return F


def positions(model: Model, X):
    """Marker positions of the state X: X itself, or X_ref + X for a displacement model."""
    X = _f64(X)
    P = np.zeros_like(X)
    lib().ibo_positions(model.ref(), _ptr(X), _ptr(P))
    return P


def initial_state(wl, displacement=False):
    """The workload's initial marker state: X0, or X0 - X_ref as displacements."""
    return _f64(wl.X0 - wl.X_ref) if displacement else _f64(wl.X0).copy()


def energy(model: Model, X):
    X = _f64(X)
    return lib().ibo_energy(model.ref(), _ptr(X))


def spread(N, L, X, F, Nz=None):
    X, F = _f64(X), _f64(F)
    Nz = _nz(N, Nz)
    Fg = np.zeros((3, Nz, N, N))
    lib().ibo_spread(C.c_int(N), C.c_int(Nz), C.c_double(L), C.c_int64(X.shape[1]), _ptr(X), _ptr(F), _ptr(Fg))
    return Fg


def interp(N, L, X, u):
    X, u = _f64(X), _f64(u)
    U = np.zeros_like(X)
    lib().ibo_interp(C.c_int(N), C.c_int(_grid_nz(N, u)), C.c_double(L), C.c_int64(X.shape[1]), _ptr(X), _ptr(u), _ptr(U))
    return U


def advect(N, L, u):
    u = _f64(u)
    A = np.zeros_like(u)
    lib().ibo_advect(C.c_int(N), C.c_int(_grid_nz(N, u)), C.c_double(L), _ptr(u), _ptr(A))
    return A


def probe(X, X0, idx, dirs):
    """Displacement of markers idx along unit directions dirs (Sec. 5 diagnostics):
    d[i] = sum_c (X[c, idx[i]] - X0[c, idx[i]]) dirs[c, i], written out term by term."""
    X, X0, dirs = _f64(X), _f64(X0), _f64(dirs)
    idx = np.asarray(idx, dtype=np.int64)
    d = np.zeros(len(idx))
    for i, q in enumerate(idx):
        for c in range(3):
            d[i] += (X[c, q] - X0[c, q]) * dirs[c, i]
    return d


def advect_adjoint(N, L, u, r):
    """(dA/du)^T r for the upwind advection A of `advect`, linearised at u with
    every branch frozen (the transpose the adjoint step needs when convect = 1)."""
    u, r = _f64(u), _f64(r)
    out = np.zeros_like(u)
    lib().ibo_advect_adjoint(C.c_int(N), C.c_int(_grid_nz(N, u)), C.c_double(L), _ptr(u), _ptr(r), _ptr(out))
    return out


def fft3(x, sign=-1):
    """Complex 3-D DFT of an (Nz, N, N) array (no normalisation)."""
    x = np.asarray(x)
    Nz, N = x.shape[0], x.shape[1]
    if x.ndim != 3 or x.shape[2] != N:
        raise ValueError("fft3: an (Nz, N, N) array expected")
    re = _f64(x.real).copy()
    im = _f64(x.imag if np.iscomplexobj(x) else np.zeros_like(re)).copy()
    lib().ibo_fft3(C.c_int(N), C.c_int(Nz), _ptr(re), _ptr(im), C.c_int(sign))
    return re + 1j * im


def fluid(N, L, rho, mu, dt, convect, u, Fg=None, return_imag=False):
    u = _f64(u)
    un = np.zeros_like(u)
    Fp = None
    if Fg is not None:
        Fg = _f64(Fg)
        Fp = _ptr(Fg)
    im = lib().ibo_fluid(C.c_int(N), C.c_int(_grid_nz(N, u)), C.c_double(L), C.c_double(rho), C.c_double(mu), C.c_double(dt),
                         C.c_int(convect), _ptr(u), Fp, _ptr(un))
    return (un, im) if return_imag else un


def step(model: Model, wl, X, u, t, N=None, convect=None, return_force=False):
    """One time step; returns new (X, u) (inputs are not modified)."""
    N = wl.N if N is None else N
    conv = wl.convect if convect is None else convect
    X = _f64(X).copy()
    u = _f64(u).copy()
    F = np.zeros_like(X)
    lib().ibo_step(model.ref(), C.c_int(N), C.c_int(_grid_nz(N, u)), C.c_double(wl.L), C.c_double(wl.rho), C.c_double(wl.mu),
                   C.c_double(wl.dt), C.c_int(conv), C.c_double(t), _ptr(X), _ptr(u), _ptr(F))
    return (X, u, F) if return_force else (X, u)


def run(wl, n_steps, X=None, u=None, N=None, k=None, convect=None, t0_step=0, callback=None, displacement=False):
    """n_steps time steps from (X, u) (default: the workload's initial state, fluid at rest);
    with ``displacement`` the marker state is D = X - X_ref."""
    N = wl.N if N is None else N
    model = Model(wl, k, displacement)
    X = (initial_state(wl, displacement) if X is None else _f64(X)).copy()
    u = np.zeros((3, wl.nz * N // wl.N, N, N)) if u is None else _f64(u).copy()
    for n in range(t0_step, t0_step + n_steps):
        X, u = step(model, wl, X, u, n * wl.dt, N=N, convect=convect)
        if callback is not None:
            callback(n + 1, X, u)
    return X, u


def adjoint_step(model: Model, wl, X_n, u_np1, t, Xbar, ubar, kbar, N=None, convect=0, u_n=None):
    """Adjoint of one step: returns (Xbar_n, ubar_n, kbar + contribution).  With
    convect = 1 the step's starting velocity u_n is required (the upwind branches
    are frozen at its signs)."""
    N = wl.N if N is None else N
    X_n, u_np1 = _f64(X_n), _f64(u_np1)
    Xb = _f64(Xbar).copy()
    ub = _f64(ubar).copy()
    kb = _f64(kbar).copy()
    if convect and u_n is None:
        raise ValueError("adjoint_step: convect = 1 needs u_n")
    un = _f64(u_n) if convect else None
    lib().ibo_adjoint_step_u(model.ref(), C.c_int(N), C.c_int(_grid_nz(N, u_np1)), C.c_double(wl.L), C.c_double(wl.rho),
                             C.c_double(wl.mu), C.c_double(wl.dt), C.c_double(t), C.c_int(1 if convect else 0),
                             _ptr(X_n), _ptr(un) if convect else None, _ptr(u_np1), _ptr(Xb), _ptr(ub), _ptr(kb))
    return Xb, ub, kb


def gradient_k(wl, n_steps, loss_idx, N=None, k=None, X0=None, convect=0, progress=None, displacement=False):
    """Loss L = (1/|W|) sum_{q in W} |X_q^T - X_q^0|^2 after n_steps steps (Stokes,
    or with the upwind advection when convect = 1) from (X0, u = 0), and its
    gradient with respect to the per-marker stiffness k, by the adjoint step run
    backwards over stored states.  Returns (L, kbar, Xbar0, ubar0).
    ``progress(phase, n)``, when given, is called after every step of the
    forward ("forward") and reverse ("adjoint") sweeps.  With ``displacement``
    the marker state (and X0) are displacements from X_ref; the loss is the
    same (X^T - X^0 = D^T - D^0)."""
    N = wl.N if N is None else N
    model = Model(wl, k, displacement)
    X0 = initial_state(wl, displacement) if X0 is None else _f64(X0)
    idx = np.asarray(loss_idx, dtype=np.int64)
    Xs, us = [X0.copy()], [np.zeros((3, wl.nz * N // wl.N, N, N))]
    for n in range(n_steps):
        Xn, un = step(model, wl, Xs[-1], us[-1], n * wl.dt, N=N, convect=convect)
        Xs.append(Xn)
        us.append(un)
        if progress is not None:
            progress("forward", n)
    d = Xs[-1][:, idx] - X0[:, idx]
    L = float((d * d).sum() / len(idx))
    Xb = np.zeros_like(X0)
    Xb[:, idx] = 2.0 * d / len(idx)
    ub = np.zeros_like(us[0])
    kb = np.zeros(wl.M)
    for n in reversed(range(n_steps)):
        Xb, ub, kb = adjoint_step(model, wl, Xs[n], us[n + 1], n * wl.dt, Xb, ub, kb, N=N, convect=convect,
                                  u_n=us[n])
        if progress is not None:
            progress("adjoint", n)
    return L, kb, Xb, ub
