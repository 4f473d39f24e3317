"""Seeded synthetic workloads for the immersed-boundary time step.

This module is the model generator: it builds marker positions, lattice
topology, material weights and drive patterns, the way the paper's separate
model-generation software writes geometry and material files before the
solver starts (Sec. 3.3, Sec. 4).  It holds none of the time step's
arithmetic (no force law, no delta function, no fluid solve), so both the
GPU library and the CPU oracle can consume its output.

Geometry stands in for the measured cochlea (Sec. 4), which is not available:
a tapered helicoidal strip (the basilar membrane, BM) inside a coiled tube
wall, in the paper's proportions (1 unit = 1 cm; BM about 3.5 cm long, its
width growing from 150 um to 560 um).  The window is a patch of the wall
near the base that carries a sinusoidal force along the outward wall normal
(Sec. 4, oval-window drive).

Units are CGS: rho = 1, mu = 0.01 for every workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Lattice:
    """A rectangular material lattice Q (Sec. 3.2): markers first + i2*n1 + i1.

    i1 runs along direction 1 (0..n1-1, fastest), i2 along direction 2
    (0..n2-1, periodic when ``periodic2``).  ``Ks``/``Kb`` are the stretch and
    bend moduli applied to every lattice edge / triple.
    """
    first: int
    n1: int
    n2: int
    periodic2: bool
    Ks: float
    Kb: float


@dataclass
class Workload:
    name: str
    N: int                 # grid points along x and y (and z, unless Nz is set)
    L: float               # box edge along x and y; h = L / N in every direction
    rho: float
    mu: float
    dt: float
    n_steps: int
    convect: int           # 1: upwind advection term on; 0: Stokes (linear) step
    X0: np.ndarray         # (3, M) float64 initial marker positions
    w: np.ndarray          # (M,) area weight (Delta q) per marker
    k: np.ndarray          # (M,) stiffness multiplier per marker
    X_ref: np.ndarray      # (3, M) reference shape: tether targets, rest geometry
    kappa: np.ndarray      # (M,) tether stiffness density (0 = untethered)
    lattices: list = field(default_factory=list)
    spring_ab: np.ndarray = None      # (2, S) int32 marker pairs
    spring_rest: np.ndarray = None    # (S,) float64 rest lengths
    K_spring: float = 0.0
    drive_idx: np.ndarray = None      # (D,) int32 driven markers
    drive_dir: np.ndarray = None      # (3, D) float64 unit directions
    drive_A: float = 0.0
    drive_freq: float = 0.0
    meta: dict = field(default_factory=dict)
    Nz: int = 0            # grid points along z: 0 means N (the cube); N / 2 is the half-cube of Sec. 4

    @property
    def M(self) -> int:
        return int(self.X0.shape[1])

    @property
    def nz(self) -> int:
        return int(self.Nz) if self.Nz else int(self.N)

    @property
    def grid_shape(self) -> tuple:
        """Shape of one grid field, [component, z, y, x]."""
        return (3, self.nz, self.N, self.N)

    @property
    def h(self) -> float:
        return self.L / self.N

    def with_grid(self, N: int) -> "Workload":
        """Same markers and time step on another grid size (a replica)."""
        import copy
        wl = copy.copy(self)
        wl.N = int(N)
        if self.Nz:
            wl.Nz = int(N) * int(self.Nz) // int(self.N)
            wl.name = f"{self.name}@{N}x{N}x{wl.Nz}"
        else:
            wl.name = f"{self.name}@{N}^3"
        return wl


def _empty_int(shape):
    return np.zeros(shape, dtype=np.int32)


# --------------------------------------------------------------------------
# closed spherical shell (icosphere)
# --------------------------------------------------------------------------
def icosphere(subdiv: int):
    """Vertices (V,3) on the unit sphere and faces (F,3) of a subdivided icosahedron."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def _edges_from_faces(faces):
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]])
    e.sort(axis=1)
    return np.unique(e, axis=0)


def config1(N: int = 32) -> Workload:
    """Closed spherical shell of Hookean springs, stretched 10% along x, fluid at rest.

    Periodic 32^3 grid on the unit cube, rho = 1, mu = 0.01, dt = 1e-3,
    10 steps; icosphere subdivision 4 (2,562 markers, 7,680 edges), radius
    0.25 about the cube centre; spring stiffness 1e3, rest length equal to the
    unstretched edge length.
    """
    v, f = icosphere(4)
    R, c = 0.25, 0.5
    rest_pos = (c + R * v).T.copy()                     # (3, M) unstretched
    X0 = rest_pos.copy()
    X0[0] = c + 1.1 * (X0[0] - c)                      # 10% stretch along x
    edges = _edges_from_faces(f)
    rest = np.linalg.norm(rest_pos[:, edges[:, 1]] - rest_pos[:, edges[:, 0]], axis=0)
    M = X0.shape[1]
    area = 4.0 * math.pi * R * R / M
    return Workload(
        name="shell32", N=N, L=1.0, rho=1.0, mu=0.01, dt=1e-3, n_steps=10, convect=1,
        X0=X0, w=np.full(M, area), k=np.ones(M), X_ref=rest_pos, kappa=np.zeros(M),
        lattices=[], spring_ab=np.ascontiguousarray(edges.T.astype(np.int32)),
        spring_rest=rest, K_spring=1e3,
        drive_idx=_empty_int(0), drive_dir=np.zeros((3, 0)), drive_A=0.0, drive_freq=0.0,
        meta={"faces": f})


# --------------------------------------------------------------------------
# helicoidal membrane in a coiled tube
# --------------------------------------------------------------------------
_TURNS = 2.5


def _centre(s):
    th = 2.0 * math.pi * _TURNS * s
    R = 0.30 - 0.18 * s
    C = np.stack([0.5 + R * np.cos(th), 0.5 + R * np.sin(th), 0.20 + 0.60 * s])
    dth = 2.0 * math.pi * _TURNS
    dC = np.stack([-0.18 * np.cos(th) - R * dth * np.sin(th),
                   -0.18 * np.sin(th) + R * dth * np.cos(th),
                   np.full_like(s, 0.60)])
    er = np.stack([np.cos(th), np.sin(th), np.zeros_like(s)])
    return C, dC, er


# flat spiral of the half-cube model (Sec. 4): 1.5 turns in the plane z = 1/4
_FLAT_TURNS = 1.5


def _centre_flat(s):
    th = 2.0 * math.pi * _FLAT_TURNS * s
    R = 0.38 - 0.28 * s
    C = np.stack([0.5 + R * np.cos(th), 0.5 + R * np.sin(th), np.full_like(s, 0.25)])
    dth = 2.0 * math.pi * _FLAT_TURNS
    dC = np.stack([-0.28 * np.cos(th) - R * dth * np.sin(th),
                   -0.28 * np.sin(th) + R * dth * np.cos(th),
                   np.zeros_like(s)])
    er = np.stack([np.cos(th), np.sin(th), np.zeros_like(s)])
    return C, dC, er


def helicoid_in_tube(nb1, nb2, nw1, nw2, win1, win2, *, N, dt, n_steps, freq,
                     Ks=50.0, Kb=3e-4, kappa=1e5, drive_A=1e2, jitter_seed=None,
                     convect=1, name="helix", window=None, flat=False) -> Workload:
    """Tapered helicoidal strip ('BM', nb1 x nb2) inside a coiled tube wall (nw1 x nw2).

    BM centre line C(s) = (1/2 + R cos th, 1/2 + R sin th, 0.2 + 0.6 s), th = 5 pi s
    (2.5 turns), R = 0.30 - 0.18 s; the strip spans +-b(s)/2 along the radial
    direction, b = 0.015 + 0.041 s.  BM stretch/bend stiffness multiplier
    k = exp(-3 s) (times 1 + 0.05 U(-1,1) when ``jitter_seed`` is given); its two
    long edges are tethered.  The wall is a tube of radius a = 0.10 - 0.04 s
    around C(s), every marker tethered to its initial position.  The window
    patch (wall i1 < win1, i2 < win2) is driven along the outward normal.

    ``window = nw`` replaces the driven wall patch by the window model of
    Sec. 4: a flat square lattice of nw x nw markers (spacing h/2) in the
    plane tangent to the wall at s = 0.03, whose markers outside the inscribed
    circle are held by tethers and whose markers inside move freely, with
    stretch and bend moduli Ks, Kb, under the sinusoidal force along the
    outward normal.

    ``flat = True`` builds the half-cube model of Sec. 4 instead: the grid is
    N x N x N/2 (box 1 x 1 x 1/2) and the membrane is flat, its centre line
    the planar spiral (1/2 + R cos th, 1/2 + R sin th, 1/4), th = 3 pi s
    (1.5 turns), R = 0.38 - 0.28 s, the strip spanning the radial direction
    within that plane; the tube radius is a = 0.07 - 0.03 s so that the
    coils stay apart and the tube stays inside 0 < z < 1/2.
    """
    centre = _centre_flat if flat else _centre
    tube_a = (lambda s_: 0.07 - 0.03 * s_) if flat else (lambda s_: 0.10 - 0.04 * s_)
    # ---- basilar membrane lattice, fibre by fibre (the membrane's fibres run
    # across its width): index = i1 * nb2 + i2 for station i1 < nb1 along the
    # length and position i2 < nb2 across ----
    s = np.linspace(0.0, 1.0, nb1)
    C, dC, er = centre(s)
    b = 0.015 + 0.041 * s
    eta = np.linspace(-0.5, 0.5, nb2)
    BM = C[:, None, :] + eta[None, :, None] * (b * er)[:, None, :]      # (3, nb2, nb1)
    ds_len = np.linalg.norm(dC, axis=0) / (nb1 - 1)
    w_bm = np.broadcast_to(ds_len * b / (nb2 - 1), (nb2, nb1))
    k_bm = np.broadcast_to(np.exp(-3.0 * s), (nb2, nb1)).copy()
    if jitter_seed is not None:
        rng = np.random.default_rng(jitter_seed)
        k_bm *= 1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=k_bm.shape)
    kap_bm = np.zeros((nb2, nb1))
    kap_bm[0, :] = kappa
    kap_bm[-1, :] = kappa
    s_bm = np.broadcast_to(s, (nb2, nb1))

    # ---- tube wall lattice (periodic around): index = M_bm + i2 * nw1 + i1 ----
    sw = np.linspace(0.0, 1.0, nw1)
    Cw, dCw, erw = centre(sw)
    t = dCw / np.linalg.norm(dCw, axis=0)
    n1 = erw - (erw * t).sum(0) * t
    n1 /= np.linalg.norm(n1, axis=0)
    n2 = np.cross(t.T, n1.T).T
    a = tube_a(sw)
    ph = 2.0 * math.pi * np.arange(nw2) / nw2
    nrm = (np.cos(ph)[:, None, None] * n1.T[None, :, :]
           + np.sin(ph)[:, None, None] * n2.T[None, :, :])                 # (nw2, nw1, 3)
    WALL = (Cw.T[None, :, :] + a[None, :, None] * nrm).transpose(2, 0, 1)   # (3, nw2, nw1)
    dsw_len = np.linalg.norm(dCw, axis=0) / (nw1 - 1)
    w_w = np.broadcast_to(dsw_len * 2.0 * math.pi * a / nw2, (nw2, nw1))

    M_bm, M_w = nb1 * nb2, nw1 * nw2
    BM = BM.transpose(0, 2, 1)                      # (3, nb1, nb2): across-width fastest
    w_bm, k_bm, kap_bm, s_bm = (a.T for a in (w_bm, k_bm, kap_bm, s_bm))
    X0 = np.concatenate([BM.reshape(3, M_bm), WALL.reshape(3, M_w)], axis=1)
    X0 = np.ascontiguousarray(X0)
    w = np.concatenate([w_bm.reshape(-1), w_w.reshape(-1)])
    k = np.concatenate([k_bm.reshape(-1), np.ones(M_w)])
    kap = np.concatenate([kap_bm.reshape(-1), np.full(M_w, kappa)])

    lattices = [Lattice(0, nb2, nb1, False, Ks, Kb), Lattice(M_bm, nw1, nw2, True, 0.0, 0.0)]
    meta = {"bm_first": 0, "bm_along": nb1, "bm_across": nb2, "wall_first": M_bm,
            "wall_n1": nw1, "wall_n2": nw2, "s_bm": s_bm.reshape(-1).copy()}
    if window is None:
        i2w, i1w = np.meshgrid(np.arange(win2), np.arange(win1), indexing="ij")
        didx = (M_bm + i2w * nw1 + i1w).reshape(-1).astype(np.int32)
        ddir = nrm[i2w.reshape(-1), i1w.reshape(-1), :].T.copy()
    else:
        # window lattice: index = M_bm + M_w + j * nw + i, i along the tube, j around it
        nwin = int(window)
        s0 = np.array([0.03])
        C0, dC0, er0 = centre(s0)
        t0 = (dC0 / np.linalg.norm(dC0, axis=0))[:, 0]
        m1 = er0[:, 0] - (er0[:, 0] @ t0) * t0
        m1 /= np.linalg.norm(m1)                      # outward normal of the wall at phase 0
        m2 = np.cross(t0, m1)
        wc = C0[:, 0] + tube_a(s0[0]) * m1
        d = 0.5 / N                                   # spacing h/2
        off = (np.arange(nwin) - 0.5 * (nwin - 1)) * d
        oj, oi = np.meshgrid(off, off, indexing="ij")
        WIN = wc[:, None, None] + oi[None] * t0[:, None, None] + oj[None] * m2[:, None, None]
        inside = (oi ** 2 + oj ** 2 <= (0.5 * (nwin - 1) * d) ** 2).reshape(-1)
        M_win = nwin * nwin
        X0 = np.ascontiguousarray(np.concatenate([X0, WIN.reshape(3, M_win)], axis=1))
        w = np.concatenate([w, np.full(M_win, d * d)])
        k = np.concatenate([k, np.ones(M_win)])
        kap = np.concatenate([kap, np.where(inside, 0.0, kappa)])
        first = M_bm + M_w
        lattices.append(Lattice(first, nwin, nwin, False, Ks, Kb))
        didx = (first + np.flatnonzero(inside)).astype(np.int32)
        ddir = np.ascontiguousarray(np.repeat(m1[:, None], len(didx), axis=1))
        meta.update({"window_first": first, "window_n": nwin, "window_inside": np.flatnonzero(inside),
                     "window_normal": m1.copy()})
    return Workload(
        name=name, N=N, L=1.0, rho=1.0, mu=0.01, dt=dt, n_steps=n_steps, convect=convect,
        X0=X0, w=np.ascontiguousarray(w), k=np.ascontiguousarray(k), X_ref=X0.copy(),
        kappa=np.ascontiguousarray(kap), lattices=lattices,
        spring_ab=np.zeros((2, 0), np.int32), spring_rest=np.zeros(0), K_spring=0.0,
        drive_idx=didx, drive_dir=np.ascontiguousarray(ddir), drive_A=drive_A,
        drive_freq=float(freq), meta=meta, Nz=N // 2 if flat else 0)


def config2(N: int = 128) -> Workload:
    """128^3 grid; BM 800 x 250 (200k) + wall 1000 x 300 (300k); window 20 x 100; 1 kHz; dt 5e-5 x 200."""
    return helicoid_in_tube(800, 250, 1000, 300, 20, 100, N=N, dt=5e-5, n_steps=200,
                            freq=1000.0, name="helix128")


C3_FREQS = (200.0, 500.0, 1000.0, 1500.0)


def config3(N: int = 256, freq: float = C3_FREQS[2]) -> Workload:
    """256^3 grid; BM 1200 x 500 (600k) + wall 1800 x 500 (900k) = 1.5M markers; +-5% k jitter (seed 0)."""
    return helicoid_in_tube(1200, 500, 1800, 500, 36, 167, N=N, dt=2.5e-5, n_steps=500,
                            freq=freq, jitter_seed=0, name="helix256")


def bm_index(wl: Workload, station, across) -> np.ndarray:
    """Marker ids of BM points (station along the length, position across the width)."""
    st, ac = np.meshgrid(np.atleast_1d(station), np.atleast_1d(across), indexing="ij")
    return (wl.meta["bm_first"] + st * wl.meta["bm_across"] + ac).reshape(-1).astype(np.int64)


def bm_station(wl: Workload, q) -> np.ndarray:
    """Station along the length of BM marker ids q."""
    return (np.asarray(q) - wl.meta["bm_first"]) // wl.meta["bm_across"]


def bm_count(wl: Workload) -> int:
    return wl.meta["bm_along"] * wl.meta["bm_across"]


def loss_window(wl: Workload, lo: int = 238, hi: int = 241) -> np.ndarray:
    """BM markers at stations [lo, hi] across the full width (1,000 markers at 800 x 250)."""
    return np.sort(bm_index(wl, np.arange(lo, hi + 1), np.arange(wl.meta["bm_across"])))


def config4(N: int = 128) -> Workload:
    """Adjoint workload: helix128 geometry, Stokes step (convect = 0), 50 steps, checkpoint every 10."""
    wl = config2(N)
    wl.name, wl.n_steps, wl.convect = "adjoint128", 50, 0
    wl.meta["ckpt"] = 10
    wl.meta["loss_idx"] = loss_window(wl)
    return wl


def config5(N: int = 256) -> Workload:
    """Adjoint at scale: helix256 geometry, 100 steps, checkpoint every 20 (64^3 replica: config5(64))."""
    wl = config3(N)
    wl.name, wl.n_steps, wl.convect = f"adjoint{N}", 100, 0
    wl.meta["ckpt"] = 20
    wl.meta["loss_idx"] = loss_window(wl, 357, 359)
    return wl


def tiny_helix(N: int = 32, nb=(60, 12), nw=(80, 24), dt=2e-4, n_steps=10, window=None) -> Workload:
    """A scaled-down helix for fast parity tests (same structure, few markers)."""
    return helicoid_in_tube(nb[0], nb[1], nw[0], nw[1], 4, 6, N=N, dt=dt, n_steps=n_steps,
                            freq=1000.0, jitter_seed=0, name=f"helix_tiny{N}", window=window)


def window128(N: int = 128) -> Workload:
    """The 128^3 helix with the window model of Sec. 4 (a 48 x 48 lattice, free
    inside its inscribed circle, fixed outside) in place of the driven wall patch."""
    return helicoid_in_tube(800, 250, 1000, 300, 20, 100, N=N, dt=5e-5, n_steps=200,
                            freq=1000.0, name="window128", window=48)


def halfcube(N: int = 256) -> Workload:
    """The half-cube model of Sec. 4 on an N x N x N/2 grid (256 x 256 x 128:
    the grid of the paper's reported runs): flat spiral membrane 1200 x 500 in
    a coiled tube wall 1800 x 500, 1.5M markers, the drive and time step of
    the 256^3 helix."""
    return helicoid_in_tube(1200, 500, 1800, 500, 36, 167, N=N, dt=2.5e-5, n_steps=500,
                            freq=1000.0, jitter_seed=0, name=f"halfcube{N}", flat=True)


def tiny_halfcube(N: int = 32, nb=(60, 12), nw=(80, 24), dt=2e-4, n_steps=10) -> Workload:
    """A scaled-down half-cube model for fast parity tests (N x N x N/2)."""
    return helicoid_in_tube(nb[0], nb[1], nw[0], nw[1], 4, 6, N=N, dt=dt, n_steps=n_steps,
                            freq=1000.0, jitter_seed=0, name=f"halfcube_tiny{N}", flat=True)


def random_markers(M: int, seed: int = 2, lo: float = 0.0, hi: float = 1.0):
    """Uniform random marker positions and forces (seed 2 is used for test fields)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, size=(3, M))
    F = rng.standard_normal((3, M))
    return X, F


def random_field(N: int, seed: int = 2, comps: int = 3, Nz: int | None = None):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((comps, N if Nz is None else Nz, N, N))


def smooth_field(N: int, seed: int = 2, Nz: int | None = None, kmax: int = 6, terms: int = 12):
    """A smooth periodic random field (3, Nz, N, N): per component, a sum of
    ``terms`` plane waves with integer wave numbers in [-kmax, kmax] along each
    axis (periodic on the N x N x Nz grid), normalised to max |value| = 1."""
    Nz = N if Nz is None else int(Nz)
    rng = np.random.default_rng(seed)
    z = np.arange(Nz)[:, None, None] / Nz
    y = np.arange(N)[None, :, None] / N
    x = np.arange(N)[None, None, :] / N
    out = np.zeros((3, Nz, N, N))
    for c in range(3):
        for _ in range(terms):
            kx, ky, kz = rng.integers(-kmax, kmax + 1, size=3)
            a, ph = rng.standard_normal(), rng.uniform(0.0, 2.0 * math.pi)
            out[c] += a * np.cos(2.0 * math.pi * (kx * x + ky * y + kz * z) + ph)
    return out / np.abs(out).max()


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
