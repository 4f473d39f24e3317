"""GPU parity on grids whose z length carries a factor 3 (n x n x 3n/4: z
transforms of length 24, 48, 96 and 192, done in registers as 3 decimated
power-of-two DFTs combined with radix-3 butterflies), against the oracle,
whose DFT along such a length is pinned to the cube's radix-2 FFT.

Tolerances as for the cube and the half-cube: binning bit-exact; FP64 1e-12
per kernel and 1e-10 over steps; mixed 2e-6 per kernel and 1e-5 over steps.
"""
import math

import numpy as np
import pytest
import torch

from paper_math_0301321_amd import workloads as W
from tests.gpu_util import announce, dev, host, rel_max

pytestmark = pytest.mark.gpu

TOL1 = {"fp64": 1e-12, "fp32": 2e-6}


@pytest.fixture(scope="module")
def ibm():
    from paper_math_0301321_amd import ib
    ib.load_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return ib


def _fd(prec):
    return torch.float32 if prec == "fp32" else torch.float64


def _free(N, X, convect=1):
    M = X.shape[1]
    return W.Workload(name="free_3q", N=N, L=1.0, rho=1.0, mu=0.01, dt=1e-3, n_steps=1, convect=convect,
                      X0=X, w=np.ones(M), k=np.ones(M), X_ref=X.copy(), kappa=np.zeros(M), Nz=3 * N // 4)


def _flat(N, n_steps=6):
    """The flat-membrane model in a box of height 3/4 (the membrane at z = 1/4)."""
    wl = W.tiny_halfcube(N, n_steps=n_steps)
    wl.Nz = 3 * N // 4
    wl.name = f"flat_3q{N}"
    return wl


def _markers(N, M, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.3, 1.3, size=(3, M))
    X[2] = rng.uniform(-0.2, 0.95, size=M)
    on = rng.random(M) < 0.1
    X[:, on] = np.round(X[:, on] * N) / N
    return X, rng.standard_normal((3, M))


@pytest.mark.parametrize("N", [32, 64])
def test_bin_bit_exact(ibm, oracle_mod, N):
    X, _ = _markers(N, 20000, 60 + N)
    wl = _free(N, X)
    announce("3q bin", N)
    ctx = ibm.Context(wl, "fp32")
    keys, perm = ctx.bin(dev(X))
    torch.cuda.synchronize()
    ok, op = oracle_mod.bin_markers(N, 1.0, X, Nz=3 * N // 4)
    assert np.array_equal(host(keys).astype(np.int64) & 0xFFFFFFFF, ok.astype(np.int64))
    assert np.array_equal(perm.cpu().numpy(), op)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [32, 64])
def test_spread_and_interp_parity(ibm, oracle_mod, prec, N):
    X, F = _markers(N, 4000, 70 + N)
    announce("3q spread/interp", prec, N)
    ctx = ibm.Context(_free(N, X), prec)
    Fg = host(ctx.spread(dev(X), dev(F)))
    assert rel_max(Fg, oracle_mod.spread(N, 1.0, X, F, Nz=3 * N // 4)) < TOL1[prec]
    u = W.random_field(N, seed=71, Nz=3 * N // 4)
    U = host(ctx.interp(dev(X), dev(u, _fd(prec))))
    uo = u.astype(np.float32).astype(np.float64) if prec == "fp32" else u
    assert rel_max(U, oracle_mod.interp(N, 1.0, X, uo)) < TOL1[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_fluid_parity(ibm, oracle_mod, prec, N):
    nz = 3 * N // 4
    u = 0.5 * W.random_field(N, seed=72, Nz=nz)
    F = 100.0 * W.random_field(N, seed=73, Nz=nz)
    if prec == "fp32":
        u, F = u.astype(np.float32).astype(np.float64), F.astype(np.float32).astype(np.float64)
    wl = _free(N, np.zeros((3, 0)))
    announce("3q fluid", prec, N, nz)
    ctx = ibm.Context(wl, prec)
    ut = dev(u, _fd(prec))
    ctx.fluid(ut, dev(F, _fd(prec)))
    uo = oracle_mod.fluid(N, 1.0, wl.rho, wl.mu, wl.dt, 1, u, F)
    assert rel_max(host(ut), uo) < TOL1[prec]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
@pytest.mark.parametrize("m", [1, 7, 48])
def test_z_mode_decay_256x256x192(ibm, prec, tol, m):
    """u_x = sin(2 pi m z / 192 + 0.3), divergence-free and untouched by the
    advection: one step multiplies it by 1 / (1 + nu dt (4/h^2) sin^2(pi m / 192))
    (m = 96 would be the Nyquist mode; 48 a quarter of the way)."""
    n, nz = 256, 192
    wl = _free(n, np.zeros((3, 0)))
    announce("3q z mode", prec, m)
    ctx = ibm.Context(wl, prec)
    u = ctx.new_grid()
    z = torch.arange(nz, dtype=torch.float64, device="cuda")
    u[0] = torch.sin(2.0 * math.pi * m * z / nz + 0.3).view(nz, 1, 1).to(u.dtype).expand(nz, n, n)
    u0 = u[0].double().clone()
    ctx.fluid(u)
    torch.cuda.synchronize()
    h = 1.0 / n
    g = 1.0 / (1.0 + wl.mu / wl.rho * wl.dt * (4.0 / h ** 2) * math.sin(math.pi * m / nz) ** 2)
    err = (u[0].double() - g * u0).abs().max().item() / (g * u0).abs().max().item()
    assert err < tol, (prec, m, err)
    assert u[1].abs().max().item() < tol and u[2].abs().max().item() < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [32, 64])
def test_step_parity_multistep(ibm, oracle_mod, prec, N):
    wl = _flat(N)
    n = wl.n_steps
    announce("3q steps", N, prec, n)
    Xo, uo = oracle_mod.run(wl, n)
    ctx = ibm.Context(wl, prec)
    X = dev(wl.X0)
    u = ctx.new_grid()
    for k in range(n):
        ctx.step(X, u, k * wl.dt)
    torch.cuda.synchronize()
    tol = 1e-10 if prec == "fp64" else 1e-5
    eX, eu = rel_max(host(X) - wl.X0, Xo - wl.X0), rel_max(host(u), uo)
    assert eX < tol and eu < tol, (N, prec, eX, eu)


@pytest.mark.parametrize("convect", [0, 1])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_adjoint_step_parity(ibm, oracle_mod, prec, tol, convect):
    wl = _flat(32)
    wl.convect = convect
    rng = np.random.default_rng(80)
    X = wl.X0 + 2e-3 * rng.standard_normal(wl.X0.shape)
    u = 0.05 * W.random_field(32, seed=81, Nz=24)
    if prec == "fp32":
        u = u.astype(np.float32).astype(np.float64)
    t = 3e-4
    m = oracle_mod.Model(wl)
    _, u1 = oracle_mod.step(m, wl, X, u, t, convect=convect)
    Xb1, ub1 = rng.standard_normal(X.shape), rng.standard_normal(u.shape)
    if prec == "fp32":
        u1 = u1.astype(np.float32).astype(np.float64)
        ub1 = ub1.astype(np.float32).astype(np.float64)
    Xbo, ubo, kbo = oracle_mod.adjoint_step(m, wl, X, u1, t, Xb1, ub1, np.zeros(wl.M), convect=convect, u_n=u)
    announce("3q adjoint", prec, convect)
    ctx = ibm.Context(wl, prec, convect=convect)
    fd = _fd(prec)
    Xb, ub, kb = dev(Xb1), dev(ub1, fd), torch.zeros(wl.M, dtype=torch.float64, device="cuda")
    ctx.adjoint_step(dev(X), dev(u1, fd), t, Xb, ub, kb, u_n=dev(u, fd) if convect else None)
    torch.cuda.synchronize()
    assert rel_max(host(Xb) - Xb1, Xbo - Xb1) < tol
    assert rel_max(host(ub), ubo) < tol
    assert rel_max(host(kb), kbo) < tol


def test_full_size_steps_256x256x192(ibm, oracle_mod):
    """The 1.5M-marker flat model in a 256 x 256 x 192 box: three steps from rest
    (the drive on from the second) in both precisions against the oracle."""
    wl = W.halfcube(256)
    wl.Nz = 192
    announce("3q full size", wl.N, wl.nz, wl.M)
    Xo, uo = oracle_mod.run(wl, 3)
    assert np.abs(uo).max() > 0 and np.abs(Xo - wl.X0).max() > 0
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        ctx = ibm.Context(wl, prec)
        X = dev(wl.X0)
        u = ctx.new_grid()
        for k in range(3):
            ctx.step(X, u, k * wl.dt)
        torch.cuda.synchronize()
        eX, eu = rel_max(host(X) - wl.X0, Xo - wl.X0), rel_max(host(u), uo)
        print(f"[gpu-case] 256x256x192 {prec}: rel u {eu:.3e}, rel dX {eX:.3e}", flush=True)
        assert eX < tol and eu < tol, (prec, eX, eu)
