"""The largest grid the library takes (n = 512): properties that hold at any size.

A full oracle comparison at 512^3 would need several GB of FP64 fields on the
host; instead these tests check what the mathematics fixes exactly:
  * binning: bit-exact against the oracle (markers only, cheap at any n);
  * fluid step: a single Fourier mode u_x = sin(2 pi m y / n), divergence-free
    and constant along x, is left alone by the projection and by the upwind
    advection (its x difference is zero and u_y = u_z = 0), so one step
    multiplies it by 1 / (1 + nu dt lambda_m), lambda_m = (4/h^2) sin^2(pi m/n)
    (eqs. discreteNS1-2);
  * spread: sum_x F h^3 = sum_q F_q per component (the weights sum to one);
  * interpolation: a constant field is interpolated exactly.
"""
import math

import numpy as np
import pytest
import torch

from paper_math_0301321_amd import workloads as W
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

NMAX = 512


@pytest.fixture(scope="module")
def ibm():
    from paper_math_0301321_amd import ib
    ib.load_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return ib


def _wl(X, convect=1):
    M = X.shape[1]
    return W.Workload(name="free512", N=NMAX, L=1.0, rho=1.0, mu=0.01, dt=1e-4, n_steps=1, convect=convect,
                      X0=X, w=np.ones(M), k=np.ones(M), X_ref=X.copy(), kappa=np.zeros(M))


def _markers(M, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.2, 1.2, size=(3, M)), rng.standard_normal((3, M))


def test_bin_bit_exact_512(ibm, oracle_mod):
    X, _ = _markers(50000, 512)
    wl = _wl(X)
    announce("bin", NMAX, wl.M)
    ctx = ibm.Context(wl, "fp32")
    keys, perm = ctx.bin(dev(X))
    torch.cuda.synchronize()
    ok, op = oracle_mod.bin_markers(NMAX, 1.0, X)
    assert np.array_equal(host(keys).astype(np.int64) & 0xFFFFFFFF, ok.astype(np.int64))
    assert np.array_equal(perm.cpu().numpy(), op)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
@pytest.mark.parametrize("convect", [0, 1])
def test_fluid_single_mode_512(ibm, prec, tol, convect):
    wl = _wl(np.zeros((3, 0)), convect)
    n, m = NMAX, 37
    h = wl.L / n
    announce("fluid single mode", prec, n, convect)
    ctx = ibm.Context(wl, prec)
    dt_ = torch.float32 if prec == "fp32" else torch.float64
    u = torch.zeros((3, n, n, n), dtype=dt_, device="cuda")
    y = torch.arange(n, dtype=torch.float64, device="cuda")
    mode = torch.sin(2.0 * math.pi * m * y / n)                    # along y: index [c][z][y][x]
    u[0] = mode.view(1, n, 1).to(dt_).expand(n, n, n)
    u0 = u[0].double().clone()
    ctx.fluid(u)
    torch.cuda.synchronize()
    lam = 4.0 / h ** 2 * math.sin(math.pi * m / n) ** 2
    g = 1.0 / (1.0 + wl.mu / wl.rho * wl.dt * lam)
    want = g * u0
    err = (u[0].double() - want).abs().max().item() / want.abs().max().item()
    assert err < tol, (prec, convect, err, g)
    assert u[1].abs().max().item() < tol and u[2].abs().max().item() < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_spread_total_and_interp_constant_512(ibm, prec, tol):
    X, F = _markers(200000, 5120)
    wl = _wl(X)
    h3 = (wl.L / NMAX) ** 3
    announce("spread/interp 512", prec, wl.M)
    ctx = ibm.Context(wl, prec)
    Fg = ctx.spread(dev(X), dev(F))
    tot = Fg.double().sum(dim=(1, 2, 3)).cpu().numpy() * h3
    want = F.sum(axis=1)
    assert np.abs(tot - want).max() <= tol * np.abs(F).sum(axis=1).max(), (tot, want)
    dt_ = torch.float32 if prec == "fp32" else torch.float64
    c = torch.tensor([0.25, -1.5, 3.0], dtype=torch.float64)
    u = c.to(dt_).view(3, 1, 1, 1).expand(3, NMAX, NMAX, NMAX).contiguous().cuda()
    U = host(ctx.interp(dev(X), u))
    err = np.abs(U - c.numpy()[:, None]).max() / np.abs(c.numpy()).max()
    assert err < (1e-14 if prec == "fp64" else 1e-6), (prec, err)
