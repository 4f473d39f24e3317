"""GPU: update of the marker partition between binnings (ib_bin_reuse).

Binning keeps the last sorted order, tile ranges and work list when no marker
changed cell, moves the few markers that did into place (rebuilding the work
list only if one changed tile), and sorts in full with more than 4096 such
markers; the choice is made on the device.  The partition must be bitwise the
oracle's after every kind of change (markers crossing cell and tile
boundaries, crossing the periodic boundary, moving within their cell,
returning, many at once), and whole steps must be bitwise those of a context
that sorts in full every time.
"""
import numpy as np
import pytest
import torch

from paper_math_0301321_amd import workloads as W
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ibm():
    from paper_math_0301321_amd import ib
    ib.load_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return ib


def _check_bin(ctx, oracle_mod, wl, X):
    keys, perm = ctx.bin(dev(X))
    torch.cuda.synchronize()
    ok, op = oracle_mod.bin_markers(wl.N, wl.L, X, Nz=wl.nz)
    assert np.array_equal(host(keys).astype(np.int64) & 0xFFFFFFFF, ok.astype(np.int64))
    assert np.array_equal(perm.cpu().numpy(), op)


def _moved(wl, X0, seed):
    """X0 with a few markers across cell boundaries (one across a tile face,
    one across the periodic boundary), a few within their cell."""
    rng = np.random.default_rng(seed)
    h = wl.L / wl.N
    X = X0.copy()
    idx = rng.choice(wl.M, size=12, replace=False)
    X[0, idx[:4]] += 1.01 * h                       # one cell along x
    X[1, idx[4:6]] -= 8.5 * h                       # a tile along y
    X[2, idx[6]] = -0.25 * h                        # wraps to the last cell along z
    X[0, idx[7]] = wl.L + 0.1 * h                   # wraps to the first cell along x
    c = np.floor(X[:, idx[8:]] / h)
    X[:, idx[8:]] = (c + 0.5) * h                   # moved within the cell (or not at all)
    return X


def _within_tiles(wl, X0, seed, count=6):
    """X0 with a few markers moved one cell along x inside their tile."""
    rng = np.random.default_rng(seed)
    h = wl.L / wl.N
    c = np.floor(X0[0] / h).astype(np.int64) % wl.N
    cand = np.flatnonzero(c % 8 < 7)
    idx = rng.choice(cand, size=count, replace=False)
    X = X0.copy()
    X[0, idx] = (c[idx] + 1.5) * h
    return X


def _scattered(wl, X0, seed, count):
    """X0 with `count` markers moved by up to 1.5 cells in random directions."""
    rng = np.random.default_rng(seed)
    h = wl.L / wl.N
    X = X0.copy()
    idx = rng.choice(wl.M, size=count, replace=False)
    X[:, idx] += rng.uniform(-1.5 * h, 1.5 * h, size=(3, count))
    return X


@pytest.mark.parametrize("case", ["helix_tiny", "halfcube_tiny", "helix128"])
def test_partition_follows_cell_changes(ibm, oracle_mod, case):
    wl = {"helix_tiny": W.tiny_helix, "halfcube_tiny": W.tiny_halfcube, "helix128": W.config2}[case]()
    announce("bin reuse", case, wl.N, wl.nz, wl.M)
    ctx = ibm.Context(wl, "fp32")
    X0 = wl.X0
    X1 = _moved(wl, X0, seed=5)
    Xt = _within_tiles(wl, X0, seed=6)
    Xs = _scattered(wl, X0, seed=7, count=min(3000, wl.M // 2))
    Xm = _scattered(wl, X0, seed=8, count=wl.M // 2 if wl.M > 9000 else wl.M)   # above 4096 movers
    # build, keep, change, keep, change back, change, within tiles, scattered, many
    for X in (X0, X0, X1, X1, X0, X1, X0, Xt, Xt, X0, Xs, X0, Xm, Xs, Xm, X0):
        _check_bin(ctx, oracle_mod, wl, X)
    # a context that rebuilds every time agrees
    ctx2 = ibm.Context(wl, "fp32")
    ctx2.bin_reuse(False)
    for X in (X1, X1, X0):
        _check_bin(ctx2, oracle_mod, wl, X)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("speed", [0.3, 0.004])
def test_steps_with_reuse_equal_steps_that_rebuild(ibm, prec, speed):
    """Markers carried across cells by a uniform flow of `speed` cells per
    step: at 0.3 most markers change cell every step (full sorts), at 0.004 a
    few do (the markers are moved into place, some across tiles); reuse on
    and off give bitwise the same trajectory."""
    wl = W.tiny_helix()
    h = wl.L / wl.N
    announce("bin reuse steps", prec, speed, wl.N, wl.M)
    out = []
    for reuse in (True, False):
        ctx = ibm.Context(wl, prec)
        ctx.bin_reuse(reuse)
        X = dev(wl.X0)
        u = ctx.new_grid()
        u[0] += speed * h / wl.dt
        u[2] += 0.2 * speed * h / wl.dt
        for n in range(12):
            ctx.step(X, u, n * wl.dt)
        torch.cuda.synchronize()
        out.append((X.clone(), u.clone()))
    (Xa, ua), (Xb, ub) = out
    assert torch.equal(Xa, Xb) and torch.equal(ua, ub)
    # the markers did cross cells
    c0 = np.floor(wl.X0 / h)
    c1 = np.floor(host(Xa) / h)
    crossed = (c0 != c1).any(axis=0).sum()
    assert crossed > (wl.M // 2 if speed > 0.1 else 10)
