"""GPU: the step replayed as a HIP graph (ib_graph_enable) against the same
step launched kernel by kernel.  The kernels are deterministic (no atomics,
fixed summation orders), so every replay must agree bitwise with the eager
step at the same time t; the drive amplitude changes every step, so a replay
that kept a stale amplitude would differ.  Between replays the test does its
own eager work (host copies, a synchronisation, an eager step on another
context)."""
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


def _eager_states(ibm, wl, prec, n0, n_steps):
    ctx = ibm.Context(wl, prec)
    X = dev(wl.X0)
    u = ctx.new_grid()
    out = []
    for n in range(n0, n0 + n_steps):
        ctx.step(X, u, n * wl.dt)
        torch.cuda.synchronize()
        out.append((host(X), host(u)))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", ["shell32", "helix_tiny", "helix128", "halfcube64"])
def test_graph_replays_match_eager(ibm, prec, case):
    wl = {"shell32": W.config1, "helix_tiny": W.tiny_helix, "helix128": W.config2,
          "halfcube64": lambda: W.tiny_halfcube(64)}[case]()
    n0, n = 1, 6
    announce("graph replays", case, prec)
    ref = _eager_states(ibm, wl, prec, n0, n)
    ctx = ibm.Context(wl, prec)
    ctx.graph_enable(True)
    other = ibm.Context(wl, prec)           # eager work between the replays
    Xo, uo = dev(wl.X0), other.new_grid()
    X = dev(wl.X0)
    u = ctx.new_grid()
    for k in range(n):
        ctx.step(X, u, (n0 + k) * wl.dt)
        other.step(Xo, uo, 0.5 * wl.dt)
        torch.cuda.synchronize()
        assert np.array_equal(host(X), ref[k][0]), (case, prec, k)
        assert np.array_equal(host(u), ref[k][1]), (case, prec, k)
    cap, lau = ctx.graph_stats()
    assert (cap, lau) == (1, n), (cap, lau)


def test_graph_recaptures_on_new_pointers_and_material(ibm):
    wl = W.tiny_helix()
    announce("graph recapture")
    ref = _eager_states(ibm, wl, "fp32", 0, 4)
    ctx = ibm.Context(wl, "fp32")
    ctx.graph_enable(True)
    X = dev(wl.X0)
    u = ctx.new_grid()
    ctx.step(X, u, 0.0)
    ctx.step(X, u, wl.dt)
    # new arrays holding the same state: a second capture, same results
    X2, u2 = X.clone(), u.clone()
    ctx.step(X2, u2, 2 * wl.dt)
    # a stiffness array with the same values: the material pointer changes, the graph is dropped
    ctx.set_stiffness(ctx.k.clone())
    ctx.step(X2, u2, 3 * wl.dt)
    torch.cuda.synchronize()
    assert np.array_equal(host(X2), ref[3][0]) and np.array_equal(host(u2), ref[3][1])
    assert ctx.graph_stats() == (3, 4)
    # off: eager launches again, the same trajectory
    ctx.graph_enable(False)
    X3, u3 = dev(wl.X0), ctx.new_grid()
    for k in range(4):
        ctx.step(X3, u3, k * wl.dt)
    torch.cuda.synchronize()
    assert np.array_equal(host(X3), ref[3][0]) and ctx.graph_stats() == (3, 4)


def test_graph_with_force_output(ibm, oracle_mod):
    """F_lag_out is part of the captured launches: each replay writes f^n."""
    wl = W.tiny_helix()
    announce("graph F_out")
    ctx = ibm.Context(wl, "fp64")
    ctx.graph_enable(True)
    X = dev(wl.X0)
    u = ctx.new_grid()
    F = torch.empty_like(X)
    m = oracle_mod.Model(wl)
    for k in range(3):
        Xk = host(X)
        ctx.step(X, u, (k + 1) * wl.dt, F_out=F)
        torch.cuda.synchronize()
        Fo = oracle_mod.force(m, Xk, (k + 1) * wl.dt)
        assert np.abs(host(F) - Fo).max() <= 1e-12 * np.abs(Fo).max()
