"""GPU: checkpoint and resume.

The state of a run is (X, u, n): the step is a function of the marker state,
the velocity and the time t = n dt alone (the partition and every scratch
array are rebuilt from them).  Saving (X, u, n) to a file, dropping the
context and continuing in a new one reproduces the uninterrupted run bitwise.
"""
import numpy as np
import pytest
import torch

from paper_math_0301321_amd import workloads as W
from tests.gpu_util import announce, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ibm():
    from paper_math_0301321_amd import ib
    ib.load_library()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return ib


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", ["helix_tiny", "halfcube_tiny"])
@pytest.mark.parametrize("graph", [False, True])
def test_resume_from_saved_state_is_bitwise(ibm, tmp_path, prec, case, graph):
    wl = W.tiny_helix() if case == "helix_tiny" else W.tiny_halfcube()
    announce("resume", case, prec, "graph" if graph else "eager", wl.N, wl.nz, wl.M)
    n_total, n_save = 10, 6
    u0 = 0.3 * W.smooth_field(wl.N, seed=11, Nz=wl.nz)
    fdt = torch.float32 if prec == "fp32" else torch.float64

    def new_ctx():
        ctx = ibm.Context(wl, prec)
        if graph:
            ctx.graph_enable(True)
        return ctx

    # the uninterrupted run
    ctx = new_ctx()
    X, u = dev(wl.X0), dev(u0, fdt)
    for n in range(n_total):
        ctx.step(X, u, n * wl.dt)
    torch.cuda.synchronize()
    X_ref, u_ref = X.clone(), u.clone()
    del ctx

    # n_save steps, the state to a file, a fresh context, the rest
    ctx = new_ctx()
    X, u = dev(wl.X0), dev(u0, fdt)
    for n in range(n_save):
        ctx.step(X, u, n * wl.dt)
    torch.cuda.synchronize()
    path = tmp_path / "state.npz"
    np.savez(path, X=X.cpu().numpy(), u=u.cpu().numpy(), n=np.int64(n_save))
    del ctx, X, u
    torch.cuda.synchronize()
    with np.load(path) as f:
        Xs, us, n0 = f["X"], f["u"], int(f["n"])
    ctx = new_ctx()
    X = torch.as_tensor(Xs, device="cuda").contiguous()
    u = torch.as_tensor(us, device="cuda").contiguous()
    assert X.dtype == torch.float64 and u.dtype == fdt
    for n in range(n0, n_total):
        ctx.step(X, u, n * wl.dt)
    torch.cuda.synchronize()
    assert torch.equal(X, X_ref) and torch.equal(u, u_ref)
    assert not torch.equal(X_ref, dev(wl.X0))        # the run moved the markers
