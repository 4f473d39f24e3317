"""GPU: the adjoint step is repeatable bitwise.

Every kernel of the adjoint step is a gather with a fixed summation order (no
floating-point atomics), so two adjoint steps from the same state and
cotangents give bitwise the same Xbar, ubar and kbar.  So does an adjoint step
in a fresh context, whose binning of X^n starts from a full sort, against one
in a context that has stepped before, whose partition was updated in place.
"""
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
def test_adjoint_step_repeatable_bitwise(ibm, prec, case):
    wl = W.tiny_helix() if case == "helix_tiny" else W.tiny_halfcube()
    announce("adjoint repeat", case, prec, wl.N, wl.nz, wl.M)
    fdt = torch.float32 if prec == "fp32" else torch.float64
    n0 = 4
    ctx = ibm.Context(wl, prec, convect=1)
    X = dev(wl.X0)
    u = dev(0.3 * W.smooth_field(wl.N, seed=5, Nz=wl.nz), fdt)
    for n in range(n0):
        ctx.step(X, u, n * wl.dt)
    X_n, u_n = X.clone(), u.clone()
    ctx.step(X, u, n0 * wl.dt)                     # u is now u^{n+1}
    g = torch.Generator().manual_seed(9)
    Xb0 = (1e-3 * torch.randn(tuple(X.shape), generator=g, dtype=torch.float64)).cuda()
    ub0 = (1e-3 * torch.randn(tuple(u.shape), generator=g, dtype=torch.float64)).to(fdt).cuda()

    def adjoint(c):
        Xb, ub = Xb0.clone(), ub0.clone()
        kb = torch.zeros(wl.M, dtype=torch.float64, device="cuda")
        c.adjoint_step(X_n, u, n0 * wl.dt, Xb, ub, kb, u_n=u_n)
        torch.cuda.synchronize()
        return Xb, ub, kb

    a = adjoint(ctx)
    b = adjoint(ctx)
    c = adjoint(ibm.Context(wl, prec, convect=1))
    for name, x, y, z in zip(("Xbar", "ubar", "kbar"), a, b, c):
        assert torch.equal(x, y), f"{name}: two adjoint steps in one context differ"
        assert torch.equal(x, z), f"{name}: a fresh context's adjoint step differs"
    # the cotangents did change: the comparison is not between untouched inputs
    assert not torch.equal(a[0], Xb0) and not torch.equal(a[1], ub0)
    assert a[2].abs().max().item() > 0.0
