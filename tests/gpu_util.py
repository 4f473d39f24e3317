"""Helpers for the GPU parity tests: device transfer and error measures."""
import numpy as np
import torch

from paper_math_0301321_amd import workloads as W


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


def host(t):
    return t.detach().double().cpu().numpy()


def rel_max(got, want):
    """max |got - want| / max |want|.

    Refuses an empty or all-zero reference: a comparison against zeros would
    pass without comparing anything."""
    got, want = np.asarray(got, dtype=np.float64), np.asarray(want, dtype=np.float64)
    if got.shape != want.shape:
        raise AssertionError(f"shape mismatch: {got.shape} vs {want.shape}")
    scale = np.abs(want).max() if want.size else 0.0
    if not scale > 0.0:
        raise AssertionError("the reference is empty or all zeros: nothing would be compared")
    return np.abs(got - want).max() / scale


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)


def run_from(ibm, wl, prec, X0, u0, n0, n_steps):
    """n_steps GPU steps from (X0, u0) at t = n0 dt."""
    ctx = ibm.Context(wl, prec)
    X = dev(X0)
    u = dev(u0, (torch.float32 if prec == "fp32" else torch.float64)) if u0 is not None else ctx.new_grid()
    for n in range(n0, n0 + n_steps):
        ctx.step(X, u, n * wl.dt)
    torch.cuda.synchronize()
    return host(X), host(u)


FULL_SIZE_STARTS = {
    # from rest: the first step has no force (every term at rest, drive sin 0),
    # the drive is on from the second; three steps
    "rest": dict(u0=None, n0=0, n_steps=3),
    # a smooth random flow of amplitude 0.5 at t = 3 dt: advection at full size,
    # markers carried off their reference shape (tethers, stretch, bend loaded)
    "flow": dict(u0="smooth", n0=3, n_steps=2),
}


def full_size_case(oracle_mod, wl, start):
    """Oracle trajectory for one of FULL_SIZE_STARTS; returns (u0, Xo, uo)."""
    cfg = FULL_SIZE_STARTS[start]
    u0 = 0.5 * W.smooth_field(wl.N, seed=61, Nz=wl.nz) if cfg["u0"] == "smooth" else None
    Xo, uo = oracle_mod.run(wl, cfg["n_steps"], u=u0, t0_step=cfg["n0"])
    # the comparison must not be vacuous
    assert np.abs(uo).max() > 1e-3 and np.abs(Xo - wl.X0).max() > 1e-7, (np.abs(uo).max(), np.abs(Xo - wl.X0).max())
    return u0, Xo, uo
