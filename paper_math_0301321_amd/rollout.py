"""Differentiable multi-step rollout of the IB time step (checkpointed adjoint).

``IBRollout.apply(k, X0, u0, ctx, n_steps, ckpt_every)`` runs ``n_steps`` time
steps on the GPU with per-marker stiffness ``k`` and returns the final state
``(X_T, u_T)``.  Its backward pass is the hand-written adjoint step of the
library (``ib_adjoint_step``) run in reverse: the forward pass keeps the state
every ``ckpt_every`` steps; the backward pass re-runs each segment from its
checkpoint, keeping that segment's states, and then walks the segment
backwards.  Gradients flow to ``k`` (the stiffness multipliers of the
material force), ``X0`` and ``u0``.

With ``convect = 1`` the upwind advection is differentiated with each branch
frozen at the side the step's starting velocity selects; the segment replay
keeps that velocity for the adjoint.
"""
from __future__ import annotations

import torch


class IBRollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, k, X0, u0, ibctx, n_steps: int, ckpt_every: int, t0: float = 0.0):
        if n_steps < 0 or ckpt_every < 1:
            raise ValueError("need n_steps >= 0 and ckpt_every >= 1")
        dt = float(ibctx.wl.dt)
        kk = k.detach().contiguous()
        ibctx.set_stiffness(kk)
        X = X0.detach().clone().contiguous()
        u = u0.detach().clone().contiguous()
        ckpts = []
        for n in range(n_steps):
            if n % ckpt_every == 0:
                ckpts.append((n, X.clone(), u.clone()))
            ibctx.step(X, u, t0 + n * dt)
        fctx.ibctx, fctx.n_steps, fctx.ckpt_every, fctx.t0, fctx.dt = ibctx, n_steps, ckpt_every, t0, dt
        fctx.ckpts = ckpts
        fctx.save_for_backward(kk)
        return X, u

    @staticmethod
    def backward(fctx, gX, gu):
        (kk,) = fctx.saved_tensors
        ibctx = fctx.ibctx
        ibctx.set_stiffness(kk)
        M = kk.numel()
        Xbar = (gX if gX is not None else torch.zeros((3, M), dtype=torch.float64, device=kk.device)).clone()
        ubar = (gu if gu is not None else ibctx.new_grid()).to(ibctx.fluid_dtype).clone().contiguous()
        Xbar = Xbar.contiguous()
        kbar = torch.zeros(M, dtype=torch.float64, device=kk.device)
        dt, t0 = fctx.dt, fctx.t0
        for start, Xc, uc in reversed(fctx.ckpts):
            end = min(start + fctx.ckpt_every, fctx.n_steps)
            X, u = Xc.clone(), uc.clone()
            seg = []
            conv = ibctx.convect != 0
            for n in range(start, end):
                Xn = X.clone()
                un = u.clone() if conv else None
                ibctx.step(X, u, t0 + n * dt)
                seg.append((Xn, un, u.clone()))      # X^n, u^n (with advection), u^{n+1}
            for n in reversed(range(start, end)):
                Xn, un, unp1 = seg[n - start]
                ibctx.adjoint_step(Xn, unp1, t0 + n * dt, Xbar, ubar, kbar, u_n=un)
        return kbar, Xbar, ubar, None, None, None, None


def rollout(k, X0, u0, ibctx, n_steps: int, ckpt_every: int, t0: float = 0.0):
    """Functional form of :class:`IBRollout`."""
    return IBRollout.apply(k, X0, u0, ibctx, n_steps, ckpt_every, t0)


def membrane_loss(X, X_ref, idx):
    """Mean-square displacement of the markers ``idx``: (1/|W|) sum |X_q - X_ref_q|^2."""
    d = X[:, idx] - X_ref[:, idx]
    return (d * d).sum() / idx.numel()
