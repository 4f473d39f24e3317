"""Diagnostics of the paper's experiments (Sec. 5): the basilar membrane's
displacement along its centre line, recorded every few steps, and its
envelope (the largest displacement each point reaches).

The displacement is taken along the membrane's normal, the direction in
which it is driven to move; the library's ``ib_probe`` computes it on the GPU
for the chosen markers each time it is called, and keeps the running maximum.
"""
from __future__ import annotations

import numpy as np
import torch


def bm_centre_line(wl):
    """Marker ids of the membrane's centre line (the middle position across its
    width at every station along its length) and the unit normal of the
    membrane there, from the reference shape: the cross product of the tangent
    along the length and the direction across the width."""
    nb1, nb2, first = wl.meta["bm_along"], wl.meta["bm_across"], wl.meta["bm_first"]
    st = np.arange(nb1)
    mid = nb2 // 2
    idx = first + st * nb2 + mid
    Y = wl.X_ref
    along = Y[:, first + np.minimum(st + 1, nb1 - 1) * nb2 + mid] - Y[:, first + np.maximum(st - 1, 0) * nb2 + mid]
    across = Y[:, first + st * nb2 + nb2 - 1] - Y[:, first + st * nb2]
    n = np.cross(along.T, across.T).T
    n /= np.linalg.norm(n, axis=0)
    return idx.astype(np.int32), np.ascontiguousarray(n)


def run_with_output(ctx, wl, X, u, n_steps: int, every: int = 10, t0_step: int = 0, path=None):
    """Run ``n_steps`` time steps from (X, u) (advanced in place) and record the
    centre line's normal displacement every ``every`` steps.

    Returns a dict with ``step`` (the step count of each record), ``disp``
    (records x stations), ``envelope`` (stations: the largest |displacement|
    over the recorded steps) and ``station_s`` (arc-length position of each
    station); with ``path`` the same arrays are written to an ``.npz`` file."""
    idx_h, n_h = bm_centre_line(wl)
    dev = X.device
    idx = torch.as_tensor(idx_h, device=dev)
    dirs = torch.as_tensor(n_h, dtype=torch.float64, device=dev).contiguous()
    X0 = torch.as_tensor(wl.X0, dtype=torch.float64, device=dev).contiguous()
    env = torch.zeros(len(idx_h), dtype=torch.float64, device=dev)
    steps, recs = [], []
    for k in range(n_steps):
        ctx.step(X, u, (t0_step + k) * wl.dt)
        if (k + 1) % every == 0:
            recs.append(ctx.probe(X, X0, idx, dirs, env=env).cpu().numpy())
            steps.append(t0_step + k + 1)
    out = {"step": np.asarray(steps, dtype=np.int64),
           "disp": np.asarray(recs).reshape(len(recs), len(idx_h)),
           "envelope": env.cpu().numpy(),
           "station_s": np.linspace(0.0, 1.0, wl.meta["bm_along"])}
    if path is not None:
        np.savez(path, **out)
    return out
