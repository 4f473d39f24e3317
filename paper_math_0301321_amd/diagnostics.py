"""Diagnostics of the paper's experiments (Sec. 5): the basilar membrane's
displacement along its centre line, recorded every few steps, and its
envelope (the largest displacement each point reaches).

The displacement is taken along the membrane's normal, the direction in
which it is driven to move; the library's ``ib_probe`` computes it on the GPU
for the chosen markers each time it is called, and keeps the running maximum.

The paper's runs also write every material point's position every tenth
step (Sec. 5).  ``run_with_output(positions=path)`` does that into one
``.npy`` array (records x 3 x M, FP64): at each output step the positions are
copied on the device (the next step moves them in place), then to pinned
host memory on a second stream while the following steps run, and written to
the file by a host thread.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

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


class _PositionSink:
    """Overlapped device-to-host output of whole marker arrays into an .npy file.

    Two slots, each a device snapshot, a pinned host buffer and a copy-done
    event: a record is snapshotted on the stream the steps run on, copied to
    the host on a copy stream (default priority) and written by one host
    thread; a slot is reused only after its previous record was written."""

    def __init__(self, path, n_records, M, device, step_stream):
        self.mm = np.lib.format.open_memmap(path, mode="w+", dtype=np.float64, shape=(n_records, 3, M))
        self.step_stream = step_stream
        self.copy_stream = torch.cuda.Stream(device=device)
        self.snap = [torch.empty((3, M), dtype=torch.float64, device=device) for _ in range(2)]
        self.host = [torch.empty((3, M), dtype=torch.float64, pin_memory=True) for _ in range(2)]
        self.done = [torch.cuda.Event() for _ in range(2)]
        self.pending = [None, None]
        self.pool = ThreadPoolExecutor(max_workers=1)
        self.r = 0

    def _write(self, slot, r):
        self.done[slot].synchronize()
        self.mm[r] = self.host[slot].numpy()

    def put(self, X):
        slot = self.r % 2
        if self.pending[slot] is not None:
            self.pending[slot].result()              # its previous record is on disk
        with torch.cuda.stream(self.step_stream):
            self.snap[slot].copy_(X)
        self.copy_stream.wait_stream(self.step_stream)
        with torch.cuda.stream(self.copy_stream):
            self.host[slot].copy_(self.snap[slot], non_blocking=True)
            self.done[slot].record(self.copy_stream)
        self.pending[slot] = self.pool.submit(self._write, slot, self.r)
        self.r += 1

    def close(self):
        for f in self.pending:
            if f is not None:
                f.result()
        self.pool.shutdown()
        self.mm.flush()
        del self.mm


def _ctx_stream(ctx, device):
    """The torch stream object for the stream the context launches on."""
    return torch.cuda.ExternalStream(ctx.stream, device=device) if ctx.stream else torch.cuda.default_stream(device)


def run_with_output(ctx, wl, X, u, n_steps: int, every: int = 10, t0_step: int = 0, path=None, positions=None):
    """Run ``n_steps`` time steps from (X, u) (advanced in place) and record the
    centre line's normal displacement every ``every`` steps.

    Returns a dict with ``step`` (the step count of each record), ``disp``
    (records x stations), ``envelope`` (stations: the largest |displacement|
    over the recorded steps) and ``station_s`` (arc-length position of each
    station); with ``path`` the same arrays are written to an ``.npz`` file.
    With ``positions`` (a path), every marker's position at each recorded step
    is written to that ``.npy`` file as an array (records x 3 x M), the
    device-to-host copies overlapping the following steps."""
    idx_h, n_h = bm_centre_line(wl)
    dev = X.device
    idx = torch.as_tensor(idx_h, device=dev)
    dirs = torch.as_tensor(n_h, dtype=torch.float64, device=dev).contiguous()
    X0 = torch.as_tensor(wl.X0, dtype=torch.float64, device=dev).contiguous()
    env = torch.zeros(len(idx_h), dtype=torch.float64, device=dev)
    sink = None
    if positions is not None:
        sink = _PositionSink(positions, n_steps // every, X.shape[1], dev, _ctx_stream(ctx, dev))
    steps, recs = [], []
    try:
        for k in range(n_steps):
            ctx.step(X, u, (t0_step + k) * wl.dt)
            if (k + 1) % every == 0:
                recs.append(ctx.probe(X, X0, idx, dirs, env=env))
                if sink is not None:
                    sink.put(X)
                steps.append(t0_step + k + 1)
    finally:
        if sink is not None:
            sink.close()
    out = {"step": np.asarray(steps, dtype=np.int64),
           "disp": torch.stack(recs).cpu().numpy() if recs else np.zeros((0, len(idx_h))),
           "envelope": env.cpu().numpy(),
           "station_s": np.linspace(0.0, 1.0, wl.meta["bm_along"])}
    if path is not None:
        np.savez(path, **out)
    return out
