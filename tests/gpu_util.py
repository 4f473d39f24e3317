"""Helpers for the GPU parity tests: device transfer and error measures."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


def host(t):
    return t.detach().double().cpu().numpy()


def rel_max(got, want):
    """max |got - want| / max |want| (0/0 -> 0)."""
    got, want = np.asarray(got, dtype=np.float64), np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max() if want.size else 0.0
    err = np.abs(got - want).max() if want.size else 0.0
    return 0.0 if scale == 0.0 and err == 0.0 else err / (scale if scale > 0 else 1.0)


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)
