"""Helpers for GPU tests: move seeded numpy inputs to the device and back."""
import numpy as np


def to_dev(a: np.ndarray):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(-1).copy())
    return t.to("cuda")


def from_dev(t, dtype, shape):
    return t.cpu().numpy().view(dtype).reshape(shape)


def packed_vis(acc, nchan, ninput):
    """int32 device accumulator -> numpy int64 [F][P][2]."""
    P = ninput * (ninput + 1) // 2
    return acc.cpu().numpy().astype(np.int64).reshape(nchan, P, 2)


def banner(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
