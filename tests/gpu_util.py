"""Helpers for the GPU parity tests (torch for device memory only)."""
import numpy as np
import torch


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
