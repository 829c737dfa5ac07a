"""Helpers shared by the GPU tests: device upload and error measures."""
import sys

import numpy as np
import torch


def say(*msg):
    print(*msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """Norm-wise relative difference ||a - b||_F / ||b||_F."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
