"""Helpers shared by the GPU parity tests (numpy <-> device tensors)."""
import numpy as np
import torch

TOL = {"fp64": 1e-10, "mixed": 1e-4}


def dev():
    return torch.device("cuda:0")


def to_dev(x, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).ravel(), dtype=dt, device=dev())


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def empty(n, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.full((int(n),), float("nan"), dtype=dt, device=dev())


def zeros(n, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.zeros(int(n), dtype=dt, device=dev())


def rel(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def flag(msg):
    """Name the case on stdout before a GPU step (flushes)."""
    print(msg, flush=True)
