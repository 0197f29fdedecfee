"""Shared helpers of the GPU parity tests: device transfer, layouts, and a guard that fails
loudly (instead of skipping) when a GPU is visible but the HIP library is not built."""

import sys

import numpy as np
import torch

DEV = "cuda:0"


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def half(full, Nx):
    """Half spectrum (m_x = 0..floor(Nx/2)) of full FFT-ordered arrays (last axis x)."""
    return np.ascontiguousarray(full[..., : Nx // 2 + 1])


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def cdtype(prec):
    return torch.complex128 if prec == "f64" else torch.complex64


def rdtype(prec):
    return torch.float64 if prec == "f64" else torch.float32
