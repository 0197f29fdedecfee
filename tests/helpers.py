"""Small array helpers for tests: layouts and random divergence-free fields (no method arithmetic
beyond what each test states)."""

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def random_real_field_hat(Ns, d, seed):
    """Fourier coefficients (FFT order) of a random real vector field sampled on the N^d grid."""
    rng = np.random.default_rng(seed)
    shp = tuple(reversed([int(n) for n in Ns]))
    u = rng.standard_normal((d,) + shp)
    axes = tuple(range(1, d + 1))
    return np.fft.fftn(u, axes=axes) / float(np.prod(shp))
