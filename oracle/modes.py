"""Truncated Fourier mode sets K_N (Sec. 3.1, eq. kNh) -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np


def mode_numbers(N):
    """Integer mode numbers m of K_N in FFT order (k = 2*pi*m/L).

    Even N: m in {-N/2, ..., N/2-1}; odd N: m in {-(N-1)/2, ..., (N-1)/2}
    (eq. kNh).  FFT order lists m = 0, 1, ... first, then the negative modes,
    so the zero mode is the first entry (Sec. 3.1, remark after eq.
    fourier_spectral_sol).
    """
    N = int(N)
    npos = (N + 1) // 2
    i = np.arange(N)
    return np.where(i < npos, i, i - N)


def spectral_shape(Ns):
    """numpy shape of a scalar spectral array for per-axis mode counts Ns=(N_x, N_y[, N_z])."""
    return tuple(int(n) for n in reversed(Ns))


def wavevector(Ns, L):
    """Per-axis wavenumber arrays k_a = 2*pi*m_a/L broadcastable to spectral_shape(Ns).

    Returns a list [k_x, k_y, (k_z)] in physical-axis order.
    """
    d = len(Ns)
    out = []
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = int(Ns[a])
        out.append((2.0 * np.pi / L) * mode_numbers(Ns[a]).astype(np.float64).reshape(shape))
    return out


def ksquared(Ns, L):
    """|k|^2 on K_N (true value, 0 at k = 0)."""
    k = wavevector(Ns, L)
    out = np.zeros(spectral_shape(Ns))
    for ka in k:
        out = out + ka * ka
    return out


def nyquist_mask(Ns):
    """Boolean mask of modes with any component m_a = -N_a/2 (even N_a only).

    Reading of the paper: for even N the set K_N holds -N/2 but not +N/2
    (eq. kNh), so a real field cannot keep that mode; the fluid update zeroes
    it, leaving the symmetric set of N-1 modes per axis that Sec. 4
    analyses for odd N.
    """
    d = len(Ns)
    mask = np.zeros(spectral_shape(Ns), dtype=bool)
    for a in range(d):
        n = int(Ns[a])
        if n % 2 == 0:
            shape = [1] * d
            shape[d - 1 - a] = n
            mask = mask | (mode_numbers(n) == -n // 2).reshape(shape)
    return mask
