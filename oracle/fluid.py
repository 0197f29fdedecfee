"""Fourier-space fluid operators -- oracle side.

Test infrastructure only (see the package docstring).

All vector fields are full-spectrum arrays of shape (d, N_z, N_y, N_x) (2D:
(2, N_y, N_x)) over K_N in FFT order.
"""

import numpy as np
import scipy.fft as sfft

from .modes import mode_numbers, wavevector, ksquared, nyquist_mask


def project(P, Ns, L):
    """Leray projection Q = P - k (k.P)/|k|^2 with |k|^2 := 1 at k = 0 (Alg. 2; Sec. 3.1).

    At k = 0 the projection is the identity (k = 0 there), as the paper
    obtains by setting the first entry of the |k|^2 matrix to one.
    """
    k = wavevector(Ns, L)
    k2 = ksquared(Ns, L)
    k2 = np.where(k2 == 0.0, 1.0, k2)
    kdotP = sum(k[a] * P[a] for a in range(len(Ns)))
    return np.stack([P[a] - k[a] * kdotP / k2 for a in range(len(Ns))])


def stokeslet(fhat, Ns, L, mu):
    """Steady periodic Stokes solve uhat = (1/mu)(I/|k|^2 - k k^T/|k|^4) fhat (Sec. 6.1, eq. stokeslet).

    The k = 0 mode of uhat is set to zero (the mean flow is undetermined by the
    steady equations; the paper requires zero net force, eq. force_vanish).
    """
    k = wavevector(Ns, L)
    k2 = ksquared(Ns, L)
    nz = k2 != 0.0
    k2s = np.where(nz, k2, 1.0)
    kdotf = sum(k[a] * fhat[a] for a in range(len(Ns)))
    out = np.stack([np.where(nz, (fhat[a] / k2s - k[a] * kdotf / (k2s * k2s)) / mu, 0.0)
                    for a in range(len(Ns))])
    return out


def stokes_pressure(fhat, Ns, L):
    """phat = k.fhat / (i |k|^2), phat(0) = 0 (Sec. 6.1, eq. stokeslet, second line)."""
    k = wavevector(Ns, L)
    k2 = ksquared(Ns, L)
    nz = k2 != 0.0
    kdotf = sum(k[a] * fhat[a] for a in range(len(Ns)))
    return np.where(nz, kdotf / (1j * np.where(nz, k2, 1.0)), 0.0)


def pressure(fhat, uhat, Ns, L, rho, npad=None):
    """phat = -i k.(fhat - rho shat(uhat)) / |k|^2, phat(0) = 0 (Sec. 3, eq. pressure_poisson_k), shat the
    advective nonlinear term of eq. nonlinear_physical (three-halves rule); uhat = None gives the
    Stokes pressure -i k.fhat / |k|^2."""
    k = wavevector(Ns, L)
    k2 = ksquared(Ns, L)
    nz = k2 != 0.0
    g = np.array(fhat, dtype=np.complex128)
    if uhat is not None:
        g = g - rho * nonlinear(uhat, Ns, L, npad)
    kg = sum(k[a] * g[a] for a in range(len(Ns)))
    return np.where(nz, -1j * kg / np.where(nz, k2, 1.0), 0.0)


def _embed(a, Ns, npad):
    """Zero-pad a K_N array (FFT order) into a K_Npad array (centred padding, Sec. 3.1)."""
    d = len(Ns)
    out = np.zeros(tuple(reversed(npad)), dtype=np.complex128)
    idx = [np.mod(mode_numbers(Ns[d - 1 - b]), npad[d - 1 - b]) for b in range(d)]
    out[np.ix_(*idx)] = a
    return out


def _truncate(a, Ns, npad):
    """Restrict a K_Npad array to the modes of K_N (operator T_N, eq. nonlinear_kspace)."""
    d = len(Ns)
    idx = [np.mod(mode_numbers(Ns[d - 1 - b]), npad[d - 1 - b]) for b in range(d)]
    return a[np.ix_(*idx)]


def default_pad(Ns):
    """Padded length per axis: 2N, which satisfies Ntilde > 3N/2 (Sec. 3.1) for any input."""
    return tuple(2 * int(n) for n in Ns)


def nonlinear(uhat, Ns, L, npad=None):
    """Dealiased advective term shat = T_N H( H^-1(uhat) . H^-1(i k uhat) ) (eqs. nonlinear_physical, nonlinear_kspace).

    Three-halves rule: zero-pad to Ntilde > 3N/2 per axis, inverse FFT to
    physical values, multiply s_alpha = sum_beta u_beta d_beta u_alpha, FFT
    back, truncate to K_N.  H^-1 evaluates the Fourier series on the padded
    grid, so H^-1 = Ntilde^d * ifftn and H = fftn / Ntilde^d.
    """
    d = len(Ns)
    npad = default_pad(Ns) if npad is None else tuple(int(n) for n in npad)
    for n, p in zip(Ns, npad):
        if 2 * p <= 3 * int(n):
            raise ValueError("padded length must exceed 3N/2")
    kpad = wavevector(npad, L)  # wavenumbers of K_Npad, indices agree with the embedding
    vol = float(np.prod(npad))
    axes = tuple(range(d))
    u = [sfft.ifftn(_embed(uhat[a], Ns, npad), axes=axes, workers=-1) * vol for a in range(d)]
    out = []
    for al in range(d):
        ua_hat = _embed(uhat[al], Ns, npad)
        s = np.zeros_like(u[0])
        for be in range(d):
            grad = sfft.ifftn(1j * kpad[be] * ua_hat, axes=axes, workers=-1) * vol
            s += u[be] * grad
        out.append(_truncate(sfft.fftn(s, axes=axes, workers=-1) / vol, Ns, npad))
    return np.stack(out)


def nonlinear_convolution(uhat, Ns, L):
    """shat by the truncated convolution sum over K_N x K_N (Sec. 3.1; tiny N only).

    shat_alpha(k) = sum_{k1 + k2 = k} sum_beta uhat_beta(k1) * (i k2_beta) uhat_alpha(k2),
    for k, k1, k2 in K_N.  O(N^{2d}) -- the cost the paper avoids with FFTs.
    """
    d = len(Ns)
    shp = tuple(reversed([int(n) for n in Ns]))
    ms = [mode_numbers(Ns[a]) for a in range(d)]
    # flat list of modes (physical order) matching C order of spectral arrays
    grids = np.meshgrid(*[ms[d - 1 - b] for b in range(d)], indexing="ij")
    mflat = np.stack([grids[d - 1 - a].ravel() for a in range(d)], axis=1)
    lookup = {tuple(m): q for q, m in enumerate(mflat)}
    uf = uhat.reshape(d, -1)
    out = np.zeros_like(uf)
    kfac = 2.0 * np.pi / L
    for q1, m1 in enumerate(mflat):
        for q2, m2 in enumerate(mflat):
            q = lookup.get(tuple(m1 + m2))
            if q is None:
                continue
            for al in range(d):
                acc = 0j
                for be in range(d):
                    acc += uf[be, q1] * (1j * kfac * m2[be]) * uf[al, q2]
                out[al, q] += acc
    return out.reshape((d,) + shp)


def vhat(fhat, uhat, Ns, L, rho, npad=None):
    """V-hat(fhat, uhat) = (I - k k^T/|k|^2)(fhat/rho - shat(uhat)) (Alg. 2; eq. fourier_spectral_sol)."""
    P = fhat / rho - nonlinear(uhat, Ns, L, npad)
    return project(P, Ns, L)


def zero_nyquist(a, Ns):
    """Zero every mode with a component m_a = -N_a/2 (even N); see modes.nyquist_mask."""
    out = a.copy()
    out[..., nyquist_mask(Ns)] = 0.0
    return out


def ns_update(fhat, uhat, Ns, L, rho, mu, dt, npad=None):
    """The two Fourier updates of one Alg. 1 step (eqs. spatial_2 and spatial_3).

    uhat_half = (dt/2 V(fhat, uhat) + uhat) / (1 + a)
    uhat_new  = (dt V(fhat, uhat_half) + (1 - a) uhat) / (1 + a),  a = mu dt |k|^2 / (2 rho).

    Reading: the |k|^2 := 1 substitution at k = 0 belongs to the projection
    only; the viscous factor uses the true |k|^2 = 0 there, which is what the
    momentum identity of Sec. 5.3 requires.  Both results are Nyquist-zeroed
    (modes.nyquist_mask).  Returns (uhat_half, uhat_new).
    """
    a = mu * dt * ksquared(Ns, L) / (2.0 * rho)
    uh = (0.5 * dt * vhat(fhat, uhat, Ns, L, rho, npad) + uhat) / (1.0 + a)
    uh = zero_nyquist(uh, Ns)
    un = (dt * vhat(fhat, uh, Ns, L, rho, npad) + (1.0 - a) * uhat) / (1.0 + a)
    un = zero_nyquist(un, Ns)
    return uh, un
