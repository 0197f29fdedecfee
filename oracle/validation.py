"""Closed forms of the paper's validation problems -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import step


def poiseuille_velocity(y, t, D, f0, mu, rho, terms=2000):
    """Channel flow from rest under a uniform force f0 between no-slip walls y = 0 and y = D
    (Sec. 6.2.2, eq. poiseuille_velo): the sine series over odd modes lambda = (2k+1) pi / D."""
    y = np.asarray(y, dtype=np.float64)
    u = np.zeros_like(y)
    for k in range(terms):
        n = 2 * k + 1
        lam = n * np.pi / D
        u += 4.0 * f0 / (mu * lam * lam * n * np.pi) * (1.0 - np.exp(-mu / rho * lam * lam * t)) * np.sin(lam * y)
    return u


def poiseuille_flux(t, D, f0, mu, rho, terms=2000):
    """Flux through the channel, the integral of poiseuille_velocity over [0, D] (eq. poiseuille_flux)."""
    phi = 0.0
    for k in range(terms):
        n = 2 * k + 1
        lam = n * np.pi / D
        phi += 8.0 * f0 / (mu * lam ** 3 * n * np.pi) * (1.0 - np.exp(-mu / rho * lam * lam * t))
    return phi


def poiseuille_steady_flux(D, f0, mu):
    """Phi_eq = f0 D^3 / (12 mu) (eq. steady_poiseuille_flux)."""
    return f0 * D ** 3 / (12.0 * mu)


def effective_width(flux_eq, f0, mu):
    """Channel width D_e = (12 mu Phi_eq / f0)^(1/3) that carries the steady flux Phi_eq."""
    return (12.0 * mu * flux_eq / f0) ** (1.0 / 3.0)


def circle_pressure_jump(F, r, L):
    """Normal-force circle in Stokes flow (Sec. 6.1): zero-mean pressure outside (p1) and inside (p2) a
    circle of radius r carrying an outward normal force F per unit theta."""
    return F / r * np.pi * r * r / (L * L), -F / r * (L * L - np.pi * r * r) / (L * L)


def poiseuille_steady_velocity(y, D, f0, mu):
    """u_eq(y) = f0 y (D - y) / (2 mu) (eq. steady_poiseuille_velo)."""
    y = np.asarray(y, dtype=np.float64)
    return f0 / (2.0 * mu) * y * (D - y)


def steady_wall_system(A, Nb, f0, L, rcond=1e-8):
    """Equilibrium of a fixed straight wall in Stokes flow driven by a uniform force f0 along x
    (Sec. 6.2.2, the steady channel with D = L: one wall at y = 0 and periodicity).

    A is the (2 Nb, 2 Nb) matrix of the Stokes map from wall strengths to wall velocities (unit
    strength on one component of one point per column, rows and columns point-major).  Unknowns:
    the strengths S and the mean flow ubar, which the periodic Stokes solve leaves free.  Equations:
    no slip at every wall point, A S + ubar = 0, and the balance of the k = 0 mode,
    sum_i S_i + f0 L^2 e_x = 0.  A has null directions (the alternating pattern sits on the zeroed
    Nyquist mode; a uniform normal load is carried by pressure), so the minimum-norm solution is
    returned, with singular values below rcond relative cut.  Returns (S (Nb, 2), ubar (2,))."""
    n = 2 * Nb
    M = np.zeros((n + 2, n + 2))
    M[:n, :n] = A
    M[0:n:2, n] = 1.0
    M[1:n:2, n + 1] = 1.0
    M[n, 0:n:2] = 1.0
    M[n + 1, 1:n:2] = 1.0
    rhs = np.zeros(n + 2)
    rhs[n] = -f0 * L * L
    sol = np.linalg.lstsq(M, rhs, rcond=rcond)[0]
    return sol[:n].reshape(Nb, 2), sol[n:]


def steady_channel_errors(ux, ubar_x, N, f0, mu, L):
    """Relative 2-norm errors of the steady channel velocity ux[y][x] (grid values, mean flow
    included) against eq. steady_poiseuille_velo with width D = L, and with the effective width
    D_e from the flux; the effective channel is centred, its walls at y = Delta_e / 2 and
    L - Delta_e / 2, zero flow outside.  Returns (err_D, err_De, D_e)."""
    y = np.arange(N) * (L / N)
    ue = np.broadcast_to(poiseuille_steady_velocity(y, L, f0, mu)[:, None], ux.shape)
    err_d = np.linalg.norm(ux - ue) / np.linalg.norm(ue)
    De = effective_width(ubar_x * L, f0, mu)
    off = 0.5 * (L - De)
    yy = y - off
    ue2 = np.where((yy > 0.0) & (yy < De), poiseuille_steady_velocity(yy, De, f0, mu), 0.0)
    ue2 = np.broadcast_to(ue2[:, None], ux.shape)
    err_de = np.linalg.norm(ux - ue2) / np.linalg.norm(ue2)
    return err_d, err_de, De


def wall_points(N, L):
    """The wall y = 0 sampled at the grid spacing, N_b = N (Sec. 6.2.2, steady channel)."""
    return np.stack([np.arange(N) * (L / N), np.zeros(N)], axis=1)


def steady_channel(N, f0, mu, L=1.0):
    """Steady channel with D = L on an N x N grid: assemble the wall's Stokes matrix column by
    column from the oracle's Stokes map, solve steady_wall_system, and return
    (S, ubar, uhat, ux) with uhat the coefficients of the strengths' flow (zero mean) and ux[y][x]
    the x velocity on the grid, mean flow included."""
    X = wall_points(N, L)
    A = np.zeros((2 * N, 2 * N))
    for j in range(N):
        for a in range(2):
            S = np.zeros((N, 2))
            S[j, a] = 1.0
            A[:, 2 * j + a] = step.stokes_map(X, S, (N, N), L, mu)[0].ravel()
    S, ubar = steady_wall_system(A, N, f0, L)
    _, uhat = step.stokes_map(X, S, (N, N), L, mu)
    ux = np.real(np.fft.ifft2(uhat[0])) * (N * N) + ubar[0]
    return S, ubar, uhat, ux
