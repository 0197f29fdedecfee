"""Closed forms of the paper's validation problems -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np


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
