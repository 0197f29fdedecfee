"""Diagnostics of the FSIB state (Secs. 5.1-5.4, 6.2) -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from .modes import wavevector, ksquared


def net_force(F, w):
    """sum_j w_j F_j: L^d times the zero mode of fhat (Sec. 5.3)."""
    return np.sum((np.asarray(w) * np.ones(F.shape[0]))[:, None] * F, axis=0)


def kinetic_energy(uhat, L, rho):
    """E_K = (rho/2) L^d sum_k |uhat(k)|^2 (Sec. 5.4)."""
    d = uhat.shape[0]
    return 0.5 * rho * float(L) ** d * float(np.sum(np.abs(uhat) ** 2))


def dissipation(uhat, Ns, L, mu):
    """Viscous dissipation rate mu L^d sum_k |k|^2 |uhat(k)|^2 (Sec. 5.4).

    Reading: the paper's final energy law drops the L^d factor that its
    earlier line (eq. kine_energ_derivative) carries; the factor is kept.
    """
    d = uhat.shape[0]
    return mu * float(L) ** d * float(np.sum(ksquared(Ns, L) * np.sum(np.abs(uhat) ** 2, axis=0)))


def power(F, w, U):
    """sum_j w_j F_j . U_j, equal to L^d sum_k fhat(k) . conj(uhat(k)) (eq. pote_energ_derivative)."""
    return float(np.sum((np.asarray(w) * np.ones(F.shape[0]))[:, None] * F * U))


def divergence_residual(uhat, Ns, L):
    """max_k |k . uhat(k)| / max_k |k| |uhat(k)| (Sec. 5.1); 0 for a field without nonzero modes.

    Normalised by the largest mode rather than mode by mode, so that modes that are zero up to
    rounding do not dominate.
    """
    k = wavevector(Ns, L)
    kd = np.abs(sum(k[a] * uhat[a] for a in range(len(Ns))))
    kn = np.sqrt(ksquared(Ns, L))
    un = np.sqrt(np.sum(np.abs(uhat) ** 2, axis=0))
    den = float(np.max(kn * un))
    return float(np.max(kd)) / den if den > 0 else 0.0


def enclosed_area(X):
    """Signed area enclosed by a closed polygon (shoelace formula), counter-clockwise positive."""
    x, y = X[:, 0], X[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def enclosed_volume(X, tris):
    """Volume enclosed by a closed triangulated surface, V = (1/6) sum_{(i,j,k)} X_i . (X_j x X_k) (Sec. 6.2.2).

    Reading: the paper prints the triple product of (X_j - X_k, X_k - X_i,
    X_i - X_j); those three vectors sum to zero, so that product vanishes
    identically.  The signed-tetrahedron sum it describes (origin-free for a
    closed surface, triangles counter-clockwise seen from outside) is the one
    used here.
    """
    tris = np.asarray(tris, dtype=np.int64)
    A, B, C = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    return float(np.sum(A * np.cross(B, C))) / 6.0
