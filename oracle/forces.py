"""Immersed-boundary force laws and their energies -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np


def tension_force_2d(X, K):
    """Closed elastic curve: F_j = K (X_{j+1} + X_{j-1} - 2 X_j) / dtheta^2 (Sec. 6.2.1, eq. elstic_force_2d).

    theta_j = j dtheta, dtheta = 2*pi/M, indices periodic.  X is the unfolded
    (continuous) curve; the force uses differences only, so it is
    translation-equivariant.  This is a force density per unit theta: the
    spread uses quadrature weights w_j = dtheta (eq. force_spreading_quad).
    """
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    dth = 2.0 * np.pi / M
    return K * (np.roll(X, -1, axis=0) + np.roll(X, 1, axis=0) - 2.0 * X) / (dth * dth)


def tension_energy_2d(X, K):
    """E = (K/2) sum_j |X_{j+1} - X_j|^2 / dtheta, whose gradient gives w_j F_j = -dE/dX_j with w_j = dtheta."""
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    dth = 2.0 * np.pi / M
    D = np.roll(X, -1, axis=0) - X
    return 0.5 * K * float(np.sum(D * D)) / dth


def surface_tension_force_3d(X, tris, gamma):
    """Surface tension: F_i = -(gamma/2) sum_{(i,j,k) in Delta_i} (X_j - X_k) x n_ijk (Sec. 6.2.3).

    Each triangle (i, j, k) is visited in its three cyclic rotations; n_ijk is
    the unit normal by the right-hand rule of (X_i, X_j, X_k).  This is the
    nodal force -dE/dX_i of E = gamma * (sum of triangle areas), so the spread
    uses quadrature weights w_i = 1.
    """
    X = np.asarray(X, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    A, B, C = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n, axis=1)[:, None]
    F = np.zeros_like(X)
    np.add.at(F, tris[:, 0], -0.5 * gamma * np.cross(B - C, n))
    np.add.at(F, tris[:, 1], -0.5 * gamma * np.cross(C - A, n))
    np.add.at(F, tris[:, 2], -0.5 * gamma * np.cross(A - B, n))
    return F


def surface_area(X, tris):
    """Sum of triangle areas (the surface-tension energy is gamma times this, Sec. 6.2.3)."""
    X = np.asarray(X, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    A, B, C = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    return 0.5 * float(np.sum(np.linalg.norm(np.cross(B - A, C - A), axis=1)))


def surface_tension_energy_3d(X, tris, gamma):
    return gamma * surface_area(X, tris)


def tension_force_2d_jvp(V, K):
    """Directional derivative dF(X)[V] of the closed-curve tension force (Sec. 6.2.1): the force is
    linear in X, so it is the same second difference applied to V.  The Jacobian is symmetric (the
    force is minus the gradient of a quadratic energy), so this is also the transpose product."""
    return tension_force_2d(V, K)


def surface_tension_force_3d_jvp(X, tris, gamma, V):
    """Directional derivative dF(X)[V] of the surface-tension force (Sec. 6.2.3).

    Per triangle (i, j, k) the force on i is -(gamma/2) (X_j - X_k) x n with n = m/|m|,
    m = (X_j - X_i) x (X_k - X_i).  Differentiating along V:
      d(X_j - X_k) = V_j - V_k,   dm = (V_j - V_i) x (X_k - X_i) + (X_j - X_i) x (V_k - V_i),
      dn = (dm - n (n . dm)) / |m|.
    F = -gamma grad(area), so the Jacobian is minus gamma times the Hessian of the area: symmetric,
    and this is also the transpose product used by the adjoint.
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    out = np.zeros_like(X)
    for r in range(3):  # the three cyclic rotations (i, j, k) of each triangle
        i, j, k = tris[:, r], tris[:, (r + 1) % 3], tris[:, (r + 2) % 3]
        a, b = X[j] - X[i], X[k] - X[i]
        da, db = V[j] - V[i], V[k] - V[i]
        m = np.cross(a, b)
        nm = np.linalg.norm(m, axis=1)[:, None]
        n = m / nm
        dm = np.cross(da, b) + np.cross(a, db)
        dn = (dm - n * np.sum(n * dm, axis=1)[:, None]) / nm
        df = np.cross(da - db, n) + np.cross(a - b, dn)
        np.add.at(out, i, -0.5 * gamma * df)
    return out


def mesh_edges(tris):
    """Undirected edges (E, 2) of a triangulation, each once with i < j, sorted."""
    tris = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def spring_stiffness(X0, tris, sigma):
    """Edge stiffness of the elastic sphere (Sec. 6.2.3): for edge AB, the sum over the two triangles
    ABC that share it of (sigma/8)(a0^2 + b0^2 - c0^2)/S0, with c0 = |AB|, a0 = |BC|, b0 = |AC| and S0 the
    triangle's area, all in the reference configuration X0.  Returns (edges (E,2), K (E,))."""
    X0 = np.asarray(X0, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    edges = mesh_edges(tris)
    index = {(int(i), int(j)): n for n, (i, j) in enumerate(edges)}
    K = np.zeros(len(edges))
    for t in tris:
        for r in range(3):
            A, B, C = t[r], t[(r + 1) % 3], t[(r + 2) % 3]  # edge AB, opposite vertex C
            c2 = np.sum((X0[A] - X0[B]) ** 2)
            a2 = np.sum((X0[B] - X0[C]) ** 2)
            b2 = np.sum((X0[A] - X0[C]) ** 2)
            S0 = 0.5 * np.linalg.norm(np.cross(X0[B] - X0[A], X0[C] - X0[A]))
            K[index[(min(A, B), max(A, B))]] += sigma / 8.0 * (a2 + b2 - c2) / S0
    return edges, K


def spring_force(X, edges, K):
    """F_i = sum_{j linked with i} K_ij (X_j - X_i) (Sec. 6.2.3)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.zeros_like(X)
    i, j = edges[:, 0], edges[:, 1]
    D = K[:, None] * (X[j] - X[i])
    np.add.at(F, i, D)
    np.add.at(F, j, -D)
    return F


def spring_energy(X, edges, K):
    """sum over edges of (K_ij / 2) |X_i - X_j|^2, whose negative gradient is spring_force."""
    X = np.asarray(X, dtype=np.float64)
    D = X[edges[:, 0]] - X[edges[:, 1]]
    return 0.5 * float(np.sum(K * np.sum(D * D, axis=1)))


def elastic_energy(X, X0, tris, sigma):
    """The elastic energy of eq. total_elastic_energy, per triangle: (sigma/2) sum over the cyclic
    permutations of a^2 (b0^2 + c0^2 - a0^2) / (8 S0)."""
    X = np.asarray(X, dtype=np.float64)
    X0 = np.asarray(X0, dtype=np.float64)
    E = 0.0
    for t in np.asarray(tris, dtype=np.int64):
        P, P0 = X[t], X0[t]
        sq = [np.sum((P[(r + 1) % 3] - P[(r + 2) % 3]) ** 2) for r in range(3)]    # side opposite vertex r
        sq0 = [np.sum((P0[(r + 1) % 3] - P0[(r + 2) % 3]) ** 2) for r in range(3)]
        S0 = 0.5 * np.linalg.norm(np.cross(P0[1] - P0[0], P0[2] - P0[0]))
        for r in range(3):
            E += sq[r] * (sq0[(r + 1) % 3] + sq0[(r + 2) % 3] - sq0[r]) / (8.0 * S0)
    return 0.5 * sigma * E


def target_force(X, target, K):
    """Target points (Sec. 6.2.2): F_i = K (Xtarget_i - X_i)."""
    return K * (np.asarray(target, dtype=np.float64) - np.asarray(X, dtype=np.float64))
