"""One FSIB time step (Alg. 1) and the steady-Stokes variant -- oracle side.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import nudft, fluid, forces
from .modes import nyquist_mask


class ForceLaw:
    """A force model F(X) with its quadrature weights w_j.

    kind "tension2d": closed curve, eq. elstic_force_2d, w_j = dtheta = 2*pi/M.
    kind "surface3d": triangulated surface tension (Sec. 6.2.3), w_j = 1.
    """

    def __init__(self, kind, K, tris=None):
        self.kind = kind
        self.K = float(K)
        self.tris = None if tris is None else np.asarray(tris, dtype=np.int64)

    def __call__(self, X):
        M = X.shape[0]
        if self.kind == "tension2d":
            return forces.tension_force_2d(X, self.K), 2.0 * np.pi / M
        if self.kind == "surface3d":
            return forces.surface_tension_force_3d(X, self.tris, self.K), 1.0
        raise ValueError(self.kind)


def spread_force(X, F, w, Ns, L):
    """fhat(k) = L^-d sum_j w_j F_j exp(-i k.X_j), k in K_N (eq. force_spreading_quad); shape (d, spectral)."""
    d = X.shape[1]
    c = (np.asarray(w) * np.ones(X.shape[0]))[None, :] * np.asarray(F, dtype=np.float64).T
    return nudft.type1(X, c.astype(np.complex128), Ns, L, scale=float(L) ** (-d))


def interp_velocity(X, uhat, Ns, L):
    """U_j = sum_{k in K_N} uhat(k) exp(i k.X_j) (eq. velo_intp_fini); returns the real part, (M, d).

    For Nyquist-zeroed Hermitian uhat the sum is real up to rounding.
    """
    return np.real(nudft.type2(X, uhat, Ns, L)).T.copy()


def stokes_velocity(X, force, Ns, L, mu):
    """Steady Stokes boundary velocity U(X) = interp(Stokeslet(spread(F(X))), X) (Sec. 6.1).

    Reading: the Stokes variant drops the time derivative and nonlinear term,
    so the fluid velocity is a function of the boundary configuration.
    Returns (U, uhat), uhat Nyquist-zeroed.
    """
    F, w = force(X)
    fhat = spread_force(X, F, w, Ns, L)
    uhat = fluid.stokeslet(fhat, Ns, L, mu)
    uhat[:, nyquist_mask(Ns)] = 0.0
    return interp_velocity(X, uhat, Ns, L), uhat


def stokes_step(X, U, force, Ns, L, mu, dt):
    """Midpoint step for the Stokes variant (eqs. spatial_1 and spatial_4 with U from stokes_velocity).

    Returns (X_new, U_new, uhat_new) where U_new = U(X_new) is U^m of the next step.
    """
    Xh = X + 0.5 * dt * U
    Uh, _ = stokes_velocity(Xh, force, Ns, L, mu)
    Xn = X + dt * Uh
    Un, uhat = stokes_velocity(Xn, force, Ns, L, mu)
    return Xn, Un, uhat


def ns_step(X, U, uhat, force, Ns, L, rho, mu, dt, npad=None, return_mid=False):
    """One step of Alg. 1 (Navier-Stokes).

    X^{m+1/2} = X^m + dt/2 U^m                              (eq. spatial_1)
    F^{m+1/2} = F(X^{m+1/2}); fhat from the type-1 sum      (eq. force_spreading_quad)
    uhat^{m+1/2}, uhat^{m+1} by the two Fourier updates      (eqs. spatial_2, spatial_3)
    U^{m+1/2} = interp(uhat^{m+1/2}, X^{m+1/2})
    X^{m+1}   = X^m + dt U^{m+1/2}                          (eq. spatial_4)
    U^{m+1}   = interp(uhat^{m+1}, X^{m+1})

    Reading: Alg. 1 does not say where U^{m+1/2} and U^{m+1} are evaluated;
    they are taken at X^{m+1/2} and X^{m+1} respectively, the latter being the
    U^m of the next step.
    """
    Xh = X + 0.5 * dt * U
    F, w = force(Xh)
    fhat = spread_force(Xh, F, w, Ns, L)
    uh, un = fluid.ns_update(fhat, uhat, Ns, L, rho, mu, dt, npad)
    Uh = interp_velocity(Xh, uh, Ns, L)
    Xn = X + dt * Uh
    Un = interp_velocity(Xn, un, Ns, L)
    if return_mid:
        return Xn, Un, un, dict(Xh=Xh, F=F, w=w, fhat=fhat, uhat_half=uh, U_half=Uh)
    return Xn, Un, un


def stokes_map(X, S, Ns, L, mu):
    """Velocity at X of point strengths S (M, d) at X: U = interp(Stokeslet(spread(S)), X), Nyquist
    modes zeroed (Sec. 6.1 with the strengths given instead of a force law).  Returns (U, uhat)."""
    uhat = fluid.stokeslet(spread_force(X, S, 1.0, Ns, L), Ns, L, mu)
    uhat[:, nyquist_mask(Ns)] = 0.0
    return interp_velocity(X, uhat, Ns, L), uhat


def stokes_map_grad(X, S, GU, Ns, L, mu):
    """Gradients of a loss of U = stokes_map(X, S) given GU = dL/dU.

    U_j = sum_l K(X_j - X_l) S_l with K(r) = L^-d sum_k G(k) exp(i k.r), G the Stokeslet: K is
    even and symmetric, so grad_S = stokes_map(X, GU) and
    grad_X[j, b] = sum_a GU[j, a] d_b u_a(X_j) + S[j, a] d_b v_a(X_j), with u the flow of S and v
    the flow of GU; d_b of a field is the type-2 sum of i k_b times its coefficients.
    """
    d = X.shape[1]
    _, uh = stokes_map(X, S, Ns, L, mu)
    V, vh = stokes_map(X, GU, Ns, L, mu)
    gX = np.zeros_like(X)
    for b in range(d):
        du = interp_velocity(X, nudft._ik_weighted(uh, Ns, L, b), Ns, L)
        dv = interp_velocity(X, nudft._ik_weighted(vh, Ns, L, b), Ns, L)
        gX[:, b] = np.sum(GU * du + S * dv, axis=1)
    return V, gX


def _force_jvp(force, X, V):
    """dF(X)[V] of the force law (also its transpose product: the Jacobians are symmetric)."""
    if force.kind == "tension2d":
        return forces.tension_force_2d_jvp(V, force.K)
    return forces.surface_tension_force_3d_jvp(X, force.tris, force.K, V)


def stokes_trajectory(X0, force, Ns, L, mu, dt, steps):
    """X after `steps` midpoint steps of the Stokes variant from X0 (stokes_step, U^0 = U(X0))."""
    X = np.array(X0, dtype=np.float64)
    for _ in range(steps):
        U, _ = stokes_velocity(X, force, Ns, L, mu)
        Xh = X + 0.5 * dt * U
        Uh, _ = stokes_velocity(Xh, force, Ns, L, mu)
        X = X + dt * Uh
    return X


def trajectory_loss(XT, target):
    """Squared distance of the final positions to their targets, sum_j |X_j(T) - Xtarget_j|^2."""
    D = XT - target
    return float(np.sum(D * D))


def stokes_trajectory_grad(X0, force, Ns, L, mu, dt, steps, target):
    """Loss of stokes_trajectory and its gradients with respect to X0 and the stiffness K.

    Reverse sweep over the steps (each step: U0 = U(X), Xh = X + dt/2 U0, Xn = X + dt U(Xh)), with
    U(X) = stokes_map(X, w F(X; K)).  The adjoint of one velocity evaluation, given GU = dL/dU:
    (gS, gX) from stokes_map_grad, then gX += w dF(X)^T gS (symmetric Jacobian) and
    gK += w <gS, F(X; 1)> (F is linear in K).  The forward positions are stored per step.
    Returns (loss, gX0, gK).
    """
    unit = ForceLaw(force.kind, 1.0, force.tris)
    Xs = [np.array(X0, dtype=np.float64)]
    Xhs = []
    for _ in range(steps):
        X = Xs[-1]
        U, _ = stokes_velocity(X, force, Ns, L, mu)
        Xh = X + 0.5 * dt * U
        Uh, _ = stokes_velocity(Xh, force, Ns, L, mu)
        Xhs.append(Xh)
        Xs.append(X + dt * Uh)
    loss = trajectory_loss(Xs[-1], target)

    def velocity_vjp(X, GU):
        F, w = force(X)
        gS, gX = stokes_map_grad(X, w * F, GU, Ns, L, mu)
        gX = gX + w * _force_jvp(force, X, gS)
        F1, _ = unit(X)
        return gX, w * float(np.sum(gS * F1))

    g = 2.0 * (Xs[-1] - target)
    gK = 0.0
    for s in range(steps - 1, -1, -1):
        gXh, k1 = velocity_vjp(Xhs[s], dt * g)
        gX0, k0 = velocity_vjp(Xs[s], 0.5 * dt * gXh)
        g = g + gXh + gX0
        gK += k1 + k0
    return loss, g, gK
