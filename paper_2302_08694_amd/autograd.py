"""Differentiable nonuniform transforms (torch.autograd) on the library's kernels.

    nufft_type1(plan, X, c, scale=1.0)  -> fhat   (fsib_spread)
    nufft_type2(plan, X, fhat)          -> c      (fsib_interp)
    stokes_velocity(plan, X, S, mu)     -> U      (force spread, Stokeslet, velocity interpolation)
    ForceLaw(kind, ...)(X, K)           -> F      (fsib_compute_force; backward fsib_force_jvp)
    stokes_force_velocity(plan, X, K, force, mu) -> U of the force law's strengths
    stokes_trajectory(plan, X0, K, force, mu, dt, steps) -> X(T), checkpointed per step

Backward (App. A, eqs. type1 and type2; gradients of complex arrays are dL/dRe + i dL/dIm):
  type-1: grad_c = scale * type2(grad_fhat);
          grad_X[:, a] = scale * Re( conj(type2(i k_a grad_fhat)) * c )
  type-2: grad_fhat = type1(grad_c);
          grad_X[:, a] = Re( conj(grad_c) * type2(i k_a fhat) )
The adjoint transforms are the library's own spread and interp; the i k_a weighting and the per-point
combination are library kernels too (fsib_spectral_scale, fsib_grad_combine), so every step runs on
the device.  Positions are FP64; the plan's precision applies to everything else.  stokes_trajectory
runs the library's own Stokes time step (fsib_step) forward and the adjoint of its midpoint rule
backward, recomputing each step's velocities from per-step checkpoints.
"""

import math

import torch
import torch.utils.checkpoint


class _Type1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, c, plan, scale):
        X = X.detach().contiguous()
        c = c.detach().contiguous()
        ctx.save_for_backward(X, c)
        ctx.plan, ctx.scale = plan, float(scale)
        return plan.spread(X, c, scale)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        X, c = ctx.saved_tensors
        plan, s = ctx.plan, ctx.scale
        g = g.contiguous()
        gX = gc = None
        if ctx.needs_input_grad[1]:
            gc = plan.interp(X, plan.spectral_scale(g, -1, s)).reshape(c.shape)
        if ctx.needs_input_grad[0]:
            gX = torch.empty((X.shape[0], plan.dim), dtype=torch.float64, device=X.device)
            for a in range(plan.dim):
                h = plan.interp(X, plan.spectral_scale(g, a, 1.0))
                plan.grad_combine(h, c, gX, a, s)
        return gX, gc, None, None


class _Type2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, fhat, plan):
        X = X.detach().contiguous()
        fhat = fhat.detach().contiguous()
        ctx.save_for_backward(X, fhat)
        ctx.plan = plan
        return plan.interp(X, fhat)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        X, fhat = ctx.saved_tensors
        plan = ctx.plan
        g = g.contiguous()
        gX = gf = None
        if ctx.needs_input_grad[1]:
            gf = plan.spread(X, g, 1.0).reshape(fhat.shape)
        if ctx.needs_input_grad[0]:
            gX = torch.empty((X.shape[0], plan.dim), dtype=torch.float64, device=X.device)
            for a in range(plan.dim):
                dv = plan.interp(X, plan.spectral_scale(fhat, a, 1.0))
                plan.grad_combine(g, dv, gX, a, 1.0)
        return gX, gf, None


def nufft_type1(plan, X, c, scale=1.0):
    """fhat = scale * sum_j c_j exp(-i k.X_j), differentiable in X and c."""
    return _Type1.apply(X, c, plan, scale)


def nufft_type2(plan, X, fhat):
    """c_j = sum_k fhat(k) exp(+i k.X_j), differentiable in X and fhat."""
    return _Type2.apply(X, fhat, plan)


class _StokesVelocity(torch.autograd.Function):
    """U(X, S) = velocity at X of the periodic Stokes flow driven by point strengths S at X
    (fsib_force_spread with scale L^-d, the Stokeslet of fsib_fluid_step, fsib_velocity_interp)."""

    @staticmethod
    def _velocity(plan, params, X, S):
        fh = plan.force_spread(X, S, plan.L ** (-plan.dim))
        uh = torch.zeros((plan.dim,) + plan.half_shape, dtype=plan.cdtype, device=X.device)
        plan.fluid_step(params, fh, uh)
        return plan.velocity_interp(X, uh), uh

    @staticmethod
    def forward(ctx, X, S, plan, mu):
        from ._binding import FluidParams
        X = X.detach().contiguous()
        S = S.detach().contiguous()
        params = FluidParams("stokes", mu=mu)
        U, uh = _StokesVelocity._velocity(plan, params, X, S)
        ctx.save_for_backward(X, S, uh)
        ctx.plan, ctx.params = plan, params
        return U

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, GU):
        # The map S -> U is symmetric (the Stokeslet G(k) is real, symmetric and even in k), so
        # grad_S = U(X, GU); and grad_X[j, b] = sum_a GU[j, a] d_b u_a(X_j) + S[j, a] d_b v_a(X_j),
        # u the flow of S, v the flow of GU (derivatives by i k_b on the half spectra).
        X, S, uh = ctx.saved_tensors
        plan, params = ctx.plan, ctx.params
        GU = GU.contiguous().to(plan.rdtype)
        V, vh = _StokesVelocity._velocity(plan, params, X, GU)
        gX = None
        if ctx.needs_input_grad[0]:
            gX = torch.empty((X.shape[0], plan.dim), dtype=torch.float64, device=X.device)
            for b in range(plan.dim):
                du = plan.velocity_interp(X, plan.spectral_scale(uh, b, 1.0, half=True))
                dv = plan.velocity_interp(X, plan.spectral_scale(vh, b, 1.0, half=True))
                plan.grad_combine(GU, du, gX, b, 1.0, u2=S, v2=dv)
        return gX, (V if ctx.needs_input_grad[1] else None), None, None


def stokes_velocity(plan, X, S, mu):
    """Boundary velocity U(X, S) of point strengths S (M, dim) at X (Stokes), differentiable in X
    and S; plan needs fluid = 1."""
    return _StokesVelocity.apply(X, S, plan, mu)


class _UnitForce(torch.autograd.Function):
    """F(X) of a force law at unit stiffness (fsib_compute_force); backward g -> dF(X)^T g
    (fsib_force_jvp: both force laws are minus an energy gradient, so the Jacobian is symmetric)."""

    @staticmethod
    def forward(ctx, X, force):
        from ._binding import compute_force
        X = X.detach().contiguous()
        ctx.save_for_backward(X)
        ctx.force = force
        return compute_force(force, X)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        from ._binding import force_jvp
        (X,) = ctx.saved_tensors
        return force_jvp(ctx.force, X, g.contiguous().to(torch.float64)), None


class ForceLaw:
    """A built-in force law with its stiffness K as a separate (differentiable) factor:
    F(X; K) = K F(X; 1), quadrature weight w (2 pi / M for the closed curve, 1 for the surface)."""

    def __init__(self, kind, tris=None, v2t_ptr=None, v2t_idx=None, aux=None):
        from ._binding import Force
        self.kind = kind
        self.unit = Force(kind, 1.0, tris, v2t_ptr, v2t_idx, aux)

    def weight(self, M):
        return 2.0 * math.pi / M if self.kind == "tension2d" else 1.0

    def __call__(self, X, K):
        return K * _UnitForce.apply(X, self.unit)


def stokes_force_velocity(plan, X, K, force, mu):
    """U(X) = stokes_velocity(X, w K F(X; 1)): the Stokes boundary velocity of a force law, differentiable
    in X (through the transforms and the force Jacobian) and in K."""
    S = (force.weight(X.shape[0]) * force(X, K)).to(plan.rdtype)
    return stokes_velocity(plan, X, S, mu)


class _StokesTrajectory(torch.autograd.Function):
    """X(T) after `steps` Stokes steps from X0.  The forward pass is the library's own time step
    (fsib_velocity for U^0, then fsib_step: X^{m+1/2} = X^m + dt/2 U(X^m), X^{m+1} = X^m + dt
    U(X^{m+1/2}), Sec. 6.1 with eqs. spatial_1 and spatial_4), keeping the positions at the start of
    each step.  The backward pass sweeps the steps in reverse; per step it recomputes the two
    velocities with the differentiable velocity map and applies the adjoint of the midpoint rule:
    for g = dL/dX^{m+1}, dL/dX^m = g + a + b with a = (dt U_{X^{m+1/2}})^T g and
    b = (dt/2 U_{X^m})^T a, and dL/dK gathers the K-derivatives of both velocity products."""

    @staticmethod
    def forward(ctx, X0, K, plan, force, mu, dt, steps):
        from ._binding import FluidParams, Force
        forceK = Force(force.kind, float(K), *force.unit._keep)
        params = FluidParams("stokes", mu=mu, dt=dt)
        X = X0.detach().clone().contiguous()
        M, d = X.shape
        U = torch.empty((M, d), dtype=plan.rdtype, device=X.device)
        uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device=X.device)
        plan.velocity(params, forceK, X, uh, out=U)  # U^0 = U(X^0)
        ckpts = []
        for _ in range(steps):
            ckpts.append(X.clone())
            plan.step(params, forceK, X, U, uh)
        ctx.ckpts = ckpts
        ctx.K = K.detach()
        ctx.plan, ctx.force, ctx.mu, ctx.dt = plan, force, mu, dt
        return X

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gX):
        plan, force, mu, dt = ctx.plan, ctx.force, ctx.mu, ctx.dt
        g = gX.detach().to(torch.float64).contiguous()
        gK = torch.zeros((), dtype=torch.float64, device=g.device)
        for Xm in reversed(ctx.ckpts):
            with torch.enable_grad():
                x = Xm.detach().requires_grad_(True)
                k = ctx.K.detach().requires_grad_(True)
                U = stokes_force_velocity(plan, x, k, force, mu).to(torch.float64)
                xh = (Xm + (0.5 * dt) * U.detach()).requires_grad_(True)  # X^{m+1/2} as the step forms it
                Uh = stokes_force_velocity(plan, xh, k, force, mu).to(torch.float64)
                a, aK = torch.autograd.grad(Uh, (xh, k), dt * g)
                b, bK = torch.autograd.grad(U, (x, k), (0.5 * dt) * a)
            g = g + a + b
            gK = gK + aK + bK
        ctx.ckpts = None
        return g, (gK.reshape(ctx.K.shape) if ctx.needs_input_grad[1] else None), None, None, None, None, None


def stokes_trajectory(plan, X0, K, force, mu, dt, steps, checkpoint=True):
    """X after `steps` midpoint steps of the Stokes variant from X0 -- the library's fsib_step -- as a
    function differentiable in X0 and K (a 0-dimensional float64 tensor).

    The forward pass keeps the positions at the start of every step (one (M, dim) array per step) and
    the backward pass recomputes each step's velocities from them.  `checkpoint` is accepted for
    compatibility; both values give this checkpointed form."""
    if not torch.is_tensor(K):
        K = torch.tensor(float(K), dtype=torch.float64, device=X0.device)
    return _StokesTrajectory.apply(X0, K, plan, force, mu, dt, int(steps))
