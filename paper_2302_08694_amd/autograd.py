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
the device.  Positions are FP64; the plan's precision applies to everything else.  The time stepping
of stokes_trajectory (X + dt U, the factor w K) is composed from torch elementwise operations, which
torch differentiates.
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


def stokes_trajectory(plan, X0, K, force, mu, dt, steps, checkpoint=True):
    """X after `steps` midpoint steps of the Stokes variant from X0 (the steps of fsib_step for the
    Stokes model: Xh = X + dt/2 U(X), X <- X + dt U(Xh)), differentiable in X0 and K.

    With checkpoint=True only the positions at the start of each step are kept for the backward
    pass; the step is recomputed from them (torch.utils.checkpoint), so memory grows by one (M, dim)
    array per step."""

    def one_step(X, K):
        U = stokes_force_velocity(plan, X, K, force, mu).to(torch.float64)
        Xh = X + (0.5 * dt) * U
        Uh = stokes_force_velocity(plan, Xh, K, force, mu).to(torch.float64)
        return X + dt * Uh

    X = X0
    for _ in range(steps):
        if checkpoint:
            X = torch.utils.checkpoint.checkpoint(one_step, X, K, use_reentrant=False)
        else:
            X = one_step(X, K)
    return X
