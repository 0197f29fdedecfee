"""MI355X (gfx950) Fourier spectral immersed boundary (FSIB) hot path.

A thin Python binding over the C ABI of ``libfsib.so`` (declared in ``include/fsib.h``): it
checks tensor shapes/dtypes/devices, passes raw device pointers and the current HIP stream, and
turns status codes into exceptions.  Every step of the computation runs in the library's HIP
kernels; there is no Python or CPU fallback -- importing this package without the built library,
or calling it without a GPU, raises.

Entry points (same names as the C ABI):

    Plan(dim, n_modes, L=1.0, prec="f64", tol=1e-6, ntrans=1, max_points=..., fluid=False,
         navier_stokes=False)
    plan.spread(X, c, scale=1.0)            type-1 (App. A eq. type1)
    plan.interp(X, fhat)                    type-2 (App. A eq. type2)
    plan.force_spread(X, S, scale)          FSIB force spreading (Sec. 3.1), half spectra
    plan.velocity_interp(X, uhat)           FSIB velocity interpolation (Sec. 3.1)
    plan.fluid_step(params, fhat, uhat)     Alg. 1 Fourier update / Stokeslet
    plan.velocity(params, force, X, uhat)   U at X (U^0 for the first step)
    plan.step(params, force, X, U, uhat)    one Alg. 1 step
    Group(plans).steps(params, forces, X, U, uhat, n)  Stokes steps of plans of different N, one launch
                                            per stage over all of them
    compute_force(force, X)                 built-in force laws
    force_jvp(force, X, V)                  their Jacobian products (adjoint)
    spring_stiffness(X0, tris, ...)         edge springs of the elastic sphere (set-up)
    plan.pressure(params, fhat, uhat)       pressure half spectrum
    plan.spectral_scale / plan.grad_combine adjoint building blocks

Differentiable wrappers (torch.autograd) are in ``paper_2302_08694_amd.autograd``; batched
independent 2D Stokes simulations in ``paper_2302_08694_amd.batch``.
"""

from ._binding import (  # noqa: F401
    FSIBError,
    Plan,
    Group,
    FluidParams,
    Force,
    compute_force,
    force_jvp,
    spring_stiffness,
    device_count,
    library_path,
    load_library,
    version,
    DIAG_COUNT,
)
