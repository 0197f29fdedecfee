"""The paper's validation problems on the GPU path (Sec. 6), and parity of the pieces they need:
edge springs with cotangent stiffness (Sec. 6.2.3), target points (Sec. 6.2.2), the pressure
(eq. pressure_poisson_k, eq. stokeslet), the uniform body force.  Parity bars as for the other
transforms (FP64 1e-10 relative, FP32 1e-5); physics checks state their own bars from the paper's
closed forms or its reported behaviour."""

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import fluid, forces, step, validation
from oracle.modes import nyquist_mask, spectral_shape
from tests.gpu_helpers import announce, dev, host, half, rel_l2, cdtype, rdtype

pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-10, "f32": 1e-5}
TOL = {"f64": 1e-11, "f32": 1e-5}


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _spring_force(F, X0, tris, sigma):
    M = X0.shape[0]
    tp, ti = wl.vertex_triangle_csr(tris, M)
    npt, nid = wl.vertex_neighbor_csr(tris, M)
    kij = F.spring_stiffness(dev(X0), dev(tris), dev(tp), dev(ti), dev(npt), dev(nid))
    return F.Force("springs", sigma, dev(tris), dev(npt), dev(nid), aux=kij), kij, npt, nid


def test_spring_stiffness_force_and_jvp(F):
    announce("edge springs stiffness / force / jvp")
    X0, tris = wl.icosphere(3, 1 / 3, (0.5, 0.5, 0.5))
    X0 = X0 + 0.003 * np.random.default_rng(5).standard_normal(X0.shape)  # irregular reference
    force, kij, npt, nid = _spring_force(F, X0, tris, 1.7)
    edges, K = forces.spring_stiffness(X0, tris, 1.0)
    lookup = {(int(i), int(j)): k for (i, j), k in zip(edges, K)}
    ref = np.array([lookup[(min(i, int(j)), max(i, int(j)))] for i in range(X0.shape[0])
                    for j in nid[npt[i]:npt[i + 1]]])
    e0 = rel_l2(host(kij), ref)
    rng = np.random.default_rng(6)
    Y = X0 + 0.02 * rng.standard_normal(X0.shape)
    V = rng.standard_normal(X0.shape)
    e1 = rel_l2(host(F.compute_force(force, dev(Y))), forces.spring_force(Y, edges, 1.7 * K))
    e2 = rel_l2(host(F.force_jvp(force, dev(Y), dev(V))), forces.spring_force(V, edges, 1.7 * K))
    print(f"springs: stiffness {e0:.2e} force {e1:.2e} jvp {e2:.2e}")
    assert max(e0, e1, e2) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_target_force_and_jvp(F, dim):
    announce(f"target force dim={dim}")
    rng = np.random.default_rng(7)
    X, T, V = (rng.standard_normal((57, dim)) for _ in range(3))
    force = F.Force("target", 40.0, aux=dev(T))
    e1 = rel_l2(host(F.compute_force(force, dev(X))), forces.target_force(X, T, 40.0))
    e2 = rel_l2(host(F.force_jvp(force, dev(X), dev(V))), -40.0 * V)
    assert max(e1, e2) < 1e-15


def _real_spectrum(rng, Ns, comps):
    """Spectra of real random fields on the N grid (FFT order, x fastest), -N/2 modes zeroed."""
    shape = (comps,) + tuple(reversed(Ns))
    a = np.fft.fftn(rng.standard_normal(shape), axes=tuple(range(1, len(Ns) + 1))) / np.prod(Ns)
    a[:, nyquist_mask(Ns)] = 0.0
    return a


@pytest.mark.parametrize("model", ["stokes", "navier_stokes"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns", [(24, 20), (12, 10, 14)])
def test_pressure_matches_oracle(F, model, prec, Ns):
    announce(f"pressure {model} {prec} N={Ns}")
    d = len(Ns)
    rng = np.random.default_rng(8)
    f = _real_spectrum(rng, Ns, d)
    u = fluid.project(_real_spectrum(rng, Ns, d), Ns, 1.0)
    ns = model == "navier_stokes"
    ref = fluid.pressure(f, u if ns else None, Ns, 1.0, 0.7)
    ref[nyquist_mask(Ns)] = 0.0
    plan = F.Plan(d, Ns, prec=prec, tol=TOL[prec], max_points=16, fluid=True, navier_stokes=ns)
    params = F.FluidParams(model, rho=0.7, mu=0.3, dt=1e-3)
    p = plan.pressure(params, dev(half(f, Ns[0]), cdtype(prec)), dev(half(u, Ns[0]), cdtype(prec)) if ns else None)
    err = rel_l2(host(p), half(ref, Ns[0]))
    print(f"pressure {model} {prec} {Ns}: {err:.2e}")
    assert err < BAR[prec]
    plan.close()


def _circle(F, N, Nb, kind):
    """Stokes flow of a circle r = L/8 at the centre carrying a uniform normal (outward) or tangent
    (clockwise) force of unit magnitude per unit theta (Sec. 6.1); returns (fhat, uhat, phat) on host."""
    X = wl.circle_2d(Nb, center=(0.5, 0.5), r=0.125)
    th = 2 * np.pi * np.arange(Nb) / Nb
    n = np.stack([np.cos(th), np.sin(th)], axis=1)
    Fo = n if kind == "normal" else np.stack([np.sin(th), -np.cos(th)], axis=1)
    S = (2 * np.pi / Nb) * Fo
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=Nb, fluid=True)
    params = F.FluidParams("stokes", mu=1.0)
    fh = plan.force_spread(dev(X), dev(S), 1.0)
    uh = torch.zeros_like(fh)
    plan.fluid_step(params, fh, uh)
    ph = plan.pressure(params, fh)
    out = host(fh), host(uh), host(ph)
    plan.close()
    return X, S, out


def _grid_values(phat_half, N):
    return np.fft.irfft2(phat_half, s=(N, N)) * N * N  # [y][x]


def test_circle_normal_force_pressure_jump(F):
    """Sec. 6.1: u = 0 and a pressure jump F/r across the circle, p = p1 outside and p2 inside with zero
    mean.  The GPU pressure matches the oracle's; at the centre and the corner the truncated series
    approaches p2 and p1 at first order in N."""
    p1, p2 = validation.circle_pressure_jump(1.0, 0.125, 1.0)
    errs = []
    for N in (32, 64, 128):
        announce(f"circle normal N={N}")
        X, S, (fh, uh, ph) = _circle(F, N, 2 * N, "normal")
        from oracle.step import spread_force
        f_full = spread_force(X, S, 1.0, (N, N), 1.0)
        f_full[:, nyquist_mask((N, N))] = 0.0
        pref = fluid.pressure(f_full, None, (N, N), 1.0, 1.0)
        ep = rel_l2(ph, half(pref, N))
        umax = np.abs(uh).max() / np.abs(fh).max()
        pg = _grid_values(ph, N)
        ec, eo = abs(pg[N // 2, N // 2] - p2), abs(pg[0, 0] - p1)
        print(f"normal circle N={N}: phat vs oracle {ep:.2e}, max|uhat|/max|fhat| {umax:.2e}, "
              f"p(centre) {pg[N // 2, N // 2]:.5f} (p2 {p2:.5f}), p(corner) {pg[0, 0]:.5f} (p1 {p1:.5f})")
        assert ep < 1e-10 and umax < 1e-12
        errs.append(ec)
        assert eo < 0.02 * abs(p1 - p2)
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1]  # first-order approach (ratio ~2)


def test_circle_tangent_force_constant_pressure(F):
    """Sec. 6.1: a tangent force is divergence free, so the pressure is constant (zero) while the
    circle drives a rotating flow."""
    announce("circle tangent N=64")
    N = 64
    _, _, (fh, uh, ph) = _circle(F, N, 2 * N, "tangent")
    _, _, (_, _, ph_n) = _circle(F, N, 2 * N, "normal")
    ratio = np.abs(ph).max() / np.abs(ph_n).max()
    print(f"tangent circle: max|phat| / normal case {ratio:.2e}, max|uhat| {np.abs(uh).max():.3e}")
    assert ratio < 1e-9 and np.abs(uh).max() > 1e-3


def _channel_flux(uh, N):
    """Flux through the channel L/4 < y < 3L/4 of u_x averaged over x, from the half spectrum (Ny, Hx):
    sum over m_y of uhat_x(0, m_y) times the integral of exp(2 pi i m_y y) over the channel."""
    m = np.fft.fftfreq(N, 1.0 / N)
    w = np.where(m == 0, 0.5, 0.0).astype(complex)
    nz = m != 0
    w[nz] = (np.exp(2j * np.pi * m[nz] * 0.75) - np.exp(2j * np.pi * m[nz] * 0.25)) / (2j * np.pi * m[nz])
    return float(np.real(np.sum(uh[0][:, 0] * w)))


def run_channel(F, N, K, dt, T, f0=100.0, mu=0.1, rho=1.0, record=()):
    """Sec. 6.2.2: walls of target points at y = L/4 and 3L/4 (N_b = 2N, spacing h = L/N), uniform body
    force f0 along x, from rest; Navier-Stokes steps with fsib_step.  Returns the flux at the
    requested times and at T."""
    x = np.arange(N) / N
    T0 = np.concatenate([np.stack([x, np.full(N, 0.25)], 1), np.stack([x, np.full(N, 0.75)], 1)])
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-10, max_points=2 * N, fluid=True, navier_stokes=True)
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt, body=(f0, 0.0))
    force = F.Force("target", K, aux=dev(T0))
    X = dev(T0.copy())
    uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128, device="cuda:0")
    U = plan.velocity(params, force, X, uh)
    steps = int(round(T / dt))
    marks = {int(round(t / dt)): t for t in record}
    out = {}
    for s in range(1, steps + 1):
        plan.step(params, force, X, U, uh)
        if s in marks:
            out[marks[s]] = _channel_flux(host(uh), N)
    out[T] = _channel_flux(host(uh), N)
    disp = float(torch.abs(X - dev(T0)).max())
    plan.close()
    return out, disp


def test_channel_flow_flux_and_effective_width(F):
    """Sec. 6.2.2, L = 1, mu = 0.1, rho = 1, f0 = 100, D = L/2.  The flux rises from zero like the
    analytic series and settles below Phi_eq; the effective width D_e = (12 mu Phi_eq / f0)^(1/3) of
    the settled flux lies within a fraction of a mode spacing h of D (the paper reports
    D - D_e -> about 0.4 h for FSIB)."""
    D, f0, mu, rho = 0.5, 100.0, 0.1, 1.0
    phi_eq = validation.poiseuille_steady_flux(D, f0, mu)
    res = {}
    for N in (16, 32):
        announce(f"channel N={N}")
        flux, disp = run_channel(F, N, K=2e3, dt=1e-4, T=3.0, record=(0.05, 0.2, 1.0))
        De = validation.effective_width(flux[3.0], f0, mu)
        res[N] = (D - De) * N
        ana = {t: validation.poiseuille_flux(t, D, f0, mu, rho) for t in flux}
        print(f"channel N={N}: flux " + ", ".join(f"t={t}: {flux[t]:.5f} (series {ana[t]:.5f})" for t in sorted(flux))
              + f"; Phi_eq {phi_eq:.5f}; (D - D_e)/h = {res[N]:.3f}; max wall displacement {disp:.2e}")
        assert 0.0 < flux[3.0] < phi_eq
        assert all(0.0 < flux[t] <= ana[t] * 1.02 for t in flux)
        assert 0.05 < res[N] < 1.0
    assert abs(res[32] - res[16]) < 0.5 * res[16]  # settles to a fixed multiple of h


def _sine_flow(plan, N):
    """uhat of u = (sin 2 pi z, 0, sin 2 pi y) (Sec. 6.2.3's initial flow) on the half spectrum."""
    uh = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype)
    uh[0, 1, 0, 0] = -0.5j   # sin(2 pi z): modes m_z = +-1
    uh[0, N - 1, 0, 0] = 0.5j
    uh[2, 0, 1, 0] = -0.5j   # sin(2 pi y): modes m_y = +-1
    uh[2, 0, N - 1, 0] = 0.5j
    return uh.to("cuda:0")


def run_sphere(F, N, level, dt, T, model, prec="f64", tol=1e-8):
    """Sphere of radius L/3 at the centre (icosahedral, `level` refinements) in Navier-Stokes flow
    started from the sine flow, rho = 1, mu = 0.01, sigma = gamma = 1; elastic springs ("springs") or
    surface tension ("surface3d").  Returns (uhat on host, volume history)."""
    X0, tris = wl.icosphere(level, 1.0 / 3.0, (0.5, 0.5, 0.5))
    M = X0.shape[0]
    if model == "springs":
        force = _spring_force(F, X0, tris, 1.0)[0]
    else:
        tp, ti = wl.vertex_triangle_csr(tris, M)
        force = F.Force("surface3d", 1.0, dev(tris), dev(tp), dev(ti))
    plan = F.Plan(3, (N, N, N), prec=prec, tol=tol, max_points=M, fluid=True, navier_stokes=True)
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=dt)
    X = dev(X0)
    uh = _sine_flow(plan, N)
    U = plan.velocity(params, force, X, uh)
    diag = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda:0")
    vols = []
    for _ in range(int(round(T / dt))):
        plan.step(params, force, X, U, uh, diag)
        vols.append(diag[10].clone())
    out = host(uh)
    vol = np.array([float(v) for v in vols])
    plan.close()
    return out, vol


def test_elastic_sphere_conserves_volume(F):
    """Sec. 6.2.3: N = 32, four refinements, dt = 1e-3, the sphere stretched by the sine flow and pulled
    back by its springs; the enclosed volume stays at its initial value (the paper's figure shows no
    drift for FSIB against a steady leak for IB)."""
    announce("elastic sphere volume N=32 level 4")
    X0, tris = wl.icosphere(4, 1.0 / 3.0, (0.5, 0.5, 0.5))
    v0 = forces_volume(X0, tris)
    _, vol = run_sphere(F, 32, 4, 1e-3, 1.0, "springs")
    drift = np.abs(vol / v0 - 1.0)
    print(f"elastic sphere: V/V0 - 1 at t = 0.25, 0.5, 1: {vol[249] / v0 - 1:.2e}, {vol[499] / v0 - 1:.2e}, "
          f"{vol[-1] / v0 - 1:.2e}; max {drift.max():.2e}")
    assert drift.max() < 2e-3


def forces_volume(X, tris):
    A, B, C = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", A, np.cross(B, C)))) / 6.0


def _field_on_coarse_grid(uh, N, n):
    """Velocity of a half spectrum evaluated at the n^3 grid points (a subset of the N^3 grid)."""
    u = np.fft.irfftn(uh, s=(N, N, N), axes=(1, 2, 3)) * N ** 3
    step = N // n
    return u[:, ::step, ::step, ::step]


@pytest.mark.parametrize("model", ["springs", "surface3d"])
def test_sphere_second_order_convergence(F, model):
    """Sec. 6.2.3 convergence studies: from N = 4, one refinement, dt = 4e-3 to T = 0.2, each
    refinement doubling N, halving dt and refining the mesh once; the velocity on the coarse grid
    converges at second order (successive differences shrink by about 4)."""
    runs = []
    for r in range(5):
        N, level, dt = 4 * 2 ** r, 1 + r, 4e-3 / 2 ** r
        announce(f"sphere convergence {model} N={N} level={level}")
        uh, _ = run_sphere(F, N, level, dt, 0.2, model)
        runs.append(_field_on_coarse_grid(uh, N, 4))
    d = [np.linalg.norm(runs[i + 1] - runs[i]) / np.linalg.norm(runs[-1]) for i in range(4)]
    ratios = [d[i] / d[i + 1] for i in range(3)]
    print(f"sphere {model}: successive differences {', '.join(f'{x:.2e}' for x in d)}; ratios "
          f"{', '.join(f'{x:.2f}' for x in ratios)}")
    assert ratios[-1] > 3.0 and ratios[-2] > 2.5


def test_circle_navier_stokes_conserves_area(F):
    """Sec. 6.2.1 (2D circle with sine flow): r = L/4, N = 64, N_b = 202, dt = 1e-3, K = 1, rho = 1,
    mu = 0.01, u0 = (0, sin 2 pi x), T = 10.  The force law would shrink the curve to a point; the
    enclosed area stays at its initial value (the paper shows no leak for FSIB)."""
    announce("2D NS circle area N=64 T=10")
    N, Nb, dt = 64, 202, 1e-3
    X0 = wl.circle_2d(Nb, center=(0.5, 0.5), r=0.25)
    a0 = 0.5 * float(np.sum(X0[:, 0] * np.roll(X0[:, 1], -1) - np.roll(X0[:, 0], -1) * X0[:, 1]))
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-10, max_points=Nb, fluid=True, navier_stokes=True)
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=dt)
    force = F.Force("tension2d", 1.0)
    X = dev(X0)
    uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128)
    uh[1, 0, 1] = -0.5j  # sin(2 pi x) in u_y: m_x = 1 (the half spectrum holds m_x >= 0 only)
    uh = uh.to("cuda:0")
    U = plan.velocity(params, force, X, uh)
    diag = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda:0")
    areas = []
    for s in range(int(round(10.0 / dt))):
        plan.step(params, force, X, U, uh, diag)
        if s % 100 == 99:
            areas.append(diag[10].clone())
    a = np.array([float(v) for v in areas])
    drift = np.abs(a / a0 - 1.0)
    Xf = host(X)
    rad = np.linalg.norm(Xf - Xf.mean(axis=0), axis=1)
    print(f"2D NS circle: A/A0 - 1 at t = 1, 5, 10: {a[9] / a0 - 1:.2e}, {a[49] / a0 - 1:.2e}, {a[-1] / a0 - 1:.2e}; "
          f"max {drift.max():.2e}; final radius spread {rad.max() - rad.min():.2e}")
    assert drift.max() < 1e-3
    plan.close()


def test_temporal_second_order_2d_navier_stokes(F):
    """Sec. 5 / Alg. 1 temporal convergence (the 2D circle with sine flow of Sec. 6.2.1, N = 64,
    202 points): dt = 0.002 halved three times to t = 0.1; successive differences of the positions
    and of the velocity field shrink by about 4 (second order)."""
    announce("temporal convergence 2D NS")
    N, Nb, T = 64, 202, 0.1
    X0 = wl.circle_2d(Nb, center=(0.5, 0.5), r=0.25)
    outs = []
    for dt in (2e-3, 1e-3, 5e-4, 2.5e-4):
        plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=Nb, fluid=True, navier_stokes=True)
        params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=dt)
        force = F.Force("tension2d", 1.0)
        X = dev(X0)
        uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128)
        uh[1, 0, 1] = -0.5j
        uh = uh.to("cuda:0")
        U = plan.velocity(params, force, X, uh)
        for _ in range(int(round(T / dt))):
            plan.step(params, force, X, U, uh)
        outs.append((host(X), host(uh)))
        plan.close()
    dX = [np.linalg.norm(outs[i + 1][0] - outs[i][0]) for i in range(3)]
    dU = [np.linalg.norm(outs[i + 1][1] - outs[i][1]) for i in range(3)]
    rX = [dX[i] / dX[i + 1] for i in range(2)]
    rU = [dU[i] / dU[i + 1] for i in range(2)]
    print(f"temporal convergence: position ratios {rX[0]:.2f} {rX[1]:.2f}; velocity ratios {rU[0]:.2f} {rU[1]:.2f}")
    assert all(3.5 < r < 4.5 for r in rX + rU)


def _steady_channel_gpu(F, N, f0, mu, L=1.0):
    """The steady channel with D = L through the HIP path: the wall's Stokes matrix is assembled one
    column per launch sequence (spread of a unit strength, Stokes solve, interpolation at the wall),
    the small bordered system is solved on the host, and the strengths' flow is computed once more on
    the GPU.  Returns (S, ubar, ux[y][x] with the mean flow)."""
    X = dev(validation.wall_points(N, L))
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=N, fluid=True)
    params = F.FluidParams("stokes", mu=mu)
    A = np.zeros((2 * N, 2 * N))
    for j in range(N):
        for a in range(2):
            S = torch.zeros((N, 2), dtype=torch.float64, device="cuda:0")
            S[j, a] = 1.0
            fh = plan.force_spread(X, S, 1.0)
            uh = torch.zeros_like(fh)
            plan.fluid_step(params, fh, uh)
            A[:, 2 * j + a] = host(plan.velocity_interp(X, uh)).ravel()
    S, ubar = validation.steady_wall_system(A, N, f0, L)
    fh = plan.force_spread(X, dev(S), 1.0)
    uh = torch.zeros_like(fh)
    plan.fluid_step(params, fh, uh)
    ux = _grid_values(host(uh)[0], N) + ubar[0]
    plan.close()
    return S, ubar, ux


def test_steady_channel_matches_oracle_and_converges(F):
    """Sec. 6.2.2, steady channel with D = L (one wall at y = 0), N_b = N, f0 = 100, mu = 0.1.
    Parity of the strengths, mean flow and velocity field with the oracle (the bordered solve
    amplifies the FP64 transform error by the wall matrix's condition number, a few hundred, so the
    bar is 1e-8); then the paper's orders up to N = 512: first order against D, faster than 1.4
    against the effective width D_e, and D - D_e about 0.4 h."""
    f0, mu, L = 100.0, 0.1, 1.0
    for N in (16, 64):
        announce(f"steady channel parity N={N}")
        S, ubar, ux = _steady_channel_gpu(F, N, f0, mu, L)
        So, ubo, _, uxo = validation.steady_channel(N, f0, mu, L)
        assert rel_l2(S, So) < 1e-8
        assert np.abs(ubar - ubo).max() < 1e-8 * np.abs(ubo).max()
        assert rel_l2(ux, uxo) < 1e-8
    res = []
    for N in (32, 64, 128, 256, 512):
        announce(f"steady channel N={N}")
        S, ubar, ux = _steady_channel_gpu(F, N, f0, mu, L)
        e, d, De = validation.steady_channel_errors(ux, ubar[0], N, f0, mu, L)
        print(f"steady channel N={N}: err(D) {e:.3e} err(D_e) {d:.3e} (L - D_e)/h {(L - De) * N:.3f}")
        res.append((e, d, De, N))
    for (e0, d0, _, _), (e1, d1, _, _) in zip(res, res[1:]):
        assert 0.8 < np.log2(e0 / e1) < 1.3
        assert np.log2(d0 / d1) > 1.4
    assert all(0.35 < (L - De) * N < 0.5 for _, _, De, N in res)


def _circle_stokes_gpu(F, N, Nb, kind):
    """_circle's Stokes solve returning the points, strengths, the velocity at the points and the x
    velocity and pressure on the grid ([y][x], host)."""
    X, S, (fh, uh, ph) = _circle(F, N, Nb, kind)
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=Nb, fluid=True)
    U = host(plan.velocity_interp(dev(X), dev(uh)))
    plan.close()
    return X, S, U, _grid_values(uh[0], N), _grid_values(ph, N)


def test_circle_exponential_convergence_in_the_number_of_points(F):
    """Sec. 6.1 (exponential accuracy of the spreading quadrature): N = 128 fixed, N_b = 4 ... 128;
    the x velocity of the tangent case and the pressure of the normal case on the vertical centreline,
    against N_b = 512, fall faster than any power of N_b (each doubling gains more than the one
    before) and reach rounding level once N_b resolves the band of the modes on the circle.  The
    GPU velocity at the points matches the oracle at N_b = 32."""
    N = 128
    _, _, _, u_ref, _ = _circle_stokes_gpu(F, N, 512, "tangent")
    _, _, _, _, p_ref = _circle_stokes_gpu(F, N, 512, "normal")
    eu, ep = [], []
    for Nb in (4, 8, 16, 32, 64, 128):
        announce(f"circle N=128 N_b={Nb}")
        X, S, U, ug, _ = _circle_stokes_gpu(F, N, Nb, "tangent")
        _, _, _, _, pg = _circle_stokes_gpu(F, N, Nb, "normal")
        eu.append(rel_l2(ug[:, N // 2], u_ref[:, N // 2]))
        ep.append(rel_l2(pg[:, N // 2], p_ref[:, N // 2]))
        if Nb == 32:
            Uo, _ = step.stokes_map(X, S, (N, N), 1.0, 1.0)
            assert rel_l2(U, Uo) < 1e-10
    print("circle centreline errors vs N_b = 512: u " + ", ".join(f"{e:.2e}" for e in eu)
          + "; p " + ", ".join(f"{e:.2e}" for e in ep))
    for e in (eu, ep):
        gains = [e[i] / e[i + 1] for i in range(len(e) - 2)]
        assert all(g2 > g1 for g1, g2 in zip(gains[1:], gains[2:]))  # accelerating
        assert e[-2] < 0.05 * e[2] and e[-1] < 1e-9


def test_circle_stokes_first_order_with_coupled_refinement(F):
    """Sec. 6.1 (spatial convergence, FSIB half): the tangent case from N = 8, N_b = 4, both doubled
    eight times to N = 2048; the velocity at the points, compared with the next refinement at the
    shared points, converges at first order.  Parity with the oracle at N = 128."""
    errs, prev = [], None
    for k in range(9):
        N, Nb = 8 << k, 4 << k
        announce(f"circle coupled N={N} N_b={Nb}")
        X, S, U, _, _ = _circle_stokes_gpu(F, N, Nb, "tangent")
        if N == 128:
            Uo, _ = step.stokes_map(X, S, (N, N), 1.0, 1.0)
            assert rel_l2(U, Uo) < 1e-10
        if prev is not None:
            errs.append(rel_l2(U[::2], prev))
        prev = U
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    print("coupled refinement: errors " + ", ".join(f"{e:.2e}" for e in errs)
          + "; ratios " + ", ".join(f"{x:.2f}" for x in ratios))
    assert all(1.7 < x < 2.4 for x in ratios[2:])


def _half_spectrum_l2_diff(hc, Nc, hf, Nf):
    """Relative L2 norm over the box of the difference of two velocity fields given by their half
    spectra (2, N, N/2 + 1) at N = Nc < Nf (Parseval: the coarse modes sit at the same mode numbers
    of the fine spectrum; m_x > 0 columns count twice)."""
    e = hf.copy()
    rows = np.arange(Nc)
    rows = np.where(rows < Nc // 2, rows, rows - Nc + Nf)  # mode number m_y -> fine row
    e[:, rows, : hc.shape[-1]] -= hc
    w = np.full(hf.shape[-1], 2.0)
    w[0] = 1.0
    return float(np.sqrt(np.sum(np.abs(e) ** 2 * w) / np.sum(np.abs(hf) ** 2 * w)))


def test_circle_navier_stokes_space_time_convergence(F):
    """Sec. 6.2.1 (space and time refined together, FSIB half): the circle with sine flow from N = 8,
    dt = 1e-3, N_b = 26, halving dt and doubling N and N_b up to N = 512, to t = 0.1; successive
    relative L2 differences of the velocity field over the box.  The paper fits order 3/2, which is
    what a velocity with a kink along the curve gives in the box L2 norm: the error is O(h) in a band
    of width O(h) around the curve, O(h^{3/2}) in L2.  Bars, fixed from that reasoning: the least-squares
    order over N = 16 to 256 within 3/2 +- 1/4, and every successive order from N = 16 on above one
    (the first-order floor of the method at the points).  Last runs: successive orders 0.89, 1.39,
    1.44, 1.33, 1.22 (1.13 at N = 1024), falling toward one on the finest grids, where the points'
    first-order error (the Stokes velocity at the points converges at first order) takes over."""
    T = 0.1
    spectra = []
    for k in range(7):
        N, Nb, dt = 8 << k, 26 << k, 1e-3 / (1 << k)
        announce(f"2D NS space-time N={N} N_b={Nb} dt={dt:g}")
        X0 = wl.circle_2d(Nb, center=(0.5, 0.5), r=0.25)
        plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=Nb, fluid=True, navier_stokes=True)
        params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=dt)
        force = F.Force("tension2d", 1.0)
        X = dev(X0)
        uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128)
        uh[1, 0, 1] = -0.5j
        uh = uh.to("cuda:0")
        U = plan.velocity(params, force, X, uh)
        for _ in range(int(round(T / dt))):
            plan.step(params, force, X, U, uh)
        spectra.append((N, host(uh)))
        plan.close()
    errs = [_half_spectrum_l2_diff(spectra[i][1], spectra[i][0], spectra[i + 1][1], spectra[i + 1][0])
            for i in range(len(spectra) - 1)]
    orders = [float(np.log2(errs[i] / errs[i + 1])) for i in range(len(errs) - 1)]
    print("2D NS space-time: L2 differences " + ", ".join(f"{e:.3e}" for e in errs)
          + "; orders " + ", ".join(f"{o:.2f}" for o in orders))
    # least-squares slope of log(err) against log(N) over the differences N = 16/32 .. 256/512
    ns = np.log2([spectra[i][0] for i in range(1, 5)])
    fit = -float(np.polyfit(ns, np.log2(errs[1:5]), 1)[0])
    print(f"2D NS space-time: fitted order over N = 16..256: {fit:.2f}")
    assert 1.25 < fit < 1.75 and all(o > 1.0 for o in orders[1:])


def test_circle_pressure_jump_width_settles_to_a_fixed_multiple_of_h(F):
    """Sec. 6.1 (boundary resolution, FSIB half): the normal-force circle with N and N_b refined
    together (h_b about h); the width of the pressure jump on the vertical centreline, jump height
    over the steepest slope between neighbouring grid values, settles to a fixed multiple of h.  The
    paper reports about 2 h from a fit it does not state; the steepest grid difference gives 1.69 h
    here (the jump spans little more than one cell)."""
    p1, p2 = validation.circle_pressure_jump(1.0, 0.125, 1.0)
    widths = []
    for N in (32, 64, 128, 256):
        announce(f"jump width N={N}")
        Nb = int(round(2 * np.pi * 0.125 * N))
        _, _, (_, _, ph) = _circle(F, N, Nb, "normal")
        col = _grid_values(ph, N)[:, N // 2]
        slope = np.max(np.abs(np.diff(col))) * N
        widths.append(abs(p1 - p2) / slope * N)
    print("jump width / h: " + ", ".join(f"{w:.3f}" for w in widths))
    assert all(1.4 < w < 2.2 for w in widths)
    assert abs(widths[-1] - widths[-2]) < 0.05


def test_circle_trivial_solution_below_and_above_the_transition(F):
    """Sec. 6.1 (coupling of N and N_b): N_b = 64 fixed, N = 4 ... 512.  Below the transition
    (h_b = 2 pi r / N_b < L / N, N <= 64) the normal-force circle's velocity at the points is zero to
    the transform tolerance (the oracle's direct sums give 1e-16); above it the boundary leaks and the
    velocity grows (oracle: 6.7e-4, 7.3e-3, 1.3e-2 at N = 128, 256, 512), which the GPU path
    reproduces."""
    from oracle import step as ostep
    M = 64
    X = wl.circle_2d(M, center=(0.5, 0.5), r=0.125)
    th = 2 * np.pi * np.arange(M) / M
    S = (2 * np.pi / M) * np.stack([np.cos(th), np.sin(th)], axis=1)
    for N in (4, 8, 16, 32, 64, 128, 256, 512):
        announce(f"transition N={N}")
        plan = F.Plan(2, (N, N), prec="f64", tol=1e-12, max_points=M, fluid=True)
        params = F.FluidParams("stokes", mu=1.0)
        fh = plan.force_spread(dev(X), dev(S), 1.0)
        uh = torch.zeros_like(fh)
        plan.fluid_step(params, fh, uh)
        U = host(plan.velocity_interp(dev(X), uh))
        plan.close()
        umax = float(np.abs(U).max())
        if N <= 64:
            assert umax < 1e-10, (N, umax)
        else:
            Uo, _ = ostep.stokes_map(X, S, (N, N), 1.0, 1.0)
            assert umax > 1e-4 and rel_l2(U, Uo) < 1e-8, (N, umax)
        print(f"transition N={N}: max|U| {umax:.2e}")
