"""GPU parity of the FSIB coupling, fluid update, force laws and Alg. 1 against the oracle.

Bar: relative l2 <= 1e-10 with the GPU in FP64 (plan tol 1e-11), and the stated FP32 errors
(plan tol 1e-5) below.  Trajectories compare the displacement X(T) - X(0), U and uhat.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import diagnostics, fluid, forces, nudft, step
from oracle.modes import nyquist_mask, spectral_shape
from tests.gpu_helpers import announce, cdtype, dev, half, host, rdtype, rel_l2
from tests.helpers import random_real_field_hat

pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-10, "f32": 1e-5}
TOL = {"f64": 1e-11, "f32": 1e-5}


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _divfree_hat(Ns, seed, L=1.0):
    uh = random_real_field_hat(Ns, len(Ns), seed)
    return fluid.zero_nyquist(fluid.project(uh, Ns, L), Ns)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns,M", [((32, 24), 300), ((16, 20, 12), 700)])
def test_force_spread(F, prec, Ns, M):
    announce(f"force_spread {prec} N={Ns} M={M}")
    d = len(Ns)
    L = 1.1
    rng = np.random.default_rng(21)
    X = rng.random((M, d)) * 3 - 1
    Fo = rng.standard_normal((M, d))
    w = 0.37
    ref = half(step.spread_force(X, Fo, w, Ns, L), Ns[0])
    if Ns[0] % 2 == 0:
        # the last half-spectrum entry holds wavenumber m_x = +N_x/2 (outside K_N): the direct sum
        # over the other axes with strengths modulated by exp(-i pi N_x x / L)
        mod = np.exp(-1j * np.pi * Ns[0] * np.mod(X[:, 0], L) / L)
        c = (w * Fo).T * mod[None, :]
        ref[..., -1] = nudft.type1(X[:, 1:], c, Ns[1:], L, scale=L ** (-d))
    plan = F.Plan(d, Ns, L=L, prec=prec, tol=TOL[prec], max_points=M, fluid=True)
    out = host(plan.force_spread(dev(X), dev(w * Fo, rdtype(prec)), scale=L ** (-d)))
    err = rel_l2(out, ref)
    print(f"force_spread {prec} {Ns} rel_l2={err:.3e}")
    assert err < BAR[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns,M", [((32, 24), 300), ((16, 20, 12), 700), ((15, 16, 9), 400)])
def test_velocity_interp(F, prec, Ns, M):
    announce(f"velocity_interp {prec} N={Ns} M={M}")
    d = len(Ns)
    rng = np.random.default_rng(22)
    X = rng.random((M, d))
    uh = _divfree_hat(Ns, 23)
    ref = step.interp_velocity(X, uh, Ns, 1.0)
    plan = F.Plan(d, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True)
    out = host(plan.velocity_interp(dev(X), dev(half(uh, Ns[0]), cdtype(prec))))
    err = rel_l2(out, ref)
    print(f"velocity_interp {prec} {Ns} rel_l2={err:.3e}")
    assert err < BAR[prec]


def test_curve_tension_force(F):
    announce("curve tension force")
    rng = np.random.default_rng(24)
    X = workloads.ellipse_2d(200, (0.3, 0.7)) + 0.01 * rng.standard_normal((200, 2)) + 5.0
    force = F.Force("tension2d", 1.7)
    out = host(F.compute_force(force, dev(X)))
    ref = forces.tension_force_2d(X, 1.7)
    assert rel_l2(out, ref) < 1e-13


def test_surface_tension_force(F):
    announce("surface tension force")
    X, tris = workloads.latlong_sphere(20, 24, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    rng = np.random.default_rng(25)
    X = X + 0.002 * rng.standard_normal(X.shape)
    ptr, idx = workloads.vertex_triangle_csr(tris, X.shape[0])
    force = F.Force("surface3d", 0.9, dev(tris), dev(ptr), dev(idx))
    out = host(F.compute_force(force, dev(X)))
    ref = forces.surface_tension_force_3d(X, tris, 0.9)
    assert rel_l2(out, ref) < 1e-13


@pytest.mark.parametrize("K", [200, 1200])
def test_surface_tension_force_high_degree(F, K):
    """A bipyramid: two apexes joined to a ring of K vertices, so the apexes have degree K.  With K = 200
    the first workgroup's 32 vertices hold 520 triangle terms, spread over its lanes; with K = 1200
    they hold 2,520, past what a workgroup keeps in LDS, and take the per-vertex path."""
    announce(f"surface tension force, bipyramid of {K} ring vertices")
    rng = np.random.default_rng(27)
    t = 2 * np.pi * np.arange(K) / K
    ring = np.stack([0.5 + 0.3 * np.cos(t), 0.5 + 0.25 * np.sin(t), 0.5 + 0.01 * rng.standard_normal(K)], axis=1)
    X = np.concatenate([[[0.5, 0.5, 0.8], [0.5, 0.5, 0.2]], ring]) + 1e-3 * rng.standard_normal((K + 2, 3))
    i = np.arange(K)
    a, b = 2 + i, 2 + (i + 1) % K
    tris = np.concatenate([np.stack([np.zeros(K, int), a, b], 1), np.stack([np.ones(K, int), b, a], 1)]).astype(np.int32)
    ptr, idx = workloads.vertex_triangle_csr(tris, X.shape[0])
    force = F.Force("surface3d", 1.3, dev(tris), dev(ptr), dev(idx))
    out = host(F.compute_force(force, dev(X)))
    ref = forces.surface_tension_force_3d(X, tris, 1.3)
    assert rel_l2(out, ref) < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns", [(16, 12), (12, 10, 8), (9, 10, 11)])
def test_fluid_step_stokes(F, prec, Ns):
    announce(f"fluid stokes {prec} N={Ns}")
    d = len(Ns)
    L, mu = 1.0, 0.7
    fh = random_real_field_hat(Ns, d, 26)
    ref = fluid.stokeslet(fh, Ns, L, mu)
    ref[:, nyquist_mask(Ns)] = 0.0
    plan = F.Plan(d, Ns, L=L, prec=prec, tol=TOL[prec], max_points=8, fluid=True)
    u = torch.zeros((d,) + plan.half_shape, dtype=cdtype(prec), device="cuda")
    plan.fluid_step(F.FluidParams("stokes", mu=mu), dev(half(fh, Ns[0]), cdtype(prec)), u)
    err = rel_l2(host(u), half(ref, Ns[0]))
    assert err < (1e-13 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns", [(16, 12), (12, 10, 8), (16, 16, 16), (9, 10, 11)])
def test_fluid_step_navier_stokes(F, prec, Ns):
    """Both Fourier updates of Alg. 1 with the dealiased nonlinear term (oracle pads to 2N)."""
    announce(f"fluid NS {prec} N={Ns}")
    d = len(Ns)
    L, rho, mu, dt = 1.0, 1.2, 0.05, 0.02
    u0 = _divfree_hat(Ns, 27) * 3.0
    fh = random_real_field_hat(Ns, d, 28) * 10.0
    mid_ref, new_ref = fluid.ns_update(fh, u0, Ns, L, rho, mu, dt)
    plan = F.Plan(d, Ns, L=L, prec=prec, tol=TOL[prec], max_points=8, fluid=True, navier_stokes=True)
    u = dev(half(u0, Ns[0]), cdtype(prec))
    mid = torch.zeros_like(u)
    plan.fluid_step(F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt), dev(half(fh, Ns[0]), cdtype(prec)), u, mid)
    e1 = rel_l2(host(mid), half(mid_ref, Ns[0]))
    e2 = rel_l2(host(u), half(new_ref, Ns[0]))
    print(f"fluid NS {prec} {Ns} mid {e1:.3e} new {e2:.3e}")
    assert max(e1, e2) < (1e-13 if prec == "f64" else 1e-6)


def _run_gpu(F, plan, params, force, X0, U0, uh0, nsteps, diag=False):
    X = dev(X0)
    U = dev(U0, plan.rdtype)
    uh = dev(uh0, plan.cdtype)
    dg = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda") if diag else None
    for _ in range(nsteps):
        plan.step(params, force, X, U, uh, dg)
    return host(X), host(U), host(uh), (host(dg) if diag else None)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_stokes2d_ellipse_trajectory(F, prec):
    """2D Stokes, N = 32^2, M = 128 ellipse (semi-axes 0.3/0.2, seeded centre), K = 1, mu = 1, dt = 1e-3, 10 steps."""
    announce(f"stokes2d trajectory {prec}")
    case = workloads.stokes2d_case()
    Ns, L, mu, dt, K = case["N"], case["L"], case["mu"], case["dt"], case["K"]
    X0 = case["X"]
    M = X0.shape[0]
    law = step.ForceLaw("tension2d", K)
    U0, _ = step.stokes_velocity(X0, law, Ns, L, mu)
    X, U = X0.copy(), U0.copy()
    for _ in range(10):
        X, U, uh = step.stokes_step(X, U, law, Ns, L, mu, dt)
    plan = F.Plan(2, Ns, L=L, prec=prec, tol=TOL[prec], max_points=M, fluid=True)
    params = F.FluidParams("stokes", mu=mu, dt=dt)
    force = F.Force("tension2d", K)
    uh_g = torch.zeros((2,) + plan.half_shape, dtype=plan.cdtype, device="cuda")
    U0_g = plan.velocity(params, force, dev(X0), uh_g)
    assert rel_l2(host(U0_g), U0) < BAR[prec]
    Xg, Ug, uhg, dg = _run_gpu(F, plan, params, force, X0, host(U0_g), host(uh_g), 10, diag=True)
    ex = rel_l2(Xg - X0, X - X0)
    eu = rel_l2(Ug, U)
    eh = rel_l2(uhg, half(uh, Ns[0]))
    print(f"stokes2d {prec}: dX {ex:.3e} U {eu:.3e} uhat {eh:.3e}")
    assert max(ex, eu, eh) < BAR[prec] * (1 if prec == "f64" else 3)
    # diagnostics of the last step: Stokes energy identity (power = dissipation) and net force ~ 0
    assert abs(dg[8] - dg[7]) < (1e-9 if prec == "f64" else 1e-4) * abs(dg[7])
    if prec == "f64":
        assert abs(dg[10] - diagnostics.enclosed_area(X)) < 1e-12


def _ns3d_small(n_rings=10, n_lon=12, N=16):
    X, tris = workloads.latlong_sphere(n_rings, n_lon, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    return X, tris, (N, N, N)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ns3d_surface_tension_trajectory(F, prec):
    """3D Navier-Stokes, ellipsoid with surface tension, rho = 1, mu = 0.01; 5 steps from rest."""
    announce(f"ns3d trajectory {prec}")
    X0, tris, Ns = _ns3d_small()
    M = X0.shape[0]
    L, rho, mu, dt, K = 1.0, 1.0, 0.01, 2e-3, 1.0
    law = step.ForceLaw("surface3d", K, tris)
    shp = spectral_shape(Ns)
    uh = np.zeros((3,) + shp, dtype=complex)
    U = np.zeros((M, 3))
    X = X0.copy()
    for _ in range(5):
        X, U, uh = step.ns_step(X, U, uh, law, Ns, L, rho, mu, dt)
    plan = F.Plan(3, Ns, L=L, prec=prec, tol=TOL[prec], max_points=M, fluid=True, navier_stokes=True)
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", K, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt)
    Xg, Ug, uhg, dg = _run_gpu(F, plan, params, force, X0, np.zeros((M, 3)),
                               np.zeros((3,) + plan.half_shape, complex), 5, diag=True)
    ex = rel_l2(Xg - X0, X - X0)
    eu = rel_l2(Ug, U)
    eh = rel_l2(uhg, half(uh, Ns[0]))
    print(f"ns3d {prec}: dX {ex:.3e} U {eu:.3e} uhat {eh:.3e}")
    assert max(ex, eu, eh) < BAR[prec] * (1 if prec == "f64" else 3)
    if prec == "f64":
        assert abs(dg[10] - diagnostics.enclosed_volume(X, tris)) < 1e-12
        assert dg[9] < 1e-12  # k.uhat = 0
        assert np.max(np.abs(dg[0:3])) < 1e-12  # zero net force of surface tension
        assert abs(dg[6] - diagnostics.kinetic_energy(uh, L, rho)) < 1e-10 * dg[6]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ns2d_sine_flow_trajectory(F, prec):
    """2D Navier-Stokes circle in a sine shear flow (Sec. 6.2.1 setup, small N), 6 steps."""
    announce(f"ns2d trajectory {prec}")
    Ns = (24, 24)
    M = 60
    X0 = workloads.ellipse_2d(M, (0.5, 0.5), 0.25, 0.25)
    L, rho, mu, dt, K = 1.0, 1.0, 0.01, 1e-3, 1.0
    shp = spectral_shape(Ns)
    uh0 = np.zeros((2,) + shp, dtype=complex)
    uh0[1][0, 1] = 1 / 2j
    uh0[1][0, -1] = -1 / 2j
    law = step.ForceLaw("tension2d", K)
    U0 = step.interp_velocity(X0, uh0, Ns, L)
    X, U, uh = X0.copy(), U0.copy(), uh0.copy()
    for _ in range(6):
        X, U, uh = step.ns_step(X, U, uh, law, Ns, L, rho, mu, dt)
    plan = F.Plan(2, Ns, L=L, prec=prec, tol=TOL[prec], max_points=M, fluid=True, navier_stokes=True)
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt)
    force = F.Force("tension2d", K)
    uhg0 = dev(half(uh0, Ns[0]), plan.cdtype)
    U0g = host(plan.velocity(params, force, dev(X0), uhg0))
    assert rel_l2(U0g, U0) < BAR[prec]
    Xg, Ug, uhg, _ = _run_gpu(F, plan, params, force, X0, U0g, half(uh0, Ns[0]), 6)
    ex = rel_l2(Xg - X0, X - X0)
    eu = rel_l2(Ug, U)
    eh = rel_l2(uhg, half(uh, Ns[0]))
    print(f"ns2d {prec}: dX {ex:.3e} U {eu:.3e} uhat {eh:.3e}")
    assert max(ex, eu, eh) < BAR[prec] * (1 if prec == "f64" else 3)


def test_translation_invariance_gpu(F):
    """Shift every point by r: the GPU trajectory shifts by r to within the NUFFT tolerance (Sec. 5.2)."""
    announce("translation invariance gpu")
    X0, tris, Ns = _ns3d_small()
    M = X0.shape[0]
    plan = F.Plan(3, Ns, prec="f64", tol=1e-11, max_points=M, fluid=True, navier_stokes=True)
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", 1.0, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=2e-3)
    r = np.array([0.31415926535, 0.27182818284, 0.14142135623])
    z = np.zeros((3,) + plan.half_shape, complex)
    Xa, _, _, _ = _run_gpu(F, plan, params, force, X0, np.zeros((M, 3)), z, 4)
    Xb, _, _, _ = _run_gpu(F, plan, params, force, X0 + r, np.zeros((M, 3)), z, 4)
    assert rel_l2(Xb - r - X0, Xa - X0) < 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ns_overlap_matches_serial_and_graph_replays(F, prec):
    """The point side of each Navier-Stokes half step runs on the plan's second stream (tuning knob
    overlap = 1, the default) or on the caller's stream (overlap = 0): the two agree to rounding
    (spreading sums in the order the sort's counting atomics leave).  The forked step also records
    into a HIP graph (the fork and join become parallel branches); every replay of two captured steps,
    with eager work and synchronisations in between, matches the same steps run eagerly."""
    announce(f"ns overlap {prec}")
    X0, tris, Ns = _ns3d_small()
    M = X0.shape[0]
    plan = F.Plan(3, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True, navier_stokes=True)
    assert plan.tuning()["overlap"] == 1
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", 1.0, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=2e-3)
    U0, uh0 = np.zeros((M, 3)), np.zeros((3,) + plan.half_shape, complex)
    ref = _run_gpu(F, plan, params, force, X0, U0, uh0, 5)[:3]
    plan.tuning(overlap=0)
    ser = _run_gpu(F, plan, params, force, X0, U0, uh0, 5)[:3]
    bar = 1e-12 if prec == "f64" else 1e-5

    def same(r, s):  # displacements, velocities, spectra
        return max(rel_l2(r[0] - X0, s[0] - X0), rel_l2(r[1], s[1]), rel_l2(r[2], s[2]))

    assert same(ref, ser) < bar
    with pytest.raises(ValueError):
        plan.tuning(overlapp=1)
    with pytest.raises(F.FSIBError):
        plan.tuning(overlap=2)
    plan.tuning(overlap=1)
    # graph capture of two forked steps
    X, U, uh = dev(X0), dev(U0, plan.rdtype), dev(uh0, plan.cdtype)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        plan.step(params, force, X, U, uh)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    X.copy_(dev(X0))
    U.zero_()
    uh.zero_()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(2):
            plan.step(params, force, X, U, uh)
    for rep in range(3):
        X.copy_(dev(X0))
        U.zero_()
        uh.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (host(X), host(U), host(uh))
        eager = _run_gpu(F, plan, params, force, X0, U0, uh0, 2)[:3]
        assert same(got, eager) < bar, rep
    g = None
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_steps_call_matches_single_steps(F, prec):
    """fsib_steps(n) against n fsib_step calls (3D Navier-Stokes with the step interpolation deferred
    onto the second stream between steps, with and without overlap; 2D Stokes), to rounding; nsteps
    = 0 is a no-op and a negative count an error; a graph of one 3-step call replays like the eager
    call."""
    announce(f"steps call {prec}")
    X0, tris, Ns = _ns3d_small()
    M = X0.shape[0]
    bar = 1e-12 if prec == "f64" else 1e-5
    plan = F.Plan(3, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True, navier_stokes=True)
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", 1.0, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=2e-3)

    def run(n_calls, per_call):
        X, U = dev(X0), torch.zeros((M, 3), dtype=plan.rdtype, device="cuda")
        uh = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype, device="cuda")
        dg = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda")
        for _ in range(n_calls):
            if per_call == 1:
                plan.step(params, force, X, U, uh, dg)
            else:
                plan.steps(params, force, X, U, uh, per_call, dg)
        return host(X) - X0, host(U), host(uh), host(dg)

    def diff(a, b):
        return max(rel_l2(x, y) for x, y in zip(a, b))

    ref = run(6, 1)
    for ov in (1, 0):
        plan.tuning(overlap=ov)
        assert diff(run(1, 6), ref) < bar
        assert diff(run(2, 3), ref) < bar
    plan.tuning(overlap=1)
    X, U = dev(X0), torch.zeros((M, 3), dtype=plan.rdtype, device="cuda")
    uh = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype, device="cuda")
    plan.steps(params, force, X, U, uh, 0)
    assert torch.equal(X, dev(X0)) and not bool(U.abs().max() > 0)
    with pytest.raises(F.FSIBError):
        plan.steps(params, force, X, U, uh, -1)
    # graph of one 3-step call
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.steps(params, force, X, U, uh, 3)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.steps(params, force, X, U, uh, 3)
    want = run(1, 3)[:3]
    for rep in range(3):
        X.copy_(dev(X0))
        U.zero_()
        uh.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert diff((host(X) - X0, host(U), host(uh)), want) < bar, rep
        run(1, 1)  # eager work between replays
    g = None
    plan.close()
    # 2D Stokes
    case = workloads.stokes2d_case()
    X2 = case["X"]
    plan = F.Plan(2, case["N"], L=case["L"], prec=prec, tol=TOL[prec], max_points=X2.shape[0], fluid=True)
    p2 = F.FluidParams("stokes", mu=case["mu"], dt=case["dt"])
    f2 = F.Force("tension2d", case["K"])
    outs = []
    for per in (1, 4):
        X = dev(X2)
        uh = torch.zeros((2,) + plan.half_shape, dtype=plan.cdtype, device="cuda")
        U = plan.velocity(p2, f2, X, uh)
        for _ in range(4 // per):
            if per == 1:
                plan.step(p2, f2, X, U, uh)
            else:
                plan.steps(p2, f2, X, U, uh, per)
        outs.append((host(X) - X2, host(U), host(uh)))
    assert diff(outs[0], outs[1]) < bar
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_navier_stokes_steps_without_points(F, prec):
    """An empty point set (M = 0: the fluid alone) through fsib_step and fsib_steps, with both stream
    modes: the field follows the oracle's steps of Alg. 1 with no boundary force; the diagnostics
    stay finite."""
    announce(f"ns without points {prec}")
    Ns = (16, 16, 16)
    L, rho, mu, dt = 1.0, 1.0, 0.02, 5e-3
    u0 = _divfree_hat(Ns, 31) * 2.0
    law = step.ForceLaw("surface3d", 1.0, np.zeros((0, 3), dtype=np.int32))
    X, U, uh = np.zeros((0, 3)), np.zeros((0, 3)), u0.copy()
    for _ in range(4):
        X, U, uh = step.ns_step(X, U, uh, law, Ns, L, rho, mu, dt)
    plan = F.Plan(3, Ns, L=L, prec=prec, tol=TOL[prec], max_points=8, fluid=True, navier_stokes=True)
    empty_i = dev(np.zeros((0, 3), dtype=np.int32))
    force = F.Force("surface3d", 1.0, empty_i, dev(np.zeros(1, dtype=np.int32)), dev(np.zeros(0, dtype=np.int32)))
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt)
    for ov in (1, 0):
        plan.tuning(overlap=ov)
        for per in (1, 4):
            Xg = dev(np.zeros((0, 3)))
            Ug = torch.zeros((0, 3), dtype=plan.rdtype, device="cuda")
            ug = dev(half(u0, Ns[0]), cdtype(prec))
            dg = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda")
            if per == 1:
                for _ in range(4):
                    plan.step(params, force, Xg, Ug, ug, dg)
            else:
                plan.steps(params, force, Xg, Ug, ug, 4, dg)
            e = rel_l2(host(ug), half(uh, Ns[0]))
            print(f"ns without points {prec} overlap={ov} per-call={per}: uhat {e:.3e}")
            assert e < BAR[prec] and np.all(np.isfinite(host(dg)))
    plan.close()
