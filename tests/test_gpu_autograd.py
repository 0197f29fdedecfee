"""Gradients of the differentiable transforms against the oracle's gradients (themselves pinned by
finite differences of the direct sums, tests/test_oracle_grad.py)."""

import numpy as np
import pytest
import torch

from oracle import nudft
from oracle.modes import spectral_shape
from tests.gpu_helpers import announce, cdtype, dev, host, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-6}
BAR = {"f64": 1e-9, "f32": 2e-4}


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns,M", [((24, 20), 150), ((12, 10, 14), 120)])
def test_type1_gradients(F, prec, Ns, M):
    from paper_2302_08694_amd.autograd import nufft_type1
    announce(f"autograd type-1 {prec} N={Ns}")
    d = len(Ns)
    rng = np.random.default_rng(61)
    X0 = rng.uniform(-0.5, 1.5, (M, d))
    c0 = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    w = rng.standard_normal(spectral_shape(Ns)) + 1j * rng.standard_normal(spectral_shape(Ns))
    scale = 0.8
    plan = F.Plan(d, Ns, prec=prec, tol=TOL[prec], max_points=M)
    X = dev(X0).requires_grad_(True)
    c = dev(c0, cdtype(prec)).requires_grad_(True)
    f = nufft_type1(plan, X, c, scale)
    loss = torch.real(torch.sum(torch.conj(dev(w, cdtype(prec))) * f))  # Re sum conj(w) f
    loss.backward()
    gc_ref, gX_ref = nudft.type1_grad(X0, c0, w, Ns, 1.0, scale)
    e1, e2 = rel_l2(host(c.grad), gc_ref), rel_l2(host(X.grad), gX_ref)
    print(f"type-1 grads {prec} {Ns}: c {e1:.2e} X {e2:.2e}")
    assert max(e1, e2) < BAR[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns,M", [((24, 20), 150), ((12, 10, 14), 120)])
def test_type2_gradients(F, prec, Ns, M):
    from paper_2302_08694_amd.autograd import nufft_type2
    announce(f"autograd type-2 {prec} N={Ns}")
    d = len(Ns)
    rng = np.random.default_rng(62)
    X0 = rng.uniform(-0.5, 1.5, (M, d))
    shp = spectral_shape(Ns)
    f0 = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    w = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    plan = F.Plan(d, Ns, prec=prec, tol=TOL[prec], max_points=M)
    X = dev(X0).requires_grad_(True)
    f = dev(f0, cdtype(prec)).requires_grad_(True)
    c = nufft_type2(plan, X, f)
    loss = torch.real(torch.sum(torch.conj(dev(w, cdtype(prec))) * c))
    loss.backward()
    gf_ref, gX_ref = nudft.type2_grad(X0, f0, w, Ns, 1.0)
    e1, e2 = rel_l2(host(f.grad), gf_ref), rel_l2(host(X.grad), gX_ref)
    print(f"type-2 grads {prec} {Ns}: fhat {e1:.2e} X {e2:.2e}")
    assert max(e1, e2) < BAR[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("Ns,M", [((24, 20), 100), ((12, 10, 14), 90)])
def test_stokes_velocity_gradients(F, prec, Ns, M):
    from oracle import step
    from paper_2302_08694_amd.autograd import stokes_velocity
    announce(f"autograd stokes velocity {prec} N={Ns}")
    d = len(Ns)
    rng = np.random.default_rng(63)
    X0 = rng.uniform(-0.5, 1.5, (M, d))
    S0 = rng.standard_normal((M, d))
    W = rng.standard_normal((M, d))
    mu = 0.7
    plan = F.Plan(d, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True)
    rd = torch.float64 if prec == "f64" else torch.float32
    X = dev(X0).requires_grad_(True)
    S = dev(S0, rd).requires_grad_(True)
    U = stokes_velocity(plan, X, S, mu)
    U_ref, _ = step.stokes_map(X0, S0, Ns, 1.0, mu)
    assert rel_l2(host(U), U_ref) < BAR[prec]
    torch.sum(dev(W, rd) * U).backward()
    gS_ref, gX_ref = step.stokes_map_grad(X0, S0, W, Ns, 1.0, mu)
    e1, e2 = rel_l2(host(S.grad), gS_ref), rel_l2(host(X.grad), gX_ref)
    print(f"stokes velocity grads {prec} {Ns}: S {e1:.2e} X {e2:.2e}")
    assert max(e1, e2) < BAR[prec]
    plan.close()


def _wobbly_sphere(n_rings, n_lon, seed):
    import workloads as wl
    X, tris = wl.latlong_sphere(n_rings, n_lon, radius=0.2, center=(0.5, 0.5, 0.5))
    return X + 0.01 * np.random.default_rng(seed).standard_normal(X.shape), tris


def _surface_force(F, K, X, tris):
    import workloads as wl
    ptr, idx = wl.vertex_triangle_csr(tris, X.shape[0])
    return F.Force("surface3d", K, dev(tris), dev(ptr), dev(idx))


def test_force_jvp_surface_and_curve(F):
    from oracle import forces
    announce("force jvp surface3d / tension2d")
    X0, tris = _wobbly_sphere(12, 16, 71)
    rng = np.random.default_rng(72)
    V0 = rng.standard_normal(X0.shape)
    out = host(F.force_jvp(_surface_force(F, 1.3, X0, tris), dev(X0), dev(V0)))
    e = rel_l2(out, forces.surface_tension_force_3d_jvp(X0, tris, 1.3, V0))
    X2, V2 = rng.standard_normal((37, 2)), rng.standard_normal((37, 2))
    out2 = host(F.force_jvp(F.Force("tension2d", 0.7), dev(X2), dev(V2)))
    e2 = rel_l2(out2, forces.tension_force_2d_jvp(V2, 0.7))
    print(f"force jvp: surface {e:.2e} curve {e2:.2e}")
    assert e < 1e-13 and e2 < 1e-13


def _trajectory_case(kind):
    import workloads as wl
    if kind == "surface3d":
        X, tris = _wobbly_sphere(5, 8, 73)
        target = 0.5 + (X - 0.5) * np.array([1.2, 1.0, 0.8])
        return dict(X=X, tris=tris, target=target, N=(12, 12, 12), K=1.0, mu=1.0, dt=2e-2, steps=3)
    X = wl.ellipse_2d(40, center=(0.43, 0.57), a=0.3, b=0.2)
    target = wl.ellipse_2d(40, center=(0.5, 0.5), a=0.25, b=0.25)
    return dict(X=X, tris=None, target=target, N=(24, 24), K=0.8, mu=1.0, dt=1e-2, steps=4)


@pytest.mark.parametrize("checkpoint", [True, False])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["surface3d", "tension2d"])
def test_stokes_trajectory_gradients(F, kind, prec, checkpoint):
    from oracle import step
    from paper_2302_08694_amd.autograd import ForceLaw, stokes_trajectory
    announce(f"autograd stokes trajectory {kind} {prec} checkpoint={checkpoint}")
    c = _trajectory_case(kind)
    X0, tris, d = c["X"], c["tris"], c["X"].shape[1]
    loss_ref, gX_ref, gK_ref = step.stokes_trajectory_grad(
        X0, step.ForceLaw(kind, c["K"], tris), c["N"], 1.0, c["mu"], c["dt"], c["steps"], c["target"])
    plan = F.Plan(d, c["N"], prec=prec, tol=TOL[prec], max_points=X0.shape[0], fluid=True)
    if kind == "surface3d":
        import workloads as wl
        ptr, idx = wl.vertex_triangle_csr(tris, X0.shape[0])
        law = ForceLaw(kind, dev(tris), dev(ptr), dev(idx))
    else:
        law = ForceLaw(kind)
    X = dev(X0).requires_grad_(True)
    K = torch.tensor(c["K"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    XT = stokes_trajectory(plan, X, K, law, c["mu"], c["dt"], c["steps"], checkpoint=checkpoint)
    loss = torch.sum((XT - dev(c["target"])) ** 2)
    loss.backward()
    el = abs(float(loss) - loss_ref) / loss_ref
    eX = rel_l2(host(X.grad), gX_ref)
    eK = abs(float(K.grad) - gK_ref) / abs(gK_ref)
    print(f"trajectory grads {kind} {prec} ckpt={checkpoint}: loss {el:.2e} X0 {eX:.2e} K {eK:.2e}")
    assert max(el, eX, eK) < BAR[prec]
    plan.close()


def test_diff_stokes_fullsize_against_finite_differences(F):
    """64^3 modes, 10,000 lat-long sphere points, 20 checkpointed steps, loss = squared distance of
    the final positions to the target ellipsoid.  Adjoint gradients (FP32 and FP64 plans) against
    central differences of the FP64 forward (tol 1e-10), on K and 16 seeded position components.
    dL/dX0 = 2 (X_T - target) + (the part through the flow); the part through the flow is also
    compared on its own, relative to its own size."""
    import workloads as wl
    from paper_2302_08694_amd.autograd import ForceLaw, stokes_trajectory
    c = wl.diff_stokes3d_case()
    X0, tris, M = c["X"], c["tris"], c["X"].shape[0]
    announce(f"autograd full size N={c['N']} M={M} steps={c['steps']}")
    ptr, idx = wl.vertex_triangle_csr(tris, M)
    law = ForceLaw("surface3d", dev(tris), dev(ptr), dev(idx))
    tgt = dev(c["target"])
    rng = np.random.default_rng(55)
    comps = [(int(j), int(a)) for j, a in zip(rng.integers(0, M, 16), rng.integers(0, 3, 16))]
    plans = {p: F.Plan(3, c["N"], prec=p, tol=(1e-10 if p == "f64" else 1e-6), max_points=M, fluid=True)
             for p in ("f64", "f32")}

    def run(prec, X, K, grad):
        XT = stokes_trajectory(plans[prec], X, K, law, c["mu"], c["dt"], c["steps"], checkpoint=True)
        loss = torch.sum((XT - tgt) ** 2)
        if grad:
            loss.backward()
        return float(loss), XT.detach()

    def loss_difference(Xa, Ka, Xb, Kb):
        # L(a) - L(b) = sum (A - B)(A + B - 2 target): the same central difference, without the
        # rounding of two separately summed losses (about eps |L| sqrt(3M), 1e-13 here)
        A, B = run("f64", Xa, Ka, False)[1], run("f64", Xb, Kb, False)[1]
        return float(torch.sum((A - B) * (A + B - 2.0 * tgt)))

    grads = {}
    for prec in ("f64", "f32"):
        X = dev(X0).requires_grad_(True)
        K = torch.tensor(c["K"], dtype=torch.float64, device="cuda:0", requires_grad=True)
        loss, XT = run(prec, X, K, True)
        grads[prec] = (host(X.grad), float(K.grad), host(XT), loss)
    with torch.no_grad():
        Kd = torch.tensor(c["K"], dtype=torch.float64, device="cuda:0")
        hK = 1e-4
        fdK = loss_difference(dev(X0), Kd + hK, dev(X0), Kd - hK) / (2 * hK)
        # the polar fans of the lat-long mesh have edges of ~2.5e-4 (ring 0 at polar angle pi/200):
        # h must stay well below them for the O(h^2) term of the force law to be negligible
        h = 1e-6
        fdX = []
        for j, a in comps:
            Xp, Xm = X0.copy(), X0.copy()
            Xp[j, a] += h
            Xm[j, a] -= h
            fdX.append(loss_difference(dev(Xp), Kd, dev(Xm), Kd) / (2 * h))
    fdX = np.array(fdX)
    XT64 = grads["f64"][2]
    ident = np.array([2.0 * (XT64[j, a] - c["target"][j, a]) for j, a in comps])
    flow_fd = fdX - ident
    errs = {}
    for prec in ("f64", "f32"):
        gX, gK, _, loss = grads[prec]
        g = np.array([gX[j, a] for j, a in comps])
        e_full = np.abs(g - fdX).max() / np.abs(fdX).max()
        e_flow = np.abs((g - ident) - flow_fd).max() / np.abs(flow_fd).max()
        e_K = abs(gK - fdK) / abs(fdK)
        print(f"full size {prec}: loss {loss:.10e} dL/dK {gK:.6e} (fd {fdK:.6e}, err {e_K:.2e}); "
              f"dL/dX0 err {e_full:.2e}; flow part err {e_flow:.2e} (|flow part| {np.abs(flow_fd).max():.2e})")
        errs[prec] = (e_full, e_flow, e_K)
        worst = int(np.argmax(np.abs((g - ident) - flow_fd)))
        print(f"  worst component {comps[worst]} (ring {comps[worst][0] // 100}): adjoint flow part "
              f"{g[worst] - ident[worst]:.6e} fd {flow_fd[worst]:.6e}")
    for prec, bars in (("f64", (1e-7, 1e-4, 1e-4)), ("f32", (1e-4, 2e-2, 2e-2))):
        assert all(e < b for e, b in zip(errs[prec], bars)), (prec, errs[prec])
    for p in plans.values():
        p.close()
