"""Multi-instance plans (ninst > 1): independent Stokes simulations of one N advanced by shared
launches, against single-instance plans (same kernels, one instance at a time) and the oracle's
time steps per instance."""

import numpy as np
import pytest
import torch

import workloads
from oracle import step
from tests.gpu_helpers import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _cases2d(N, Ms, seed):
    rng = np.random.default_rng(seed)
    out = []
    for M in Ms:
        a = rng.uniform(0.15, 0.3)
        X = workloads.ellipse_2d(M, center=tuple(rng.random(2)), a=a, b=a / rng.uniform(1, 3),
                                 rotation=rng.uniform(0, np.pi))
        out.append(X)
    return out


def _run_single(F, X0, N, prec, tol, mu, dt, K, steps):
    plan = F.Plan(2, (N, N), prec=prec, tol=tol, max_points=X0.shape[0], fluid=True)
    params = F.FluidParams("stokes", mu=mu, dt=dt)
    force = F.Force("tension2d", K)
    X = dev(X0)
    uh = torch.zeros((2,) + plan.half_shape, dtype=plan.cdtype, device="cuda:0")
    U = plan.velocity(params, force, X, uh)
    for _ in range(steps):
        plan.step(params, force, X, U, uh)
    out = host(X), host(U), host(uh)
    plan.close()
    return out


@pytest.mark.parametrize("prec,tol,bar", [("f64", 1e-11, 1e-12), ("f32", 1e-5, 1e-5)])
def test_instances_match_single_plans_2d(F, prec, tol, bar):
    N, Ms, mu, dt, K, steps = 32, [50, 128, 77, 200, 3], 1.0, 1e-3, 1.0, 5
    announce(f"instances 2D {prec} N={N} M={Ms}")
    Xs = _cases2d(N, Ms, 91)
    plan = F.Plan(2, (N, N), prec=prec, tol=tol, max_points=sum(Ms), fluid=True, ninst=len(Ms))
    plan.set_instances(Ms)
    params = F.FluidParams("stokes", mu=mu, dt=dt)
    force = F.Force("tension2d", K)
    X = dev(np.concatenate(Xs))
    uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device="cuda:0")
    U = plan.velocity(params, force, X, uh)
    for _ in range(steps):
        plan.step(params, force, X, U, uh)
    Xg, Ug, uhg = host(X), host(U), host(uh)
    plan.close()
    off = np.concatenate([[0], np.cumsum(Ms)])
    worst = 0.0
    for i, X0 in enumerate(Xs):
        Xr, Ur, uhr = _run_single(F, X0, N, prec, tol, mu, dt, K, steps)
        sl = slice(off[i], off[i + 1])
        e = max(rel_l2(Xg[sl] - X0, Xr - X0), rel_l2(Ug[sl], Ur), rel_l2(uhg[i], uhr))
        worst = max(worst, e)
    print(f"instances 2D {prec}: worst relative difference to single plans {worst:.2e}")
    assert worst < bar


def test_instances_match_oracle_2d(F):
    """FP64 instances against the oracle's midpoint Stokes steps (direct sums), per instance."""
    N, Ms, mu, dt, K, steps = 16, [40, 64, 23], 1.0, 1e-3, 1.0, 3
    announce(f"instances 2D oracle N={N} M={Ms}")
    Xs = _cases2d(N, Ms, 92)
    plan = F.Plan(2, (N, N), prec="f64", tol=1e-11, max_points=sum(Ms), fluid=True, ninst=len(Ms))
    plan.set_instances(Ms)
    params = F.FluidParams("stokes", mu=mu, dt=dt)
    force = F.Force("tension2d", K)
    X = dev(np.concatenate(Xs))
    uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device="cuda:0")
    U = plan.velocity(params, force, X, uh)
    for _ in range(steps):
        plan.step(params, force, X, U, uh)
    Xg = host(X)
    plan.close()
    off = np.concatenate([[0], np.cumsum(Ms)])
    law = step.ForceLaw("tension2d", K)
    worst = 0.0
    for i, X0 in enumerate(Xs):
        Xr = X0.copy()
        Ur, _ = step.stokes_velocity(Xr, law, (N, N), 1.0, mu)
        for _ in range(steps):
            Xr, Ur, _ = step.stokes_step(Xr, Ur, law, (N, N), 1.0, mu, dt)
        worst = max(worst, rel_l2(Xg[off[i]:off[i + 1]] - X0, Xr - X0))
    print(f"instances vs oracle: worst displacement error {worst:.2e}")
    assert worst < 1e-10


def test_instances_surface_tension_3d(F):
    """Two spheres as instances of one 3D plan, triangles indexed over the concatenated points."""
    announce("instances 3D surface tension")
    N, mu, dt, K, steps = 16, 1.0, 1e-3, 1.0, 3
    A, ta = workloads.latlong_sphere(6, 8, radius=0.2, center=(0.4, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    B, tb = workloads.latlong_sphere(5, 7, radius=0.15, center=(0.6, 0.4, 0.55), scale=(1.0, 1.3, 0.9))
    X0 = np.concatenate([A, B])
    tris = np.concatenate([ta, tb + A.shape[0]]).astype(np.int32)
    ptr, idx = workloads.vertex_triangle_csr(tris, X0.shape[0])
    plan = F.Plan(3, (N,) * 3, prec="f64", tol=1e-11, max_points=X0.shape[0], fluid=True, ninst=2)
    plan.set_instances([A.shape[0], B.shape[0]])
    params = F.FluidParams("stokes", mu=mu, dt=dt)
    force = F.Force("surface3d", K, dev(tris), dev(ptr), dev(idx))
    X = dev(X0)
    uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device="cuda:0")
    U = plan.velocity(params, force, X, uh)
    for _ in range(steps):
        plan.step(params, force, X, U, uh)
    Xg = host(X)
    plan.close()
    worst = 0.0
    for (P, t, sl) in ((A, ta, slice(0, A.shape[0])), (B, tb, slice(A.shape[0], X0.shape[0]))):
        law = step.ForceLaw("surface3d", K, t)
        Xr = P.copy()
        Ur, _ = step.stokes_velocity(Xr, law, (N,) * 3, 1.0, mu)
        for _ in range(steps):
            Xr, Ur, _ = step.stokes_step(Xr, Ur, law, (N,) * 3, 1.0, mu, dt)
        worst = max(worst, rel_l2(Xg[sl] - P, Xr - P))
    print(f"instances 3D vs oracle: worst displacement error {worst:.2e}")
    assert worst < 1e-10


def test_instance_errors(F):
    plan = F.Plan(2, (16, 16), prec="f64", tol=1e-8, max_points=100, fluid=True, ninst=3)
    params = F.FluidParams("stokes", mu=1.0, dt=1e-3)
    force = F.Force("tension2d", 1.0)
    X = dev(np.random.default_rng(1).random((30, 2)))
    uh = torch.zeros(plan.field_shape, dtype=plan.cdtype, device="cuda:0")
    with pytest.raises(F.FSIBError):  # instances not set
        plan.velocity(params, force, X, uh)
    with pytest.raises(F.FSIBError):  # offsets beyond max_points
        plan.set_instances([50, 50, 50])
    plan.set_instances([10, 10, 10])
    with pytest.raises(F.FSIBError):  # M differs from the instances' total
        plan.velocity(params, force, X[:20].contiguous(), uh)
    with pytest.raises(F.FSIBError):  # one-instance calls are refused
        plan.spread(X, torch.zeros(30, dtype=plan.cdtype, device="cuda:0"))
    plan.set_instances([10, 18, 2])
    with pytest.raises(F.FSIBError):  # a closed curve needs >= 3 points
        plan.velocity(params, force, X, uh)
    plan.close()


def test_group_batch_matches_per_instance_batch(F):
    """The 64-case batched workload's grouping (here 12 cases, seeded) against one plan per case."""
    from paper_2302_08694_amd.batch import StokesBatch, StokesGroupBatch
    announce("group batch vs per-instance batch")
    cases = workloads.batched_stokes2d(count=12, seed=4, sizes=(32, 64), m_range=(64, 512))
    a = StokesBatch(cases, prec="f64", tol=1e-10, streams=4)
    b = StokesGroupBatch(cases, prec="f64", tol=1e-10)
    a.step(5)
    b.step(5)
    worst = 0.0
    for it, Xb, c in zip(a.items, b.positions(), cases):
        worst = max(worst, rel_l2(host(Xb) - c["X"], host(it["X"]) - c["X"]))
    b.reset()
    b.capture(5)
    for _ in range(2):
        b.reset()
        b.replay()
        torch.cuda.synchronize()
        for it, Xb, c in zip(a.items, b.positions(), cases):
            worst = max(worst, rel_l2(host(Xb) - c["X"], host(it["X"]) - c["X"]))
    print(f"group batch vs per-instance: {worst:.2e}")
    a.close()
    b.close()
    assert worst < 1e-11


def test_tuning_knobs_keep_results(F):
    """Changing the launch-shape knobs (fsib_plan_tuning) changes speed only: a 3D NUFFT pair and a
    2D multi-instance step agree to rounding across settings; the autotuner leaves a valid setting."""
    import workloads as wl
    from oracle.modes import spectral_shape
    from paper_2302_08694_amd.tune import autotune
    announce("tuning knobs")
    X0, c0 = wl.nufft_points(3000, seed=7, dim=3)
    f0 = wl.random_modes(spectral_shape((24, 24, 24)), 8)
    plan = F.Plan(3, (24, 24, 24), prec="f64", tol=1e-10, max_points=3000)
    X, c, f = dev(X0), dev(c0), dev(f0)
    base = plan.tuning()
    assert base["split"] == 256  # the creation value of a plan of at most 2^18 points
    r0 = (host(plan.spread(X, c)), host(plan.interp(X, f)))
    for knobs in ({"xcd_chunk_spread": 0, "xcd_chunk_interp": 0}, {"xcd_chunk_spread": 64, "split": 2048},
                  {"xcd_chunk_interp": 256, "split": 600}, {"interp_points": 1}, {"interp_points": 16}):
        plan.tuning(**{**base, **knobs})
        r = (host(plan.spread(X, c)), host(plan.interp(X, f)))
        assert rel_l2(r[0], r0[0]) < 1e-13 and rel_l2(r[1], r0[1]) < 1e-15
    with pytest.raises(F.FSIBError):
        plan.tuning(split=128)  # below the creation value
    with pytest.raises(F.FSIBError):
        plan.tuning(interp_points=3)
    res = autotune(plan, lambda: (plan.spread(X, c), plan.interp(X, f)), reps=1)
    assert res["best"] == plan.tuning()
    print(f"autotune chose {res['best']} ({len(res['trials'])} trials)")
    plan.close()


def test_environment_knobs_at_creation(F, monkeypatch):
    """FSIB_SPREAD_SPLIT and the XCD chunk variables replace the defaults when a plan is created
    (split below the default, its scratch sized for it; out-of-range chunks ignored); results agree
    to rounding with a default plan's."""
    import workloads as wl
    announce("environment knobs at plan creation")
    X0, c0 = wl.nufft_points(3000, seed=7, dim=3)
    X, c = dev(X0), dev(c0)
    ref_plan = F.Plan(3, (24, 24, 24), prec="f64", tol=1e-10, max_points=3000)
    ref = host(ref_plan.spread(X, c))
    ref_plan.close()
    monkeypatch.setenv("FSIB_SPREAD_SPLIT", "96")
    monkeypatch.setenv("FSIB_XCD_CHUNK_INTERP", "0")
    monkeypatch.setenv("FSIB_XCD_CHUNK_SPREAD", "5000")
    plan = F.Plan(3, (24, 24, 24), prec="f64", tol=1e-10, max_points=3000)
    t = plan.tuning()
    assert (t["split"], t["xcd_chunk_interp"], t["xcd_chunk_spread"]) == (96, 0, 16)
    assert rel_l2(host(plan.spread(X, c)), ref) < 1e-13
    plan.close()
