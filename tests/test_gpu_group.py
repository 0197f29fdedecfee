"""Groups of plans of different N stepped together (fsib_group_steps): every stage of the Stokes step
(Sec. 6.1, eq. stokeslet, with the midpoint update of eqs. spatial_1 and spatial_4) is one launch over
all plans.

* Against the same plans stepped one by one (fsib_step per plan on its own stream): the arithmetic per
  plan is the same; only the order of points inside a bin (atomic run claims) may differ, so the
  bars are 1e-12 (FP64) and 1e-6 (FP32).
* Against the CPU oracle's Stokes steps (direct sums) for FP64 at tol 1e-11: 1e-10.
* Graph capture: every replay of a captured group step against the eager group step, with eager
  work and synchronisations between the replays.
* Mixed launch shapes: fine-grid lengths without compile-time passes or with other thread counts
  (the stages fall back to one launch per plan), one-instance plans beside multi-instance ones, and
  3D plans with the surface force (the force stage falls back to the plans' own launches).
* Deterministic plans: a group's steps equal the plans' own steps bitwise, and repeat bitwise.
* Refusals: plans of different precision or kernel width, Navier-Stokes plans, more than 8 plans.
"""

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


def _cases():
    return workloads.batched_stokes2d(count=10, seed=4, sizes=(32, 64, 128), m_range=(48, 300))


def _compare(a, b, rep, label):
    for i, (Xa, Xb, X0) in enumerate(zip(a.positions(), b.positions(), [c["X"] for c in a.cases])):
        ex = rel_l2(host(Xa) - X0, host(Xb) - X0)
        assert ex < rep, f"{label}: case {i} dX {ex:.3e}"
    for ga, gb in zip(a.groups, b.groups):
        eu = rel_l2(host(ga["U"]), host(gb["U"]))
        eh = rel_l2(host(ga["uh"]), host(gb["uh"]))
        assert max(eu, eh) < rep, f"{label}: N={ga['plan'].n_modes} U {eu:.3e} uhat {eh:.3e}"


def _batch(cases, prec, tol, fused):
    from paper_2302_08694_amd.batch import StokesGroupBatch
    b = StokesGroupBatch(cases, prec=prec, tol=tol, fused=fused)
    b.cases = cases
    return b


@pytest.mark.parametrize("prec,tol,rep", [("f64", 1e-11, 1e-12), ("f32", 1e-5, 1e-6)])
def test_group_matches_plans_stepped_alone(F, prec, tol, rep):
    announce(f"group of plans of N 32/64/128 against per-plan steps, {prec}")
    cases = _cases()
    fused = _batch(cases, prec, tol, True)
    alone = _batch(cases, prec, tol, False)
    assert len(fused.groups) == 3 and fused.lanes == 1
    fused.step(3)
    for _ in range(3):  # each plan on its own (fsib_step)
        for g in alone.groups:
            g["plan"].step(g["params"], g["force"], g["X"], g["U"], g["uh"])
    torch.cuda.synchronize()
    _compare(fused, alone, rep, "fused vs alone")
    if prec == "f64":
        for c, X in zip(cases, fused.positions()):
            law = step.ForceLaw("tension2d", c["K"])
            Xo = c["X"].copy()
            Uo, _ = step.stokes_velocity(Xo, law, c["N"], 1.0, c["mu"])
            for _ in range(3):
                Xo, Uo, _ = step.stokes_step(Xo, Uo, law, c["N"], 1.0, c["mu"], c["dt"])
            e = rel_l2(host(X) - c["X"], Xo - c["X"])
            print(f"group f64 N={c['N'][0]} M={c['X'].shape[0]}: dX vs oracle {e:.2e}")
            assert e < 1e-10
    fused.close()
    alone.close()


def test_group_lanes_and_autotune(F):
    """Two lanes (two library groups on two streams) and the autotuner's choice agree with one lane."""
    announce("group lanes and autotune, FP64")
    cases = _cases()
    one = _batch(cases, "f64", 1e-11, True)
    two = _batch(cases, "f64", 1e-11, True)
    two.set_lanes(2)
    assert two.lanes == 2 and sorted(len(gs) for _, gs in two.lane_groups) == [1, 2]
    one.step(2)
    two.step(2)
    torch.cuda.synchronize()
    _compare(two, one, 1e-12, "two lanes vs one")
    tuned = _batch(cases, "f64", 1e-11, True)
    res = tuned.autotune(reps=1)
    assert set(res["lanes"]) == {1, 2, 3} and tuned.lanes in (1, 2, 3)
    for _, gs in tuned.lane_groups:  # one spreading variant per lane
        assert len({g["plan"].tuning()["spread_threads"] for g in gs}) == 1
    tuned.step(2)
    torch.cuda.synchronize()
    _compare(tuned, one, 1e-12, "autotuned vs one lane")
    for b in (one, two, tuned):
        b.close()


def test_group_graph_replays(F):
    announce("group steps captured in a HIP graph, FP32")
    cases = _cases()
    eager = _batch(cases, "f32", 1e-5, True)
    snaps = []
    for _ in range(2):
        eager.step(2)
        torch.cuda.synchronize()
        snaps.append([(host(g["X"]), host(g["U"])) for g in eager.groups])
    gb = _batch(cases, "f32", 1e-5, True)
    gb.capture(2)
    for r in range(2):
        gb.replay()
        torch.cuda.synchronize()
        for g, (Xe, Ue) in zip(gb.groups, snaps[r]):
            X0 = host(g["X0"])
            assert rel_l2(host(g["X"]) - X0, Xe - X0) < 1e-6
            assert rel_l2(host(g["U"]), Ue) < 1e-6
        junk = torch.randn(1 << 16, device="cuda")
        float(junk.abs().sum().item())
        torch.cuda.synchronize()
    eager.close()
    gb.close()


def _plan_state(F, p, params, force, X0):
    X = dev(X0)
    uh = torch.zeros(p.field_shape, dtype=p.cdtype, device="cuda")
    U = p.velocity(params, force, X, uh)
    return X, U, uh


def test_group_mixed_launch_shapes_2d(F):
    """N = 40 (fine grid 80: no compile-time passes, 250-thread passes) beside N = 32 and a
    two-instance N = 24 plan; every stage falls back or fuses as its shapes allow."""
    announce("group with mixed FFT launch shapes, 2D FP64")
    specs = [((40, 40), 1, [120]), ((32, 32), 1, [90]), ((24, 24), 2, [60, 75])]
    plans, params, forces, states, ref = [], [], [], [], []
    for k, (N, ni, Ms) in enumerate(specs):
        Xs = [workloads.ellipse_2d(m, center=(0.4 + 0.05 * k + 0.02 * i, 0.55), a=0.25, b=0.15) for i, m in enumerate(Ms)]
        X0 = np.concatenate(Xs)
        p = F.Plan(2, N, prec="f64", tol=1e-11, max_points=X0.shape[0], fluid=True, ninst=ni)
        if ni > 1:
            p.set_instances(Ms)
        prm = F.FluidParams("stokes", mu=1.0 + 0.5 * k, dt=1e-3 * (k + 1))
        frc = F.Force("tension2d", 1.0 + k)
        plans.append(p)
        params.append(prm)
        forces.append(frc)
        states.append(_plan_state(F, p, prm, frc, X0))
        ref.append(_plan_state(F, p, prm, frc, X0))
    for p, prm, frc, (X, U, uh) in zip(plans, params, forces, ref):
        p.step(prm, frc, X, U, uh)
        p.step(prm, frc, X, U, uh)
    grp = F.Group(plans)
    grp.steps(params, forces, [s[0] for s in states], [s[1] for s in states], [s[2] for s in states], 2)
    torch.cuda.synchronize()
    for (X, U, uh), (Xr, Ur, uhr) in zip(states, ref):
        assert rel_l2(host(X), host(Xr)) < 1e-13
        assert rel_l2(host(U), host(Ur)) < 1e-12
        assert rel_l2(host(uh), host(uhr)) < 1e-12
    grp.close()
    for p in plans:
        p.close()


def test_group_3d_surface(F):
    """Two 3D Stokes plans of different N with the surface-tension force (its stage runs per plan)."""
    announce("group of two 3D plans (N 12 and 16), FP64")
    plans, params, forces, states, ref = [], [], [], [], []
    for k, N in enumerate((12, 16)):
        X0, tris = workloads.latlong_sphere(6 + k, 8, radius=0.2, center=(0.5, 0.5 - 0.05 * k, 0.5))
        ptr, idx = workloads.vertex_triangle_csr(tris, X0.shape[0])
        p = F.Plan(3, (N, N, N), prec="f64", tol=1e-9, max_points=X0.shape[0], fluid=True)
        prm = F.FluidParams("stokes", mu=1.0, dt=2e-3)
        frc = F.Force("surface3d", 1.0, dev(tris), dev(ptr), dev(idx))
        plans.append(p)
        params.append(prm)
        forces.append(frc)
        states.append(_plan_state(F, p, prm, frc, X0))
        ref.append(_plan_state(F, p, prm, frc, X0))
    for p, prm, frc, (X, U, uh) in zip(plans, params, forces, ref):
        for _ in range(2):
            p.step(prm, frc, X, U, uh)
    grp = F.Group(plans)
    grp.steps(params, forces, [s[0] for s in states], [s[1] for s in states], [s[2] for s in states], 2)
    torch.cuda.synchronize()
    for (X, U, uh), (Xr, Ur, uhr) in zip(states, ref):
        assert rel_l2(host(X), host(Xr)) < 1e-13
        assert rel_l2(host(U), host(Ur)) < 1e-12
    grp.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_group_deterministic_bitwise(F, prec):
    """Deterministic plans of N = 24, 32 (two instances) and 40: group steps equal each plan's own
    fsib_step bitwise, and a second run repeats them bitwise."""
    announce(f"deterministic group bitwise {prec}")
    tol = 1e-10 if prec == "f64" else 1e-5
    specs = [((24, 24), 1, [90]), ((32, 32), 2, [70, 64]), ((40, 40), 1, [120])]
    def build():
        plans, params, forces, states = [], [], [], []
        for k, (N, ni, Ms) in enumerate(specs):
            Xs = [workloads.ellipse_2d(m, center=(0.45 + 0.03 * i, 0.5 + 0.02 * k), a=0.22, b=0.14) for i, m in enumerate(Ms)]
            X0 = np.concatenate(Xs)
            p = F.Plan(2, N, prec=prec, tol=tol, max_points=X0.shape[0], fluid=True, ninst=ni, deterministic=True)
            if ni > 1:
                p.set_instances(Ms)
            prm = F.FluidParams("stokes", mu=1.0, dt=2e-3)
            frc = F.Force("tension2d", 1.0)
            plans.append(p)
            params.append(prm)
            forces.append(frc)
            states.append(_plan_state(F, p, prm, frc, X0))
        return plans, params, forces, states
    runs = []
    for _ in range(2):
        plans, params, forces, states = build()
        grp = F.Group(plans)
        grp.steps(params, forces, [s[0] for s in states], [s[1] for s in states], [s[2] for s in states], 3)
        torch.cuda.synchronize()
        runs.append([(host(X), host(U), host(uh)) for X, U, uh in states])
        grp.close()
        for p in plans:
            p.close()
    plans, params, forces, states = build()
    for p, prm, frc, (X, U, uh) in zip(plans, params, forces, states):
        for _ in range(3):
            p.step(prm, frc, X, U, uh)
    alone = [(host(X), host(U), host(uh)) for X, U, uh in states]
    for p in plans:
        p.close()
    for a, b, c in zip(runs[0], runs[1], alone):
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
            assert np.array_equal(x.view(np.uint8), z.view(np.uint8))


def test_group_refusals(F):
    announce("group refusals")
    a = F.Plan(2, (16, 16), prec="f64", tol=1e-8, max_points=64, fluid=True)
    b = F.Plan(2, (32, 32), prec="f32", tol=1e-5, max_points=64, fluid=True)
    c = F.Plan(2, (32, 32), prec="f64", tol=1e-4, max_points=64, fluid=True)  # another kernel width
    d = F.Plan(2, (32, 32), prec="f64", tol=1e-8, max_points=64, fluid=True, navier_stokes=True)
    e = F.Plan(2, (32, 32), prec="f64", tol=1e-8, max_points=64, fluid=True, deterministic=True)
    F.Group([a, e]).close()  # deterministic plans may join
    for other in (b, c, d):
        with pytest.raises(F.FSIBError):
            F.Group([a, other])
    with pytest.raises(F.FSIBError):
        F.Group([a, a])
    many = [F.Plan(2, (16, 16), prec="f64", tol=1e-8, max_points=16, fluid=True) for _ in range(9)]
    with pytest.raises(F.FSIBError):
        F.Group(many)
    g = F.Group(many[:8])
    g.close()
    for p in [a, b, c, d, e] + many:
        p.close()
