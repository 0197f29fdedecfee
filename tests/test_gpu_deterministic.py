"""Deterministic plans (fsib_plan_opts.deterministic = 1): every output bitwise reproducible.

The method itself is deterministic (Alg. 1, Sec. 3.3); the only order-dependent sums of the GPU path
are the spreading sums, whose order follows the points' order inside each bin.  A deterministic plan
orders every bin by original point index, so:
  * two runs of the same transform give bitwise-equal outputs, on a point set crowded into a few
    bins (where the atomic run claims of the default sort arrive in varying order);
  * Navier-Stokes and Stokes trajectories are bitwise equal between runs, between eager execution and
    HIP graph replays, and between an uninterrupted run and one saved to the host and resumed;
  * the deterministic plan agrees with the default plan to rounding and with the oracle to tol.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import nudft
from tests.gpu_helpers import announce, cdtype, dev, host, rdtype, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


def _crowded_points(M, seed):
    """Half the points inside one small ball (a few bins), half uniform."""
    rng = np.random.default_rng(seed)
    X = rng.random((M, 3))
    X[: M // 2] = 0.37 + 0.01 * rng.standard_normal((M // 2, 3))
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return X, c


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_transforms_bitwise_repeatable(F, prec):
    announce(f"deterministic type-1/type-2 repeat {prec}")
    Ns = (24, 20, 16)
    X, c = _crowded_points(20000, 61)
    tol = 1e-9 if prec == "f64" else 1e-5
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=X.shape[0], deterministic=True)
    Xd, cd = dev(X), dev(c, cdtype(prec))
    outs = [host(plan.spread(Xd, cd)) for _ in range(4)]
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint8), outs[0].view(np.uint8))
    f = workloads.random_modes(tuple(reversed(Ns)), 62)
    fd = dev(f, cdtype(prec))
    outs2 = [host(plan.interp(Xd, fd)) for _ in range(3)]
    for o in outs2[1:]:
        assert np.array_equal(o.view(np.uint8), outs2[0].view(np.uint8))
    # against the oracle and the default plan
    ref = nudft.type1(X, c, Ns)
    assert rel_l2(outs[0], ref) < (1e-8 if prec == "f64" else 1e-5)
    plain = F.Plan(3, Ns, prec=prec, tol=tol, max_points=X.shape[0])
    o_plain = host(plain.spread(Xd, cd))
    assert rel_l2(outs[0], o_plain) < (1e-13 if prec == "f64" else 1e-6)
    plan.close()
    plain.close()


def _ns3d_small(F, deterministic, prec="f64"):
    X0, tris = workloads.latlong_sphere(40, 40, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    M = X0.shape[0]
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    plan = F.Plan(3, (32, 32, 32), prec=prec, tol=1e-9 if prec == "f64" else 1e-5, max_points=M, fluid=True,
                  navier_stokes=True, deterministic=deterministic)
    force = F.Force("surface3d", 1.0, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=1.0, mu=0.01, dt=5e-4)
    return plan, force, params, X0


def _state(plan, X0, prec):
    X = dev(X0)
    U = torch.zeros((X0.shape[0], 3), dtype=rdtype(prec), device="cuda")
    uh = torch.zeros((3,) + plan.half_shape, dtype=cdtype(prec), device="cuda")
    return X, U, uh


def _same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ns_trajectory_bitwise(F, prec):
    announce(f"deterministic NS trajectory: repeat, graph replay, checkpoint/resume {prec}")
    plan, force, params, X0 = _ns3d_small(F, True, prec)
    # two uninterrupted runs of 6 steps
    runs = []
    for _ in range(2):
        X, U, uh = _state(plan, X0, prec)
        plan.steps(params, force, X, U, uh, 6)
        runs.append((host(X), host(U), host(uh)))
    for a, b in zip(runs[0], runs[1]):
        assert _same(a, b)
    # checkpoint after 3 steps: state to host and back, then 3 more steps
    X, U, uh = _state(plan, X0, prec)
    for _ in range(3):
        plan.step(params, force, X, U, uh)
    saved = (host(X).copy(), host(U).copy(), host(uh).copy())
    del X, U, uh
    torch.cuda.synchronize()
    X, U, uh = dev(saved[0]), dev(saved[1]), dev(saved[2])
    for _ in range(3):
        plan.step(params, force, X, U, uh)
    for a, b in zip((host(X), host(U), host(uh)), runs[0]):
        assert _same(a, b)
    # HIP graph: 6 steps captured once, replayed three times with eager work in between
    X, U, uh = _state(plan, X0, prec)
    Xi, Ui, uhi = X.clone(), U.clone(), uh.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.steps(params, force, X, U, uh, 6)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.steps(params, force, X, U, uh, 6)
    for _ in range(3):
        X.copy_(Xi)
        U.copy_(Ui)
        uh.copy_(uhi)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((host(X), host(U), host(uh)), runs[0]):
            assert _same(a, b)
        plan.steps(params, force, X, U, uh, 1)  # eager work between replays
        torch.cuda.synchronize()
    del g
    # the default plan agrees to rounding
    plain, force2, _, _ = _ns3d_small(F, False, prec)
    X, U, uh = _state(plain, X0, prec)
    plain.steps(params, force2, X, U, uh, 6)
    disp = runs[0][0] - X0
    err = np.linalg.norm(host(X) - runs[0][0]) / np.linalg.norm(disp)
    print(f"deterministic vs default plan, 6 NS steps {prec}: displacement rel err {err:.2e}")
    assert err < (1e-10 if prec == "f64" else 1e-4)
    plan.close()
    plain.close()


def test_stokes2d_bitwise(F):
    announce("deterministic 2D Stokes trajectory repeat")
    case = workloads.stokes2d_case()
    X0 = case["X"]
    M = X0.shape[0]
    plan = F.Plan(2, case["N"], prec="f64", tol=1e-12, max_points=M, fluid=True, deterministic=True)
    force = F.Force("tension2d", case["K"])
    params = F.FluidParams("stokes", mu=case["mu"], dt=case["dt"])
    res = []
    for _ in range(2):
        X = dev(X0)
        U = torch.zeros((M, 2), dtype=torch.float64, device="cuda")
        uh = torch.zeros((2,) + plan.half_shape, dtype=torch.complex128, device="cuda")
        plan.velocity(params, force, X, uh, out=U)
        plan.steps(params, force, X, U, uh, 10)
        res.append((host(X), host(U), host(uh)))
    for a, b in zip(*res):
        assert _same(a, b)
    plan.close()
