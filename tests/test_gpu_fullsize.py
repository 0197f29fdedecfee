"""GPU parity at the full benchmark sizes, on outputs the oracle can compute one by one.

3D Navier-Stokes workload: N = 128^3, M = 40,000 lat-long ellipsoid points, surface tension.
  * force spreading of the surface force at 512 sampled modes (direct sums),
  * velocity interpolation of a random real field at 256 sampled points (direct sums),
  * both Fourier updates of Alg. 1 on all 128^3 modes (the oracle pads to 200 > 3N/2),
  * one full Alg. 1 step: invariants that hold at any size (k.u = 0, zero net force, constant
    mean flow, volume conserved to the time-step error).
NUFFT micro-benchmark: N = 256^3, M = 2,000,000 points (half uniform, half on a sphere of radius
0.2), complex N(0,1) strengths; type-1 at 256 sampled modes and type-2 at 128 sampled points, in
FP32 at tol 1e-5 and FP64 at tol 1e-10 (the launch configuration the bench uses).

Bars: FP64 <= 1e-10 relative l2 over the sample (tol 1e-11 plans for the 1e-10 bar; the tol 1e-10
NUFFT case is held to 1e-9), FP32 <= 1e-5.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import diagnostics, fluid, nudft, step
from oracle.modes import mode_numbers, spectral_shape
from tests.gpu_helpers import announce, cdtype, dev, half, host, rdtype, rel_l2
from tests.helpers import random_real_field_hat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


@pytest.fixture(scope="module")
def ns3d():
    case = workloads.ns3d_case()
    X, tris = case["X"], case["tris"]
    ptr, idx = workloads.vertex_triangle_csr(tris, X.shape[0])
    case.update(ptr=ptr, idx=idx)
    return case


def _sample_modes(Ns, K, seed, half_x=False):
    rng = np.random.default_rng(seed)
    idx = []
    for a, n in enumerate(Ns):
        hi = n // 2 if (half_x and a == 0) else n  # m_x < N/2 for half spectra
        idx.append(rng.integers(0, hi, K))
    m = np.stack([mode_numbers(n)[i] for n, i in zip(Ns, idx)], axis=1)
    return idx, m


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_force_spread_full_size(F, ns3d, prec):
    announce(f"full-size force spread {prec}")
    X = ns3d["X"]
    M = X.shape[0]
    Ns = ns3d["N"]
    rng = np.random.default_rng(31)
    S = rng.standard_normal((M, 3))
    tol = 1e-11 if prec == "f64" else 1e-5
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=M, fluid=True)
    out = host(plan.force_spread(dev(X), dev(S, rdtype(prec)), scale=1.0))
    (ix, iy, iz), m = _sample_modes(Ns, 512, 32, half_x=True)
    got = out[:, iz, iy, ix]
    ref = np.stack([nudft.type1_at_modes(X, S[:, a], m) for a in range(3)])
    err = rel_l2(got, ref)
    print(f"full-size force spread {prec}: rel_l2 {err:.3e}")
    assert err < (1e-10 if prec == "f64" else 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_velocity_interp_full_size(F, ns3d, prec):
    announce(f"full-size velocity interp {prec}")
    X = ns3d["X"]
    M = X.shape[0]
    Ns = ns3d["N"]
    uh = fluid.zero_nyquist(random_real_field_hat(Ns, 3, 33), Ns)
    tol = 1e-11 if prec == "f64" else 1e-5
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=M, fluid=True)
    U = host(plan.velocity_interp(dev(X), dev(half(uh, Ns[0]), cdtype(prec))))
    sel = np.random.default_rng(34).choice(M, 256, replace=False)
    ref = step.interp_velocity(X[sel], uh, Ns, 1.0)
    err = rel_l2(U[sel], ref)
    print(f"full-size velocity interp {prec}: rel_l2 {err:.3e}")
    assert err < (1e-10 if prec == "f64" else 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fluid_update_full_size(F, prec):
    announce(f"full-size fluid update {prec}")
    Ns = (128, 128, 128)
    L, rho, mu, dt = 1.0, 1.0, 0.01, 5e-4
    u0 = fluid.zero_nyquist(fluid.project(random_real_field_hat(Ns, 3, 35), Ns, L), Ns) * 20.0
    fh = random_real_field_hat(Ns, 3, 36) * 100.0
    mid_ref, new_ref = fluid.ns_update(fh, u0, Ns, L, rho, mu, dt, npad=(200, 200, 200))
    plan = F.Plan(3, Ns, prec=prec, tol=1e-11 if prec == "f64" else 1e-5, max_points=8, fluid=True,
                  navier_stokes=True)
    u = dev(half(u0, Ns[0]), cdtype(prec))
    mid = torch.zeros_like(u)
    plan.fluid_step(F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt), dev(half(fh, Ns[0]), cdtype(prec)), u, mid)
    e1 = rel_l2(host(mid), half(mid_ref, Ns[0]))
    e2 = rel_l2(host(u), half(new_ref, Ns[0]))
    print(f"full-size fluid update {prec}: mid {e1:.3e} new {e2:.3e}")
    assert max(e1, e2) < (1e-12 if prec == "f64" else 1e-5)
    plan.close()


@pytest.mark.parametrize("stages", [2, 3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fluid_update_192_lines_flat_box(F, prec, stages):
    """Lines of 192 dealiasing points on a flat mode box (128 x 10 x 6 modes, dealiasing grid
    192 x 16 x 10), both products kernels (tuning nl_stages: 16 x 12 in registers, 8 x 8 x 3 through
    LDS), against the oracle's update."""
    announce(f"fluid update, 192-point lines, flat box {prec}, {stages} stages")
    Ns = (128, 10, 6)
    L, rho, mu, dt = 1.0, 1.0, 0.01, 5e-4
    u0 = fluid.zero_nyquist(fluid.project(random_real_field_hat(Ns, 3, 37), Ns, L), Ns) * 20.0
    fh = random_real_field_hat(Ns, 3, 38) * 100.0
    mid_ref, new_ref = fluid.ns_update(fh, u0, Ns, L, rho, mu, dt, npad=(200, 16, 10))
    plan = F.Plan(3, Ns, prec=prec, tol=1e-11 if prec == "f64" else 1e-5, max_points=8, fluid=True,
                  navier_stokes=True)
    nd = plan.info()["n_dealias"]
    assert tuple(nd) == (192, 16, 10), nd
    plan.tuning(nl_stages=stages)
    with pytest.raises(F.FSIBError):
        plan.tuning(nl_stages=1)
    assert plan.tuning()["nl_stages"] == stages
    u = dev(half(u0, Ns[0]), cdtype(prec))
    mid = torch.zeros_like(u)
    plan.fluid_step(F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt), dev(half(fh, Ns[0]), cdtype(prec)), u, mid)
    e1 = rel_l2(host(mid), half(mid_ref, Ns[0]))
    e2 = rel_l2(host(u), half(new_ref, Ns[0]))
    print(f"fluid update {Ns} dealias {nd} {prec} {stages} stages: mid {e1:.3e} new {e2:.3e}")
    assert max(e1, e2) < (1e-12 if prec == "f64" else 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fluid_update_products_z_fused(F, prec):
    """128 modes and 192 dealiasing points along z: the products' last pass and the update run as one
    kernel; a narrow box (12 x 10 x 128 modes, 70 (ky, kx) columns, the last workgroup partly
    filled, a uniform body force) against the oracle's update, both half and full step."""
    announce(f"fluid update, fused z pass, narrow box {prec}")
    Ns = (12, 10, 128)
    L, rho, mu, dt = 1.0, 1.0, 0.01, 5e-4
    u0 = fluid.zero_nyquist(fluid.project(random_real_field_hat(Ns, 3, 39), Ns, L), Ns) * 20.0
    fh = random_real_field_hat(Ns, 3, 40) * 100.0
    body = np.array([0.3, -0.2, 0.1])
    fh_ref = fh.copy()
    fh_ref[:, 0, 0, 0] += body  # a uniform body force is an extra k = 0 force density
    mid_ref, new_ref = fluid.ns_update(fh_ref, u0, Ns, L, rho, mu, dt, npad=(20, 16, 200))
    plan = F.Plan(3, Ns, prec=prec, tol=1e-11 if prec == "f64" else 1e-5, max_points=8, fluid=True,
                  navier_stokes=True)
    assert tuple(plan.info()["n_dealias"]) == (18, 16, 192)
    u = dev(half(u0, Ns[0]), cdtype(prec))
    mid = torch.zeros_like(u)
    plan.fluid_step(F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt, body=tuple(body)),
                    dev(half(fh, Ns[0]), cdtype(prec)), u, mid)
    e1 = rel_l2(host(mid), half(mid_ref, Ns[0]))
    e2 = rel_l2(host(u), half(new_ref, Ns[0]))
    print(f"fluid update {Ns} fused z pass {prec}: mid {e1:.3e} new {e2:.3e}")
    assert max(e1, e2) < (1e-12 if prec == "f64" else 1e-5)
    plan.close()


def test_step_invariants_full_size(F, ns3d):
    """One Alg. 1 step at the benchmark size: k.u = 0, zero net force, constant mean flow, volume."""
    announce("full-size step invariants f64")
    X0, tris = ns3d["X"], ns3d["tris"]
    M = X0.shape[0]
    plan = F.Plan(3, ns3d["N"], prec="f64", tol=1e-11, max_points=M, fluid=True, navier_stokes=True)
    force = F.Force("surface3d", ns3d["K"], dev(tris), dev(ns3d["ptr"]), dev(ns3d["idx"]))
    params = F.FluidParams("navier_stokes", rho=ns3d["rho"], mu=ns3d["mu"], dt=ns3d["dt"])
    X = dev(X0)
    U = torch.zeros((M, 3), dtype=torch.float64, device="cuda")
    uh = torch.zeros((3,) + plan.half_shape, dtype=torch.complex128, device="cuda")
    dg = torch.zeros(F.DIAG_COUNT, dtype=torch.float64, device="cuda")
    V0 = diagnostics.enclosed_volume(X0, tris)
    for _ in range(3):
        plan.step(params, force, X, U, uh, dg)
    d = host(dg)
    Xh = host(X)
    assert np.all(np.isfinite(Xh))
    assert d[9] < 1e-13                                   # k.uhat = 0 (Sec. 5.1)
    assert np.max(np.abs(d[0:3])) < 1e-12                 # sum_j F_j = 0
    assert np.max(np.abs(d[3:6])) < 1e-15                 # uhat(0) stays 0 (Sec. 5.3)
    assert abs(d[10] - diagnostics.enclosed_volume(Xh, tris)) < 1e-12
    assert abs(d[10] - V0) < 1e-6 * V0                    # divergence-free flow conserves volume
    # force law on the device equals the oracle's at the final positions
    Fg = host(F.compute_force(force, X))
    from oracle import forces
    assert rel_l2(Fg, forces.surface_tension_force_3d(Xh, tris, ns3d["K"])) < 1e-13
    plan.close()


@pytest.fixture(scope="module")
def nufft_micro():
    X, c = workloads.nufft_points(2_000_000, seed=3, dim=3)
    return X, c


@pytest.mark.parametrize("prec,tol,bar", [("f32", 1e-5, 1e-5), ("f64", 1e-10, 1e-9), ("f64", 1e-5, 1e-5)])
def test_nufft_micro_type1_sampled(F, nufft_micro, prec, tol, bar):
    announce(f"NUFFT micro type-1 {prec} tol {tol}")
    X, c = nufft_micro
    M = X.shape[0]
    Ns = (256, 256, 256)
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=M)
    out = host(plan.spread(dev(X), dev(c, cdtype(prec))))
    (ix, iy, iz), m = _sample_modes(Ns, 128, 37)
    ref = nudft.type1_at_modes(X, c, m)
    err = rel_l2(out[iz, iy, ix], ref)
    print(f"NUFFT micro type-1 {prec} tol {tol}: rel_l2 {err:.3e}")
    assert err < bar
    plan.close()


@pytest.mark.parametrize("prec,tol,bar", [("f32", 1e-5, 1e-5), ("f64", 1e-10, 1e-9)])
def test_nufft_micro_type2_sampled(F, nufft_micro, prec, tol, bar):
    announce(f"NUFFT micro type-2 {prec} tol {tol}")
    X, _ = nufft_micro
    M = X.shape[0]
    Ns = (256, 256, 256)
    f = workloads.random_modes(spectral_shape(Ns), 38)
    plan = F.Plan(3, Ns, prec=prec, tol=tol, max_points=M)
    out = host(plan.interp(dev(X), dev(f, cdtype(prec))))
    sel = np.random.default_rng(39).choice(M, 128, replace=False)
    ref = nudft.type2(X[sel], f, Ns)
    err = rel_l2(out[sel], ref)
    print(f"NUFFT micro type-2 {prec} tol {tol}: rel_l2 {err:.3e}")
    assert err < bar
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_longest_fft_lines_2d(F, prec):
    """The longest fine-grid lines one workgroup holds: N = 2048^2 in 2D oversamples to 4096-point
    lines (about 136 KiB of LDS per line in FP64).  Type-1 at 256 sampled modes and type-2 at 64
    sampled points against direct sums; lines of 8192 points are refused at plan creation."""
    announce(f"2D N=2048 long FFT lines {prec}")
    Ns = (2048, 2048)
    X, c = workloads.nufft_points(4000, seed=41, dim=2)
    M = X.shape[0]
    tol = 1e-11 if prec == "f64" else 1e-5
    bar = 1e-10 if prec == "f64" else 1e-5
    plan = F.Plan(2, Ns, prec=prec, tol=tol, max_points=M)
    assert plan.info()["n_fine"] == (4096, 4096)
    out = host(plan.spread(dev(X), dev(c, cdtype(prec))))
    (ix, iy), m = _sample_modes(Ns, 256, 42)
    e1 = rel_l2(out[iy, ix], nudft.type1_at_modes(X, c, m))
    f = workloads.random_modes(spectral_shape(Ns), 43)
    got = host(plan.interp(dev(X), dev(f, cdtype(prec))))
    sel = np.random.default_rng(44).choice(M, 64, replace=False)
    e2 = rel_l2(got[sel], nudft.type2(X[sel], f, Ns))
    print(f"2D N=2048 {prec}: type-1 rel_l2 {e1:.3e}, type-2 rel_l2 {e2:.3e}")
    assert e1 < bar and e2 < bar
    plan.close()
    with pytest.raises(F.FSIBError, match="LDS budget"):
        F.Plan(2, (4096, 4096), prec=prec, tol=tol, max_points=16)
    with pytest.raises(F.FSIBError, match="dealiasing length"):
        F.Plan(2, Ns, prec=prec, tol=tol, max_points=16, fluid=True, navier_stokes=True)
