"""The low-memory form: fine grid oversampled by 1.25 instead of 2 (about 4x fewer grid bytes in 3D)
with a wider Kaiser-Bessel kernel, against the oracle's direct sums and time steps.  Bars at the
plan's tolerance: FP64 at tol 1e-8, 1e-8 relative; FP32 at tol 1e-3 (the lowest it accepts at this
oversampling), 1e-3."""

import numpy as np
import pytest

import workloads
from oracle import nudft, step
from oracle.modes import spectral_shape
from tests.gpu_helpers import announce, cdtype, dev, half, host, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-8, "f32": 1e-3}
BAR = {"f64": 1e-8, "f32": 1e-3}


@pytest.fixture(scope="module")
def F():
    import paper_2302_08694_amd as F
    assert F.device_count() > 0, "no HIP device visible"
    return F


CASES = [(2, (32, 32), 1000, 1), (2, (17, 24), 777, 2), (3, (16, 16, 16), 2000, 3), (3, (24, 13, 18), 1501, 4),
         (3, (64, 64, 64), 20000, 5)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M,seed", CASES)
def test_lowmem_type1_type2(F, prec, dim, Ns, M, seed):
    announce(f"lowmem type1/type2 {prec} dim={dim} N={Ns} M={M}")
    X, c = workloads.nufft_points(M, seed=seed, dim=dim)
    f = workloads.random_modes(spectral_shape(Ns), seed + 100)
    plan = F.Plan(dim, Ns, prec=prec, tol=TOL[prec], max_points=M, upsampfac=1.25)
    info = plan.info()
    for a in range(dim):  # the fine grid is the smallest allowed size >= 1.25 N (and >= 2w)
        assert info["n_fine"][a] >= max(int(np.ceil(1.25 * Ns[a])), 2 * info["w"])
        assert info["n_fine"][a] < 2 * Ns[a] or Ns[a] < 32
    e1 = rel_l2(host(plan.spread(dev(X), dev(c, cdtype(prec)))), nudft.type1(X, c, Ns))
    e2 = rel_l2(host(plan.interp(dev(X), dev(f, cdtype(prec)))), nudft.type2(X, f, Ns))
    print(f"lowmem {prec} N={Ns}: w={info['w']} n_fine={info['n_fine'][:dim]} type1 {e1:.2e} type2 {e2:.2e}")
    assert max(e1, e2) < BAR[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lowmem_ns3d_trajectory(F, prec):
    """3D Navier-Stokes ellipsoid with surface tension, 5 steps from rest, in the low-memory form."""
    announce(f"lowmem ns3d trajectory {prec}")
    X0, tris = workloads.latlong_sphere(10, 12, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    Ns, M = (16, 16, 16), X0.shape[0]
    rho, mu, dt, K = 1.0, 0.01, 2e-3, 1.0
    law = step.ForceLaw("surface3d", K, tris)
    uh = np.zeros((3,) + spectral_shape(Ns), dtype=complex)
    U = np.zeros((M, 3))
    X = X0.copy()
    for _ in range(5):
        X, U, uh = step.ns_step(X, U, uh, law, Ns, 1.0, rho, mu, dt)
    plan = F.Plan(3, Ns, prec=prec, tol=TOL[prec], max_points=M, fluid=True, navier_stokes=True, upsampfac=1.25)
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", K, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt)
    import torch
    Xg, Ug = dev(X0), dev(np.zeros((M, 3)), plan.rdtype)
    uhg = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype, device="cuda:0")
    for _ in range(5):
        plan.step(params, force, Xg, Ug, uhg)
    ex = rel_l2(host(Xg) - X0, X - X0)
    eh = rel_l2(host(uhg), half(uh, Ns[0]))
    print(f"lowmem ns3d {prec}: dX {ex:.2e} uhat {eh:.2e}")
    assert max(ex, eh) < 3 * BAR[prec]
    plan.close()


@pytest.mark.parametrize("upsampfac,tol,w", [(2.0, 1e-7, 9), (1.25, 1e-5, 10), (2.0, 1e-8, 10)])
@pytest.mark.parametrize("dim,Ns,M,seed", [(2, (40, 36), 1500, 11), (3, (24, 20, 18), 3001, 12)])
def test_kernel_widths_nine_and_ten(F, upsampfac, tol, w, dim, Ns, M, seed):
    """FP64 plans whose kernel width is 9 or 10 (the interpolation's 9- and 10-lane rows)."""
    announce(f"widths: upsampfac={upsampfac} tol={tol} dim={dim}")
    X, c = workloads.nufft_points(M, seed=seed, dim=dim)
    f = workloads.random_modes(spectral_shape(Ns), seed + 100)
    plan = F.Plan(dim, Ns, prec="f64", tol=tol, max_points=M, upsampfac=upsampfac)
    assert plan.info()["w"] == w
    e1 = rel_l2(host(plan.spread(dev(X), dev(c, cdtype("f64")))), nudft.type1(X, c, Ns))
    e2 = rel_l2(host(plan.interp(dev(X), dev(f, cdtype("f64")))), nudft.type2(X, f, Ns))
    print(f"w={w} sigma={upsampfac} dim={dim}: type1 {e1:.2e} type2 {e2:.2e} (tol {tol:g})")
    assert max(e1, e2) < tol
    plan.close()


# Oversampling 1.5 (the automatic choice of FP32 3D plans at tol >= 1e-5 with few points): FP32 at tol
# 1e-5 and FP64 at tol 1e-9, against the oracle's direct sums to the tolerance.
TOL15 = {"f64": 1e-9, "f32": 1e-5}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dim,Ns,M,seed", CASES)
def test_sigma15_type1_type2(F, prec, dim, Ns, M, seed):
    announce(f"oversampling 1.5 type1/type2 {prec} dim={dim} N={Ns} M={M}")
    X, c = workloads.nufft_points(M, seed=seed, dim=dim)
    f = workloads.random_modes(spectral_shape(Ns), seed + 200)
    plan = F.Plan(dim, Ns, prec=prec, tol=TOL15[prec], max_points=M, upsampfac=1.5)
    info = plan.info()
    for a in range(dim):
        assert info["n_fine"][a] >= max(int(np.ceil(1.5 * Ns[a])), 2 * info["w"])
    e1 = rel_l2(host(plan.spread(dev(X), dev(c, cdtype(prec)))), nudft.type1(X, c, Ns))
    e2 = rel_l2(host(plan.interp(dev(X), dev(f, cdtype(prec)))), nudft.type2(X, f, Ns))
    print(f"sigma 1.5 {prec} N={Ns}: w={info['w']} n_fine={info['n_fine'][:dim]} type1 {e1:.2e} type2 {e2:.2e}")
    assert max(e1, e2) < TOL15[prec]
    plan.close()


def test_sigma15_automatic_choice(F):
    announce("oversampling 1.5 chosen for 3D plans with few points: FP64 tol >= 1e-6, FP32 tol >= 1e-4")
    for prec, tol, nf in (("f64", 1e-5, 192), ("f64", 1e-7, 256), ("f32", 1e-4, 192), ("f32", 1e-5, 256)):
        p = F.Plan(3, (128, 128, 128), prec=prec, tol=tol, max_points=40000, fluid=True, navier_stokes=True)
        assert tuple(p.info()["n_fine"]) == (nf, nf, nf), (prec, tol)
        p.close()
    p32b = F.Plan(3, (128, 128, 128), prec="f32", tol=1e-4, max_points=2_000_000)  # many points: 2.0
    assert tuple(p32b.info()["n_fine"]) == (256, 256, 256)
    p32b.close()
    with pytest.raises(F.FSIBError):
        F.Plan(3, (32, 32, 32), prec="f32", tol=1e-6, max_points=10, upsampfac=1.5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sigma15_ns3d_trajectory(F, prec):
    """3D Navier-Stokes ellipsoid with surface tension, 5 steps from rest, at oversampling 1.5."""
    announce(f"oversampling 1.5 ns3d trajectory {prec}")
    X0, tris = workloads.latlong_sphere(10, 12, radius=0.25, center=(0.5, 0.5, 0.5), scale=(1.2, 1.0, 0.8))
    Ns, M = (16, 16, 16), X0.shape[0]
    rho, mu, dt, K = 1.0, 0.01, 2e-3, 1.0
    law = step.ForceLaw("surface3d", K, tris)
    uh = np.zeros((3,) + spectral_shape(Ns), dtype=complex)
    U = np.zeros((M, 3))
    X = X0.copy()
    for _ in range(5):
        X, U, uh = step.ns_step(X, U, uh, law, Ns, 1.0, rho, mu, dt)
    plan = F.Plan(3, Ns, prec=prec, tol=TOL15[prec], max_points=M, fluid=True, navier_stokes=True, upsampfac=1.5)
    ptr, idx = workloads.vertex_triangle_csr(tris, M)
    force = F.Force("surface3d", K, dev(tris), dev(ptr), dev(idx))
    params = F.FluidParams("navier_stokes", rho=rho, mu=mu, dt=dt)
    import torch
    Xg, Ug = dev(X0), dev(np.zeros((M, 3)), plan.rdtype)
    uhg = torch.zeros((3,) + plan.half_shape, dtype=plan.cdtype, device="cuda:0")
    for _ in range(5):
        plan.step(params, force, Xg, Ug, uhg)
    ex = rel_l2(host(Xg) - X0, X - X0)
    eh = rel_l2(host(uhg), half(uh, Ns[0]))
    print(f"sigma 1.5 ns3d {prec}: dX {ex:.2e} uhat {eh:.2e}")
    assert max(ex, eh) < 3 * TOL15[prec]
    plan.close()
