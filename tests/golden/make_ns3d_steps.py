"""Write the oracle's state after three full-size 3D Navier-Stokes steps (Alg. 1, Sec. 3.3) as a text
fixture, for the GPU trajectory parity tests.

Workload: the lat-long ellipsoid of 40,000 points (radius 0.25 stretched to axes 0.3/0.25/0.2 about
the box centre), N = 128^3 modes, surface tension K = 1, rho = 1, mu = 0.01, dt = 5e-4, uhat^0 = 0,
U^0 = 0.  The oracle takes the steps with direct nonuniform Fourier sums and the three-halves-rule
nonlinear term; nothing here calls the HIP library.

Stored (samples drawn from default_rng(20261203)):
  * the displacement X^3 - X^0 and the velocity U^3 at 1024 sampled points,
  * uhat^3 at 512 sampled modes of the half spectrum (m_x < N/2),
  * the norms of the whole displacement and of U^3, the kinetic energy and the enclosed volume.

Run:  python tests/golden/make_ns3d_steps.py   (about 5-10 minutes on 8 cores)
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import diagnostics, step  # noqa: E402
from oracle.modes import mode_numbers, spectral_shape  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ns3d_128_three_steps.json")
STEPS = 3
SAMPLE_SEED = 20261203


def main():
    case = workloads.ns3d_case()
    X0, tris, Ns = case["X"], case["tris"], case["N"]
    L, rho, mu, dt = case["L"], case["rho"], case["mu"], case["dt"]
    M = X0.shape[0]
    force = step.ForceLaw("surface3d", case["K"], tris)
    X = X0.copy()
    U = np.zeros((M, 3))
    uhat = np.zeros((3,) + spectral_shape(Ns), dtype=np.complex128)
    t0 = time.time()
    for s in range(STEPS):
        X, U, uhat = step.ns_step(X, U, uhat, force, Ns, L, rho, mu, dt)
        print(f"step {s + 1}: {time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    pts = np.sort(rng.choice(M, 1024, replace=False))
    ix = rng.integers(0, Ns[0] // 2, 512)
    iy = rng.integers(0, Ns[1], 512)
    iz = rng.integers(0, Ns[2], 512)
    disp = X - X0
    uh_s = uhat[:, iz, iy, ix]
    out = {
        "source": "Oracle trajectory of Alg. 1 (Sec. 3.3): three Navier-Stokes steps of the 40,000-point "
                  "lat-long ellipsoid with surface tension (Sec. 6.2.3) at N = 128^3, direct nonuniform "
                  "Fourier sums (App. A, eqs. type1 and type2) and the three-halves-rule nonlinear term "
                  "(Sec. 3.1).  Written by tests/golden/make_ns3d_steps.py from oracle/ and workloads.py only.",
        "N": list(Ns), "L": L, "rho": rho, "mu": mu, "dt": dt, "K": case["K"], "steps": STEPS,
        "points": pts.tolist(),
        "disp": disp[pts].tolist(),
        "U": U[pts].tolist(),
        "modes_index_zyx": np.stack([iz, iy, ix], axis=1).tolist(),
        "modes_m_xyz": np.stack([mode_numbers(Ns[0])[ix], mode_numbers(Ns[1])[iy],
                                 mode_numbers(Ns[2])[iz]], axis=1).tolist(),
        "uhat_re": uh_s.real.tolist(),
        "uhat_im": uh_s.imag.tolist(),
        "disp_norm": float(np.linalg.norm(disp)),
        "U_norm": float(np.linalg.norm(U)),
        "kinetic_energy": diagnostics.kinetic_energy(uhat, L, rho),
        "volume": diagnostics.enclosed_volume(X, tris),
        "volume0": diagnostics.enclosed_volume(X0, tris),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT} ({time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()
