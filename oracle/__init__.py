"""Plain FP64 CPU oracle for the Fourier spectral immersed boundary (FSIB) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call it.  It shares no code with the HIP library.

What it computes (Chen & Peskin, "A Fourier spectral immersed boundary method
with exact translation invariance, improved boundary resolution, and a
divergence-free velocity field"):

* ``nudft``  -- the type-1 and type-2 nonuniform Fourier sums written out as
  direct sums (App. A, eqs. type1 and type2; Sec. 3.1 eqs.
  force_spreading_quad and velo_intp_fini).  No NUFFT, no grid, no kernel.
* ``fluid``  -- Leray projection, periodic Stokeslet (eq. stokeslet),
  dealiased nonlinear term by the three-halves rule (eqs. nonlinear_physical
  and nonlinear_kspace), V-hat (Alg. 2) and the Alg. 1 Fourier update.
* ``forces`` -- 2D elastic tension (eq. elstic_force_2d) and 3D surface
  tension (Sec. 6.2.3) with their energies.
* ``step``   -- one Alg. 1 time step (Navier-Stokes) and the steady-Stokes
  variant of Sec. 6.1, in the paper's order.
* ``diagnostics`` -- momentum, energy, divergence, enclosed area/volume.

Every array is float64 / complex128.  Spectral arrays hold the truncated mode
set K_N (eq. kNh) in FFT order with numpy shape ``(N_z, N_y, N_x)`` (x index
fastest), component-major for vector fields: ``(d, N_z, N_y, N_x)``.

Readings of the paper where it is silent or garbled are listed in each
function's docstring.  Parity pins: see ``tests/test_oracle_*.py``; one
function has no independent pin and says "parity unpinned" in its docstring
(``forces.latlong`` geometry is a workload choice, not part of the method).
"""

from . import modes, nudft, fluid, forces, step, diagnostics  # noqa: F401
