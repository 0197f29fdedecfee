"""C ABI checks that need no GPU: the library loads, exports every entry point declared in
include/fsib.h, validates arguments before touching a device, and reports the missing device."""

import ctypes
import os
import re

import pytest

from paper_2302_08694_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fsib.h")).read()
    return sorted(set(re.findall(r"\b(fsib_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = B.load_library()
    names = _declared()
    assert "fsib_spread" in names and "fsib_step" in names and len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_status_strings():
    lib = B.load_library()
    assert b"gfx950" in lib.fsib_version()
    for s in range(8):
        assert lib.fsib_status_string(s)
    assert lib.fsib_status_string(99) == b"unknown status"


def _opts(**kw):
    o = dict(dim=3, n_modes=(16, 16, 16), L=1.0, prec=0, tol=1e-6, upsampfac=2.0, ntrans=1, max_points=100,
             fluid=0, navier_stokes=0, ninst=0, deterministic=0)
    o.update(kw)
    return B._Opts(o["dim"], (ctypes.c_int64 * 3)(*o["n_modes"]), o["L"], o["prec"], o["tol"], o["upsampfac"],
                   o["ntrans"], o["max_points"], o["fluid"], o["navier_stokes"], o["ninst"],
                   o["deterministic"])


@pytest.mark.parametrize("kw,status", [
    (dict(dim=1), 1), (dict(dim=4), 1), (dict(n_modes=(1, 16, 16)), 1), (dict(L=0.0), 1), (dict(L=float("nan")), 1),
    (dict(prec=7), 1), (dict(upsampfac=1.7), 1), (dict(upsampfac=1.5, prec=1, tol=1e-6), 2), (dict(upsampfac=1.25, tol=1e-10), 2), (dict(upsampfac=1.25, prec=1, tol=1e-4), 2), (dict(ntrans=0), 1), (dict(max_points=-1), 1),
    (dict(navier_stokes=1, fluid=0), 1),
    (dict(ninst=2), 1), (dict(ninst=2, fluid=1, navier_stokes=1), 1), (dict(ninst=2, fluid=1, ntrans=2), 1),
    (dict(ninst=5000, fluid=1), 1), (dict(ninst=-1), 1), (dict(deterministic=2), 1),
    (dict(prec=1, tol=1e-10), 2), (dict(prec=0, tol=1e-16), 2), (dict(tol=0.5), 2),
])
def test_plan_argument_errors_come_before_device_use(kw, status):
    lib = B.load_library()
    h = ctypes.c_void_p()
    assert lib.fsib_plan_create(ctypes.byref(_opts(**kw)), ctypes.byref(h)) == status
    assert h.value is None
    assert lib.fsib_last_error()


def test_null_arguments_rejected():
    lib = B.load_library()
    assert lib.fsib_plan_create(None, None) == 1
    assert lib.fsib_plan_destroy(None) == 1
    assert lib.fsib_spread(None, 0, None, None, None, 1.0, None) == 1
    assert lib.fsib_interp(None, 0, None, None, None, None) == 1
    assert lib.fsib_step(None, None, None, 0, None, None, None, None, None) == 1
    f = B._Force(99, 1.0, None, 0, None, None)
    assert lib.fsib_compute_force(ctypes.byref(f), 3, 10, None, None, None) == 1


@pytest.mark.skipif(B.device_count() > 0, reason="only meaningful on a host without a GPU")
def test_no_device_reported():
    lib = B.load_library()
    assert lib.fsib_device_count() == 0
    h = ctypes.c_void_p()
    assert lib.fsib_plan_create(ctypes.byref(_opts()), ctypes.byref(h)) == 3


def test_adjoint_helpers_reject_null_plan():
    lib = B.load_library()
    assert lib.fsib_spectral_scale(None, 0, 0, 1.0, None, None, None) == 1
    assert lib.fsib_grad_combine(None, 0, 0, None, None, None, None, 1.0, None, 0, None) == 1


def test_force_jvp_rejects_bad_arguments():
    lib = B.load_library()
    f = B._Force(99, 1.0, None, 0, None, None)
    assert lib.fsib_force_jvp(ctypes.byref(f), 3, 10, None, None, None, None) == 1
    g = B._Force(B.FSIB_FORCE_CURVE_TENSION, 1.0, None, 0, None, None)
    assert lib.fsib_force_jvp(ctypes.byref(g), 2, 10, None, None, None, None) == 1
    assert lib.fsib_force_jvp(ctypes.byref(g), 4, 10, None, None, None, None) == 1
    assert lib.fsib_force_jvp(ctypes.byref(g), 2, -1, None, None, None, None) == 1
    assert lib.fsib_force_jvp(ctypes.byref(g), 2, 0, None, None, None, None) == 0  # nothing to do


def test_new_force_kinds_and_pressure_reject_bad_arguments():
    lib = B.load_library()
    for kind in (B.FSIB_FORCE_EDGE_SPRINGS, B.FSIB_FORCE_TARGET):
        f = B._Force(kind, 1.0, None, 0, None, None, None)  # no CSR / no targets
        assert lib.fsib_compute_force(ctypes.byref(f), 3, 10, None, None, None) == 1
        assert lib.fsib_force_jvp(ctypes.byref(f), 2, 10, None, None, None, None) == 1
        assert lib.fsib_compute_force(ctypes.byref(f), 3, 0, None, None, None) == 0  # nothing to do
    assert lib.fsib_pressure(None, None, None, None, None, None) == 1


def test_fluid_params_layout():
    # the C struct is {int; double rho, mu, dt; double body[3]}
    assert ctypes.sizeof(B._Params) == 8 + 3 * 8 + 3 * 8
    assert B._Params.body.offset == 32
    assert ctypes.sizeof(B._Force) == 7 * 8


def test_set_instances_rejects_null_plan():
    lib = B.load_library()
    assert lib.fsib_plan_set_instances(None, None) == 1


def test_tuning_rejects_null_arguments():
    lib = B.load_library()
    t = B._Tuning(0, 0, 512, 1, 8, 0, 0)
    assert lib.fsib_plan_tuning(None, ctypes.byref(t), 1) == 1


def test_tuning_struct_matches_header():
    """The binding's tuning struct lists the header's fields in order (seven ints)."""
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "fsib.h")).read()
    body = hdr[hdr.index("/* Launch-shape knobs of a plan"):hdr.index("} fsib_tuning;")]
    fields = re.findall(r"^\s*int (\w+);", body, re.M)
    assert fields == [k for k, _ in B._Tuning._fields_]
    assert ctypes.sizeof(B._Tuning) == 4 * len(fields) == 28


def test_group_calls_reject_bad_arguments():
    lib = B.load_library()
    h = ctypes.c_void_p()
    assert lib.fsib_group_create(0, None, ctypes.byref(h)) == 1
    assert lib.fsib_group_create(9, None, ctypes.byref(h)) == 1
    assert lib.fsib_group_create(1, None, ctypes.byref(h)) == 1
    assert h.value is None
    null = (ctypes.c_void_p * 2)(None, None)
    assert lib.fsib_group_create(2, null, ctypes.byref(h)) == 1
    assert lib.fsib_group_create(1, null, None) == 1
    assert lib.fsib_group_steps(None, None, None, None, None, None, None, 1, None) == 1
    assert lib.fsib_group_destroy(None) == 0
