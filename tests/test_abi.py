"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and rejects bad arguments before it
touches a device."""
import ctypes
import os

import pytest

from paper_2106_03872_amd import ks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    syms = ks.header_symbols()
    assert {"ks_ham_apply", "ks_propagate_step", "ks_density", "ks_reduce", "ks_orthonormalize",
            "ks_system_create", "ks_system_destroy", "ks_system_set_vloc",
            "ks_system_set_projectors", "ks_last_error"} <= set(syms)
    lib = ks.library()
    for s in syms:
        assert hasattr(lib, s), s


def test_exports_match_header_exactly():
    # every exported ks_* function is declared in the header
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", ks.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T ks_" in line}
    assert exported == set(ks.header_symbols())


def _create(n, L, ecut, prec=0, max_norb=4):
    h = ctypes.c_void_p()
    st = ks.library().ks_system_create((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*L), ecut, prec,
                                       max_norb, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("n,L,ecut,prec,max_norb,expect", [
    ((16, 16, 24), (10, 10, 10), 10.0, 0, 4, ks.KS_EINVAL),        # n1 != n2
    ((16, 17, 17), (10, 10, 10), 10.0, 0, 4, ks.KS_EUNSUPPORTED),  # 17 has no kernel
    ((16, 16, 16), (10, -1, 10), 10.0, 0, 4, ks.KS_EINVAL),        # bad cell
    ((16, 16, 16), (10, 10, 10), 10.0, 0, 0, ks.KS_EINVAL),        # max_norb
    ((16, 16, 16), (10, 10, 10), 10.0, 7, 4, ks.KS_EUNSUPPORTED),  # precision
    ((0, 16, 16), (10, 10, 10), 10.0, 0, 4, ks.KS_EINVAL),         # empty grid
])
def test_create_rejects_bad_arguments(n, L, ecut, prec, max_norb, expect):
    st, h = _create(n, L, ecut, prec, max_norb)
    assert st == expect
    assert not h.value
    assert ks.library().ks_last_error(None)


def test_null_system_calls_fail_cleanly():
    lib = ks.library()
    assert lib.ks_ham_apply(None, 1, None, None, None) == ks.KS_EINVAL
    assert lib.ks_density(None, 1, None, None, None, None) == ks.KS_EINVAL
    assert lib.ks_propagate_step(None, 1, None, 0.1, 1, None, None, None) == ks.KS_EINVAL
    assert lib.ks_autotune(None, 1, None, None) == ks.KS_EINVAL
    assert lib.ks_hartree(None, None, None, 0, None) == ks.KS_EINVAL
    assert lib.ks_dipole(None, None, None, None) == ks.KS_EINVAL
    assert lib.ks_state_kick(None, None, None) == ks.KS_EINVAL
    assert lib.ks_state_propagate_etrs(None, 0.1, 1, None, None, None, None) == ks.KS_EINVAL
    assert lib.ks_state_eigensolve(None, 1, None, None, None) == ks.KS_EINVAL
    assert lib.ks_system_set_tuning(None, None) == ks.KS_EINVAL
    lib.ks_system_destroy(None)


def test_build_entry_points_exist():
    import importlib.util
    spec = importlib.util.spec_from_file_location("ge", os.path.join(ROOT, "__graft_entry__.py"))
    ge = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(ge)
    assert callable(ge.build) and callable(ge.smoke)


def test_footprint_caps_the_pass_at_the_grid_limit():
    """A pass holds at most 65535 orbitals (the y extent of a launch grid):
    the planner counts the default chunk and any larger chunk as 65535."""
    n, L = (8, 12, 12), (4.8, 7.2, 7.2)
    fp = lambda chunk: ks.plan_footprint(n, L, 10.0, 100000, 100, chunk=chunk)
    assert fp(0) == fp(65535) == fp(200000)
    assert fp(65534) < fp(65535)
