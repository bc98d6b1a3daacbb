"""The C ABI library loads and exports every function include/wwbi.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wwbi.h")
LIB = os.path.join(ROOT, "paper_2108_01786_amd", "libwwbi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wwbi_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for must in ("wwbi_create", "wwbi_destroy", "wwbi_solve_phi", "wwbi_solve_gamma",
                 "wwbi_adjoint_phi", "wwbi_solve_phi_multi", "wwbi_tangent_phi", "wwbi_spectral",
                 "wwbi_debug_matrix", "wwbi_matvec", "wwbi_status_str", "wwbi_default_opts",
                 "wwbi_tangential_energy", "wwbi_solve_gamma_t", "wwbi_stage_rhs",
                 "wwbi_rk_step", "wwbi_boundary_velocity", "wwbi_interior_eval",
                 "wwbi_interior_velocity", "wwbi_pressure"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwwbi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwwbi.so not built")
def test_host_only_helpers():
    """Functions that touch no device: default options and status strings."""
    from paper_2108_01786_amd import wwbi
    o = wwbi.make_opts()
    assert o.tol == 1e-13 and o.restart == 100 and o.precision == wwbi.FP64
    assert wwbi.status_str(wwbi.EINVAL_ORIENTATION).startswith("invalid argument")
    assert wwbi.status_str(wwbi.NOT_CONVERGED) == "not converged"
    assert "Fourier tail" in wwbi.status_str(wwbi.WARN_UNDERRESOLVED)
    assert "30" in wwbi.status_str(wwbi.EINVAL_RANGE)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwwbi.so not built")
def test_struct_layouts_match_header():
    """ctypes mirrors of the option and report structs have the C sizes."""
    from paper_2108_01786_amd import wwbi
    assert ctypes.sizeof(wwbi._Opts) == 8 + 8 + 4 * 8 + 8
    assert ctypes.sizeof(wwbi.Report) == 4 * 4 + 8 * 6 + 4 * 2 + 8 * 3 + 4 * 2 + 8 * 32
