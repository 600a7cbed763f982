"""CPU checks of the C ABI: the library loads, exports every function that
include/pdep.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1501_03141_amd import pdep


@pytest.fixture(scope="module")
def lib():
    return pdep.load()


def test_exports_every_declared_function(lib):
    names = pdep.header_functions()
    assert {"pdep_setup", "chi0_apply", "chi0_apply_raw", "pdep_eigs", "pdep_destroy",
            "pdep_last_error", "pdep_default_opts", "pdep_get_info", "pdep_get_gvectors",
            "pdep_get_orbitals"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_default_opts(lib):
    o = pdep.Opts()
    lib.pdep_default_opts(C.byref(o))
    assert o.precision == pdep.PDEP_FP64 and o.cg_tol == 1e-10 and o.precond == 1
    assert o.cg_maxit == 2000 and o.refine_maxit == 8 and o.flags == 0 and o.rhs_tile == 0


def _setup(lib, L=(10.0, 10.0, 10.0), n=(16, 16, 16), ecut=5.0, n_v=4, vloc=None, precision=0):
    cell = pdep.Cell((C.c_double * 3)(*L), (C.c_int * 3)(*n), ecut)
    o = pdep.Opts()
    lib.pdep_default_opts(C.byref(o))
    o.n_v = n_v
    o.precision = precision
    v = np.zeros(int(np.prod(n))) if vloc is None else vloc
    h = C.c_void_p()
    rc = lib.pdep_setup(C.byref(cell), v.ctypes.data, C.byref(o), None, None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [dict(n=(16, 16, 7)), dict(n=(16, 16, 256)), dict(L=(10.0, -1.0, 10.0)),
                                dict(ecut=-1.0), dict(n_v=0), dict(precision=7),
                                dict(ecut=80.0)])
def test_setup_rejects_bad_arguments(lib, kw):
    rc, h = _setup(lib, **kw)
    assert rc == pdep.PDEP_EINVAL
    assert h.value is None
    assert len(lib.pdep_last_error()) > 0


def test_setup_rejects_nan_potential(lib):
    v = np.zeros(16 ** 3)
    v[5] = math.nan
    rc, h = _setup(lib, vloc=v)
    assert rc == pdep.PDEP_EINVAL
    assert b"NaN" in lib.pdep_last_error()


def test_null_arguments(lib):
    h = C.c_void_p()
    assert lib.pdep_setup(None, None, None, None, None, C.byref(h)) == pdep.PDEP_EINVAL
    assert lib.chi0_apply(None, 1, None, None, None) == pdep.PDEP_EINVAL
    assert lib.pdep_get_info(None, None) == pdep.PDEP_EINVAL
    assert lib.pdep_qp_energies(None, 1, None, 1, None, None, None, None, 0, None, None, None) == pdep.PDEP_EINVAL
    assert lib.pdep_destroy(None) == pdep.PDEP_OK


def test_header_parser_finds_declarations():
    names = pdep.header_functions()
    assert "chi0_apply" in names and "pdep_setup" in names
