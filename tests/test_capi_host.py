"""Host-side checks of the C-ABI library: it loads, exports every declared
entry point, and its host-only calls (G-sphere, status strings, validation
before any launch) behave as documented. No device work is started."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rpa.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rpa_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1307_8052_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("HIP library not built: run python -m paper_1307_8052_amd.build")
    return _capi.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "rpa_ec" in names and "rpa_chi0" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for code in range(-7, 1):
        assert L.rpa_status_string(code)
    assert b"positive definite" in L.rpa_status_string(-5)


@pytest.mark.parametrize("cfg", ["cfg0", "cfg1q1", "tiny_oblique"])
def test_gsphere_matches_oracle(cfg):
    import paper_1307_8052_amd as rpa
    if cfg == "cfg0":
        w = synth.config0(n_occ=1, n_unocc=2)
        A, q, e, grid = w.A, w.qpoints[0].q, w.qpoints[0].ecut, w.grid
    elif cfg == "cfg1q1":
        A = np.diag([12.0, 12.0, 13.0])
        q = np.array([0.1 * 2 * np.pi / 12.0, 0.0, 0.0])
        e, grid = synth.ecut_for_count(A, q, 1500), (48, 48, 48)
    else:
        A = np.array([[7.0, 0.0, 0.0], [1.0, 6.5, 0.0], [0.5, 0.3, 8.0]])
        q, e, grid = np.array([0.05, -0.02, 0.03]), 1.7, (16, 16, 16)
    got = rpa.gsphere(A, grid, q, e)
    ref = oracle.gsphere(A, q, e)
    if cfg == "tiny_oblique":
        assert sorted(map(tuple, got.tolist())) == sorted(map(tuple, ref.tolist()))
    else:
        assert np.array_equal(got, ref)


def test_gsphere_capacity_error(L):
    import paper_1307_8052_amd as rpa
    from paper_1307_8052_amd import _capi
    cell = rpa._cell(np.eye(3) * 10.0, (16, 16, 16))
    q = np.zeros(3)
    ng = ctypes.c_int(0)
    out = np.zeros((2, 3), dtype=np.int32)
    rc = L.rpa_gsphere(ctypes.byref(cell), q.ctypes.data_as(_capi.P_f64), 2.0,
                       out.ctypes.data_as(_capi.P_i32), 2, ctypes.byref(ng))
    assert rc == _capi.RPA_ERR_SHAPE and ng.value > 2


def test_create_rejects_unsupported_grid(L):
    import paper_1307_8052_amd as rpa
    from paper_1307_8052_amd import _capi
    h = ctypes.c_void_p()
    cell = rpa._cell(np.eye(3) * 10.0, (14, 16, 16))  # 14 = 2 * 7
    assert L.rpa_create(ctypes.byref(h), ctypes.byref(cell), 0, 0) == _capi.RPA_ERR_UNSUPPORTED
    assert b"14" in L.rpa_last_error(None)
    assert L.rpa_create(None, ctypes.byref(cell), 0, 0) == _capi.RPA_ERR_INPUT
