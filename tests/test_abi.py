"""The C ABI library loads, exports what include/fct.h declares, and rejects
bad inputs on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fct.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fct_[A-Za-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def fct():
    from paper_2309_14584_amd import fct as mod
    return mod


def test_header_symbols_exported(fct):
    names = _declared()
    assert "fct_plan_create" in names and "fct_solve" in names
    lib = ctypes.CDLL(fct.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(fct.EXPORTED) == names


def test_abi_version_and_strings(fct):
    assert fct.abi_version() == fct.ABI_VERSION == 3
    assert fct._status_string(fct.FCT_ERANK) == b"FCT_ERANK"
    assert fct._status_string(99) == b"FCT_UNKNOWN"


def _create(fct, S, G, flags=0):
    S = np.ascontiguousarray(S, dtype=np.int32)
    G = np.ascontiguousarray(G, dtype=np.int32)
    h = ctypes.c_void_p()
    st = fct._plan_create(S.shape[1] if S.ndim == 2 else 0, S.shape[0],
                          S.ctypes.data_as(ctypes.c_void_p), G.shape[0],
                          G.ctypes.data_as(ctypes.c_void_p), flags, None, ctypes.byref(h))
    return st, fct._last_error().decode(), h


def test_host_validation_errors(fct):
    S = np.array([[0, 0], [1, 0], [0, 1]])
    assert _create(fct, S, np.array([[-1, 2]]))[0] == fct.FCT_EINVAL
    assert _create(fct, S, np.array([[64, 2]]))[0] == fct.FCT_EINVAL
    st, msg, _ = _create(fct, np.array([[0, 0], [1, 0], [1, 0]]), np.array([[3, 3]]))
    assert st == fct.FCT_EINVAL and "equal" in msg
    assert _create(fct, np.array([[0, -1]]), np.array([[3, 3]]))[0] == fct.FCT_EINVAL
    st, msg, _ = _create(fct, np.zeros((1, 129)), np.zeros((1, 129)))
    assert st == fct.FCT_EINVAL and "D=129" in msg


def test_rank_precheck(fct):
    # degrees 0..6 on the same N=3 grid twice: 0 and 6 alias on every grid
    S = np.arange(7)[:, None]
    st, msg, _ = _create(fct, S, np.array([[3], [3]]))
    assert st == fct.FCT_ERANK and "dimension 0" in msg


def test_python_binding_refuses_missing_library(tmp_path):
    """The binding raises on import when the shared library is absent."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2309_14584_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2309_14584_amd", "fct.py"), pkg / "fct.py")
    (pkg / "__init__.py").write_text("")
    r = subprocess.run([sys.executable, "-c", "import paper_2309_14584_amd.fct"],
                       cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0 and "libfct is not built" in r.stderr


def test_gauss_rank_precheck_and_flags(fct):
    """Host checks of a Gauss-grid plan (before any device work): T_{N+1}
    vanishing on every grid, degrees equal up to sign, unknown flags."""
    G = fct.FCT_PLAN_GAUSS
    st, msg, _ = _create(fct, np.array([[0], [3]]), np.array([[2], [2]]), G)
    assert st == fct.FCT_ERANK and "vanishes" in msg
    st, msg, _ = _create(fct, np.arange(4)[:, None], np.array([[1], [1]]), G)
    assert st == fct.FCT_ERANK
    # grids N = 0 (node x = 0) and N = 1: T_3 = -T_1 on both (T_1 and T_3
    # vanish at x = 0), so degree 3 repeats degree 1 up to sign
    st, msg, _ = _create(fct, np.arange(4)[:, None], np.array([[0], [1]]), G)
    assert st == fct.FCT_ERANK and "degree 3" in msg and "up to sign" in msg
    st, msg, _ = _create(fct, np.array([[0], [1]]), np.array([[3]]), 8)
    assert st == fct.FCT_EINVAL and "flags" in msg


def test_rows_by_member_flag_checks(fct):
    S = np.array([[0, 0], [1, 0], [0, 1]])
    st, msg, _ = _create(fct, S, np.array([[3, 3]]),
                         fct.FCT_PLAN_GAUSS | fct.FCT_PLAN_ROWS_BY_MEMBER)
    assert st == fct.FCT_EINVAL and "combine" in msg
