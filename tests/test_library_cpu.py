"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared_functions()
    for n in ["mf_mesh_create", "mf_space_create", "mf_op_create", "mf_op_apply", "mf_op_apply_range",
              "mf_op_diagonal", "mf_cg_solve", "mf_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1903_08243_amd import api
    path = api.library_path()
    if not os.path.exists(path):
        pytest.skip("libmf.so not built")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_errors_without_device_work():
    """Validation paths return MF_E* codes before touching the GPU."""
    import numpy as np
    from paper_1903_08243_amd import api
    if not os.path.exists(api.library_path()):
        pytest.skip("libmf.so not built")
    L = api.load_library()
    h = ctypes.c_void_p()
    coords = np.zeros((4, 3))
    c2v = np.array([[0, 1, 2, 7]], dtype=np.int32)  # vertex 7 out of range
    rc = L.mf_mesh_create(api.CELL_TET, 4, coords.ctypes.data, 1, c2v.ctypes.data, ctypes.byref(h))
    assert rc == -1 and b"out of range" in L.mf_last_error()
    c2v = np.array([[0, 1, 2, 3]], dtype=np.int32)  # all vertices coincide: degenerate
    rc = L.mf_mesh_create(api.CELL_TET, 4, coords.ctypes.data, 1, c2v.ctypes.data, ctypes.byref(h))
    assert rc == -4
    rc = L.mf_mesh_create(7, 4, coords.ctypes.data, 1, c2v.ctypes.data, ctypes.byref(h))
    assert rc == -1
    # tangled hex: swap two vertices of a unit cube
    from paper_1903_08243_amd import meshgen as mg
    m = mg.hex_mesh(1)
    c2v = m.cell2vert.copy()
    c2v[0, [0, 1]] = c2v[0, [1, 0]]
    rc = L.mf_mesh_create(api.CELL_HEX, m.nverts, np.ascontiguousarray(m.coords).ctypes.data, 1,
                          c2v.ctypes.data, ctypes.byref(h))
    assert rc == -4
    # a valid mesh, then a space with a bad node index and an unsupported degree
    rc = L.mf_mesh_create(api.CELL_HEX, m.nverts, np.ascontiguousarray(m.coords).ctypes.data, 1,
                          np.ascontiguousarray(m.cell2vert).ctypes.data, ctypes.byref(h))
    assert rc == 0
    s = ctypes.c_void_p()
    c2n = np.arange(8, dtype=np.int32)
    c2n[3] = 8
    assert L.mf_space_create(h, 1, 1, c2n.ctypes.data, 8, ctypes.byref(s)) == -1
    c2n[3] = 3
    assert L.mf_space_create(h, 7, 1, c2n.ctypes.data, 8, ctypes.byref(s)) == -7
    assert L.mf_space_create(h, 1, 1, c2n.ctypes.data, 8, ctypes.byref(s)) == 0
    L.mf_space_destroy(s)
    L.mf_mesh_destroy(h)


def test_learned_precond_host_validation():
    """Channel counts, parameter counts and unreadable network files are rejected
    on the host."""
    import numpy as np
    from paper_1903_08243_amd import api
    if not os.path.exists(api.library_path()):
        pytest.skip("libmf.so not built")
    lib = api.load_library()
    for c in (4, 8, 16):
        for L in (2, 3, 6):
            assert lib.mf_cnn_nparams(c, L) == 27 * (2 * c + (2 * L - 2) * c * c)
    assert lib.mf_cnn_nparams(5, 3) == -1
    assert lib.mf_cnn_nparams(8, 1) == -1
    th = np.zeros(10, np.float32)
    h = ctypes.c_void_p()
    assert lib.mf_cnn_create(5, 3, th.ctypes.data, ctypes.byref(h)) == -7
    assert lib.mf_cnn_create(8, 9, th.ctypes.data, ctypes.byref(h)) == -7
    assert lib.mf_cnn_load(b"/nonexistent/net.bin", ctypes.byref(h)) == -1
    assert lib.mf_cnn_forward(None, 1, 5, 5, 5, None, None, None) == -1
