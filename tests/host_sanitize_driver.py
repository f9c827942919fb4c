"""Runs the library's host set-up paths (meshes, spaces with their colouring and
numbering for every cell type, the host validation of the C-ABI) against the
library path given as argv[1]; used under AddressSanitizer/UndefinedBehaviorSanitizer
by test_host_sanitize.py. Needs no GPU."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import paper_1903_08243_amd.api as api  # noqa: E402

api._LIB_PATH = sys.argv[1]
import paper_1903_08243_amd as mf  # noqa: E402
from paper_1903_08243_amd import meshgen as mg  # noqa: E402

L = mf.load_library()
spaces = 0
for k in (1, 2, 3, 6):
    m = mg.hex_mesh(4, 0.15, config=1, seed_k=k)
    sp = mf.Space.from_meshgen(mg.hex_space(m, k, ncomp=3 if k == 2 else 1, config=1))
    sp.colouring()
    sp.internal_to_user()
    spaces += 1
for k in (1, 2, 3):
    m = mg.tet_mesh(3, 0.2, config=2)
    sp = mf.Space.from_meshgen(mg.tet_space(m, k, ncomp=3, config=2))
    sp.colouring()
    sp.internal_to_user()
    m = mg.tri_mesh(8, 0.2, config=0)
    sp = mf.Space.from_meshgen(mg.tri_space(m, k, ncomp=1))
    sp.colouring()
    spaces += 2
for k in (1, 4):
    m = mg.quad_mesh(8, 0.25, config=0)
    sp = mf.Space.from_meshgen(mg.quad_space(m, k, ncomp=1))
    sp.colouring()
    spaces += 1
# host validation paths that return errors before any device work
h = ctypes.c_void_p()
coords = np.zeros((4, 3))
c2v = np.array([[0, 1, 2, 7]], dtype=np.int32)
assert L.mf_mesh_create(api.CELL_TET, 4, coords.ctypes.data, 1, c2v.ctypes.data, ctypes.byref(h)) == -1
c2v = np.array([[0, 1, 2, 3]], dtype=np.int32)
assert L.mf_mesh_create(api.CELL_TET, 4, coords.ctypes.data, 1, c2v.ctypes.data, ctypes.byref(h)) == -4
th = np.zeros(10, np.float32)
assert L.mf_cnn_create(5, 3, th.ctypes.data, ctypes.byref(h)) == -7
assert L.mf_cnn_load(b"/nonexistent/net.bin", ctypes.byref(h)) == -1
print(f"host paths ok: {spaces} spaces", flush=True)
