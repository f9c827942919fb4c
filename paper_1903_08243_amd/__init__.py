"""MI355X-native matrix-free finite element operator action (gfx950 HIP kernels).

The compute path is the C-ABI library ``libmf.so`` (declared in
``include/mf.h``); this package only marshals arguments to it. PyTorch is
used for device memory and streams. If the library has not been built the
first call raises -- there is no CPU fallback.
"""
from .api import (  # noqa: F401
    CELL_HEX, CELL_QUAD, CELL_TET, CELL_TRI, F32, F64, SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_COLOURED, SCATTER_PATCH, MASS, HELMHOLTZ, LAPLACIAN, POISSON, ELASTICITY, HYPERELASTIC,
    MFError, Mesh, Space, Operator, JacobiPrecond, LearnedPrecond, CNN, Batch, cg_solve, cnn_nparams,
    cnn_initial_weights, library_path, load_library, probe_peaks,
)
