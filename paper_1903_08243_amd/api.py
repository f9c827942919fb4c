"""ctypes binding of include/mf.h (argument marshalling only).

Every numerical step runs in libmf.so's HIP kernels. Device vectors are torch
tensors on the GPU; the binding passes their data pointers and the current
torch stream to the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

CELL_TRI, CELL_TET, CELL_HEX, CELL_QUAD = 0, 1, 2, 3
MASS, HELMHOLTZ, LAPLACIAN, POISSON, ELASTICITY, HYPERELASTIC = range(6)
F64, F32 = 0, 1
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_COLOURED, SCATTER_PATCH = 0, 1, 2, 3
_ERR = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EMESH", -5: "ENOTCONV", -6: "EBREAKDOWN",
        -7: "EUNSUPPORTED"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmf.so")
_lib = None


class MFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"MF_{_ERR.get(code, code)}: {msg}")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


class _OpInfo(ctypes.Structure):
    _fields_ = [("ncells", ctypes.c_int64), ("nnodes", ctypes.c_int64), ("ndofs", ctypes.c_int64),
                ("cell_type", ctypes.c_int), ("kind", ctypes.c_int), ("precision", ctypes.c_int),
                ("degree", ctypes.c_int), ("ncomp", ctypes.c_int), ("nq1d", ctypes.c_int),
                ("nqp", ctypes.c_int), ("dofs_per_cell", ctypes.c_int),
                ("flops_per_apply", ctypes.c_double), ("bytes_per_apply", ctypes.c_double),
                ("cell_launches", ctypes.c_int), ("ncolours", ctypes.c_int), ("clears_output", ctypes.c_int),
                ("scatter", ctypes.c_int)]


class _OpParams(ctypes.Structure):
    _fields_ = [("vertex_coef", ctypes.c_void_p), ("lam", ctypes.c_double), ("mu", ctypes.c_double),
                ("dirichlet", ctypes.c_void_p), ("scatter", ctypes.c_int), ("u0", ctypes.c_void_p)]


class CGInfo(ctypes.Structure):
    _fields_ = [("outer_iterations", ctypes.c_int), ("inner_iterations", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("rel_residual", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load_library():
    """Load libmf.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run __graft_entry__.build() "
                          "(python -m paper_1903_08243_amd.build)")
    L = ctypes.CDLL(_LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "mf_mesh_create": (I, [I, I64, P, I64, P, PP]),
        "mf_space_create": (I, [P, I, I, P, I64, PP]),
        "mf_op_create": (I, [P, I, I, I, ctypes.POINTER(_OpParams), P, PP]),
        "mf_op_apply": (I, [P, P, P, P]),
        "mf_op_apply_range": (I, [P, I64, I64, P, P, I, P]),
        "mf_op_diagonal": (I, [P, P, P]),
        "mf_op_apply_internal": (I, [P, P, P, P]),
        "mf_op_apply_range_internal": (I, [P, I64, I64, P, P, I, P]),
        "mf_space_get_permutation": (I, [P, P]),
        "mf_space_get_colouring": (I, [P, P, P, ctypes.POINTER(ctypes.c_int)]),
        "mf_op_get_info": (I, [P, ctypes.POINTER(_OpInfo)]),
        "mf_op_csr_pattern": (I, [P, P, P, P, ctypes.POINTER(I64)]),
        "mf_op_assemble_csr": (I, [P, P, P, P]),
        "mf_precond_create_jacobi": (I, [P, P, PP]),
        "mf_cg_solve": (I, [P, P, P, P, P, D, D, I, ctypes.POINTER(CGInfo), P]),
        "mf_cg_solve_noalloc": (I, [P, P, P, P, P, D, D, I, ctypes.POINTER(CGInfo), P]),
        "mf_batch_create": (I, [I, P, P, P, P, P, P, PP]),
        "mf_batch_solve": (I, [P, D, D, I, P, P]),
        "mf_batch_apply": (I, [P, I, P]),
        "mf_batch_apply_user": (I, [P, I, P, P, P]),
        "mf_batch_autotune": (I, [P, ctypes.c_char_p, P]),
        "mf_batch_get_tuning": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "mf_batch_set_tuning": (I, [P, I, I]),
        "mf_batch_destroy": (None, [P]),
        "mf_mesh_destroy": (None, [P]),
        "mf_space_destroy": (None, [P]),
        "mf_op_destroy": (None, [P]),
        "mf_precond_destroy": (None, [P]),
        "mf_precond_apply": (I, [P, P, P, P]),
        "mf_cnn_nparams": (I64, [I, I]),
        "mf_cnn_create": (I, [I, I, P, PP]),
        "mf_cnn_get_params": (I, [P, P]),
        "mf_cnn_set_params": (I, [P, P]),
        "mf_cnn_save": (I, [P, ctypes.c_char_p]),
        "mf_cnn_load": (I, [ctypes.c_char_p, PP]),
        "mf_cnn_destroy": (None, [P]),
        "mf_cnn_forward": (I, [P, I, I, I, I, P, P, P]),
        "mf_cnn_loss_grad": (I, [P, I, I, I, I, P, P, ctypes.POINTER(D), P, P]),
        "mf_cnn_train": (I, [P, I, I, P, P, I, I, P, ctypes.c_float, P, P]),
        "mf_precond_create_cnn": (I, [P, P, I, I, I, P, P, PP]),
        "mf_precond_harvest": (I, [P, P, P, I, I, P, P, P, P]),
        "mf_cnn_energy_loss_grad": (I, [P, P, P, P, ctypes.POINTER(D), P, P]),
        "mf_cnn_train_energy": (I, [P, P, P, I, P, I, P, ctypes.c_float, P, P]),
        "mf_probe_peaks": (I, [P, P]),
        "mf_last_error": (ctypes.c_char_p, []),
        "mf_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise MFError(rc, load_library().mf_last_error().decode())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=None):
    """Device pointer of a torch tensor (contiguous, on the GPU)."""
    if not t.is_cuda:
        raise ValueError("device vectors must be GPU tensors")
    if not t.is_contiguous():
        raise ValueError("device vectors must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def probe_peaks(stream=None):
    """Attainable device rates (mf_probe_peaks): HBM copy GB/s, FP64 / FP32 vector and
    FP32 / FP64 matrix TFLOP/s."""
    out = (ctypes.c_double * 5)()
    _check(load_library().mf_probe_peaks(out, _stream(stream)))
    keys = ("hbm_copy_gbs", "fp64_vector_tflops", "fp32_vector_tflops", "fp32_mfma_tflops", "fp64_mfma_tflops")
    return dict(zip(keys, list(out)))


class Mesh:
    def __init__(self, cell_type, coords, cell2vert):
        L = load_library()
        self._coords = _np(coords, np.float64)
        self._c2v = _np(cell2vert, np.int32)
        h = ctypes.c_void_p()
        _check(L.mf_mesh_create(cell_type, self._coords.shape[0], self._coords.ctypes.data,
                                self._c2v.shape[0], self._c2v.ctypes.data, ctypes.byref(h)))
        self.handle, self.cell_type = h, cell_type
        self.nverts, self.ncells = self._coords.shape[0], self._c2v.shape[0]

    @classmethod
    def from_meshgen(cls, m):
        return cls(m.cell_type, m.coords, m.cell2vert)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_mesh_destroy(self.handle)
            self.handle = None


class Space:
    def __init__(self, mesh: Mesh, degree, ncomp, cell2node, nnodes):
        L = load_library()
        c2n = _np(cell2node, np.int32)
        h = ctypes.c_void_p()
        _check(L.mf_space_create(mesh.handle, degree, ncomp, c2n.ctypes.data, int(nnodes), ctypes.byref(h)))
        self.handle, self.mesh = h, mesh
        self.degree, self.ncomp, self.nnodes = degree, ncomp, int(nnodes)
        self.ndofs = self.nnodes * ncomp

    def internal_to_user(self):
        """Host array: user node of each internal node (the library's cell-order numbering)."""
        out = np.empty(self.nnodes, dtype=np.int32)
        _check(load_library().mf_space_get_permutation(self.handle, out.ctypes.data))
        return out

    def colouring(self):
        """(internal -> user cell order, colour offsets) of the library's cell colouring."""
        L = load_library()
        n = ctypes.c_int()
        _check(L.mf_space_get_colouring(self.handle, None, None, ctypes.byref(n)))
        order = np.empty(self.mesh.ncells, dtype=np.int32)
        ptr = np.empty(n.value + 1, dtype=np.int64)
        _check(L.mf_space_get_colouring(self.handle, order.ctypes.data, ptr.ctypes.data, ctypes.byref(n)))
        return order, ptr

    @classmethod
    def from_meshgen(cls, s, mesh: Mesh | None = None):
        mesh = mesh or Mesh.from_meshgen(s.mesh)
        return cls(mesh, s.degree, s.ncomp, s.cell2node, s.nnodes)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_space_destroy(self.handle)
            self.handle = None


class Operator:
    """A matrix-free operator; apply() runs the HIP kernels on the current torch stream."""

    def __init__(self, space: Space, kind, precision=F64, nq1d=0, vertex_coef=None, lam=1.0, mu=0.5,
                 dirichlet=None, scatter=SCATTER_AUTO, stream=None, u0=None):
        L = load_library()
        self._coef = None if vertex_coef is None else _np(vertex_coef, np.float64)
        self._bc = None if dirichlet is None else _np(dirichlet, np.uint8)
        self._u0 = None if u0 is None else _np(u0, np.float64)
        pr = _OpParams(None if self._coef is None else self._coef.ctypes.data, lam, mu,
                       None if self._bc is None else self._bc.ctypes.data, scatter,
                       None if self._u0 is None else self._u0.ctypes.data)
        h = ctypes.c_void_p()
        _check(L.mf_op_create(space.handle, kind, precision, nq1d, ctypes.byref(pr), _stream(stream),
                              ctypes.byref(h)))
        self.handle, self.space = h, space
        info = _OpInfo()
        _check(L.mf_op_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _OpInfo._fields_}
        self.ndofs = info.ndofs
        self.precision = precision

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == F64 else torch.float32

    def apply(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.ndofs, dtype=self.torch_dtype, device=x.device)
        self._size(x), self._size(y)
        _check(load_library().mf_op_apply(self.handle, _dev(x, self.torch_dtype), _dev(y, self.torch_dtype),
                                          _stream(stream)))
        return y

    def apply_internal(self, x, y=None, stream=None):
        """y = A x with x, y in the space's internal numbering (no boundary permutation)."""
        import torch
        if y is None:
            y = torch.empty(self.ndofs, dtype=self.torch_dtype, device=x.device)
        self._size(x), self._size(y)
        _check(load_library().mf_op_apply_internal(self.handle, _dev(x, self.torch_dtype),
                                                   _dev(y, self.torch_dtype), _stream(stream)))
        return y

    def apply_range_internal(self, start, end, x, y, accumulate=False, stream=None):
        self._size(x), self._size(y)
        _check(load_library().mf_op_apply_range_internal(self.handle, start, end, _dev(x, self.torch_dtype),
                                                         _dev(y, self.torch_dtype), int(accumulate),
                                                         _stream(stream)))
        return y

    def apply_range(self, start, end, x, y, accumulate=False, stream=None):
        self._size(x), self._size(y)
        _check(load_library().mf_op_apply_range(self.handle, start, end, _dev(x, self.torch_dtype),
                                                _dev(y, self.torch_dtype), int(accumulate), _stream(stream)))
        return y

    def csr(self, stream=None):
        """The assembled sparse matrix (user numbering): (rowptr int64 numpy, col int32
        numpy, vals device tensor of the operator's precision)."""
        import torch
        L = load_library()
        nnz = ctypes.c_int64()
        sh = self.space.handle
        _check(L.mf_op_csr_pattern(self.handle, sh, None, None, ctypes.byref(nnz)))
        rowptr = np.empty(self.ndofs + 1, np.int64)
        col = np.empty(nnz.value, np.int32)
        _check(L.mf_op_csr_pattern(self.handle, sh, rowptr.ctypes.data, col.ctypes.data, None))
        vals = torch.empty(max(1, nnz.value), dtype=self.torch_dtype, device="cuda")[:nnz.value]
        _check(L.mf_op_assemble_csr(self.handle, sh, _dev(vals, self.torch_dtype), _stream(stream)))
        return rowptr, col, vals

    def diagonal(self, stream=None):
        import torch
        d = torch.empty(self.ndofs, dtype=self.torch_dtype, device="cuda")
        _check(load_library().mf_op_diagonal(self.handle, _dev(d), _stream(stream)))
        return d

    def _size(self, t):
        if t.numel() != self.ndofs:
            raise ValueError(f"vector has {t.numel()} entries, operator has {self.ndofs} dofs")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_op_destroy(self.handle)
            self.handle = None


class _Precond:
    def apply(self, r, z=None, stream=None):
        """z = M r (FP64 device vectors, user numbering)."""
        import torch
        if z is None:
            z = torch.empty_like(r)
        _check(load_library().mf_precond_apply(self.handle, _dev(r, torch.float64), _dev(z, torch.float64),
                                               _stream(stream)))
        return z

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_precond_destroy(self.handle)
            self.handle = None


class JacobiPrecond(_Precond):
    def __init__(self, op: Operator, stream=None):
        h = ctypes.c_void_p()
        _check(load_library().mf_precond_create_jacobi(op.handle, _stream(stream), ctypes.byref(h)))
        self.handle = h


def cnn_nparams(channels, levels):
    n = load_library().mf_cnn_nparams(channels, levels)
    if n < 0:
        raise ValueError("channels must be 4, 8 or 16 and levels 2..8")
    return n


def cnn_initial_weights(channels, levels, seed=0, scale=0.02):
    """Initial parameters: small seeded Gaussian weights, so that the network starts
    close to the identity (and the preconditioner close to Jacobi). Host float32."""
    g = np.random.default_rng([1903, 8243, seed])
    return (g.standard_normal(cnn_nparams(channels, levels)) * scale).astype(np.float32)


class CNN:
    """The learned preconditioner's network (see include/mf.h). Lattices are
    float32 device tensors shaped [batch, nz, ny, nx]."""

    def __init__(self, channels, levels, theta=None, _handle=None):
        L = load_library()
        self.channels, self.levels = channels, levels
        self.nparams = cnn_nparams(channels, levels)
        if _handle is not None:
            self.handle = _handle
            return
        th = _np(cnn_initial_weights(channels, levels) if theta is None else theta, np.float32)
        if th.size != self.nparams:
            raise ValueError(f"theta must have {self.nparams} entries")
        h = ctypes.c_void_p()
        _check(L.mf_cnn_create(channels, levels, th.ctypes.data, ctypes.byref(h)))
        self.handle = h

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        _check(load_library().mf_cnn_load(path.encode(), ctypes.byref(h)))
        with open(path, "rb") as f:  # the library validated the header
            channels, levels = (int(v) for v in np.frombuffer(f.read(16)[8:16], dtype="<i4"))
        return cls(channels, levels, _handle=h)

    def params(self):
        th = np.empty(self.nparams, np.float32)
        _check(load_library().mf_cnn_get_params(self.handle, th.ctypes.data))
        return th

    def set_params(self, theta):
        th = _np(theta, np.float32)
        if th.size != self.nparams:
            raise ValueError(f"theta must have {self.nparams} entries")
        _check(load_library().mf_cnn_set_params(self.handle, th.ctypes.data))

    def save(self, path):
        _check(load_library().mf_cnn_save(self.handle, path.encode()))

    def forward(self, x, y=None, stream=None):
        import torch
        if x.dim() != 4:
            raise ValueError("x must be [batch, nz, ny, nx]")
        if y is None:
            y = torch.empty_like(x)
        B, nz, ny, nx = x.shape
        _check(load_library().mf_cnn_forward(self.handle, B, nz, ny, nx, _dev(x, torch.float32),
                                             _dev(y, torch.float32), _stream(stream)))
        return y

    def loss_grad(self, x, t, stream=None):
        import torch
        B, nz, ny, nx = x.shape
        g = torch.empty(self.nparams, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        _check(load_library().mf_cnn_loss_grad(self.handle, B, nz, ny, nx, _dev(x, torch.float32),
                                               _dev(t, torch.float32), ctypes.byref(loss), _dev(g),
                                               _stream(stream)))
        return loss.value, g

    def train(self, r, e, order, batch, lr=1e-3, stream=None):
        """Adam steps over pairs r, e ([npairs, n, n, n] float32); order: int array of
        nsteps * batch pair indices. Returns the per-step losses (before each step)."""
        import torch
        npairs, n = r.shape[0], r.shape[1]
        order = _np(order, np.int32)
        nsteps = order.size // batch
        losses = np.zeros(max(nsteps, 1), np.float64)
        _check(load_library().mf_cnn_train(self.handle, npairs, n, _dev(r, torch.float32), _dev(e, torch.float32),
                                           nsteps, batch, order.ctypes.data, lr, losses.ctypes.data,
                                           _stream(stream)))
        return losses[:nsteps]

    def energy_loss_grad(self, precond, op, r, stream=None):
        """Energy loss (z'Az - 2 z'r) / (r'D^-1 r) of z = precond(r) and its gradient."""
        import torch
        g = torch.empty(self.nparams, dtype=torch.float32, device=r.device)
        loss = ctypes.c_double()
        _check(load_library().mf_cnn_energy_loss_grad(self.handle, precond.handle, op.handle,
                                                      _dev(r, torch.float64), ctypes.byref(loss), _dev(g),
                                                      _stream(stream)))
        return loss.value, g

    def train_energy(self, precond, op, R, order, lr=1e-3, stream=None):
        """Adam steps on the energy loss; R: [nsamples, ndofs] float64 residuals (user
        numbering), order: sample index per step. Returns the per-step losses."""
        import torch
        if R.dim() != 2 or not R.is_contiguous():
            raise ValueError("R must be a contiguous [nsamples, ndofs] tensor")
        order = _np(order, np.int32)
        losses = np.zeros(max(order.size, 1), np.float64)
        _check(load_library().mf_cnn_train_energy(self.handle, precond.handle, op.handle, R.shape[0],
                                                  _dev(R, torch.float64), order.size, order.ctypes.data, lr,
                                                  losses.ctypes.data, _stream(stream)))
        return losses[:order.size]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_cnn_destroy(self.handle)
            self.handle = None


class LearnedPrecond(_Precond):
    """z = D^-1/2 N(D^-1/2 r) on the DoF lattice of a structured hex mesh
    (shape = (nz, ny, nx); node_grid[u] = lattice index of user node u)."""

    def __init__(self, op: Operator, net: CNN, shape, node_grid, stream=None):
        ng = _np(node_grid, np.int32)
        h = ctypes.c_void_p()
        nz, ny, nx = shape
        _check(load_library().mf_precond_create_cnn(op.handle, net.handle, nz, ny, nx, ng.ctypes.data,
                                                    _stream(stream), ctypes.byref(h)))
        self.handle, self.net, self.shape = h, net, tuple(shape)

    def harvest(self, r, e, corners, n, stream=None):
        """Diagonally scaled n^3 crops of the pair (r, e) at the given corners (z, y, x)."""
        import torch
        c = _np(corners, np.int32).reshape(-1, 3)
        ro = torch.empty((c.shape[0], n, n, n), dtype=torch.float32, device=r.device)
        eo = torch.empty_like(ro)
        _check(load_library().mf_precond_harvest(self.handle, _dev(r, torch.float64), _dev(e, torch.float64),
                                                 c.shape[0], n, c.ctypes.data, _dev(ro), _dev(eo), _stream(stream)))
        return ro, eo


def cg_solve(A64: Operator, b, x, A32: Operator | None = None, precond=None, rtol=1e-10, inner_rtol=0.0,
             maxit=10000, stream=None, raise_on_error=True, noalloc=False):
    """FP64 (optionally FP32-refined) preconditioned CG; x holds the initial guess.
    noalloc: the variant that allocates nothing (vectors in the library's fixed
    device array, MF_NOALLOC_SCRATCH_BYTES per GPU)."""
    import torch
    info = CGInfo()
    fn = load_library().mf_cg_solve_noalloc if noalloc else load_library().mf_cg_solve
    rc = fn(A64.handle, None if A32 is None else A32.handle,
                                    None if precond is None else precond.handle, _dev(b, torch.float64),
                                    _dev(x, torch.float64), rtol, inner_rtol, maxit, ctypes.byref(info),
                                    _stream(stream))
    if rc != 0 and raise_on_error:
        _check(rc)
    return info.as_dict() | {"rc": rc}


class Batch:
    """Many systems solved together: one persistent launch applies every operator
    per CG iteration; iterations are replayed from a captured hipGraph.

    The device vectors b[i] (rhs) and x[i] (initial guess / solution, user
    numbering, FP64) are bound at creation and must outlive the batch."""

    def __init__(self, A64, b, x, A32=None, M=None, stream=None):
        import torch
        L = load_library()
        n = len(A64)
        if len(b) != n or len(x) != n or (A32 is not None and len(A32) != n) or (M is not None and len(M) != n):
            raise ValueError("A64, b, x (and A32, M) must have the same length")
        for t in list(b) + list(x):
            _dev(t, torch.float64)
        P = ctypes.c_void_p
        self._keep = (list(A64), list(A32 or []), list(M or []), list(b), list(x))
        a64 = (P * n)(*[a.handle.value for a in A64])
        a32 = None if A32 is None else (P * n)(*[a.handle.value for a in A32])
        mm = None if M is None else (P * n)(*[(m.handle.value if m is not None else None) for m in M])
        bb = (P * n)(*[t.data_ptr() for t in b])
        xx = (P * n)(*[t.data_ptr() for t in x])
        h = ctypes.c_void_p()
        _check(L.mf_batch_create(n, a64, a32, mm, bb, xx, _stream(stream), ctypes.byref(h)))
        self.handle, self.n = h, n
        self.refine = A32 is not None

    def solve(self, rtol=1e-10, inner_rtol=0.0, maxit=100000, stream=None, raise_on_error=True):
        infos = (CGInfo * self.n)()
        rc = load_library().mf_batch_solve(self.handle, rtol, inner_rtol, maxit, infos, _stream(stream))
        if rc != 0 and raise_on_error:
            _check(rc)
        return [i.as_dict() for i in infos], rc

    def apply(self, inner=True, stream=None):
        _check(load_library().mf_batch_apply(self.handle, int(inner), _stream(stream)))

    def apply_user(self, xs, ys, inner=True, stream=None):
        """ys[i] = A[i] xs[i] for all systems in one batched launch (user numbering)."""
        if len(xs) != self.n or len(ys) != self.n:
            raise ValueError("one x and one y per system")
        import torch
        dt = torch.float32 if (inner and self.refine) else torch.float64
        for t in list(xs) + list(ys):
            _dev(t, dt)
        P = ctypes.c_void_p
        xx = (P * self.n)(*[t.data_ptr() for t in xs])
        yy = (P * self.n)(*[t.data_ptr() for t in ys])
        _check(load_library().mf_batch_apply_user(self.handle, int(inner), xx, yy, _stream(stream)))

    def autotune(self, cache_path=None, stream=None):
        _check(load_library().mf_batch_autotune(self.handle, None if cache_path is None else cache_path.encode(),
                                                _stream(stream)))
        return self.tuning

    @property
    def tuning(self):
        per, grid = ctypes.c_int(), ctypes.c_int()
        _check(load_library().mf_batch_get_tuning(self.handle, ctypes.byref(per), ctypes.byref(grid)))
        return per.value, grid.value

    def set_tuning(self, items_per, grid):
        _check(load_library().mf_batch_set_tuning(self.handle, items_per, grid))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mf_batch_destroy(self.handle)
            self.handle = None
