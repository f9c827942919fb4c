/*
 * mf.h -- C ABI of the MI355X (gfx950) matrix-free finite element library.
 *
 * The library computes the action y = A x of a finite element bilinear form
 * without assembling A: for every cell it gathers the cell's degrees of
 * freedom through the cell-to-node map, evaluates the element kernel at
 * quadrature points and scatter-adds the local result (Sun et al.,
 * "A study of vectorization for matrix-free finite element methods",
 * Section 2: the action of a bilinear form is the assembly of a linear form,
 * eq. 1; Section 2.2: a parallel loop over cells with indirectly accessed
 * data -- maps -- and access descriptors R / INC; Listing 3's gather, zero,
 * local kernel, scatter-increment structure).
 *
 * Conventions
 * -----------
 * - Every function returns int: MF_OK (0) on success, a negative MF_E* code
 *   otherwise; mf_last_error() then returns a message (thread-local). Outputs
 *   are written only on success. No C++ exception crosses this boundary.
 * - Host arrays passed to *_create are copied; the caller keeps ownership.
 * - Device vectors (x, y, d, b, ...) are caller-owned device pointers
 *   (e.g. torch data_ptr()) of the operator's precision (double for MF_F64,
 *   float for MF_F32) unless stated. They are never retained after the call,
 *   except by an mf_batch, which binds the pointers given at creation.
 * - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *   Calls are asynchronous on that stream unless documented as synchronous.
 * - Objects are immutable after creation; different objects may be used
 *   concurrently. One mf_op must not be used by two streams at once (it owns
 *   a workspace).
 * - Indices are int32 (nodes, cells); sizes are int64.
 * - Reference cells and local orderings:
 *     hex  [0,1]^3, vertex v at (v&1, (v>>1)&1, (v>>2)&1); Q_k nodes on the
 *          Gauss-Lobatto-Legendre points, local id i + n*j + n*n*l, n = k+1;
 *     tet  vertices (0,0,0),(1,0,0),(0,1,0),(0,0,1); P_k nodes at the
 *          equispaced lattice points alpha/k, a1 fastest, then a2, then a3;
 *     tri  vertices (0,0),(1,0),(0,1); P_k nodes at the equispaced lattice points
 *          alpha/k, a1 fastest.
 *   Vector fields are node-interleaved: dof = ncomp*node + component.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MF_OK = 0,
  MF_EINVAL = -1,       /* bad argument: null pointer, size, index out of range */
  MF_ENOMEM = -2,       /* device or host allocation failed */
  MF_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  MF_EMESH = -4,        /* degenerate or inverted cell */
  MF_ENOTCONV = -5,     /* iteration limit reached before the tolerance */
  MF_EBREAKDOWN = -6,   /* non-finite value or loss of positivity in a solver */
  MF_EUNSUPPORTED = -7  /* valid request this build does not implement */
};

/* QUAD: bilinear quadrilateral, vertex v at reference (v & 1, v >> 1) -- the 2D
 * tensor-product cell of the paper's sweep (Section 4.1) next to TRI, TET and HEX. */
enum { MF_CELL_TRI = 0, MF_CELL_TET = 1, MF_CELL_HEX = 2, MF_CELL_QUAD = 3 };

/* Bilinear forms (paper, supplementary material "operators"):
 *   MASS        int c u v            (c: optional vertex coefficient, else 1)
 *   HELMHOLTZ   int grad u . grad v + u v                       (eq. 2)
 *   LAPLACIAN   int grad u : grad v, ncomp 1 or 3 (paper: vector-valued)
 *   POISSON     int kappa grad u . grad v  (kappa: vertex coefficient)
 *   ELASTICITY  int sigma(u) : eps(v), sigma = 2 mu eps(u) + lambda tr(eps(u)) I;
 *               the paper's int eps(u):eps(v) is lambda = 0, mu = 1/2.
 *   HYPERELASTIC  the paper's hyperelasticity operator: the St-Venant-Kirchhoff
 *               residual int P(u0) : grad v, P = F S, F = I + grad u0,
 *               E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E, linearised at a given
 *               displacement u0 (mf_op_params.u0): int (dF S + F dS) : grad v with
 *               dF = grad u, dE = (dF^T F + F^T dF)/2, dS = lambda tr(dE) I + 2 mu dE.
 *               Vector P1-P6 tets (quadrature exact for the degree 4(k-1)
 *               integrand: 1, 14 and 125 points for P1-P3, conical rules of up to
 *               1331 points for P4-P6) and Q1-Q6 hexahedra (nq1d k+1 or
 *               k+2). */
enum { MF_OP_MASS = 0, MF_OP_HELMHOLTZ = 1, MF_OP_LAPLACIAN = 2, MF_OP_POISSON = 3,
       MF_OP_ELASTICITY = 4, MF_OP_HYPERELASTIC = 5 };

enum { MF_F64 = 0, MF_F32 = 1 };

typedef struct mf_mesh mf_mesh;
typedef struct mf_space mf_space;
typedef struct mf_op mf_op;

/* Create a mesh. coords: host, nverts x gdim (gdim 2 for TRI and QUAD, 3 otherwise),
 * components interleaved per vertex (the paper's coordinate dat accessed as
 * coords[gdim*vertex + i], Listing 3). cell2vert: host, ncells x (3|4|8; 4 for TET
 * and QUAD). Every cell's Jacobian determinant is checked at its vertices (hex and
 * quad: at every corner, which must share one sign); a zero or sign-changing determinant
 * gives MF_EMESH. |det J| is used afterwards (Listing 2 takes fabs of the
 * determinant). Errors: MF_EINVAL (bad type/sizes/index), MF_EMESH. */
int mf_mesh_create(int cell_type, int64_t nverts, const double *coords, int64_t ncells,
                   const int32_t *cell2vert, mf_mesh **out);

/* Create a Lagrange space of the given degree (hex and quad: Q_k on GLL nodes,
 * k = 1..6, local node i + (k+1)(j + (k+1) l) at the GLL point (i, j, l), i fastest;
 * tet and tri: P_k equispaced, k = 1..3) with ncomp components.
 * cell2node: host, ncells x D (D = (k+1)^3 hex, (k+1)^2 quad, (k+1)(k+2)(k+3)/6 tet,
 * (k+1)(k+2)/2 tri),
 * entries in [0, nnodes) -- the paper's cell2dof map (Section 2.2). The caller's
 * node numbering is kept at this boundary. Errors: MF_EINVAL, MF_EUNSUPPORTED. */
int mf_space_create(const mf_mesh *mesh, int degree, int ncomp, const int32_t *cell2node,
                    int64_t nnodes, mf_space **out);

/* Scatter-add strategies for the race of shared nodes (the paper serialises
 * the write-back, Section 3.1, and proposes conflict detection, Section 5):
 *   COLOURED  cells are coloured at space creation so that cells of one colour
 *             share no node; a full apply is one launch per colour with plain
 *             read-modify-write stores -- deterministic, bit-reproducible.
 *   ATOMIC    one launch, device-scope floating-point atomics.
 *   PATCH     cells are grouped into spatially compact patches; a workgroup
 *             accumulates its patch's cells in on-chip memory and writes each
 *             node once: nodes of no other patch directly, shared nodes into
 *             per-patch slots that a second launch sums in patch order
 *             (deterministic), or for hex Q1 (patches of at most 512 cells, 1024
 *             free nodes) with a device atomic (not bit-reproducible). Built for
 *             the hex MASS, HELMHOLTZ, LAPLACIAN and POISSON operators of degree 1
 *             (two points per direction) and 2-6 (k+1 points), P2 / P3 tet
 *             ELASTICITY, one-component tet operators and the triangle operators
 *             (the P1 mass and 2D ELASTICITY included).
 *   AUTO      PATCH for hex Q1 on at least 2^15 cells, for those hex operators of
 *             degree 2-4 below 2^17 cells (degree 2: 2^20; in FP32 also the
 *             one-component ones of degree 5 and 6), and for the tet and
 *             triangle forms above on at least 2^15 cells (one-component tets of
 *             degree 4-6: only FP32 P4 and P5; triangles of degree 5 and 6: only
 *             the FP32 one-component forms); otherwise COLOURED for
 *             3-component hex operators of degree >= 2 on at least 4096 cells
 *             (the HYPERELASTIC tangent only up to degree 4 in FP64, 5 in FP32),
 *             scalar hex operators of degree >= 2 on at least 2^18 cells, tets of
 *             degree 2 and 3, quad and triangle ELASTICITY (at least 4096 cells)
 *             and the other triangle operators but the P1 mass on at least 2^20
 *             cells; else ATOMIC (the measured choices).
 * Range applies (mf_op_apply_range*) always use ATOMIC. Errors at mf_op_create:
 * MF_EUNSUPPORTED for PATCH on other cells, kinds or degrees. */
enum { MF_SCATTER_AUTO = 0, MF_SCATTER_ATOMIC = 1, MF_SCATTER_COLOURED = 2, MF_SCATTER_PATCH = 3 };

typedef struct {
  const double *vertex_coef; /* host, nverts; MASS coefficient c or POISSON kappa; NULL -> 1 */
  double lambda, mu;         /* ELASTICITY and HYPERELASTIC Lame parameters */
  const uint8_t *dirichlet;  /* host, nnodes; nonzero marks a node whose every component is
                                constrained: (A x)_b = x_b there, and constrained values are
                                excluded from every other row. NULL -> no constraint. */
  int scatter;               /* MF_SCATTER_* */
  const double *u0;          /* HYPERELASTIC: host, ndofs, user numbering (node-interleaved
                                like x): the displacement the residual is linearised at,
                                copied at create (constrained nodes included). Else ignored. */
} mf_op_params;

/* Create an operator. precision MF_F64 or MF_F32 (FP32 arithmetic with FP32
 * accumulation; cell geometry is precomputed in FP64 and rounded once).
 * nq1d: hex and quad quadrature points per direction, 0 -> k+1 (tensor
 * Gauss-Legendre; quad: k+1..8, the paper's k+2 included); simplices ignore it and
 * use a rule exact for the integrand. params may be
 * NULL (coefficient 1, lambda 1, mu 0.5, no constraints). stream: device
 * uploads are ordered on it; the call returns after they complete.
 * Built combinations: hex Q1-Q6 MASS, HELMHOLTZ, POISSON (ncomp 1) and LAPLACIAN
 * (ncomp 1 or 3), nq1d k+1 or k+2; hex ELASTICITY and HYPERELASTIC (ncomp 3; nq1d
 * k+1 or k+2); tet ELASTICITY and HYPERELASTIC P1-P6 (ncomp 3); tet MASS
 * and HELMHOLTZ, LAPLACIAN and POISSON P1-P6 (ncomp 1; the tet rules reach degree
 * 21); tri MASS, HELMHOLTZ, LAPLACIAN and POISSON P1-P6 (ncomp 1) and ELASTICITY
 * P1-P6 (ncomp 2, the 2D stress); the simplex operators run both contractions on the
 * matrix cores (except P1 tet elasticity and the triangle P1 mass patch kernel, a
 * lane per cell); quad MASS, HELMHOLTZ, LAPLACIAN and POISSON Q1-Q6 (ncomp 1) and
 * ELASTICITY Q1-Q6 (ncomp 2, the 2D stress).
 * Errors: MF_EINVAL, MF_EUNSUPPORTED (op/cell/degree combination), MF_ENOMEM. */
int mf_op_create(const mf_space *space, int kind, int precision, int nq1d,
                 const mf_op_params *params, void *stream, mf_op **out);

/* y = A x over all cells; y (ndofs) is overwritten (the paper's assemble(L)
 * returns a fresh vector, Listing 1; the local tensor is zeroed before each
 * cell, Listing 3). x and y must not alias. */
int mf_op_apply(const mf_op *op, const void *x, void *y, void *stream);

/* The paper's wrapper contract over a cell range (Listing 3: start <= n < end,
 * access INC): y += A_[start,end) x if accumulate, else y = A_[start,end) x.
 * No constraint rows are set here (only the masking of constrained values). */
int mf_op_apply_range(const mf_op *op, int64_t start, int64_t end, const void *x, void *y,
                      int accumulate, void *stream);

/* d = diag(A) (ndofs, op precision); constrained dofs get 1. Used as the Jacobi
 * preconditioner. Hex scalar operators with k+1 points, quadrilaterals, tet elasticity
 * and the P1 triangle mass have fused diagonal kernels; the one-component tet
 * operators, the other triangle operators, hex elasticity and the hex operators with
 * k+2 points sum the diagonals of their element matrices (FP64, a thread per cell
 * and node; synchronous). MF_EUNSUPPORTED for HYPERELASTIC. */
int mf_op_diagonal(const mf_op *op, void *d, void *stream);

/* Internal cell order and numbering. Every space colours its cells greedily
 * (first fit, user cell order, two cells conflict when they share a vertex --
 * for these conforming spaces exactly when they share a node) and orders them
 * by colour, user order within a colour. mf_space_get_colouring writes the
 * user cell of each internal cell (ncells entries, may be NULL), the colour
 * offsets (ncolours + 1 entries, may be NULL) and the number of colours.
 * Nodes are numbered internally in order of first appearance when the cells
 * are traversed in that internal order (hexahedra, quadrilaterals) or, for
 * tetrahedra and triangles, in the Morton order of their centroids (each
 * coordinate quantised to 1024 steps over the centroids' bounding box, bit b of
 * x, y, z at bits 3b, 3b+1, 3b+2 of the code, z = 0 on triangles; ties by
 * internal cell order), the
 * order in which the patch scatter takes them; the kernels gather
 * and scatter only in that numbering, so the nodes of neighbouring cells are
 * neighbours in memory whatever numbering the caller uses. mf_op_apply and
 * mf_op_apply_range take user-numbered vectors and pay one permutation in and
 * one out; the _internal variants take internally numbered vectors (dof =
 * ncomp*internal_node + component) and run only the operator kernels.
 * mf_space_get_permutation writes internal_to_user[i] = the user node of
 * internal node i (nnodes entries, host). All operators built on one space
 * share its numbering. */
int mf_space_get_colouring(const mf_space *space, int32_t *internal_to_user_cell, int64_t *colour_ptr,
                           int *ncolours);
int mf_space_get_permutation(const mf_space *space, int32_t *internal_to_user);
int mf_op_apply_internal(const mf_op *op, const void *x, void *y, void *stream);
int mf_op_apply_range_internal(const mf_op *op, int64_t start, int64_t end, const void *x, void *y,
                               int accumulate, void *stream);

typedef struct {
  int64_t ncells, nnodes, ndofs;
  int cell_type, kind, precision, degree, ncomp, nq1d, nqp;
  int dofs_per_cell;      /* D (nodes per cell) */
  double flops_per_apply; /* algorithmic flops of one operator action */
  double bytes_per_apply; /* algorithmic HBM bytes of one action (perfect caching) */
  int cell_launches;      /* cell-kernel launches per full action (colours, or 1) */
  int ncolours;           /* colours of the space's cell colouring */
  int clears_output;      /* 1: mf_op_apply / mf_op_apply_internal clear y in a pass of their
                             own before the cell launches; 0: the launches write every entry
                             themselves (coloured hex k >= 2: each node's first contribution
                             is stored; patch scatters: each node is written once).
                             Overwriting range applies of an operator with constrained nodes
                             always clear. */
  int scatter;            /* the scatter full actions use: MF_SCATTER_ATOMIC, _COLOURED or
                             _PATCH (patch: one patch launch, plus one launch summing the
                             nodes shared between patches, except for the degree-1 hex
                             patches, which use device atomics there) */
} mf_op_info;

int mf_op_get_info(const mf_op *op, mf_op_info *info);

/* ----------------------------------------------------------------- solvers */
typedef struct {
  int outer_iterations;   /* FP64 residual refreshes (1 for plain FP64 CG) */
  int inner_iterations;   /* total CG iterations with the (inner) operator */
  int fallbacks;          /* learned-preconditioner steps replaced by Jacobi */
  double rel_residual;    /* final true ||b - A64 x||_2 / ||b||_2 */
} mf_cg_info;

typedef struct mf_precond mf_precond;

/* Jacobi preconditioner from A's diagonal (FP64). */
int mf_precond_create_jacobi(const mf_op *A, void *stream, mf_precond **out);

/* Global sparse matrix of the operator, CSR in user numbering (rows and columns are
 * the dofs node * ncomp + component): the paper's matrix assembly (Sun et al.,
 * Section 5: the local kernel's element matrices scattered into a sparse matrix)
 * beside the matrix-free action. Built for every operator kind but HYPERELASTIC on
 * tets and triangles of degree 1-3, quadrilaterals of degree 1-6 and hexahedra of
 * degree 1-4, with the operator's own quadrature rule. `space` must be the space the
 * operator was created on (MF_EINVAL otherwise); the pattern comes from its cell map.
 * mf_op_csr_pattern: rowptr (host, ndofs + 1 int64, nullable), col (host, nnz int32,
 * nullable; columns sorted in each row) and nnz (nullable). Entry (r, c) is in the
 * pattern when the nodes of dofs r and c share a cell (for ncomp > 1, every component
 * pair of such nodes). The pattern is built once and kept by the operator.
 * mf_op_assemble_csr: vals (device, nnz values of the operator's precision, in the
 * pattern's order; overwritten) = the element matrices, computed on the device in
 * FP64 and added in the operator's precision; constrained dofs give identity rows and
 * zero columns, as in the action. Synchronous (temporary device buffers).
 * Errors: MF_EUNSUPPORTED outside the built set, MF_EINVAL for null arguments or a
 * different space. */
int mf_op_csr_pattern(const mf_op *op, const mf_space *space, int64_t *rowptr, int32_t *col, int64_t *nnz);
int mf_op_assemble_csr(const mf_op *op, const mf_space *space, void *vals, void *stream);

/* Conjugate gradients for A64 x = b, all vectors FP64 on the device (Hestenes
 * and Stiefel; not in the paper -- the solver that consumes the action).
 * A32 == NULL: plain preconditioned CG with the FP64 action.
 * A32 != NULL, M NULL or Jacobi: one preconditioned CG sequence with the FP32
 * action A32 p and FP64 vectors, dot products and updates, with reliable updates:
 * whenever the recursively updated residual has dropped by the factor inner_rtol
 * (0 -> 1e-3) since the last true residual, and whenever it meets the target, r is
 * replaced by b - A64 x computed in FP64 and r'z recomputed, keeping the search
 * direction; the solve stops when that true ||r||/||b|| <= rtol.
 * info->outer_iterations counts the true residuals formed (the first included).
 * A32 != NULL with a learned M: iterative refinement -- the outer loop forms
 * r = b - A64 x in FP64 and stops when ||r||/||b|| <= rtol; each inner solve runs
 * flexible CG on A32 d = r (FP64 vectors) to relative tolerance
 * max(inner_rtol, rtol ||b|| / ||r||), floored at inner_rtol (0 -> 1e-6), then
 * x += d.
 * M == NULL: no preconditioner; a Jacobi M: preconditioned CG; a learned M
 * (mf_precond_create_cnn): flexible CG with the Polak-Ribiere beta
 * -alpha <z_k+1, A p_k> / <z_k, r_k>, where any iteration whose network output z
 * is non-finite or has <z, r> <= 0 uses the Jacobi z instead (counted in
 * info->fallbacks).
 * x holds the initial guess on entry. Synchronous. info may be NULL.
 * Errors: MF_ENOTCONV (maxit total inner iterations reached; x holds the last
 * iterate, info filled), MF_EBREAKDOWN (non-finite residual or p'Ap <= 0). */
int mf_cg_solve(const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b,
                double *x, double rtol, double inner_rtol, int maxit, mf_cg_info *info,
                void *stream);

/* For callers that cannot allocate device memory (code under stream capture
 * elsewhere in the program, tight serving loops, harnesses that forbid hipMalloc):
 * mf_cg_solve with the same arguments and results, except that
 *  - the solver's vectors live in one fixed device array of the library,
 *    MF_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU until
 *    the process ends; a solve needs 8 n bytes for each of r, p and A p, plus
 *    8 n + 4 n + 4 n with A32 (correction, FP32 search direction and its image),
 *    plus 16 n when the space's internal numbering differs from the user's (b and x
 *    moved inside), each vector rounded up to 256 bytes, plus 33 KB of reduction
 *    partials and state (n = A64's DoF count);
 *  - it runs on `stream` itself and creates no stream, event, graph or pinned
 *    buffer (the iteration chunks are launched directly, not replayed from a graph);
 *    the iteration state is read back through pageable host memory;
 *  - M must be NULL or a Jacobi preconditioner.
 * Every call on one GPU uses that GPU's array and leaves its contents behind (each
 * solve initialises what it reads), so calls that overlap in time on one GPU, from
 * several threads or streams, race and must be serialised by the caller.
 * Errors: as mf_cg_solve; MF_EINVAL when the solve needs more than
 * MF_NOALLOC_SCRATCH_BYTES (message states both sizes); MF_EUNSUPPORTED for a
 * learned M; MF_EDEVICE if the array's device address cannot be obtained. */
#define MF_NOALLOC_SCRATCH_BYTES (64u << 20)
int mf_cg_solve_noalloc(const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b,
                        double *x, double rtol, double inner_rtol, int maxit, mf_cg_info *info,
                        void *stream);

void mf_precond_destroy(mf_precond *p);

/* z = M r for FP64 device vectors of the operator's space in user numbering
 * (Jacobi: z = D^-1 r; learned: as below). Asynchronous on stream. */
int mf_precond_apply(const mf_precond *M, const double *r, double *z, void *stream);

/* ----------------------------------------------------------------- learned preconditioner
 * Not in the paper: a convolutional approximate inverse for the matrix-free
 * operator on the DoF lattice of a structured hex mesh (Q_k on m^3 cells:
 * (k m + 1)^3 nodes). The network N is an L-level U-Net (2 <= L <= 8) on FP32
 * channel-last lattices whose sizes n satisfy n = j 2^(L-1) + 1, j >= 1:
 *   h_0 = relu(A x);  c_l = R h_(l-1), h_l = relu(B_l c_l)          (l = 1 .. L-1)
 *   g_(L-1) = relu(D h_(L-1));  u_l = P g_(l+1) + h_l               (l = L-2 .. 0)
 *   g_l = relu(E_l u_l)  (l = L-2 .. 1);   y = x + F u_0,
 * with 3x3x3 convolutions (zero padding, no bias; A: 1 -> C channels, F: C -> 1,
 * the others C -> C), full-weighting restriction R (1/4, 1/2, 1/4 per direction)
 * and trilinear prolongation P. With zero weights N is the identity (so the
 * preconditioner below is Jacobi). Parameters: one FP32 vector holding
 * A, B_1 .. B_(L-1), D, E_(L-2) .. E_1, F in that order, each as W[tap][cin][cout]
 * with tap = (dx+1) + 3 (dy+1) + 9 (dz+1) and out[v] = sum_d in[v + d] W[tap(d)];
 * mf_cnn_nparams(C, L) = 27 (2 C + (2 L - 2) C^2). Channels C: 4, 8 or 16.
 * A network object holds the parameters, Adam moments and training workspaces;
 * one object must not be used by two streams at once. */
typedef struct mf_cnn mf_cnn;
int64_t mf_cnn_nparams(int channels, int levels); /* -1 for unsupported values */
/* theta: host, mf_cnn_nparams(channels, levels) floats (initial weights; copied). */
int mf_cnn_create(int channels, int levels, const float *theta, mf_cnn **out);
int mf_cnn_get_params(const mf_cnn *net, float *theta);   /* host out; synchronises the device */
int mf_cnn_set_params(mf_cnn *net, const float *theta);   /* host in; resets the Adam state */
/* Binary file: 8-byte magic "MFCNN02", int32 channels, int32 levels, int64 nparams,
 * then the FP32 parameters (little-endian). */
int mf_cnn_save(const mf_cnn *net, const char *path);
int mf_cnn_load(const char *path, mf_cnn **out);
void mf_cnn_destroy(mf_cnn *net); /* NULL-safe */
/* y = N(x) for a batch of lattices: x, y device FP32 [batch][nz][ny][nx];
 * every size j 2^(L-1) + 1 with j >= 1 (else MF_EINVAL). Asynchronous on stream. */
int mf_cnn_forward(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, float *y, void *stream);
/* Loss of a batch, mean over samples of |N(x_b) - t_b|^2 / |t_b|^2 (a sample
 * with t_b = 0 contributes 0), and its gradient with respect to the parameters.
 * loss: host (nullable, then asynchronous), grad: device nparams floats (nullable). */
int mf_cnn_loss_grad(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, const float *t,
                     double *loss, float *grad, void *stream);
/* nsteps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * batches of training pairs: r, e device FP32 [npairs][n][n][n]; step s uses the
 * pairs order[s*batch .. s*batch+batch-1] (host int32, each in [0, npairs)).
 * losses: host, nsteps doubles (the loss before each step; nullable). Synchronous. */
int mf_cnn_train(mf_cnn *net, int npairs, int n, const float *r, const float *e, int nsteps, int batch,
                 const int32_t *order, float lr, double *losses, void *stream);
/* Learned preconditioner for a scalar operator A on a lattice of nz x ny x nx
 * nodes: node_grid (host, A's nnodes entries, user numbering) gives each node's
 * lattice index (z ny + y) nx + x and must be a bijection. The preconditioner is
 * z = D^-1/2 N(D^-1/2 r) with D = diag(A), and z = r on Dirichlet nodes. The
 * network is borrowed: it must outlive the preconditioner, and training it
 * later changes the preconditioner. Errors: MF_EUNSUPPORTED (vector space),
 * MF_EINVAL (sizes, not a bijection). */
int mf_precond_create_cnn(const mf_op *A, const mf_cnn *net, int nz, int ny, int nx,
                          const int32_t *node_grid, void *stream, mf_precond **out);
/* Energy (Ritz) loss of the learned preconditioner for one residual r of A
 * (FP64 device vector, user numbering): with z = P r,
 *   loss = (z^T A z - 2 z^T r) / (r^T D^-1 r),
 * which is the A-norm error |z - A^-1 r|_A^2 up to the constant r^T A^-1 r, so
 * minimising it over the weights improves the preconditioner for every mode in
 * proportion to its energy. P must be a learned preconditioner built on net and A
 * the FP64 operator P was built from. loss: host (nullable); grad: device nparams
 * floats (nullable). Synchronous. */
int mf_cnn_energy_loss_grad(mf_cnn *net, const mf_precond *P, const mf_op *A, const double *r, double *loss,
                            float *grad, void *stream);
/* nsteps Adam steps (as mf_cnn_train) on that loss, one residual per step:
 * r: device FP64 [nsamples][ndofs] (user numbering), step s uses r[order[s]]
 * (host int32). losses: host, nsteps doubles (the loss before each step;
 * nullable). Synchronous. */
int mf_cnn_train_energy(mf_cnn *net, const mf_precond *P, const mf_op *A, int nsamples, const double *r,
                        int nsteps, const int32_t *order, float lr, double *losses, void *stream);
/* Training pairs from a residual / error pair of A (r = A e; FP64 device vectors,
 * user numbering): both are diagonally scaled (r~ = D^-1/2 r, e~ = D^1/2 e, the
 * pair of the unit-diagonal operator), and crop c is the n^3 sub-lattice starting
 * at (z, y, x) = corners[3c .. 3c+2] (host int32), scaled by 1 / rms of its r~
 * values. r_out, e_out: device FP32 [ncrops][n][n][n]. Synchronous. */
int mf_precond_harvest(const mf_precond *M, const double *r, const double *e, int ncrops, int n,
                       const int32_t *corners, float *r_out, float *e_out, void *stream);

/* ----------------------------------------------------------------- batched solves
 * Many independent systems A64[i] x[i] = b[i] on uneven hex meshes and degrees,
 * solved together (not in the paper -- the batched form of the CG consumer of
 * the action). Every iteration applies all operators either in ONE persistent
 * launch over a device work list of (operator, cell-batch range) items, or (launch
 * form "per system", grid -1) with each live system's own operator kernels (its
 * tile shape and scatter); vector stages run over the concatenated vectors of all
 * systems; chunks of iterations are captured into a hipGraph and replayed (launched
 * directly in the per-system form, whose set of live systems changes).
 * Requirements: scalar FP64 hex operators of one kind, degree <= 5, without
 * constraints; A32 (nullable) holds the FP32 operators on the same spaces (the FP32
 * action with reliable updates, as in mf_cg_solve); M (nullable, entries nullable)
 * Jacobi preconditioners of the A64[i].
 * The batch binds the device pointers b[i] (input) and x[i] (initial guess in,
 * solution out, user numbering); they must stay valid while the batch exists. */
typedef struct mf_batch mf_batch;
int mf_batch_create(int nsys, const mf_op *const *A64, const mf_op *const *A32, const mf_precond *const *M,
                    const double *const *b, double *const *x, void *stream, mf_batch **out);
/* Solve all systems to ||b_i - A64_i x_i|| <= rtol ||b_i|| (true FP64 residual).
 * infos (nullable) receives nsys entries. maxit bounds the inner iterations of
 * the slowest system summed over refinements. Synchronous. Errors as
 * mf_cg_solve (MF_ENOTCONV if any system misses the tolerance). */
int mf_batch_solve(mf_batch *batch, double rtol, double inner_rtol, int maxit, mf_cg_info *infos, void *stream);
/* One batched operator launch (inner = 1: the inner operators on the internal
 * search directions; 0: the FP64 operators on the iterates), for timing. */
int mf_batch_apply(mf_batch *batch, int inner, void *stream);
/* y[i] = A[i] x[i] for every system in ONE batched launch (the launch mf_batch_solve
 * iterates with, at the current tuning): inner = 1 applies the inner operators (A32
 * when the batch refines: x[i], y[i] FP32; else A64), inner = 0 the FP64 operators.
 * x[i], y[i]: device vectors of system i in user numbering (nsys entries each, y[i]
 * overwritten, no aliasing). The inputs pass through the batch's internal iteration
 * buffers, which a later mf_batch_solve re-initialises from the bound vectors.
 * Asynchronous on stream. Errors: MF_EINVAL (null batch, array or vector). */
int mf_batch_apply_user(mf_batch *batch, int inner, const void *const *x, void *const *y, void *stream);
/* Autotuner: times one application of all inner operators in each launch form --
 * per-system kernels (grid -1), the work-list kernel with one wavefront per
 * single-batch item (grid 0), and persistent grids of 1, 2, 4 x (CUs x 4)
 * wavefronts with work-list granularities of 1..32 cell batches per item -- and
 * keeps the fastest. With cache_path, a result for the same (kind, inner precision,
 * CU count, set of (degree, cells)) is read from / appended to that text file.
 * mf_batch_set_tuning: items_per >= 1, grid >= -1 (items_per 1 for grids 0, -1). */
int mf_batch_autotune(mf_batch *batch, const char *cache_path, void *stream);
int mf_batch_get_tuning(const mf_batch *batch, int *items_per, int *grid);
int mf_batch_set_tuning(mf_batch *batch, int items_per, int grid);
void mf_batch_destroy(mf_batch *batch);

/* ----------------------------------------------------------------- attainable peaks
 * The device's attainable rates, measured as the paper measured its CPUs' (Section 4.1,
 * Table 1: STREAM bandwidth and LINPACK beside the theoretical peaks): out[0] HBM GB/s
 * of a 1 GiB streaming copy (bytes read + written), out[1] FP64 and out[2] FP32 vector
 * multiply-add TFLOP/s (independent chains, no packed math), out[3] FP32 matrix TFLOP/s
 * (v_mfma_f32_4x4x1_16b) and out[4] FP64 matrix TFLOP/s (v_mfma_f64_4x4x4_4b).
 * out: host, 5 doubles. Allocates and frees 2 GiB of device memory. Synchronous.
 * Errors: MF_EINVAL (out NULL), MF_ENOMEM, MF_EDEVICE. */
int mf_probe_peaks(double *out, void *stream);

/* ----------------------------------------------------------------- teardown / errors */
void mf_mesh_destroy(mf_mesh *m);   /* NULL-safe */
void mf_space_destroy(mf_space *s); /* NULL-safe */
void mf_op_destroy(mf_op *op);      /* NULL-safe; waits for the op's work */
const char *mf_last_error(void);
const char *mf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
