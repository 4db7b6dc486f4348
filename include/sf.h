/*
 * sf.h -- C ABI of the MI355X (gfx950) sum-factorised local assembly library.
 *
 * The library computes, for every hexahedral cell of a mesh, either the
 * operator action y^K = A^K u^K or the dense element matrix A^K of a bilinear
 * form, with the sum-factorisation of Homolya, Kirby & Ham, "Exposing and
 * exploiting structure: optimal code generation for high-order finite element
 * methods" (Sec. 3.2-3.5): 1-D tabulation matrices are applied one axis at a
 * time to reach the quadrature points (eq. coeff_eval), pointwise geometric
 * and coefficient factors are applied (Sec. 3.2, argument factorisation), and
 * the transposed 1-D matrices bring the result back to the local degrees of
 * freedom (eq. form_eval).
 *
 * Conventions shared by every entry point:
 *   - Reference cell [0,1]^3.  A cell's geometry is its 8 vertices, FP64,
 *     [ncells][8][3]; the reference vertex (v0,v1,v2) in {0,1}^3 is stored at
 *     index 4*v0+2*v1+v2 (the vector-Q1 coordinate field, Sec. 3.1).  The GPU
 *     kernels take AFFINE cells (x = x0 + J xi, which includes axis-aligned
 *     boxes); a cell whose remaining vertices deviate from the affine map, or
 *     whose det J <= 0, raises a device-side flag read by sf_check_errors()
 *     and its output is unspecified.  sf_set_geometry() declares boxes
 *     (faster kernels) or general trilinear cells (geometry per point).
 *   - Quadrature: nq1 Gauss-Legendre points per axis (Gauss-Lobatto-Legendre
 *     for SF_QGLL) (tensor rule, eq. tpps),
 *     point q = (q0*nq1 + q1)*nq1 + q2.  kappa, when given, is a value per
 *     cell per quadrature point, [ncells][nq1^3]; NULL means kappa = 1.
 *   - Elements (Secs. 2.4-2.7): SF_Q = Q_p on Gauss-Lobatto-Legendre nodes,
 *     SF_DQ = dQ_p on Gauss-Legendre nodes, SF_NCF = the H(div) Q^- element
 *     (RTCF on quadrilaterals) and SF_NCE = the H(curl) one.  NCF_k block c is
 *     P_k (GLL_{k+1} nodes) on axis c times dP_{k-1} (GL_k nodes) on the other
 *     axes, with value +phi e_c; NCE_k block c is dP_{k-1} on axis c and P_k
 *     elsewhere.  Local DOFs: the blocks concatenated in order, each block
 *     row-major over its per-axis indices, last axis fastest (Sec. 3.5, the
 *     indexed-buffer splitting of Concatenate; eq. rtcf_split_x/y).
 *   - Forms (row i = test function, column j = trial function, y = A u):
 *       SF_MASS     int kappa u v        (Piola-mapped for NCF / NCE)
 *       SF_LAPLACE  int kappa grad u . grad v          (SF_Q, SF_DQ, SF_QGLL)
 *       SF_HDIV     alpha * mass + beta * int kappa div u div v     (SF_NCF)
 *       SF_HCURL    alpha * mass + beta * int kappa curl u . curl v (SF_NCE)
 *     Contravariant Piola for H(div): Psi = J Psi^ / det J; covariant for
 *     H(curl): Psi = J^{-T} Psi^, curl Psi = J curl^ Psi^ / det J.
 *   - Outputs are OVERWRITTEN (the local tensor is cleared, then every
 *     contribution is added: Sec. 3.4).
 *   - All device pointers are caller-owned device memory (e.g. torch
 *     tensors); the library never frees them and keeps none after a call
 *     returns (an sf_batch keeps its job pointers until destroyed).
 *   - Calls are asynchronous on the given stream (hipStream_t passed as
 *     void*, NULL = the default stream).  Argument validation happens before
 *     any HIP call and returns an error code; no exception crosses the ABI.
 *   - A context is not thread-safe.
 */
#ifndef SF_H
#define SF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SF_OK 0
#define SF_ERR_ARG (-1)         /* NULL / negative / inconsistent argument       */
#define SF_ERR_UNSUPPORTED (-2) /* family, degree, form, nq1 or precision        */
#define SF_ERR_NOMEM (-3)       /* device or host allocation failed              */
#define SF_ERR_HIP (-4)         /* a HIP runtime call failed                     */
#define SF_ERR_GEOMETRY (-5)    /* device flag: det J <= 0, non-affine, non-box   */
#define SF_ERR_CAPACITY (-6)    /* a size exceeds a documented maximum           */

/* device error flag bits, as reported by sf_check_errors() */
#define SF_FLAG_DETJ 1      /* det J <= 0                          */
#define SF_FLAG_NONAFFINE 2 /* vertices are not an affine image      */
#define SF_FLAG_NONBOX 4    /* element matrix on a non-box cell      */

/* SF_QGLL: the Q_p element of SF_Q integrated with the (p+1)-point
 * Gauss-Lobatto-Legendre rule instead of Gauss-Legendre, so quadrature points
 * and nodes coincide (B = I): the collocated, under-integrated spectral-element
 * variant (Sec. 2.5).  Its mass matrix is diagonal (lumped); the 1-D stiffness
 * is still integrated exactly.  kappa is given at the GLL points. */
/* SF_VQ: the vector Q_p element, the scalar SF_Q basis times the three unit
 * vectors (Sec. 2.3): ndof_cell = 3 (p+1)^3, local DOF (component c, node i)
 * at c (p+1)^3 + i (three component blocks), p = 1..8, the (p+1)-point GL
 * rule, kappa scalar per point.  Forms SF_MASS (kappa u . v) and SF_LAPLACE
 * (kappa grad u : grad v); FP64 contractions and SF_F64 storage only.  Its
 * element matrices are block diagonal, the SF_Q matrix in each diagonal
 * block: computed once per cell and assigned to the three diagonal views of
 * the output after the whole output has been cleared (delta cancellation
 * across the assignment, Sec. 3.4); box cells, as for SF_Q. */
enum { SF_Q = 0, SF_DQ = 1, SF_NCF = 2, SF_NCE = 3, SF_QGLL = 4, SF_VQ = 5 };
enum { SF_MASS = 0, SF_LAPLACE = 1, SF_HDIV = 2, SF_HCURL = 3, SF_SVK = 4, SF_SVK_RESIDUAL = 5 };
/* SF_SVK / SF_SVK_RESIDUAL: the Saint Venant-Kirchhoff hyperelastic model of
 * the paper's evaluation on the VECTOR Q_p element (family SF_Q, or SF_QGLL
 * for its GLL-collocated variant; p = 1..8): the scalar basis times the unit
 * vectors (Sec. 2.3), ndof_cell = 3 (p+1)^3, local DOF (component c, node i)
 * at c (p+1)^3 + i (component-major; node numbering as for the scalar
 * element).  op.alpha = lambda, op.beta = mu (the Lame parameters).  With
 * F = I + grad u, E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E, P = F S:
 *   SF_SVK_RESIDUAL  y_(c,i) = int P(u) : grad(Psi_i e_c)  (residual form,
 *                    no body force; `u` is the displacement, kappa NULL);
 *   SF_SVK           y_(c,i) = int dP(u0; du) : grad(Psi_i e_c), the
 *                    linearised residual (eq. bilinear_form) applied to the
 *                    direction du = `u`, with dF = grad du,
 *                    dE = (dF^T F + F^T dF)/2, dS = lambda tr(dE) I + 2 mu dE,
 *                    dP = dF S + F dS; the linearisation point u0 is passed
 *                    in `kappa` (the form's coefficient) as a local vector of
 *                    the same layout, NULL for u0 = 0 (linear elasticity).
 * Quadrature: p+1 points per axis (GL for SF_Q, GLL for SF_QGLL).  FP64
 * contractions and SF_F64 storage only.  Element matrices: SF_SVK only
 * (p = 1..8; 38 MB per cell at p = 8), kappa = u0 as for the action, output
 * [ncells][ndof_cell][ndof_cell] with row = test function (c, i) and column
 * = trial function (c', j): the tangent modulus of P at u0 in every block.
 * Geometry: affine cells, or any trilinear cell under SF_GEOM_TRILINEAR (J
 * per point). */
/* contraction precision: FP64, FP32 (both VALU); BF16 / FP16 single-term MFMA
 * with FP32 accumulation; BF16X3 = operands split into three BF16 terms
 * (hi + mid + lo), six cross products per contraction, FP32 accumulation.
 * Geometry, Jacobian, inverse, determinant and the pointwise factors are FP64
 * in every mode (the pointwise product itself is FP32).  FP16 operands carry
 * FP16's range: u, the interpolated values and the pointwise products must
 * stay below 65504 in magnitude (BF16 and BF16X3 have FP32's range).  Scalar-family
 * actions in the MFMA modes (nq1 = degree + 1) group the contractions as
 * dense Kronecker products (Sec. 3.3's sums, grouped differently): one
 * (p+1)^3 x (p+1)^3 matrix per component at p <= 3, a (p+1)^2 x (p+1)^2 matrix
 * on axes 1-2 times a (p+1) x (p+1) matrix on axis 0 at p = 4..8; BF16X3 at
 * p = 8 and other nq1 use the one-axis-at-a-time MFMA kernel. */
enum { SF_FP64 = 0, SF_FP32 = 1, SF_BF16 = 2, SF_FP16 = 3, SF_BF16X3 = 4 };
/* storage type of kappa, u, y and A */
enum { SF_F64 = 0, SF_F32 = 1 };

typedef struct sf_context sf_context;
typedef struct sf_batch sf_batch;

typedef struct {
    int32_t family;    /* SF_Q, SF_DQ, SF_QGLL, SF_VQ: degree p in 1..8;  SF_NCF, SF_NCE: k in 1..6 */
    int32_t degree;
    int32_t form;      /* see above                                                 */
    int32_t nq1;       /* GL points per axis; 0 => degree + 1 (see sf_element_dims) */
    int32_t precision; /* SF_FP64 ... SF_BF16X3                                     */
    int32_t io_dtype;  /* SF_F64 or SF_F32                                           */
    double alpha;      /* SF_HDIV / SF_HCURL weights; ignored otherwise               */
    double beta;
} sf_op;

/* Create a context on HIP device `hip_device`; it owns the 1-D tables, the
 * device error flag and the tuning cache.  Returns SF_OK and *out, or an
 * error.  Make the device current before calling.  Destroy frees all of it. */
int sf_context_create(int hip_device, sf_context **out);
int sf_context_destroy(sf_context *ctx);

/* Human-readable text of a status code (static storage). */
const char *sf_status_string(int status);

/* Geometry class the caller guarantees for later calls on this context.
 * SF_GEOM_AFFINE (the default): any affine cell (parallelepipeds, boxes).
 * SF_GEOM_BOX: every cell is an axis-aligned box (J diagonal); the Q_p /
 * dQ_p actions then use kernels that exploit the diagonal factor |J| G G^T
 * (two LDS tensors per cell instead of three).  Under SF_GEOM_BOX the
 * Laplace action of a cell whose Jacobian has off-diagonal entries is
 * unspecified and raises SF_FLAG_NONBOX, except when the autotuner picked
 * the general kernel for that op (variant 3 below), which stays exact and
 * raises nothing; the mass action needs only |det J| and stays exact on any
 * affine cell.  Element matrices of SF_Q / SF_VQ then use the box kernel
 * (see assemble_element_matrix).  The SF_NCF / SF_NCE actions use diagonal
 * Piola factors (h_c^2 / |J|, |J| / h_c^2) with the pointwise stage fused into
 * the contractions; a cell with off-diagonal J raises SF_FLAG_NONBOX and only
 * the diagonal factors are applied to it (unless the autotuner picked the
 * general kernel, variant 2 of that class, which stays exact).
 * Returns SF_ERR_ARG for an unknown value. */
#define SF_GEOM_AFFINE 0
#define SF_GEOM_BOX 1
/* SF_GEOM_TRILINEAR: cells may be general trilinear hexahedra (the vector-Q1
 * coordinate field, Sec. 3.1); the Q_p / dQ_p / SF_QGLL actions then evaluate
 * J, |J| and |J| G G^T at every quadrature point (the per-point factor
 * P^{(k,l)}_q of Sec. 3.2, all six entries) in FP64 and need SF_FP64 with
 * SF_F64 storage (else SF_ERR_UNSUPPORTED); a point with det J <= 0 raises
 * SF_FLAG_DETJ.  The same holds for the SF_NCF / SF_NCE actions (Piola
 * factors J^T J / |J|, |J| G G^T and 1 / |J| per point), the vector and
 * hyperelastic forms and the scalar element matrices; every action under
 * this hint needs SF_FP64 contractions with SF_F64 storage.  The SF_NCF /
 * SF_NCE element matrices keep the box requirement. */
#define SF_GEOM_TRILINEAR 2
int sf_set_geometry(sf_context *ctx, int32_t geometry);

/*
 * Global operator action of continuous Q_p on an nx x ny x nz grid of
 * axis-aligned box cells (cell (i,j,k) is number (i*ny + j)*nz + k):
 *   y_global = sum over cells K of P_K^T A_K P_K u_global
 * (Sec. 1.1: the global operator is the sum of the cell contributions; P_K
 * gathers cell K's local DOFs).  Local DOF (i0,i1,i2) of cell (i,j,k) is the
 * lattice point (i p + i0, j p + i1, k p + i2), numbered
 * (a (ny p + 1) + b)(nz p + 1) + c — the numbering sf_dof_map_q returns.
 *   op        family SF_Q, form SF_MASS or SF_LAPLACE, SF_FP64, SF_F64
 *   vertices  device, [nx*ny*nz][8][3] FP64, boxes (others raise SF_FLAG_NONBOX)
 *   kappa     device, [nx*ny*nz][nq_cell] FP64, or NULL
 *   u_global  device, [(nx p+1)(ny p+1)(nz p+1)] FP64
 *   y_global  device, same length, overwritten (cleared by a kernel, then the
 *             cell contributions are added with FP64 atomics, so the order of
 *             the additions, and the last bits of y, vary from run to run)
 * Errors: SF_ERR_ARG, SF_ERR_UNSUPPORTED (other family / form / precision),
 * SF_ERR_CAPACITY (more than 2^40 global DOFs), SF_ERR_HIP.
 */
int assemble_action_global_q(sf_context *ctx, const sf_op *op, int32_t nx, int32_t ny, int32_t nz,
                             const double *vertices, const void *kappa, const void *u_global, void *y_global,
                             void *hip_stream);

/* Host only, no GPU needed.  Per-cell local DOF count and quadrature-point
 * count of `op` (after nq1 = 0 => degree + 1), or an error for an
 * unsupported combination.  Validation rules are exactly those of the
 * assembly entry points. */
int sf_element_dims(const sf_op *op, int32_t *ndof_cell, int32_t *nq_cell);

/*
 * Operator action, the matrix-free linear form (Sec. 1.1; Sec. 3.3,
 * eq. coeff_eval and eq. form_eval):  y[c][i] = a(psi_i, u_c) on every cell.
 *   vertices  device, [ncells][8][3] FP64
 *   kappa     device, [ncells][nq_cell] io_dtype, or NULL (kappa = 1);
 *             SF_SVK: u0 [ncells][ndof_cell] or NULL; SF_SVK_RESIDUAL: NULL
 *   u         device, [ncells][ndof_cell] io_dtype, cell-major local vector
 *   y         device, [ncells][ndof_cell] io_dtype, overwritten; must not
 *             alias u or kappa
 *   ncells    >= 0 (0 is a no-op); hip_stream: hipStream_t or NULL
 * Errors: SF_ERR_ARG (NULL context/op/pointers with ncells > 0, ncells < 0),
 * SF_ERR_UNSUPPORTED (combination not built), SF_ERR_HIP (launch failure).
 * Geometry problems are reported asynchronously through sf_check_errors().
 */
int assemble_action(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices,
                    const void *kappa, const void *u, void *y, void *hip_stream);

/*
 * Allocation-free box-cell action, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * assemble_action() on a context whose geometry is SF_GEOM_BOX, restricted
 * to the box-cell kernel: families SF_Q, SF_DQ, SF_QGLL, forms SF_MASS and
 * SF_LAPLACE, precision SF_FP64 or SF_FP32, storage SF_F64 or SF_F32
 * (SF_ERR_UNSUPPORTED otherwise); every cell must be an axis-aligned box (a
 * sheared cell raises SF_FLAG_NONBOX), whatever the context's geometry hint.
 * The call allocates nothing: the kernel's scratch (one slot of claim
 * counters) and the 1-D tables of every supported family and degree live in
 * a fixed 96 KiB device array per GPU, set up once per device by
 * sf_context_create and held until the process ends.  The counters are
 * cleared by a kernel at the start of each call; calls that overlap on one
 * GPU (different streams, or different host threads) share that array and
 * race, so they must be serialised by the caller.  Inputs of any size are
 * accepted (the scratch does not grow with ncells); degrees outside 1..8 are
 * rejected with SF_ERR_UNSUPPORTED.
 */
int assemble_action_box_noalloc(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices,
                                const void *kappa, const void *u, void *y, void *hip_stream);

/*
 * Element matrices (Sec. 3.2: argument factorisation, then sum
 * factorisation of every product, Alg. 1, with the products' final
 * contraction merged by distributivity, Sec. 3.6 pass 6):
 *   A[c][i][j] = a(psi_j, psi_i) on cell c, row i = test, column j = trial,
 *   device [ncells][ndof_cell][ndof_cell] io_dtype, overwritten.
 * Other arguments and errors as assemble_action().  FP64 contractions
 * (SF_ERR_UNSUPPORTED otherwise).  Geometry, by the context's hint:
 *   SF_Q, SF_VQ: SF_GEOM_BOX: axis-aligned boxes, the three diagonal
 *     products (a sheared cell raises SF_FLAG_NONBOX); SF_GEOM_AFFINE (the
 *     default): any affine cell, all nine products P^{(a,b)} of eq.
 *     poisson_gem with the symmetric factor |J| G G^T; SF_GEOM_TRILINEAR:
 *     trilinear cells, the same nine products with J, G and |J| at every
 *     point.
 *   SF_QGLL, SF_DQ (quadrature points = nodes, B = I, Sec. 2.5): every
 *     geometry as above, assembled from the O(n^5) structured nonzeros
 *     (delta cancellation of the identity factors); the mass matrix is
 *     diagonal.
 *   SF_NCF, SF_NCE: axis-aligned boxes (others raise SF_FLAG_NONBOX).
 *   SF_SVK: affine cells or, under SF_GEOM_TRILINEAR, trilinear cells.
 */
int assemble_element_matrix(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices,
                            const void *kappa, void *A, void *hip_stream);

/* Synchronise `hip_stream` and report (then clear) the device flags raised by
 * earlier calls: SF_OK, or SF_ERR_GEOMETRY with *flags (may be NULL)
 * receiving the OR of SF_FLAG_* bits. */
int sf_check_errors(sf_context *ctx, void *hip_stream, int32_t *flags);

/*
 * Global continuous Q_p numbering on an nx*ny*nz tensor grid of cells (the
 * assembled operator of Sec. 4.2, whose rates count these global DOFs; cell
 * (i,j,k) is number (i*ny+j)*nz+k): local node (i0,i1,i2) of cell (i,j,k) is
 * the lattice point (a,b,c) = (i*p+i0, j*p+i1, k*p+i2), numbered
 * (a*(ny*p+1)+b)*(nz*p+1)+c.  Written by a GPU kernel into map_device, int32
 * [ncells][(p+1)^3].  Returns SF_ERR_ARG for non-positive sizes,
 * SF_ERR_CAPACITY when the number of global DOFs exceeds INT32_MAX.
 */
int sf_dof_map_q(sf_context *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t p, int32_t *map_device,
                 void *hip_stream);

/* Host only.  Local number of the DOF with per-axis indices multi[0..ndim-1]
 * in block `block` of an element whose blocks have extents
 * extents[b*ndim + a] (b < nblocks): the offset of the block (sum of the
 * sizes of the blocks before it) plus the row-major index within it.  This is
 * the concatenation of Sec. 2.6 with the indexed buffers of Sec. 3.5, in any
 * dimension.  Returns the index (>= 0) or SF_ERR_ARG for out-of-range input. */
int64_t sf_concat_index(int32_t ndim, int32_t nblocks, const int32_t *extents, int32_t block,
                        const int32_t *multi);

/* Host only.  Per-block extents of the element of `op` (family and degree):
 * *nblocks in {1,3}; extents[b*3+a] functions of block b along axis a;
 * offsets[b] the block's first local index (the vector element of SF_VQ and SF_SVK:
 * three blocks of (p+1)^3, one per component). */
int sf_block_layout(const sf_op *op, int32_t *nblocks, int32_t *extents, int32_t *offsets);

/*
 * Host only.  The 1-D tables the kernels use (Sec. 1.2 and Sec. 2.5): kind 0
 * = m-point Gauss-Legendre, kind 1 = m-point Gauss-Lobatto-Legendre rule on
 * [0,1] into x[m], w[m]; sf_lagrange_table fills B[p][i] = l_i(pts[p]) and
 * D[p][i] = l_i'(pts[p]) for the Lagrange basis l_i on `nodes`
 * (B, D are [npts][nnodes], row-major).  Errors: SF_ERR_ARG.
 */
int sf_rule_1d(int32_t kind, int32_t m, double *x, double *w);
int sf_lagrange_table(int32_t nnodes, const double *nodes, int32_t npts, const double *pts, double *B,
                      double *D);

/*
 * Host only.  The contraction order chosen for one product of 1-D factors
 * (Alg. 1, MakeTensorProduct, restricted to the three axis indices of a
 * hexahedron): for an input tensor with extents in[3] contracted along every
 * axis a by a matrix of shape out[a] x in[a], try all 6 axis orders and pick
 * the cheapest (ties: first in lexicographic order).  order[3] receives the
 * axes in application order; the return value is the flop count
 * (2 * out * in * remaining extents per step), or SF_ERR_ARG.
 */
int64_t sf_plan_axis_order(const int32_t *in, const int32_t *out, int32_t *order);

/*
 * Batched persistent launch (many meshes of mixed size and degree in one
 * fused launch, captured once in a hipGraph and replayed).  Each job is one
 * action (u, y non-NULL, A NULL) or one element-matrix assembly (A non-NULL,
 * u and y NULL) over its own mesh.  Element matrices are written into an
 * arena of A_arena_cells cells, cell c going to slot c % A_arena_cells
 * (A_arena_cells <= 0 means ncells, i.e. no cycling).  sf_batch_create
 * validates every job, builds the cost-ordered tile list, captures the
 * persistent kernel into a hipGraph on an internal stream and instantiates
 * it; it does not run it.  On a context declared SF_GEOM_BOX the FP64
 * actions run the box-cell body (cells must be axis-aligned boxes, as for
 * assemble_action there); otherwise the general affine body.  Supported
 * jobs: SF_Q, SF_LAPLACE, SF_F64 storage; actions in any precision, element
 * matrices in SF_FP64.  The caller keeps every job buffer alive until
 * sf_batch_destroy.  Errors: SF_ERR_ARG, SF_ERR_UNSUPPORTED, SF_ERR_NOMEM,
 * SF_ERR_HIP.
 */
typedef struct {
    sf_op op;
    int64_t ncells;
    const double *vertices;
    const void *kappa;
    const void *u;
    void *y;
    void *A;
    int64_t A_arena_cells;
} sf_job;

int sf_batch_create(sf_context *ctx, const sf_job *jobs, int32_t njobs, sf_batch **out);
int sf_batch_launch(sf_batch *batch, void *hip_stream);
int sf_batch_destroy(sf_batch *batch);
/* number of tiles and of workgroups the batch launch uses (for reports) */
int sf_batch_info(const sf_batch *batch, int64_t *ntiles, int32_t *nworkgroups);

/*
 * Autotuner of the kernel choices the library makes per class (family,
 * degree, form, nq1, precision, storage): times, on ncells_hint synthetic
 * unit-box cells on an internal stream, the candidates of every choice that
 * applies to `op` and records the fastest in the context:
 *   "batch" (SF_Q, SF_LAPLACE, SF_F64 storage, any precision): cell groups
 *     per tile of the batched launch's actions (1, 2, 4, 8 or 16; variants
 *     0..4);
 *   "batch_matrix" (the same class with SF_FP64): cell groups per tile of
 *     the batched launch's element matrices (same variants);
 *   "standalone" (SF_Q, SF_DQ, SF_QGLL; SF_MASS, SF_LAPLACE; SF_FP64 or
 *     SF_FP32; either storage): the box-cell action kernel used under
 *     SF_GEOM_BOX (0: prefetch of the next cell group, >= 3 workgroups per
 *     CU; 1: no prefetch, >= 4; 2: prefetch, >= 2; 3: the general
 *     three-tensor kernel that SF_GEOM_AFFINE uses; 4 and 5: 128-thread
 *     workgroups with and without prefetch; 6, p = 1 only: one cell per
 *     thread in registers, no LDS);
 *   "standalone" (SF_NCF, SF_NCE; SF_FP64 or SF_FP32; either storage): the
 *     H(div) / H(curl) action kernel used under SF_GEOM_BOX (0: diagonal
 *     Piola factors with the pointwise stage fused into the contractions;
 *     1: one cell group per workgroup; 2: the persistent kernel with full
 *     per-cell Piola factors that SF_GEOM_AFFINE uses).
 * A "standalone" entry for a scalar-family action in SF_BF16, SF_FP16 or
 * SF_BF16X3 selects its kernel (0, the default: the dense Kronecker
 * kernels; 1: the one-axis-at-a-time MFMA kernel).  sf_autotune does not
 * time that choice; sf_load_tuning accepts it.
 * When cache_json_path is non-NULL the choices are merged into that JSON
 * file, keyed by architecture, family, degree, form, nq1, precision, io dtype
 * and the choice name.  Later calls with the same key use the winners.
 * Returns SF_ERR_UNSUPPORTED for an op with no tunable choice.
 * sf_tuned_variant() returns the batched action tile variant (default 2).
 */
int sf_autotune(sf_context *ctx, const sf_op *op, int64_t ncells_hint, const char *cache_json_path);
int sf_tuned_variant(sf_context *ctx, const sf_op *op, int32_t *variant);
int sf_load_tuning(sf_context *ctx, const char *cache_json_path);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
