/*
 * fem.h -- C ABI of libfem: global stiffness and mass matrices of lowest-order
 * edge elements (Nedelec curl-curl + mass, Raviart-Thomas div-div + mass) on
 * 2D triangle and 3D tetrahedron meshes, assembled on an MI355X (gfx950) GPU.
 *
 * Method: Anjam & Valdman, "Fast MATLAB assembly of FEM matrices in 2D and 3D:
 * Edge elements" (arXiv:1409.4618).
 *   - mesh structures and global dof numbering: Section 3 (first two tables);
 *   - orientation (sign) data: Section 2.3 and Section 3;
 *   - Piola maps and reference bases: Sections 2.1 (RT) and 2.2 (Nedelec);
 *   - local and global matrices: Section 2.4;
 *   - assembly call sequence (affine maps, get_faces, signs, stiffness/mass):
 *     Section 3.2.
 *
 * Conventions shared by every entry point
 *   - All ids are 0-based (the paper is 1-based).
 *   - "dev" pointers are device (HBM) pointers on the current HIP device; "host"
 *     pointers are ordinary host memory. The caller owns every buffer it passes
 *     in; the library never frees them. The library owns everything inside a
 *     handle (topology, pattern, maps, scratch) and frees it in *_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work is
 *     enqueued on it asynchronously unless the entry point says it synchronises.
 *   - A handle is not thread-safe, and its work on different streams must not
 *     overlap: lazily built data (pattern, tiles, maps) and the adjoint's
 *     per-node partial sums live in the handle. Order such calls on one stream
 *     or synchronise between them. Distinct handles are independent.
 *   - Every entry point returns a fem_status. On an error nothing is enqueued,
 *     output buffers are left untouched, and fem_last_error() returns a message
 *     (thread-local, valid until the next call on that thread). Faults detected
 *     inside an asynchronous kernel (a zero Jacobian determinant, a non-finite
 *     coordinate) set a per-handle device error word read by fem_status_query.
 *   - Global dof numbering (the paper leaves the row order open): edge rows are
 *     the sorted node pairs (lo, hi), face rows the sorted node triples
 *     (a, b, c), both in lexicographic order.
 *   - Sign data: Nedelec (2D and 3D) and 2D Raviart-Thomas use +1 for a local
 *     edge whose start node has the larger global index (Section 3 states this
 *     for 2D; the 3D local edges are 1->2, 1->3, 1->4, 2->3, 3->4, 4->2 of
 *     Figure 1). 3D Raviart-Thomas uses minus the parity of the permutation
 *     taking the local node order to (sorted face nodes, opposite node), which
 *     equals the det-based rule of Section 2.3.
 *   - The 3D Raviart-Thomas basis is the printed one, whose flux through its
 *     face is 1/2 (Section 2.1).
 *   - Coefficients: K(a) = sum_K a_K K^K and M(b) = sum_K b_K M^K with one value
 *     per element; a NULL coefficient pointer means 1 (the paper's matrices).
 *   - CSR: rowptr int64 [n_rows+1], colind int32 [nnz] ascending within a row,
 *     full (not triangular) storage, every (dof_k, dof_l) pair of every element
 *     present even when its value is zero. K and M share the pattern. Values are
 *     bitwise symmetric and deterministic: an entry with more than two element
 *     contributions is summed in ascending element order, and one with two is
 *     the same either way round (x + y == y + x in IEEE arithmetic). A mesh in
 *     which some facet (3D face, 2D edge) has more than two elements, or which
 *     repeats an element, is assembled by the row kernels, which sum every
 *     entry in ascending element order.
 */
#ifndef FEM_H
#define FEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fem_mesh_s* fem_mesh;
typedef struct fem_batch_s* fem_batch;

typedef enum {
    FEM_NEDELEC = 0,         /* H(curl): curl-curl stiffness + mass, dofs on edges        */
    FEM_RAVIART_THOMAS = 1,  /* H(div): div-div stiffness + mass, dofs on edges (2D) /
                                faces (3D)                                                 */
    FEM_KIND_RANGE_MIN = -0x7FFFFFFF - 1,  /* not kinds: they widen the enum to the range of
    FEM_KIND_RANGE_MAX = 0x7FFFFFFF         int, so any int a caller passes is a valid value
                                            (and rejected with FEM_EINVAL)                    */
} fem_kind;

typedef enum {
    FEM_OK = 0,
    FEM_EINVAL = 1,       /* bad argument: NULL pointer, dim not 2/3, kind/dim mismatch, ... */
    FEM_ERANGE = 2,       /* an element references a node id outside [0, n_nodes); in the
                             checked build (FEM_CHECK=1), also: a kernel met a map index
                             outside the array it indexes                                   */
    FEM_EDEGENERATE = 3,  /* an element has det B_K == 0 (e.g. a repeated node)            */
    FEM_ENONFINITE = 4,   /* a node coordinate or a Jacobian determinant is not finite     */
    FEM_EOVERFLOW = 5,    /* a size exceeds an index limit (int32 ids, row length > 255)   */
    FEM_ENOMEM = 6,       /* device allocation failed                                      */
    FEM_EHIP = 7,         /* a HIP runtime call failed                                     */
    FEM_ENOTREADY = 8     /* the pattern for this kind has not been built (fem_pattern)   */
} fem_status;

/* Topology: Section 3 (get_edges / get_faces / signs_edges / signs_faces).
 *   nodes  dev f64 [n_nodes][dim]   node coordinates (nodes2coord), row-major
 *   elems  dev i32 [n_elems][dim+1] element -> node ids (elems2nodes), row-major
 *   dim    2 (triangles) or 3 (tetrahedra)
 * Builds the global edge (and in 3D face) numbering, elems2edges / elems2faces
 * and the sign data by a device radix sort + unique over node-index keys, and
 * validates the mesh (node ids in range, finite coordinates, det B_K != 0).
 * Synchronises `stream` (to learn the number of edges / faces).
 * On success *out owns the topology; release it with fem_mesh_destroy.
 * Limits: n_elems * (edges per element) < 2^31, n_nodes * dim < 2^31.       */
fem_status fem_topology(const double* nodes, int64_t n_nodes, int dim,
                        const int32_t* elems, int64_t n_elems,
                        void* stream, fem_mesh* out);

/* Counts of a mesh (host outputs; any pointer may be NULL). n_faces is 0 in 2D. */
fem_status fem_mesh_counts(fem_mesh mesh, int64_t* n_nodes, int64_t* n_elems,
                           int64_t* n_edges, int64_t* n_faces, int* dim);

/* Borrowed device pointers to the topology (valid until fem_mesh_destroy):
 *   edges2nodes i32 [n_edges][2] (lo < hi), elems2edges i32 [n_elems][3|6],
 *   signs_e i8 [n_elems][3|6], faces2nodes i32 [n_faces][3] (a < b < c),
 *   elems2faces i32 [n_elems][4], signs_f i8 [n_elems][4] (3D only; NULL in 2D).
 * Any output pointer may be NULL.                                            */
fem_status fem_mesh_topology(fem_mesh mesh, const int32_t** edges2nodes,
                             const int32_t** elems2edges, const int8_t** signs_e,
                             const int32_t** faces2nodes, const int32_t** elems2faces,
                             const int8_t** signs_f);

/* One-time CSR sparsity pattern of `kind` and the per-element scatter map
 * (the global step that the paper leaves out at the end of Section 3.2).
 * Builds it on first use (synchronises `stream`), then returns borrowed device
 * pointers: rowptr i64 [n_rows+1], colind i32 [nnz]. n_rows is the number of
 * edges (Nedelec, 2D RT) or faces (3D RT). Outputs may be NULL.
 * The element pairs are sorted in chunks of whole rows (at most 2^29 pairs
 * each; the environment variable FEM_PAIR_CHUNK sets another bound), so
 * n_elems * n_local^2 may exceed 2^31 (3D Nedelec on a 60 M-tet mesh), and
 * so may nnz (rowptr is i64; colind holds column numbers, which are below
 * n_rows). FEM_EOVERFLOW if a row has more than 255 entries; a refused build
 * keeps nothing, and the other kind's pattern can still be built.            */
fem_status fem_pattern(fem_mesh mesh, fem_kind kind, void* stream,
                       int64_t* n_rows, int64_t* nnz,
                       const int64_t** rowptr, const int32_t** colind);

/* Numeric assembly (the hot path): values of K(a) and M(b) on the pattern of
 * fem_pattern(kind), Section 2.4. Asynchronous on `stream`.
 *   nodes  dev f64 [n_nodes][dim]  coordinates (may differ from fem_topology's;
 *                                  the topology is reused)
 *   a, b   dev f64 [n_elems] or NULL (= 1)
 *   K_vals dev f64 [nnz] output (may be NULL to skip K); M_vals likewise
 * Each value is written exactly once (no accumulation into the outputs).
 * FEM_ENOTREADY if fem_pattern(kind) has not been called.                  */
fem_status fem_assemble(fem_mesh mesh, fem_kind kind, const double* nodes,
                        const double* a, const double* b,
                        double* K_vals, double* M_vals, void* stream);

/* Adjoint of fem_assemble for L = sum_p gK[p] K(a)[p] + gM[p] M(b)[p]
 * (for L = u^T (K(a) + M(b)) u pass gK[p] = gM[p] = u_row(p) u_col(p)).
 * Not part of the paper: the derivative of its local matrices (Section 2.4) with
 * respect to the coefficients and the vertex coordinates. Asynchronous.
 *   gK, gM  dev f64 [nnz] upstream weights (NULL = 0)
 *   ga, gb  dev f64 [n_elems] outputs dL/da, dL/db (NULL to skip)
 *   gnodes  dev f64 [n_nodes][dim] output dL/dnodes (NULL to skip); overwritten,
 *           nodes in no element get 0.
 * Uses library-owned scratch inside the handle (allocated on first use).
 * FEM_EOVERFLOW if nnz >= 2^31 (its per-slot row starts are 32-bit); the
 * quadratic form (fem_assemble_backward_quadratic) reads no nnz-sized array
 * and has no such limit.                                                     */
fem_status fem_assemble_backward(fem_mesh mesh, fem_kind kind, const double* nodes,
                                 const double* a, const double* b,
                                 const double* gK, const double* gM,
                                 double* ga, double* gb, double* gnodes, void* stream);

/* Adjoint of the quadratic form L = u^T (K(a) + M(b)) u (the energy of a dof
 * vector u): the outputs of fem_assemble_backward with
 * gK[p] = gM[p] = u_row(p) u_col(p), up to rounding, but formed per element
 * from u at its dofs instead of from nnz-sized arrays. The element's
 * contractions are evaluated as sums of squares (for 3D Nedelec
 * |sum_k s_k u_k o_k|^2 for K and the squared Whitney field for M; for
 * Raviart-Thomas and 2D the squared divergence and field likewise), so the
 * results differ from the general entry point by a few ulps of the element
 * sums. Deterministic. Not part of the paper. Asynchronous.
 *   u       dev f64 [n_rows of fem_pattern(kind)] (edge or face values)
 *   ga, gb, gnodes as in fem_assemble_backward (NULL to skip)
 * FEM_EINVAL if u is NULL.                                                  */
fem_status fem_assemble_backward_quadratic(fem_mesh mesh, fem_kind kind, const double* nodes,
                                           const double* a, const double* b, const double* u,
                                           double* ga, double* gb, double* gnodes, void* stream);

/* Value of the quadratic form L = u^T (K(a) + M(b)) u (the energy of a dof
 * vector u for the matrices of Section 2.4), without assembling K and M: L is
 * linear in the coefficients, so L = sum_K (a_K dL/da_K + b_K dL/db_K), and
 * each element's dL/da_K, dL/db_K are the sums of squares of
 * fem_assemble_backward_quadratic. Not part of the paper (it is the forward
 * value of that adjoint). Deterministic: one partial per workgroup of 256
 * elements, each summed in a fixed tree order, then the partials in a fixed
 * order. Asynchronous on `stream`.
 *   u      dev f64 [n_rows of fem_pattern(kind)] (edge or face values)
 *   L      dev f64 [1] output
 * Uses library-owned scratch inside the handle (ceil(n_elems / 256) doubles,
 * allocated on the first call). FEM_EINVAL if nodes, u or L is NULL;
 * FEM_ENOTREADY if fem_pattern(kind) has not been called.                  */
fem_status fem_quadratic_value(fem_mesh mesh, fem_kind kind, const double* nodes,
                               const double* a, const double* b, const double* u,
                               double* L, void* stream);

/* L = u^T (K(a) + M(b)) u and its adjoint (dL/da, dL/db, dL/dnodes) in one
 * pass: fem_quadratic_value and fem_assemble_backward_quadratic fused, for a
 * forward pass whose result will be differentiated (the derivatives are then
 * ready before the backward pass asks for them; the backward only scales them
 * by the upstream factor). Not part of the paper. Arguments as in those two
 * calls; ga, gb, gnodes may be NULL (all three NULL: fem_quadratic_value).
 * L is summed in the same element order as fem_quadratic_value's; the two may
 * differ in the last bits (the element terms come from another kernel).
 * Uses the handle's scratch of fem_quadratic_value. Asynchronous.
 * FEM_EINVAL if nodes, u or L is NULL; FEM_ENOTREADY before fem_pattern.    */
fem_status fem_quadratic_value_adjoint(fem_mesh mesh, fem_kind kind, const double* nodes,
                                       const double* a, const double* b, const double* u,
                                       double* L, double* ga, double* gb, double* gnodes,
                                       void* stream);

/* Allocation-free variant of fem_quadratic_value, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, kernels and result
 * (bitwise) as fem_quadratic_value; it calls no hipMalloc, hipFree or other
 * allocating routine. Its workgroup partials live in a fixed device array
 * inside the library (4 MiB, one copy on each GPU the library runs on, held
 * until the process ends), whose device address is looked up once per device
 * on the first call there.
 *   limit  n_elems <= 2^27 (134,217,728); larger meshes get FEM_EOVERFLOW
 *          (fem_quadratic_value has no such limit)
 *   device the mesh's device must be the current device (else FEM_EINVAL)
 * Every call on one GPU shares that array: calls that overlap on one GPU (on
 * different streams, or from different threads without ordering) race and
 * give wrong values. Order them on one stream or synchronise between them.
 * Asynchronous on `stream`. FEM_EINVAL if nodes, u or L is NULL;
 * FEM_ENOTREADY if fem_pattern(kind) has not been called.                  */
fem_status fem_quadratic_value_noalloc(fem_mesh mesh, fem_kind kind, const double* nodes,
                                       const double* a, const double* b, const double* u,
                                       double* L, void* stream);

/* Sparse product on an assembled pattern: y = alpha A x + beta B x, where A and
 * B are value arrays on the same CSR pattern (for example K and M of
 * fem_assemble; B may be NULL, then y = alpha A x). Not part of the paper: the
 * operator of the linear systems its Section 4 examples solve, and the
 * derivative 2 (K + M) u of the quadratic form with respect to u.
 *   rowptr dev i64 [n_rows+1], colind dev i32 [nnz], A, B dev f64 [nnz]
 *   x      dev f64 [n_cols] (n_cols = n_rows for the patterns of fem_pattern)
 *   y      dev f64 [n_rows] output, overwritten; must not alias x
 * Every row is summed in a fixed order (deterministic). Asynchronous.
 * FEM_EINVAL for a NULL argument (n_rows > 0) or x == y.                    */
fem_status fem_csr_matvec(int64_t n_rows, const int64_t* rowptr, const int32_t* colind,
                          const double* A, const double* B, double alpha, double beta,
                          const double* x, double* y, void* stream);

/* ---------------------------------------------------------------------------
 * Integration over a mesh (Section 3.1) and the building blocks of the
 * examples of Section 4: the squared L2 norm of a function, the load vector of
 * the Nedelec basis, the H(curl) error of a discrete field, and a
 * conjugate-gradient solve on an assembled pattern.
 *
 * Quadrature: the conical-product Gauss-Legendre rule on the reference
 * triangle / tetrahedron with `quad_m` points per direction (1..8; quad_m^dim
 * points), exact for polynomials of total degree <= 2 quad_m - dim. The
 * paper's routine uses a rule of order 6; quad_m = 4 (2D) and 5 (3D) reach it.
 *
 * Functions: the paper's norm_L2 takes a function handle; here the integrand
 * is one of a compiled-in catalogue, selected by fem_function:
 *   FEM_FN_POLYNOMIAL   f(x) = sum of terms c x_1^p_1 ... x_d^p_d, each term
 *                       adding to one component of f. params: host array of
 *                       n_terms (1..32) groups of (2 + dim) doubles:
 *                       c, component (0..dim-1), p_1 .. p_dim (integers 0..30).
 *   FEM_FN_EDDY_E       the exact solution E of the 2D eddy-current example
 *                       (Section 4.2): the printed field on x1 > x2, 0 elsewhere
 *   FEM_FN_EDDY_CURL_E  its curl (scalar)
 *   FEM_FN_EDDY_F       its right-hand side F = curl_vec curl E + E (mu = kappa = 1)
 *   FEM_FN_BUBBLE_U     the bubble u = prod_i x_i (x_i - 1) of the majorant
 *                       example (Section 4.1), 2D or 3D (scalar)
 *   FEM_FN_BUBBLE_GRAD_U  its gradient (dim components)
 *   FEM_FN_BUBBLE_F     f = -Lap u (scalar)
 * The eddy and bubble functions take no params (NULL, 0); the eddy functions
 * need dim = 2.
 */
typedef enum {
    FEM_FN_POLYNOMIAL = 0,
    FEM_FN_EDDY_E = 1,
    FEM_FN_EDDY_CURL_E = 2,
    FEM_FN_EDDY_F = 3,
    FEM_FN_BUBBLE_U = 4,
    FEM_FN_BUBBLE_GRAD_U = 5,
    FEM_FN_BUBBLE_F = 6,
    FEM_FN_RANGE_MIN = -0x7FFFFFFF - 1,  /* not functions: they widen the enum to the range
    FEM_FN_RANGE_MAX = 0x7FFFFFFF         of int (any other value is rejected with FEM_EINVAL) */
} fem_function;

/* Squared L2 norm ||f||^2 = sum_K int_K |f|^2 (the paper's norm_L2, Section 3.1;
 * for a vector function the squared Euclidean norm is integrated).
 *   nodes     dev f64 [n_nodes][dim]
 *   per_elem  dev f64 [n_elems] output ||f||_K^2 (NULL to skip)
 *   total     dev f64 [1] output ||f||^2
 * Deterministic (element sums in a fixed order). Uses library-owned scratch in
 * the handle (ceil(n_elems / 256) doubles, allocated on first use).
 * Asynchronous. FEM_EINVAL for a bad function, params or quad_m.            */
fem_status fem_norm_L2(fem_mesh mesh, const double* nodes, fem_function f, const double* params,
                       int n_params, int quad_m, double* per_elem, double* total, void* stream);

/* Load vector f_i = int F . eta_i of the Nedelec basis (kind must be
 * FEM_NEDELEC; 2D and 3D), for a vector function F of the mesh dimension.
 * eta_i is the global (sign-adjusted, Piola-mapped) basis function of edge i,
 * Sections 2.2-2.3. Element integrals by the quadrature above, then each
 * entry summed over its edge's elements in ascending element order.
 *   f  dev f64 [n_edges] output, overwritten
 * Uses library-owned scratch in the handle ([n_elems][3|6] doubles).
 * Asynchronous.                                                             */
fem_status fem_load_vector(fem_mesh mesh, fem_kind kind, const double* nodes, fem_function F,
                           const double* params, int n_params, int quad_m, double* f, void* stream);

/* H(curl) error of the Nedelec field v_h with edge values v against a field E
 * with curl C: sum_K int_K |E - v_h|^2 + |C - curl v_h|^2 (the squared error
 * of the eddy-current table, Section 4.2). kind must be FEM_NEDELEC.
 *   v         dev f64 [n_edges]
 *   field     function giving E (dim components), curl giving C (2D: 1, 3D: 3
 *             components); both read `params` when they are polynomials
 *   per_elem  dev f64 [n_elems] output (NULL to skip); total dev f64 [1] output
 * Deterministic. Uses the handle's scratch of fem_norm_L2. Asynchronous.     */
fem_status fem_field_error(fem_mesh mesh, fem_kind kind, const double* nodes, const double* v,
                           fem_function field, fem_function curl, const double* params, int n_params,
                           int quad_m, double* per_elem, double* total, void* stream);

/* Solve (ca A + cb B) x = rhs by conjugate gradients with the Jacobi
 * (diagonal) preconditioner, A and B value arrays on one CSR pattern (B may
 * be NULL). Not part of the paper (its Section 4 examples solve such systems;
 * the matrix must be symmetric positive definite, as K + M is).
 *   rowptr dev i64 [n_rows+1], colind dev i32 [nnz] (square pattern)
 *   rhs    dev f64 [n_rows]; x dev f64 [n_rows]: initial guess in, solution out
 *   rtol   stop when the recursive residual r (updated by the iteration, equal
 *          to rhs - A' x up to rounding) has ||r|| <= rtol ||rhs||; tested every
 *          16 iterations
 *   iters, rel_resid  host outputs (may be NULL): iterations done and the true
 *          relative residual ||rhs - A' x|| / ||rhs|| of the returned x, formed
 *          at the end (it can stay above rtol by the rounding of A' x)
 * Deterministic: every dot product is summed in one fixed order. Allocates its
 * workspace (6 n_rows + 8229 doubles, and with B the nnz values ca A + cb B,
 * formed once so that an iteration reads one value array) for the call and
 * synchronises `stream`.
 * FEM_EINVAL for bad arguments or a non-positive diagonal entry; FEM_EHIP if
 * the iteration breaks down (p . A' p <= 0). Reaching max_iter is not an
 * error: check rel_resid. With the environment variable FEM_CG_LOG=N set, a
 * line on stderr reports the iterations and the recursive relative residual
 * at the first convergence test after every N iterations.                  */
fem_status fem_cg_solve(int64_t n_rows, const int64_t* rowptr, const int32_t* colind,
                        const double* A, const double* B, double ca, double cb, const double* rhs,
                        double* x, double rtol, int64_t max_iter, void* stream, int64_t* iters,
                        double* rel_resid);

/* ---------------------------------------------------------------------------
 * The majorant minimisation of Section 4.1: linear nodal (P1) elements for the
 * approximation v of -Lap u = f (u = 0 on the boundary), and the
 * Raviart-Thomas quantities of the majorant functional. The global
 * Raviart-Thomas basis on an element is phi_k = s_k (x - x_p) / det B_K, p the
 * vertex opposite local dof k (the Piola image of the printed basis with the
 * signed determinant, Section 2.1; with the sign data of Section 2.3 its
 * normal component is continuous), div phi_k = s_k d / det B_K.
 */

/* Nodal CSR pattern of the P1 stiffness matrix: row i holds node i and its
 * edge neighbours, columns ascending (n_rows = n_nodes, nnz = n_nodes +
 * 2 n_edges). Built on first use together with each node's list of element
 * incidences and the boundary-node flags (nodes of facets that belong to one
 * element); synchronises `stream`. Borrowed device pointers, valid until
 * fem_mesh_destroy. FEM_EOVERFLOW if nnz >= 2^31.                          */
fem_status fem_p1_pattern(fem_mesh mesh, void* stream, int64_t* n_rows, int64_t* nnz,
                          const int64_t** rowptr, const int32_t** colind);

/* P1 stiffness K_ij = sum_K a_K int_K grad(lambda_i) . grad(lambda_j) on the
 * pattern of fem_p1_pattern (a NULL = 1). Entry (i, j) is summed over the
 * elements of edge {i, j}, (i, i) over the elements of node i, each in
 * ascending element order (deterministic). K dev f64 [nnz] output.
 * FEM_ENOTREADY before fem_p1_pattern. Asynchronous.                       */
fem_status fem_p1_assemble(fem_mesh mesh, const double* nodes, const double* a, double* K,
                           void* stream);

/* P1 load vector F_i = int f lambda_i of a scalar catalogue function, by the
 * quadrature above; element values summed per node in ascending element
 * order. F dev f64 [n_nodes] output. Uses the handle's element scratch.
 * FEM_ENOTREADY before fem_p1_pattern. Asynchronous.                       */
fem_status fem_p1_load(fem_mesh mesh, const double* nodes, fem_function f, const double* params,
                       int n_params, int quad_m, double* F, void* stream);

/* Boundary condition v = 0 on the boundary nodes by symmetric elimination:
 * their rows and columns of K become those of the identity and their entries
 * of rhs 0 (either pointer may be NULL). FEM_ENOTREADY before fem_p1_pattern.
 * Asynchronous.                                                             */
fem_status fem_p1_dirichlet(fem_mesh mesh, double* K, double* rhs, void* stream);

/* Energy error sum_K int_K |g - grad v|^2 of the P1 field v (dev [n_nodes])
 * against a vector function g (the exact gradient: FEM_FN_BUBBLE_GRAD_U, or a
 * polynomial); per_elem dev [n_elems] (NULL to skip), total dev [1]. Uses the
 * handle's scratch of fem_norm_L2. Asynchronous.                           */
fem_status fem_p1_grad_error(fem_mesh mesh, const double* nodes, const double* v, fem_function g,
                             const double* params, int n_params, int quad_m, double* per_elem,
                             double* total, void* stream);

/* Right-hand side of the discrete majorant problem (Section 4.1):
 *   rhs_i = c_div int f div phi_i + c_grad int grad v . phi_i
 * over the Raviart-Thomas basis (edges in 2D, faces in 3D), for a scalar
 * function f and the P1 field v (dev [n_nodes]); the problem of Section 4.1
 * takes c_div = -(1 + beta) C^2, c_grad = 1 + 1/beta. Element values summed
 * per dof in ascending element order. rhs dev f64 [n_rows of
 * fem_pattern(FEM_RAVIART_THOMAS)] output. Uses the handle's element
 * scratch. Asynchronous.                                                    */
fem_status fem_rt_majorant_rhs(fem_mesh mesh, const double* nodes, const double* v, fem_function f,
                               const double* params, int n_params, int quad_m, double c_div,
                               double c_grad, double* rhs, void* stream);

/* The two terms of the majorant for the P1 field v and the Raviart-Thomas
 * field y (dof values, dev [n_rows]): terms[0] = ||grad v - y||^2,
 * terms[1] = ||div y + f||^2 (dev f64 [2] output), each summed in a fixed
 * order. The majorant is sqrt((1 + 1/beta) terms[0] + (1 + beta) C^2 terms[1])
 * and the optimal beta sqrt(terms[0]) / (C sqrt(terms[1])). Uses the handle's
 * scratch of fem_norm_L2. Asynchronous.                                    */
fem_status fem_majorant_terms(fem_mesh mesh, const double* nodes, const double* v, const double* y,
                              fem_function f, const double* params, int n_params, int quad_m,
                              double* terms, void* stream);

/* Synchronises the last stream used with `mesh`, returns and clears the
 * asynchronous device error word (FEM_OK, FEM_EDEGENERATE or FEM_ENONFINITE). */
fem_status fem_status_query(fem_mesh mesh);

void fem_mesh_destroy(fem_mesh mesh);

/* ---------------------------------------------------------------------------
 * Batched assembly: many meshes of uneven sizes (mixed dims and kinds) in one
 * launch (a persistent kernel over every kind), or with element-major tiles in
 * one launch per element kind present (schedules 3-4 below). Not in the paper
 * (a launch-amortisation layer over the same per-element computation).
 *   meshes  host array [n] of handles, each with fem_pattern(kinds[i]) built
 *   kinds   host array [n]
 * The batch borrows the meshes (they must outlive it).                     */
fem_status fem_batch_create(const fem_mesh* meshes, const fem_kind* kinds, int n,
                            fem_batch* out);

/* Bind the per-mesh buffers (host arrays [n] of device pointers; a/b entries
 * may be NULL = 1, K/M entries may be NULL to skip). Waits for the device to
 * be idle (a launch of the batch may still read the table), then copies a
 * small table to the device. Rebinding is allowed between launches.         */
fem_status fem_batch_bind(fem_batch batch, const double* const* nodes,
                          const double* const* a, const double* const* b,
                          double* const* K_vals, double* const* M_vals);

/* Autotuner: times every candidate (tiling with its workgroup size, schedule)
 * with the bound buffers on `stream`: element-major tiles of 256 and of 128
 * lanes with schedules 0-4, row tiles of 64/128/256 rows with schedules 0-2. Keeps
 * the fastest, and records it in the JSON cache file
 * `cache_path` (NULL = no file). If the file already holds an entry for this
 * device and batch signature, that entry is used without timing. Synchronises. */
fem_status fem_batch_tune(fem_batch batch, const char* cache_path, void* stream);

/* Which configuration the batch uses (host outputs, may be NULL):
 * tiling, schedule, workgroup size, number of work items, grid size (the
 * workgroups launched: the persistent grid, or with schedules 3-4 one per
 * work item). Schedules: 0 static stride, 1 dynamic queue, 2 LPT-sorted
 * dynamic queue (a persistent kernel over every kind); with element-major
 * tiles also 3 and 4: the items grouped by element kind, one plain-grid
 * launch per kind (one workgroup per item, the kind's own kernel and its
 * occupancy), in mesh order (3) or by decreasing cost (4; the default when
 * element-major tiles fit). Tiling
 * (`rows_per_tile`):
 *   0            element-major tiles, one element per lane, in workgroups of
 *                `threads` lanes (128 or 256: the elements per tile and the
 *                wavefronts per workgroup); rows per tile chosen per mesh so
 *                that a tile's element list fits its workgroup (the default,
 *                with 256, when every mesh's tiles fit);
 *   64, 128, 256 row tiles of that many rows, one or more lanes per row, in
 *                workgroups of 256 lanes (`threads` = 256).                 */
fem_status fem_batch_config(fem_batch batch, int* rows_per_tile, int* schedule, int* threads,
                            int64_t* n_work, int* grid);

/* Select a configuration by hand (skips tuning). FEM_EINVAL for a tiling
 * outside {0, 64, 128, 256} (or 0 when element-major tiles are unavailable),
 * a schedule outside 0..2, or `threads` other than 128/256 for element-major
 * tiles and 0/256 for row tiles. The 128-lane element-major tiles are built on
 * first use (device allocations; synchronises the device); FEM_EINVAL if some
 * mesh's tiles do not fit 128 lanes.                                          */
fem_status fem_batch_set_config(fem_batch batch, int rows_per_tile, int schedule, int threads);

/* One persistent launch over all bound meshes. Asynchronous; contains no
 * memset or allocation, so it may be captured into a HIP graph. Launches of
 * one batch, direct or replayed, must not overlap: they share a work-queue
 * counter that the last workgroup resets. Queue them on one stream or
 * synchronise between them.                                                */
fem_status fem_batch_assemble(fem_batch batch, void* stream);

/* Capture one fem_batch_assemble into a HIP graph held by the batch
 * (re-captured after bind / set_config / tune), then replay it on `stream`.
 * Before a capture, one plain launch runs on the batch's own stream, ordered
 * after the work already queued on `stream`, and is waited for.            */
fem_status fem_batch_graph_launch(fem_batch batch, void* stream);

void fem_batch_destroy(fem_batch batch);

/* Message of the last error on this thread ("" if none). */
const char* fem_last_error(void);

/* Library version string. */
const char* fem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FEM_H */
