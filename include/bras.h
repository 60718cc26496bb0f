/*
 * bras.h - C ABI of the MI355X (gfx950) BRAS mass-inverse library.
 *
 * The library solves finite-element mass systems M u = f with preconditioned
 * conjugate gradients, where M = P^T M_br P is assembled from element mass
 * matrices M_K and the broken-to-conforming map pi (eq. M_PMbrP), and the
 * preconditioner is either diag(M)^-1 (Section 2.1) or the broken-space
 * additive Schwarz inverse
 *
 *     M_bras^-1 = D^-1 P^T M_br^-1 P D^-1,   D = P^T P = diag(d_i)
 *
 * (eq. mhatinvbras_def; element-sum form eq. mass_and_bras_element_sums).
 *
 * Conventions shared by every call
 *   - Functions return BRAS_OK (0) or a negative status; they never abort and
 *     no C++ exception crosses this boundary.  bras_last_error() returns a
 *     thread-local message for the last failure on the calling thread.
 *   - "_d" arguments are device pointers (memory of the current HIP device),
 *     "_h" arguments are host pointers.  Buffers passed in are owned by the
 *     caller; the library never frees them.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *   - Conforming vectors are float64 [n] for one right-hand side, or
 *     [n][nrhs] row-major (right-hand-side index fastest) for several.
 *   - Element-local order, entity numbering and the reference simplex
 *     conv{0, e_1, .., e_d} follow the canonical convention documented with
 *     bras_dofmap().
 */
#ifndef BRAS_H
#define BRAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BRAS_OK          0
#define BRAS_EINVAL     -1   /* bad argument: null pointer, size, map entry  */
#define BRAS_ENOTSPD    -2   /* an element mass matrix failed Cholesky        */
#define BRAS_EHIP       -3   /* a HIP runtime call failed                     */
#define BRAS_ENOCONV    -4   /* PCG reached maxit before the tolerance        */
#define BRAS_EBREAKDOWN -5   /* PCG breakdown: p.q <= 0, r.z <= 0, NaN / Inf  */
#define BRAS_ENOMEM     -6   /* device allocation failed                      */

/* ---- element families (Section 3: Lagrange, Bernstein, N1curl, N2curl, RT, BDM) */
#define BRAS_H1    0         /* H1 Lagrange P_p, GLL-based nodes             */
#define BRAS_HCURL 1         /* first-kind Nedelec N1curl_k, covariant Piola */
#define BRAS_HDIV  2         /* Raviart-Thomas RT_k, contravariant Piola     */
#define BRAS_H1_BERNSTEIN 3  /* H1 P_p in the Bernstein basis p!/alpha! lambda^alpha,
                                local order as the Lagrange nodes (same multi-indices) */
#define BRAS_HCURL2 4        /* second-kind Nedelec N2curl_k = [P_k]^d, covariant Piola */
#define BRAS_HDIV2  5        /* Brezzi-Douglas-Marini BDM_k = [P_k]^d, contravariant Piola */

/* ---- element-data forms accepted by bras_setup -------------------------- */
#define BRAS_ELEM_EXPLICIT   0  /* elem_d: E x n_loc x n_loc float64 M_K, row-major */
#define BRAS_ELEM_SCALED_REF 1  /* ref_d: n_loc^2 Mhat; elem_d: E scalars c_K,
                                   M_K = c_K Mhat (affine H1, eq. h1_mass_pullback) */
#define BRAS_ELEM_METRIC_REF 2  /* ref_d: nsym x n_loc^2 symmetric tables S_p;
                                   elem_d: E x nsym metric entries G_p;
                                   M_K = sum_p G_p S_p (eqs. hcurl/hdiv_mass_pullback) */

/* ---- precision of the stored BRAS element inverses ---------------------- */
#define BRAS_FP64 0
#define BRAS_FP32 1
#define BRAS_BF16 2          /* Gram-factor form on MFMA, FP32 accumulation  */

/* ---- preconditioners for pcg_solve -------------------------------------- */
#define BRAS_PC_NONE   0
#define BRAS_PC_JACOBI 1     /* diag(M)^-1                                    */
#define BRAS_PC_BRAS   2     /* D^-1 P^T M_br^-1 P D^-1                       */

typedef struct bras_ctx* bras_handle;

/* ======================================================================== *
 * Host helpers: workload construction.  Every output is written to host
 * memory and is bit-exact reproducible from the documented definitions.
 * ======================================================================== */

/* Sizes of the structured Kuhn mesh of the unit square (dim 2: N*N squares
 * split into 2 triangles) or cube (dim 3: N^3 cubes split into the 6
 * tetrahedra containing the main diagonal).  Returns EINVAL for dim not in
 * {2,3} or N < 1. */
int bras_mesh_size(int dim, int N, int64_t* nvert_h, int64_t* ncell_h);

/* Structured mesh (the simplicial unit square / cube meshes of Section 3).
 * Vertex (i,j[,k]) has id i + (N+1)(j + (N+1)k) and coordinates (i h, ...),
 * h = 1.0/N.  Cells list ascending vertex ids: 2D square c = i + N j gives
 * triangles [v(i,j), v(i+1,j), v(i+1,j+1)] and [v(i,j), v(i,j+1), v(i+1,j+1)];
 * 3D cube c gives 6 tetrahedra, s-th = monotone lattice path through the
 * cube along the s-th permutation of the axes in lexicographic order.
 * Interior vertices move each coordinate by (jitter h)(2u - 1),
 * u = (mix64(seed + (dim vid + axis + 1) * 0x9E3779B97F4A7C15) >> 11) 2^-53,
 * mix64 = the SplitMix64 output function.
 * coords_h: [nvert][dim] float64, cells_h: [ncell][dim+1] int32 (caller
 * allocated, sizes from bras_mesh_size). */
int bras_mesh_structured(int dim, int N, double jitter, uint64_t seed,
                         double* coords_h, int32_t* cells_h);

/* Element description: n_loc and the DOFs per vertex, edge, face and cell
 * (dofs_per_entity_h[4]; 2D uses entries 0..2, entry 2 = cell).
 * Supported: H1 degree 1..6 (2D/3D), HCURL and HDIV degree 1..4 (2D/3D),
 * HCURL2 and HDIV2 degree 1..7 (2D) and 1..4 (3D). */
int bras_element_info(int family, int dim, int degree, int* n_loc_h, int* dofs_per_entity_h);

/* Reference mass tables on conv{0, e_1, .., e_d} (eq. piola_mass_pullbacks).
 * H1: ref_h[n_loc*n_loc] = Mhat_ij = int phi_i phi_j.
 * HCURL/HDIV: nsym = dim(dim+1)/2 symmetric tables, pair order
 * (0,0),(0,1),(0,2),(1,1),(1,2),(2,2) in 3D and (0,0),(0,1),(1,1) in 2D:
 * S_(a,a) = Mhat^{aa}, S_(a,b) = Mhat^{ab} + Mhat^{ba} for a < b, with
 * Mhat^{ab}_ij = int phi_i^a phi_j^b, so M_K = sum_p G_p S_p.
 * Degrees of freedom: point values at recursive GLL nodes (H1); integral
 * moments against orthonormal polynomials of each sorted-vertex entity
 * (HCURL / HDIV); for HCURL2 / HDIV2 the classical second-kind moments
 * (edges / facets against P_k, N2curl faces against RT_{k-1}, interiors
 * against RT_{k-1} (2D) / RT_{k-2} (3D) for N2curl and N1curl_{k-1} for BDM),
 * the RT / N1curl test fields being monomial spanning fields orthonormalised
 * in a fixed order.  Computed by quadrature in extended precision. */
int bras_reference_mass(int family, int dim, int degree, double* ref_h);

/* Canonical local-to-global map.  Edges / faces are the sorted vertex pairs /
 * triples of the cells numbered in lexicographic order; conforming DOFs come
 * in blocks [vertex | edge | face | cell] (2D: [vertex | edge | cell]), entity
 * e of a block owning offset + e*k + (0..k-1).  l2g_h[K][l] follows the
 * element's local order: vertices, local edges (lex pairs of local vertices),
 * local faces, interior.  cells_h must list ascending vertex ids.
 * Outputs n (number of conforming DOFs) and l2g_h [E][n_loc] int32. */
int bras_dofmap(int family, int dim, int degree, int64_t nvert, int64_t ncell,
                const int32_t* cells_h, int64_t* n_h, int32_t* l2g_h);

/* Per-element pullback coefficients on the device (eq. piola_mass_pullbacks):
 * H1    elem_d[K]         = rho_K |det J_K|
 * HCURL, HCURL2 elem_d[K][nsym] = rho_K |det J_K| J_K^-1 J_K^-T (symmetric pairs)
 * HDIV, HDIV2   elem_d[K][nsym] = rho_K J_K^T J_K / |det J_K|
 * J_K has columns v_i - v_0.  rho_d may be NULL (rho = 1).  Asynchronous. */
int bras_geometry(int family, int dim, int64_t nvert, const double* coords_d,
                  int64_t ncell, const int32_t* cells_d, const double* rho_d,
                  double* elem_d, void* stream);

/* ======================================================================== *
 * Core: setup and the operators of the hot path.
 * ======================================================================== */

/* Build a handle for the conforming space with n DOFs, E elements of n_loc
 * local DOFs, map l2g_d [E][n_loc] (device, int32), and element data in one
 * of the BRAS_ELEM_* forms (nsym is used by METRIC_REF only).  n_loc <= 120;
 * the element passes exist for the n_loc of the supported families (3..36
 * per lane, 42..105 per element on the matrix cores), EINVAL at the first
 * apply otherwise.
 * Validates the map: entries in [0, n), distinct within an element, and every
 * DOF has d_i >= 1 (P has full column rank, Section 2.2) - else EINVAL.
 * Computes d, the transpose map, diag(M), and every element's exact inverse
 * M_K^-1 in float64 (Cholesky; ENOTSPD names the first failing element),
 * folds D^-1 on both sides and stores it in apply_prec.  BRAS_BF16 requires
 * METRIC_REF or EXPLICIT and stores the Gram factor G_K = L_K^-1 D_K^-1
 * (M_K = L_K L_K^T) so that D_K^-1 M_K^-1 D_K^-1 = G_K^T G_K.
 * max_rhs (1..256) bounds nrhs in later calls and sizes the workspace; one
 * [n][max_rhs] float64 block must stay below 4 GiB (EINVAL otherwise).
 * Every input is copied; the caller may free its buffers when the call
 * returns.  Synchronous. */
int bras_setup(bras_handle* h, int64_t n, int64_t E, int n_loc, const int32_t* l2g_d,
               int form, const double* ref_d, const double* elem_d, int nsym,
               int apply_prec, int max_rhs, void* stream);

/* Replace the element coefficients (same form and sizes as at setup) and
 * recompute the element inverses and diag(M); maps are kept.  Synchronous. */
int bras_update(bras_handle h, const double* elem_d, void* stream);

/* Release every resource of the handle.  NULL is accepted. */
int bras_destroy(bras_handle h);

/* y = M_bras^-1 x = D^-1 P^T M_br^-1 P D^-1 x (eq. mhatinvbras_def).
 * x_d, y_d: [n] or [n][nrhs] float64, distinct buffers, 1 <= nrhs <= max_rhs.
 * Deterministic (no floating-point atomics); asynchronous on stream; no
 * allocation. */
int bras_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream);

/* bras_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and result (bit for bit) as bras_apply; the broken-vector
 * workspace is a fixed device array of BRAS_NOALLOC_SCRATCH_BYTES per device
 * (taken when the first handle is set up on that device and held until the
 * process ends) instead of the handle's own buffer, and the call makes no
 * allocation of any kind.  EINVAL when the workspace of the call (8 bytes per
 * broken DOF and column for float64 inverses or the scaled H1 form, 4 for
 * float32 / bfloat16 ones) exceeds that size, or when the handle's device is
 * not the current one.  All calls on one device share the array: calls that
 * overlap in time on one device (unordered streams) race and must not be
 * issued; calls ordered on one stream are safe.  Asynchronous on stream. */
#define BRAS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int bras_apply_noalloc(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream);

/* y = M x = sum_K P_K^T M_K P_K x (eq. M_PMbrP), float64 throughout.
 * Same argument rules as bras_apply. */
int mass_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream);

/* y = diag(M)^-1 x (Section 2.1).  Same argument rules as bras_apply. */
int jacobi_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream);

/* Preconditioned CG on M x = b (Section 3), independently per column.
 * pc: BRAS_PC_NONE / JACOBI / BRAS.  x_d holds the initial guess on entry and
 * the solution on exit.  Column c stops when ||r_k||_2 / ||r_0||_2 <= rtol
 * (r_k the recursive residual, r_0 = b - M x_0) or after maxit products M p.
 * With BF16 inverses the iteration uses the flexible beta
 * r_new.(z_new - z_old) / rho_old (FP32 inverses too when BRAS_OPT_FLEXIBLE
 * is 1; the default for FP32 is the standard beta).  At exit the true residual b - M x is recomputed; while it exceeds
 * rtol ||r_0|| in a column, the iteration restarts from x (iterative
 * refinement, at most BRAS_OPT_MAX_RESTART times, default 8; the products
 * of every restart count in iters_h).
 * iters_h[nrhs]: products M p per column; relres_h[nrhs]: final true
 * ||b - M x|| / ||r_0|| (host, may be NULL).  Blocking.  Returns ENOCONV if a
 * column did not reach rtol within maxit products, or if its final true
 * residual is still above rtol after the restarts, and EBREAKDOWN on
 * breakdown; x_d, iters_h and relres_h are written in every case.
 * Small problems (SCALED_REF form with n_loc of degree 1-4 H1 elements,
 * FP64, nrhs = 1, n <= 2048, 16 n + 10 n_br <= 160000, at most 1024 times
 * 2 elements (3 for n_loc 4, 1 for n_loc 20 and 35), maxit <= 100000) run
 * the whole iteration in one work-group kernel with its vectors in LDS and
 * registers, unless BRAS_OPT_SMALL_CG is 0; the operators, iteration,
 * stopping test and outputs are the same, dot products are summed in
 * another fixed order, and there is no restart (a final true residual above
 * rtol returns ENOCONV).  BRAS_INFO_SOLVE_PATH reports which path the last
 * call took. */
int pcg_solve(bras_handle h, int pc, const double* b_d, double* x_d, int nrhs,
              double rtol, int maxit, int* iters_h, double* relres_h, void* stream);

/* Density gradient for M(rho) = sum_K rho_K c_K P_K^T Mhat P_K (H1,
 * SCALED_REF): g_d[K] = -dcoef_d[K] * sum_c lam_K,c^T Mhat x_K,c, i.e.
 * dL/drho_K = -lambda_K^T (dM_K/drho_K) x_K with dcoef_d[K] = c_K = |det J_K|
 * (the adjoint identity of a linear solve).  x_d, lam_d: [n] or [n][nrhs];
 * g_d: [E].  Asynchronous. */
int bras_rho_grad(bras_handle h, const double* x_d, const double* lam_d,
                  const double* dcoef_d, double* g_d, int nrhs, void* stream);

/* ======================================================================== *
 * Introspection and options.
 * ======================================================================== */

#define BRAS_INFO_N        0   /* conforming DOFs                              */
#define BRAS_INFO_E        1   /* elements                                     */
#define BRAS_INFO_NLOC     2
#define BRAS_INFO_NBR      3   /* broken DOFs = E * n_loc                       */
#define BRAS_INFO_PREC     4
#define BRAS_INFO_FORM     5
#define BRAS_INFO_MAXRHS   6
#define BRAS_INFO_RESTARTS 7   /* refinement restarts in the last pcg_solve     */
#define BRAS_INFO_VARIANT  8   /* element-pass scheduling variant (-1: built-in) */
#define BRAS_INFO_SOLVE_PATH 9 /* last pcg_solve / fixed_point_solve /
                                  chebyshev_solve: 0 multi-pass, 1 one work-group */
#define BRAS_INFO_PATCHES  10  /* patches of the one-column operator passes
                                  (0: element / reduce form only)             */
#define BRAS_INFO_PATCH_ON 11  /* 1 when one-column passes run in patch form
                                  (a plan exists and BRAS_OPT_PATCH is 1)     */
int bras_info(bras_handle h, int what, int64_t* value_h);

/* Copy derived setup data to device buffers for inspection:
 * BRAS_EXPORT_MULT   int32 [n]   multiplicities d_i
 * BRAS_EXPORT_ROWPTR int32 [n+1] transpose-map row pointers
 * BRAS_EXPORT_SLOT   int64 [n_br] broken slots K*n_loc + l per row, ascending
 * BRAS_EXPORT_DIAG   float64 [n] diag(M) */
#define BRAS_EXPORT_MULT   0
#define BRAS_EXPORT_ROWPTR 1
#define BRAS_EXPORT_SLOT   2
#define BRAS_EXPORT_DIAG   3
int bras_export(bras_handle h, int what, void* dst_d, void* stream);

/* ---- assembled operators (eq. mass_and_bras_element_sums: M_bras^-1 has the
 * sparsity of M) ------------------------------------------------------------
 * CSR on the device: rowptr int64 [n+1], col int32 [nnz] ascending within each
 * row, val float64 [nnz].  Row i holds every DOF of every element containing
 * DOF i; entry (i, j) sums over the copies (K, l) of i in transpose-map order
 * (K*n_loc + l ascending) the element entries M_K[l][m] (BRAS_OP_MASS) or
 * d_i^-1 (M_K^-1)[l][m] d_j^-1 (BRAS_OP_BRAS, from the stored FP64 / FP32
 * inverses) with pi(K, m) = j.  Buffers are caller allocated. */
#define BRAS_OP_MASS 0
#define BRAS_OP_BRAS 1
#define BRAS_OP_JACOBI 2   /* diag(M)^-1: see bras_csr_jacobi (its own pattern) */
/* Row pointers and nnz of the pattern (the same for both operators).  EINVAL
 * when a row has more than 2048 candidate columns (max d_i * n_loc) or nnz
 * reaches 2^31.  Synchronises the stream. */
int bras_csr_rowptr(bras_handle h, int64_t* rowptr_d, int64_t* nnz_h, void* stream);
/* Columns and values for rowptr_d from bras_csr_rowptr.  EINVAL for a handle
 * storing BF16 Gram factors.  Asynchronous on the stream. */
int bras_csr_assemble(bras_handle h, int op, const int64_t* rowptr_d, int32_t* col_d, double* val_d, void* stream);
/* y = A x for a CSR matrix on the device (one column, float64): each row's
 * sum is taken in a fixed order (16 strided partial sums, then a butterfly).
 * x and y must not overlap. */
int bras_csr_apply(int64_t n, const int64_t* rowptr_d, const int32_t* col_d, const double* val_d,
                   const double* x_d, double* y_d, void* stream);
/* diag(M)^-1 (Section 2.1, the diagonal mass-inverse approximation BRAS is
 * compared with) as CSR: rowptr_d [n+1] = 0..n, col_d [n] = 0..n-1, val_d [n]
 * = 1 / M_ii.  Asynchronous on the stream. */
int bras_csr_jacobi(bras_handle h, int64_t* rowptr_d, int32_t* col_d, double* val_d, void* stream);

/* ---- sparse products for Schur-complement approximations (Section 4:
 * -St = C + G Mt^-1 G^T, eq. approx_positive_schur_general, sparse when Mt^-1
 * is the assembled M_bras^-1; formed as (G M_bras^-1) G^T, then + C, with
 * these calls) -------------------------------------------------------------
 * CSR on the device as above: int64 row pointers (non-decreasing, from 0 to
 * nnz), int32 columns ascending and distinct within each row, float64
 * values.  Output buffers are caller allocated; each call allocates
 * temporary device buffers of its own; sizes below 2^31.
 * C = A B for A (m x k) and B (k x n).  bras_spgemm_rowptr writes C's row
 * pointers c_rowptr_d [m+1] and nnz(C) (synchronises the stream);
 * bras_spgemm_fill writes C's columns (ascending) and values, each entry the
 * sum of its products a_ip b_pj taken in the order of A's columns: the same
 * result for every launch shape.  A row's candidate products are the sum
 * over its entries of the selected B row lengths; rows with at most 1024 of
 * them and at most 1024 entries are formed in LDS, longer rows through a
 * sort in device memory, in batches of at most 2^27 candidates (8 bytes
 * each for the row pointers, 24 for the fill; a row longer than a batch
 * forms one alone, below 2^31 candidates).  Both routes give the same sums.
 * Environment: BRAS_SPGEMM_BATCH (a positive integer) sets another batch
 * size; BRAS_SPGEMM_LDS_MAX (0 .. 2048) another limit for the LDS route.  EINVAL when
 * a row of A has a column outside [0, k), malformed row pointers, a row of
 * 2^31 or more candidates, nnz(C) >= 2^31, or (fill) row pointers that do
 * not match the counts.  Synchronous. */
int bras_spgemm_rowptr(int64_t m, int64_t k, const int64_t* a_rowptr_d, const int32_t* a_col_d,
                       const int64_t* b_rowptr_d, const int32_t* b_col_d, int64_t* c_rowptr_d, int64_t* nnz_h,
                       void* stream);
int bras_spgemm_fill(int64_t m, int64_t k, const int64_t* a_rowptr_d, const int32_t* a_col_d, const double* a_val_d,
                     const int64_t* b_rowptr_d, const int32_t* b_col_d, const double* b_val_d,
                     const int64_t* c_rowptr_d, int32_t* c_col_d, double* c_val_d, void* stream);
/* A^T (n x m) of A (m x n): row j of A^T lists the rows of A holding column
 * j, ascending, with their values (a stable sort by column; exact).  EINVAL
 * for malformed row pointers or a column outside [0, n).  Synchronous. */
int bras_csr_transpose(int64_t m, int64_t n, const int64_t* rowptr_d, const int32_t* col_d, const double* val_d,
                       int64_t* rowptr_t_d, int32_t* col_t_d, double* val_t_d, void* stream);
/* C = A + B for A, B (m x n), e.g. the C term of eq.
 * approx_positive_schur_general: rows merged by column; an entry present in
 * both is a + b.  bras_csr_add_rowptr writes C's row pointers and nnz(C);
 * bras_csr_add_fill its columns and values.  EINVAL for malformed row
 * pointers, nnz(C) >= 2^31, or (fill) row pointers that do not match the
 * counts.  Synchronous. */
int bras_csr_add_rowptr(int64_t m, const int64_t* a_rowptr_d, const int32_t* a_col_d, const int64_t* b_rowptr_d,
                        const int32_t* b_col_d, int64_t* c_rowptr_d, int64_t* nnz_h, void* stream);
int bras_csr_add_fill(int64_t m, const int64_t* a_rowptr_d, const int32_t* a_col_d, const double* a_val_d,
                      const int64_t* b_rowptr_d, const int32_t* b_col_d, const double* b_val_d,
                      const int64_t* c_rowptr_d, int32_t* c_col_d, double* c_val_d, void* stream);

#define BRAS_OPT_GRAPH_ITERS 0  /* most CG (or stationary) iterations launched
                                   between two host checks of the convergence
                                   flags, 1..32 (default 32); the launcher
                                   predicts the count from the observed rate
                                   and never exceeds this cap              */
#define BRAS_OPT_MAX_RESTART 1  /* refinement restarts allowed (>= 0)         */
#define BRAS_OPT_VARIANT     2  /* force a scheduling variant (-1 = built-in)  */
#define BRAS_OPT_SMALL_CG    3  /* 1 (default): single work-group pcg_solve,
                                   fixed_point_solve and chebyshev_solve for
                                   small problems; 0: always multi-pass      */
#define BRAS_OPT_PATCH       4  /* 1 (default): one-column BRAS / mass passes
                                   in patch form when the handle has patches
                                   (BRAS_INFO_PATCHES > 0); 0: element pass
                                   plus transpose-map reduce               */
#define BRAS_OPT_FLEXIBLE    5  /* BRAS-PCG beta with reduced-precision
                                   inverses: -1 (default) flexible for BF16,
                                   standard for FP32; 0 standard; 1 flexible
                                   for FP32 and BF16 (FP64: always standard) */
int bras_set_option(bras_handle h, int opt, double value);

/* ======================================================================== *
 * Stationary iterations with the same operators (Section 3).
 * ======================================================================== */

/* Power-iteration estimate of lambda_max(C M), C = BRAS (pc = BRAS_PC_BRAS)
 * or diag(M)^-1 (BRAS_PC_JACOBI), used for the fixed-point weights of
 * Section 3 (omega_diag = 1/lambda_max, omega_bras = 2/(1 + lambda_max)):
 * v_0 = v0/||v0||; for k = 1..iters: q = M v, w = C q, lambda = q.w / q.v,
 * v = w/||w||.  v0_d: [n] float64 (device, not modified).  The estimate is a
 * Rayleigh quotient of the M-self-adjoint C M, so it never exceeds
 * lambda_max.  EINVAL for a zero start vector, EBREAKDOWN on non-positive
 * products.  Synchronous. */
int bras_lambda_max(bras_handle h, int pc, const double* v0_d, int iters, double* lambda_h, void* stream);

/* Damped fixed-point iteration u_{k+1} = u_k + omega C (f - M u_k)
 * (Section 3) from u_0 = x_d, for every column independently; stops when
 * ||f - M u_k||_2 <= rtol ||f - M u_0||_2 (iters_h = k, the number of
 * updates) or after maxit updates (ENOCONV).  pc: BRAS_PC_JACOBI or
 * BRAS_PC_BRAS.  Arguments and results as pcg_solve, including the single
 * work-group path for small problems.  Synchronous. */
int fixed_point_solve(bras_handle h, int pc, double omega, const double* b_d, double* x_d, int nrhs,
                      double rtol, int maxit, int* iters_h, double* relres_h, void* stream);

/* Chebyshev semi-iteration for C M on the interval [lmin, lmax] (Section 3
 * recommends Chebyshev with the BRAS spectral interval, lmin = 1 by Cor.
 * bras_lambda_min): d_0 = C r_0 / theta; rho_0 = 1/sigma; rho_k = 1/(2 sigma -
 * rho_{k-1}); d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k/delta) C r_k;
 * u_{k+1} = u_k + d_k, with theta = (lmax + lmin)/2, delta = (lmax - lmin)/2,
 * sigma = theta/delta and r_k = f - M u_k.  No dot products besides the
 * stopping test.  Stopping, arguments and results as fixed_point_solve. */
int chebyshev_solve(bras_handle h, int pc, double lmin, double lmax, const double* b_d, double* x_d, int nrhs,
                    double rtol, int maxit, int* iters_h, double* relres_h, void* stream);

/* Time the candidate forms of this handle's operator passes on one mass +
 * one BRAS apply at nrhs columns on stream, and keep the fastest.  Candidates:
 * the element-pass scheduling variants (3D H(curl) / H(div) metric-form mass
 * passes with n_loc <= 36: row order in batches of 2 or 4 table entries,
 * diagonal order in batches of 8; scaled H1: the FP64 matrix-core product or
 * the per-row FMA product; every other handle has one) and, for nrhs = 1 on a
 * handle with patches, the patch form.  All candidates compute the same
 * operator (summation orders differ).  Read the choice back with
 * BRAS_INFO_VARIANT and BRAS_INFO_PATCH_ON; BRAS_OPT_VARIANT and
 * BRAS_OPT_PATCH override it.  Allocates two [n][nrhs] scratch vectors for
 * the duration of the call.  Synchronous. */
int bras_autotune(bras_handle h, int nrhs, void* stream);

/* Microbenchmark, not an operator pass: the two element-local Gram products
 * of the BF16 BRAS apply (U = Gtil W, Z = Gtil^T bf16(U) for 32 columns, the
 * multi-right-hand-side form of eq. mhatinvbras_def) on tiles that stay in
 * LDS, so that no HBM traffic limits them.  Launches `blocks` work-groups of
 * `iters` rounds each on stream (asynchronous); each thread writes a checksum
 * to out_d[blocks * 256] (float32, device, caller-owned).  *flops_h receives
 * the issued matrix-core FLOPs of the launch (zero-padded tiles included).
 * n_loc: 20, 36, 70 or 84 (BRAS_EINVAL otherwise).  blocks = 0 launches
 * nothing and reports the FLOPs of one round of one work-group (one element,
 * 32 columns). */
int bras_bench_bf16_local_gemm(int n_loc, int iters, int blocks, float* out_d, long long* flops_h, void* stream);

const char* bras_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BRAS_H */
