/*
 * wqfd — weighted-quadrature row assembly for cut tensor-product B-spline meshes (gfx950).
 *
 * C ABI of libwqfd.so.  Method: Marussig, "Fast formation and assembly for spline-based
 * 3D fictitious domain methods".  Mass and stiffness matrices of a degree-p, C^{p-1},
 * open-uniform-knot tensor B-spline background mesh (identity map, Section 2) cut by a
 * level-set domain, assembled row by row (one row per test function, Section 1) with
 * sum factorization and weighted quadrature (WQ, Section 1 and Section 2.2 step 1);
 * the regular part of each cut test function's support uses discontinuous weighted
 * quadrature (DWQ, Section 2.2 steps 2-6 and Eq. (1)); the rest of its support is
 * integrated element by element with Gauss rules on interior elements and octree
 * sub-cells on cut elements.
 *
 * Conventions shared by every entry point
 *  - Return value: WQ_OK (0) or a negative wq_status; a human-readable message for the
 *    last failure on the calling thread is returned by wq_last_error().
 *  - Argument errors (null pointers where data is required, dtype/which mismatch) are
 *    detected before any device work is enqueued; nothing is written in that case.
 *  - Device pointers (kappa, vals_*, G_*, dkappa) are caller-owned, contiguous, and must
 *    hold the documented number of elements of the value type (double for WQ_F64,
 *    float for WQ_F32 and WQ_BF16X3).  The library never frees caller memory.
 *  - Every call except wq_build_rules is asynchronous on the given HIP stream
 *    (hipStream_t passed as void*; NULL = the default stream).  A rules handle is
 *    immutable after wq_build_rules, so calls on different streams may share it.
 *  - Value dtypes: kappa, the matrix values, the cotangents and dkappa all use the
 *    selected dtype.  WQ rules, classification and octree geometry are always FP64;
 *    the FP32 path rounds each FP64 table entry once and accumulates in FP32.
 */
#ifndef WQFD_H
#define WQFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WQ_OK = 0,
    WQ_EINVAL = -1,       /* invalid argument (message says which) */
    WQ_ENOMEM = -2,       /* device allocation failed */
    WQ_EHIP = -3,         /* HIP runtime error (message has the HIP error string) */
    WQ_ESINGULAR = -4,    /* a WQ exactness system was rank deficient */
    WQ_EUNSUPPORTED = -5  /* valid request outside the library's limits (e.g. p > 6) */
} wq_status;

/* WQ_BF16X3 (an experiment, forward assembly only): values and kappa are float as for
 * WQ_F32; in wq_assemble_rows the direction-1 contraction of the interior rows runs on
 * the matrix cores with each FP32 operand split into two bf16 parts, x = hi + lo, and
 * products taken as hi*hi + hi*lo + lo*hi accumulated in FP32 (about 2^-16 relative per
 * product); every other step of wq_assemble_rows and cut_assemble runs as WQ_F32.
 * wq_assemble_adjoint and gauss_assemble return WQ_EUNSUPPORTED for it. */
typedef enum { WQ_F64 = 0, WQ_F32 = 1, WQ_BF16X3 = 2 } wq_dtype;

enum { WQ_MASS = 1u, WQ_STIFF = 2u };   /* 'which' bit mask */

/* Optional part bits of cut_assemble's 'which': run only the element Gauss remainder
 * and/or only the octree part (neither bit set: both).  Each part accumulates on its
 * own, so the two calls in sequence equal one call with both parts. */
enum { WQ_CUT_REMAINDER = 4u, WQ_CUT_OCTREE = 8u };

/* Background mesh: nel[d] uniform elements on [lo[d], hi[d]], degree 1 <= p <= 6, open
 * knot vectors with maximal smoothness C^{p-1} (Section 1, Section 2). */
typedef struct {
    int32_t nel[3];
    int32_t degree;
    double lo[3], hi[3];
} wq_mesh;

/* Domain Omega = {phi < 0} (Section 2.1: Omega^v, interface Gamma).
 * kind 0: no cut.  1: plane phi = (n.x - r0)/|n|.  2: ball phi = |x - c| - r0.
 * 3: torus around the axis through c parallel to z, major radius r0, minor r1. */
typedef struct {
    int32_t kind;
    double c[3], n[3], r0, r1;
} wq_levelset;

typedef struct {
    int32_t octree_levels;   /* depth of the cut-element octree, 0..5 (default 3) */
    int32_t flags;           /* 0 or WQ_OPT_HYBRID_GAUSS | WQ_OPT_GAUSS_ROWS | WQ_OPT_MOMENT_FIT | WQ_OPT_TENSOR */
} wq_options;

/* Option flag: the "Hybrid Gauss" scheme of Section 3.1 (list of compared schemes) instead of
 * DWQ.  Interior rows keep weighted quadrature; no cut row gets a DWQ box, so the whole
 * regular support of every cut row (its interior elements) is integrated by element Gauss
 * rules with sum factorization in cut_assemble.  Slots and pattern are unchanged.
 * Option flag WQ_OPT_GAUSS_ROWS (comparison, not in the paper): no weighted quadrature at all;
 * every active row is handled like a cut row without a box, i.e. wq_assemble_rows zeroes it
 * and cut_assemble integrates every interior element of its support by element Gauss rules
 * with sum factorization and its cut elements by the octree.  The result is the conventional
 * Gauss assembly (gauss_assemble), formed row by row without atomics, so that the gain of
 * weighted quadrature can be measured on the same row-owned engineering.  The slot layout
 * then holds a Gauss block for every interior element; n_rows_interior is 0. */
enum { WQ_OPT_HYBRID_GAUSS = 1, WQ_OPT_GAUSS_ROWS = 2, WQ_OPT_MOMENT_FIT = 4, WQ_OPT_TENSOR = 8 };

/* Option flag WQ_OPT_MOMENT_FIT (cheaper cut integration; the paper's cut-element scheme is
 * higher order but costly, Section 3.2): every cut element's octree rule is replaced by a rule on
 * the NK^3 = (2p+1)^3 tensor Gauss-Legendre points of the element whose weights reproduce the
 * octree rule on every polynomial of degree <= 2p in each variable (fitted at build time from
 * the octree's moments).  With kappa = 1 the matrices are the octree rule's; kappa is then needed
 * at NK^3 points per cut element instead of (p+1)^3 per octree leaf.  The octree slots of the
 * layout become these points (n_octree = n_cut_elems * NK^3, lexicographic per cut element) and
 * octree_w their weights (which may be negative).  Octree depth <= 3 only. */

/* Option flag WQ_OPT_TENSOR (Section 2 takes the identity as the geometry map and notes that
 * this loses no generality; under a map F the Laplacian stiffness has the full symmetric
 * coefficient tensor C = |det DF| DF^-1 DF^-T): the rule build adds the mixed 1D rule
 * families (1, 0) (test derivative, trial value) and (0, 1) (test value, trial derivative),
 * standard and one-sided, that wq_assemble_tensor needs.  Degrees 1..4 only. */

typedef struct wq_rules wq_rules;   /* opaque; owns its device buffers */

/* Read-only views of a rules handle (device pointers owned by the handle, valid until
 * wq_rules_free). */
typedef struct {
    int64_t n_active;        /* matrix dimension: active (non-exterior) functions */
    int64_t nnz;             /* entries per matrix */
    int64_t n_rows_interior; /* interior test functions (all support in Omega) */
    int64_t n_rows_cut;      /* cut test functions */
    int64_t n_rows_split;    /* cut functions that have a DWQ box */
    int64_t n_dwq_rules;     /* distinct one-sided 1D DWQ rules */
    int64_t n_kappa;         /* kappa slots = n_grid + n_block + n_octree */
    int64_t n_grid;          /* WQ tensor grid X1 x X2 x X3, lexicographic */
    int64_t n_block;         /* element Gauss blocks, (p+1)^3 per block element */
    int64_t n_octree;        /* octree points, (p+1)^3 per octree leaf (fitted rule: (2p+1)^3 per cut element) */
    int64_t n_block_elems;   /* elements carrying a Gauss block */
    int64_t n_cut_elems;     /* cut elements */
    int64_t n_cells;         /* octree leaves */
    int64_t n_line_blocks;   /* interior row blocks of the fast kernel */
    int64_t n_oct_xgroups;   /* octree leaves grouped by (cut element, depth, x offset) */
    int64_t n_oct_columns;   /* octree leaves grouped by (cut element, depth, x and y offsets) */
    int64_t n_rem_pairs;     /* (cut row, element Gauss remainder element) pairs */
    int64_t n_gauss_elems;   /* interior elements (inputs of gauss_assemble) */
    int32_t grid_dims[3];    /* |X_d| */
    int32_t nfun[3];         /* functions per direction, nel[d] + p */
    const int64_t* row_ptr;        /* (n_active+1) CSR row pointer */
    const int32_t* col_idx;        /* (nnz) active column indices, ascending per row */
    const int32_t* active_to_lex;  /* (n_active) lexicographic function index, first index slowest */
    const double* kappa_xyz;       /* (n_kappa, 3) slot coordinates */
    const double* octree_w;        /* (n_octree) octree weights (0 outside Omega; fitted weights under WQ_OPT_MOMENT_FIT) */
    const int32_t* block_elems;    /* (n_block_elems) lexicographic element index per block */
    const int8_t* fun_class;       /* (nfun product) 0 exterior, 1 interior, 2 cut */
    const int8_t* elem_class;      /* (nel product) 0 exterior, 1 interior, 2 cut */
    const int32_t* split;          /* (n_rows_cut, 4) d, s, high, rule (-1: no box) per cut row */
    const int32_t* cut_rows;       /* (n_rows_cut) active index of each cut row */
} wq_rules_info;

/* Builds everything that does not depend on kappa (Section 2.2 steps 1-6, Section 2.1):
 * Gauss rules, the WQ point layout (two Gauss points per inner element, all p+1 in the
 * boundary elements), 1D WQ rules for mass (00) and stiffness (11) by FP64 min-norm
 * solves, element/function classification, the CSR pattern (row I holds every active J
 * with max_d |I_d - J_d| <= p), DWQ splits and one-sided rules, element Gauss blocks,
 * octree cells and the kappa slot layout.  Synchronous: returns once the handle is ready.
 * opts may be NULL (octree_levels = 3).  On success *out receives a new handle. */
int wq_build_rules(const wq_mesh* mesh, const wq_levelset* ls, const wq_options* opts,
                   void* stream, wq_rules** out);

int wq_rules_info_get(const wq_rules* rules, wq_rules_info* out);

/* Row assembly (Section 1: sum factorization + weighted quadrature + row loop; Section
 * 2.2 DWQ for cut rows).  For every interior row writes the full WQ row; for every cut
 * row with a DWQ box writes the box part; every other cut row is set to zero.  All nnz
 * entries of each requested matrix are OVERWRITTEN.
 * kappa: (n_kappa) values at the slots.  vals_mass / vals_stiff: (nnz) outputs; each may
 * be NULL iff its bit is absent from which. */
int wq_assemble_rows(const wq_rules* rules, int dtype, uint32_t which, const void* kappa,
                     void* vals_mass, void* vals_stiff, void* stream);

/* Cut part of Eq. (1): element Gauss on the interior elements of each cut row's support
 * outside its DWQ box, and octree Gauss on every cut element.  ACCUMULATES into the
 * values (call after wq_assemble_rows on the same stream).  'which' may add the part bits
 * WQ_CUT_REMAINDER / WQ_CUT_OCTREE to run one part only. */
int cut_assemble(const wq_rules* rules, int dtype, uint32_t which, const void* kappa,
                 void* vals_mass, void* vals_stiff, void* stream);

/* Rows and the whole cut part in one call (Section 1 row loop, Section 2.2 DWQ rows, Eq. (1)
 * cut part): the same values as wq_assemble_rows followed by cut_assemble on the same stream,
 * bitwise (every row is summed in the same order), with the work spread over three streams:
 * the interior rows on the caller's stream, the cut rows and then the element Gauss remainder
 * on the handle's second stream, the cut elements' moments and local rows on a third; the
 * gather of the local rows follows on the caller's stream once all three are done.  All nnz
 * entries of each requested matrix are OVERWRITTEN.  dtype WQ_F64 or WQ_F32.  Uses the
 * stream-ordered scratch of cut_assemble.  Without the moment form (octree depth > 3), cut
 * elements or the extra streams it runs the two calls in turn.  Asynchronous on stream. */
int wq_assemble(const wq_rules* rules, int dtype, uint32_t which, const void* kappa,
                void* vals_mass, void* vals_stiff, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cut_assemble with the same arguments,
 * results and error behaviour, whose scratch (the moments and local rows of the cut
 * elements) lives in a fixed 64 MiB device array inside the library instead of a
 * stream-ordered pool.  The cut elements are processed in batches that fit the array; a
 * case where one cut element alone needs more returns WQ_EINVAL.  No hipMalloc, hipFree or
 * allocating library routine is called.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (different streams or host threads)
 * race and give wrong results; calls ordered on one stream are safe.  The array is held
 * on every device the library runs on until the process ends. */
int cut_assemble_noalloc(const wq_rules* rules, int dtype, uint32_t which, const void* kappa,
                         void* vals_mass, void* vals_stiff, void* stream);

/* Adjoint of rows + cut parts: for L = sum_IJ (G_mass_IJ M_IJ + G_stiff_IJ K_IJ),
 * dkappa[slot] = dL/dkappa(slot), summed over every use of the slot.  dkappa (n_kappa) is
 * OVERWRITTEN.  G_mass / G_stiff: (nnz) cotangents on the pattern; each may be NULL iff
 * its bit is absent from which. */
int wq_assemble_adjoint(const wq_rules* rules, int dtype, uint32_t which, const void* G_mass,
                        const void* G_stiff, void* dkappa, void* stream);

/* Stiffness matrix with a full symmetric coefficient tensor (Section 2, opening paragraph:
 * the identity geometry map lifted; Eq. (1) for the cut rows):
 *   K_IJ = int_Omega grad B_I . C grad B_J = sum_{d,e} int C_de d_d B_I d_e B_J.
 * Interior rows and the DWQ box of cut rows by weighted quadrature with sum factorization,
 * term (d, e) using the family (1, 0) in direction d, (0, 1) in direction e, (1, 1) when d = e
 * and (0, 0) elsewhere; the element Gauss remainder and the cut elements (octree, or the
 * fitted rule under WQ_OPT_MOMENT_FIT) of cut rows by element quadrature, row by row.
 * C: device array (6, n_kappa), row-major: the components C11, C22, C33, C12, C13, C23 at
 * every slot.  vals_stiff: (nnz) device output, OVERWRITTEN; the mass matrix of a map only
 * changes its scalar coefficient and comes from wq_assemble_rows / cut_assemble.  Needs rules
 * built with WQ_OPT_TENSOR (WQ_EINVAL otherwise); dtype WQ_F64 or WQ_F32.  Sums run in a
 * fixed order (no atomics).  Asynchronous on stream. */
int wq_assemble_tensor(const wq_rules* rules, int dtype, const void* C, void* vals_stiff, void* stream);

/* Conventional assembly for comparison (Section 3.1, "Standard Gauss"): element by element,
 * (p+1)^3 Gauss points on every interior element and the octree points on every cut element,
 * local matrices added into the same pattern.  OVERWRITES all nnz entries of each requested
 * matrix.  kappa_gauss: (n_gauss_elems * (p+1)^3) values at the points wq_gauss_coords lists;
 * kappa: the slot vector of the other calls (its octree slots are read).  Octree depth <= 3
 * only (WQ_EUNSUPPORTED otherwise).  Uses atomics: summation order varies. */
int gauss_assemble(const wq_rules* rules, int dtype, uint32_t which, const void* kappa_gauss, const void* kappa,
                   void* vals_mass, void* vals_stiff, void* stream);

/* Coordinates of the Gauss points of every interior element, (n_gauss_elems * (p+1)^3, 3)
 * doubles written to the caller's device buffer xyz: elements in lexicographic order, points
 * in lexicographic Gauss order (first direction slowest). */
int wq_gauss_coords(const wq_rules* rules, double* xyz, void* stream);

/* ---------------------------------------------------------------------------------------
 * L2 projection with extended B-splines (Section 3.1 test setting: mass matrix, projection
 * of a target function f, extended B-splines for a well-conditioned system; Section 3.2:
 * relative L2 error).  FP64 only.  The paper refers to other works for the extension; the
 * library reads it as follows.  Inner functions: active functions with an interior element in
 * their support; the others are outer.  The root element l of an outer function j is the
 * interior element whose centre is nearest to the centre of supp B_j (|l + p/2 - j| in
 * element units, Euclidean; the lexicographically first l on ties); its array is the block
 * l + {0..p}^3 of inner functions.  j enters the basis through its array with the
 * coefficients e_ij = lambda_j(P_i), P_i the polynomial piece of B_i on l and lambda_j the
 * dual functional of B_j (a product over the directions; on uniform knots the Lagrange
 * extrapolation weights in the index).  E (n_active x n_inner) maps the coefficients of the
 * extended basis to those of the active functions; the projection solves E^T M E c = E^T b
 * and returns u = E c.
 * --------------------------------------------------------------------------------------- */
typedef struct wq_extension wq_extension;   /* opaque; owns its device buffers */

/* Read-only views of an extension (device pointers owned by it, valid until
 * wq_extension_free). */
typedef struct {
    int64_t n_inner;               /* inner functions (columns of E) */
    int64_t n_outer;               /* outer functions */
    int64_t nnz_e;                 /* entries of E */
    const int32_t* inner_of_active;  /* (n_active) inner index of each active function, -1 if outer */
    const int32_t* outer_rows;       /* (n_outer) active index of each outer function, ascending */
    const int32_t* outer_base;       /* (n_outer, 3) base l of its array */
    const int64_t* e_ptr;            /* (n_active+1) CSR row pointer of E */
    const int32_t* e_col;            /* (nnz_e) inner indices, ascending per row */
    const double* e_val;             /* (nnz_e) values */
} wq_extension_info;

/* Load vector of the projection: b_I = sum over the quadrature points x_q of row I (the WQ or
 * DWQ box points, the element Gauss remainder, the octree points of cut elements) of the mass
 * row's test weight W_I(q) times f(x_q).  Computed as the row sums of the mass matrix
 * assembled with kappa = f, which is the same sum: the active functions of a row add up to one
 * at each of its points.  f: (n_kappa) values at the slots (device); b: (n_active) output,
 * OVERWRITTEN (device).  Uses nnz doubles of stream-ordered scratch.  Asynchronous. */
int wq_load_vector(const wq_rules* rules, const double* f, double* b, void* stream);

/* Builds the extension operator of a rules handle.  Synchronous.  Returns WQ_EINVAL when an
 * outer function exists but no (p+1)^3 block of inner functions does (mesh too coarse). */
int wq_extension_build(const wq_rules* rules, void* stream, wq_extension** out);
int wq_extension_info_get(const wq_extension* ext, wq_extension_info* out);
void wq_extension_free(wq_extension* ext);

/* u = E c with E^T M E c = E^T b by preconditioned conjugate gradients from c = 0, stopping
 * when ||r|| <= tol ||E^T b|| (checked every 8 iterations) or after max_iter iterations.  The
 * preconditioner is S R K^{-1} R^T S: K = K1 x K2 x K3 the mass matrix of all functions of the
 * background mesh (banded Cholesky factors of the 1D masses, built with the extension), R^T
 * the zero extension from the inner functions, S = diag(sqrt(diag(K)_i / diag(E^T M E)_i)).  vals_mass: (nnz) mass values (FP64, kappa = 1 for
 * the paper's projection), b: (n_active), u: (n_active) output; all device.  *iters and
 * *relres (host, may be NULL) receive the iteration count and the final relative residual.
 * ext must come from the same rules handle.  Synchronous (the host reads the residual);
 * WQ_ESINGULAR on a non-positive diagonal entry or a breakdown.  Reductions use a fixed
 * order: the result is the same on every run. */
int wq_project(const wq_rules* rules, const wq_extension* ext, const double* vals_mass, const double* b,
               double* u, double tol, int32_t max_iter, int32_t* iters, double* relres, void* stream);

/* out[0] = sum w (u_h - f)^2 and out[1] = sum w f^2 over Omega: (p+1)^3 Gauss points on every
 * interior element and the octree points on every cut element (the relative L2 error is
 * sqrt(out[0] / out[1])).  u: (n_active) coefficients; f_gauss: f at the points of
 * wq_gauss_coords (may be NULL iff n_gauss_elems = 0); f: (n_kappa) slot values of f (the
 * octree slots are read); out: 2 doubles; all device.  Asynchronous. */
int wq_l2_error(const wq_rules* rules, const double* u, const double* f_gauss, const double* f, double* out,
                void* stream);

void wq_rules_free(wq_rules* rules);
const char* wq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WQFD_H */
