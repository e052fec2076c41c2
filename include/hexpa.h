/*
 * hexpa -- matrix-free high-order hexahedral finite-element operators for
 * MI355X (gfx950), behind a plain C ABI.
 *
 * What is computed (Kolev et al., "Efficient Exascale Discretizations:
 * High-Order Finite Element Methods", 2021):
 *   - Benchmarks section: the bake-off problems BP1-BP6, CG solves of
 *     (alpha A + beta B) u = B f with homogeneous Dirichlet conditions, where
 *     A_ij = int grad phi_i . grad phi_j and B_ij = int phi_i phi_j on
 *     isoparametric Q_p bricks; Gauss rule with q = p+2 points for BP1-BP4,
 *     integration on the GLL nodes (q = p+1) for BP5-BP6; scalar (m = 1) and
 *     vector (m = 3) problems.
 *   - libCEED section, operator decomposition: the action on an L-vector is
 *     G^T B^T D B G -- element restriction G, basis evaluation B, pointwise
 *     quadrature-point operator D, then the transposes -- and the matrix is
 *     never formed. Each apply below is one fused pass of that product.
 *   - Miniapps section (Nekbone): CG with a diagonal (Jacobi) preconditioner.
 *
 * Conventions shared by every entry point:
 *   - Every function returns hx_status: HX_OK (0) or a negative code. No
 *     function aborts or throws across the ABI; hx_last_error() returns a
 *     thread-local message describing the last failure on this thread.
 *   - "host" pointers are ordinary CPU memory, read during the call only.
 *     "device" pointers are GPU memory on the current HIP device, owned by the
 *     caller, contiguous, 16-byte aligned, not aliased between input and
 *     output.
 *   - hx_stream is a hipStream_t (NULL = the default stream). Work is enqueued
 *     on it in order; entry points marked "asynchronous" return before the GPU
 *     finishes.
 *   - Handles are created and destroyed by the caller. A handle owns its
 *     device buffers (geometric factors, index arrays, work vectors) and frees
 *     them in its destroy call. An operator keeps a reference to its mesh and
 *     basis; destroy the operator first.
 *   - L-vectors hold one value per mesh node and component; for ncomp = 3 the
 *     components are interleaved: entry 3*node + c.
 *   - Calls on one handle from several host threads at once are not
 *     supported. Two operators may be used concurrently on different streams.
 */
#ifndef HEXPA_H
#define HEXPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hx_status;
enum {
  HX_OK = 0,
  HX_EINVAL = -1,       /* a null pointer, a size or an enum out of range          */
  HX_ERANGE = -2,       /* an index in elem_nodes outside [0, nnodes)              */
  HX_EUNSUPPORTED = -3, /* a valid combination this library does not implement     */
  HX_EGEOM = -4,        /* a non-positive Jacobian determinant found at setup      */
  HX_ENOCONV = -5,      /* a solve stopped at maxit; the info struct is filled     */
  HX_EBREAKDOWN = -6,   /* p'Ap <= 0, r'z <= 0 or a non-finite scalar in a solve   */
  HX_EHIP = -7,         /* a HIP runtime error; its text is in hx_last_error()     */
  HX_ENOMEM = -8        /* a device or host allocation failed                      */
};

enum { HX_GAUSS = 0, HX_GLL = 1 };          /* quadrature rule families               */
enum { HX_MASS = 0, HX_DIFFUSION = 1,       /* B and A of the bake-off problems       */
       HX_HELMHOLTZ = 2,                     /* alpha A + beta B (hx_op_create_helmholtz) */
       HX_LOR = 3 };                         /* low-order refined diffusion (hx_op_create_lor) */
/* Arithmetic precisions. HX_BF16: matrix-core products of operands rounded to
 * bfloat16, accumulated in FP32. HX_BF16_SPLIT: the same matrix cores with every
 * operand carried as hi + lo, both bfloat16 (lo the rounding error of hi), and the
 * products hi*hi + hi*lo + lo*hi accumulated in FP32 (about 16 significant bits). */
enum { HX_FP64 = 0, HX_FP32 = 1, HX_BF16 = 2, HX_BF16_SPLIT = 3 };

typedef struct hx_mesh_s *hx_mesh;
typedef struct hx_basis_s *hx_basis;
typedef struct hx_op_s *hx_op;
typedef struct hx_mlp_s *hx_mlp;  /* two-layer network (learned preconditioner) */
typedef void *hx_stream; /* hipStream_t */

/* Text of the last error on the calling thread ("" if none). Never NULL. */
const char *hx_last_error(void);

/* Library version string. */
const char *hx_version(void);

/* ------------------------------------------------------------------------ */
/* Meshes                                                                    */
/* ------------------------------------------------------------------------ */

/* Coordinates of the Q_p nodes of a mesh of trilinear bricks.
 * Benchmarks section: elements are mapped from the reference cube [-1,1]^3 by
 * x^e(r); for a trilinear brick that map is the Q_1 interpolant of its 8
 * vertices, evaluated here at the (p+1)^3 Gauss-Lobatto-Legendre nodes.
 *   p           polynomial degree, 1..8
 *   elem_verts  host, nelem*8, vertex ids; vertex a+2b+4c sits at reference
 *               corner (2a-1, 2b-1, 2c-1)
 *   verts       host, nverts*3 FP64 coordinates
 *   elem_nodes  host, nelem*(p+1)^3 node ids, element-local order i fastest
 *   node_xyz    host output, nnodes*3 FP64; nodes listed by no element are 0
 * Errors: HX_EINVAL (null, sizes, p), HX_ERANGE (an id out of range). */
hx_status hx_mesh_nodes_trilinear(int p, int64_t nelem, const int64_t *elem_verts, int64_t nverts,
                                  const double *verts, const int32_t *elem_nodes, int64_t nnodes,
                                  double *node_xyz);

/* Create a mesh: element restriction G (libCEED section) plus node coordinates.
 *   p           polynomial degree, 1..8; (p+1)^3 nodes per element
 *   nelem       number of elements, >= 1, with nelem*(p+1)^3 < 2^31
 *   nnodes      number of L-vector nodes, 1 .. 2^31-1
 *   elem_nodes  host, nelem*(p+1)^3 int32 node ids, local order
 *               (i + (p+1)(j + (p+1)k)), i along the reference r1 axis
 *   node_xyz    host, nnodes*3 FP64 coordinates of the Q_p nodes
 *   dirichlet   host, nnodes bytes, 1 = constrained node; NULL = none
 *   out         receives the handle
 * The library colors the elements so that no two elements of one color share
 * a node, and orders them internally (color-major, spatially sorted within a
 * color); this is invisible at the ABI. Device memory: nelem*(p+1)^3*4 bytes
 * of indices, nelem*(p+1)^2*2 bytes of ownership masks, nnodes*(24+1) bytes.
 * Errors: HX_EINVAL, HX_ERANGE, HX_ENOMEM, HX_EHIP. */
hx_status hx_mesh_create(int p, int64_t nelem, int64_t nnodes, const int32_t *elem_nodes,
                         const double *node_xyz, const uint8_t *dirichlet, hx_mesh *out);

typedef struct {
  int p;
  int ncolors;          /* element colors (launches per apply)                     */
  int64_t nelem;
  int64_t nnodes;
  int64_t nfree;        /* nodes with dirichlet == 0                               */
  int64_t nuntouched;   /* nodes listed by no element                              */
  int64_t max_color;    /* elements in the largest color                           */
  int64_t nstrips;      /* strips of up to 8 face-adjacent elements along r1 that
                           the degree-7 collocated apply scatters together (0: the
                           per-element scatter is used)                          */
  int64_t nstrip_colors; /* strip colors (launches per apply when nstrips > 0)   */
  int64_t nstrip_groups; /* workgroups per apply of the strip kernels: whole strips
                            of one color packed into groups of up to 8 elements  */
  int index_mode;       /* element restriction read by the fused kernels: 0 the full
                           index array; 1 one id per r1-row (every r1-row of every
                           element holds consecutive ids); 2 three numbers per
                           element (base + i + j s_j + k s_k for every element)  */
} hx_mesh_stats;

hx_status hx_mesh_get_stats(hx_mesh mesh, hx_mesh_stats *stats);

/* Element permutation chosen by the library: order[t] = caller element id of
 * internal position t; color_start has ncolors+1 entries. Host outputs of
 * nelem and ncolors+1 entries. */
hx_status hx_mesh_get_order(hx_mesh mesh, int32_t *order, int64_t *color_start);

void hx_mesh_destroy(hx_mesh mesh);

/* Host-only mesh plan: the element coloring, internal order, ownership masks,
 * index mode and strips that hx_mesh_create computes (libCEED section: the
 * element restriction G and the atomic-free form of its transpose), built on
 * the host with no HIP call and no device memory, so that the host logic can
 * be inspected where there is no GPU. Arguments and errors as hx_mesh_create
 * (no HX_EHIP). hx_mesh_get_stats, hx_mesh_get_order, hx_mesh_plan_arrays and
 * hx_mesh_destroy accept the result; operator creation rejects it (HX_EINVAL). */
hx_status hx_mesh_plan(int p, int64_t nelem, int64_t nnodes, const int32_t *elem_nodes,
                       const double *node_xyz, const uint8_t *dirichlet, hx_mesh *out);

/* Copy a plan's arrays to host buffers the caller owns (any may be NULL),
 * P = p+1, all in internal element order (hx_mesh_get_order):
 *   idx               nelem*P^3 int32, node ids, local order i + P(j + Pk)
 *   own               nelem*P^2 uint16, [t][j*P+i] bit k: element t is the first
 *                     element (internal order) listing node (i,j,k)
 *   strip_elems       nstrip_groups*8 int32: the internal positions of each
 *                     strip group's elements, -1 past its last
 *   strip_link        nstrip_groups uint8: bit w, slot w+1 continues slot w's strip
 *   strip_own         nelem*P^2 uint16, ownership in strip order (element w > 0
 *                     of a strip never owns its i = 0 face)
 *   strip_color_start nstrip_colors+1 int64, in groups
 * The strip arrays are empty (nothing copied) when nstrips == 0.
 * Errors: HX_EINVAL (null mesh, or a mesh from hx_mesh_create). */
hx_status hx_mesh_plan_arrays(hx_mesh mesh, int32_t *idx, uint16_t *own, int32_t *strip_elems,
                              uint8_t *strip_link, uint16_t *strip_own, int64_t *strip_color_start);

/* ------------------------------------------------------------------------ */
/* Bases                                                                     */
/* ------------------------------------------------------------------------ */

/* 1D basis of degree p on the GLL nodes with a q-point rule (Benchmarks
 * section: q = p+2 Gauss for BP1-BP4, q = p+1 GLL for BP5-BP6).
 *   qrule = HX_GAUSS: q in {p+1, p+2}; qrule = HX_GLL: q = p+1 (collocated).
 * Errors: HX_EINVAL (p outside 1..8, q outside the list), HX_ENOMEM. */
hx_status hx_basis_create(int p, int q, int qrule, hx_basis *out);

/* Host copies of the 1D tables, each optional (NULL = skip):
 *   nodes[p+1], qpts[q], qweights[q],
 *   interp[q*(p+1)]  interp[a*(p+1)+i] = l_i(qpts[a]),
 *   grad[q*(p+1)]    grad[a*(p+1)+i]   = l_i'(qpts[a]). */
hx_status hx_basis_get_tables(hx_basis basis, double *nodes, double *qpts, double *qweights,
                              double *interp, double *grad);

void hx_basis_destroy(hx_basis basis);

/* ------------------------------------------------------------------------ */
/* Operators                                                                 */
/* ------------------------------------------------------------------------ */

/* Coefficient kappa(x) = exp(scale * g(x) + shift),
 * g(x) = sqrt(2/M) sum_m cos(omega_m . x + phase_m): a random-Fourier-feature
 * Gaussian random field. Not in the paper; it multiplies the diffusion
 * integrand (A_ij = int kappa grad phi_i . grad phi_j). Host arrays. */
typedef struct {
  int M;
  const double *omega; /* M*3 */
  const double *phase; /* M   */
  double scale;
  double shift;
} hx_kappa_rff;

/* Create an operator: the pointwise operator D at the quadrature points
 * (libCEED section) is computed once, in FP64 on the GPU, and stored:
 *   HX_MASS       w * detJ                          (1 value per point)
 *   HX_DIFFUSION  w * kappa * detJ * J^-1 J^-T      (6 values per point)
 * ncomp is 1 (BP1/3/5) or 3 (BP2/4/6). kappa may be NULL (kappa = 1); it is
 * rejected for HX_MASS. Enqueued on s; returns after setup completes.
 * Errors: HX_EINVAL, HX_EUNSUPPORTED (p of mesh and basis differ),
 * HX_EGEOM (detJ <= 0 at some point), HX_ENOMEM, HX_EHIP. */
hx_status hx_op_create(hx_mesh mesh, hx_basis basis, int kind, int ncomp, const hx_kappa_rff *kappa,
                       hx_stream s, hx_op *out);

/* Create the Helmholtz operator alpha A + beta B of the bake-off problems
 * (Benchmarks section: the systems are (alpha A + beta B) u = B f; A the
 * diffusion operator with the optional coefficient kappa, B the mass operator,
 * both integrated with the basis's rule). Kind HX_HELMHOLTZ: stored as alpha
 * times the diffusion factors (6 values per point) plus beta * w * detJ (1 value
 * per point), computed in FP64 on the GPU in one pass; every apply evaluates
 * both terms in one fused kernel (on the GLL-collocated rule the mass term is
 * diagonal). Every entry point that takes an operator accepts it, except the
 * bf16 matrix-core apply and the learned preconditioner (HX_EUNSUPPORTED).
 *   alpha, beta  finite, >= 0, not both 0 (alpha = 0: the mass operator on the
 *                diffusion code path; beta = 0: the diffusion operator)
 * Errors: as hx_op_create; HX_EINVAL for alpha or beta out of range. */
hx_status hx_op_create_helmholtz(hx_mesh mesh, hx_basis basis, int ncomp, double alpha, double beta,
                                 const hx_kappa_rff *kappa, hx_stream s, hx_op *out);

/* Low-order refined (LOR) diffusion operator of a mesh (Preconditioning section: a
 * spectrally equivalent sparse matrix from a low-order discretization on a refined
 * mesh, by the FEM-SEM equivalence of tensor-product elements). Every element of
 * degree p is split into p^3 trilinear sub-hexahedra whose corners are its GLL
 * nodes; the matrix is the Q1 stiffness on them, integrated with the 2-point GLL
 * (vertex) rule per direction, kappa (as for hx_op_create; NULL: 1) at the
 * vertices, assembled on the device into ELL storage (width W <= 32 entries per
 * row, 19 on a lattice). The operator has the mesh's nodes: hx_op_apply (FP64),
 * hx_op_diagonal, hx_pcg_solve in HX_SOLVE_FP64 mode and the finest level of an
 * FP64 p-multigrid hierarchy accept it; FP32, bf16, E-vector and learned-map
 * entry points return HX_EUNSUPPORTED. A hierarchy whose finest level is this
 * operator preconditions the high-order operator of the same mesh nodes
 * (HX_PC_PMG). Synchronous. Device memory: W * nnodes * 12 bytes.
 * Errors: HX_EINVAL, HX_EGEOM (a sub-hex corner with a non-positive Jacobian),
 * HX_EUNSUPPORTED (p = 0 or a row longer than 32), HX_ENOMEM, HX_EHIP. */
hx_status hx_op_create_lor(hx_mesh mesh, const hx_kappa_rff *kappa, hx_stream s, hx_op *out);

/* The assembled LOR matrix, copied to the host in ELL layout: width receives W;
 * cols [W][nnodes] int32 and vals [W][nnodes] FP64 (entry k of row t at k*nnodes
 * + t; rows shorter than W repeat their own index with value 0). cols and vals
 * may be NULL (width only). Errors: HX_EINVAL (null, not an LOR operator), HX_EHIP. */
hx_status hx_op_lor_matrix(hx_op op, int *width, int32_t *cols, double *vals);

/* y = A x on the whole L-vector (no boundary condition), FP64.
 * x, y: device, nnodes*ncomp doubles. y is overwritten. Asynchronous.
 * Deterministic: the same x gives bit-identical y on every call.
 * Errors: HX_EINVAL (null), HX_EHIP. */
hx_status hx_op_apply(hx_op op, const double *x, double *y, hx_stream s);

/* y = A x in FP32 vectors. qdata_prec = HX_FP64 reads the FP64 geometric
 * factors and rounds them in registers; HX_FP32 reads an FP32 copy made at
 * the first such call (FP64 arithmetic, then rounded). Products and sums are
 * FP32. x, y: device floats. Asynchronous. Errors: HX_EINVAL, HX_ENOMEM, HX_EHIP. */
hx_status hx_op_apply_f32(hx_op op, int qdata_prec, const float *x, float *y, hx_stream s);

/* y = A x with the basis contractions on bf16 matrix cores, the pointwise
 * operator in FP32 on a bfloat16 copy of the geometric factors (made at the
 * first call). prec: HX_BF16 or HX_BF16_SPLIT (operand representation, see the
 * precision constants). x, y: device floats. HX_DIFFUSION, ncomp = 1, p + 1 <= 8
 * and q <= 8 only. Asynchronous.
 * Errors: HX_EINVAL (null pointer, bad prec), HX_EUNSUPPORTED, HX_ENOMEM, HX_EHIP. */
hx_status hx_op_apply_bf16(hx_op op, int prec, const float *x, float *y, hx_stream s);

/* E-vector action (the bake-off kernel: the element-local part only):
 * y_e[(e*ncomp + c)*(p+1)^3 + l] = (A_e x_e)_l for caller element e, FP64.
 * y_e: device, nelem*ncomp*(p+1)^3 doubles. Asynchronous. */
hx_status hx_op_apply_elem(hx_op op, const double *x, double *y_e, hx_stream s);

/* Diagonal of the assembled operator, matrix-free: diag = G^T diag(B^T D B),
 * summed over elements (Miniapps section: Nekbone's diagonal preconditioner).
 * diag: device, nnodes*ncomp doubles, overwritten. Asynchronous. */
hx_status hx_op_diagonal(hx_op op, double *diag, hx_stream s);

typedef struct {
  int p, q, qrule, kind, ncomp;
  int64_t nnodes, nelem;
  int64_t qdata_bytes;   /* FP64 geometric factors                       */
  int64_t index_bytes;   /* element restriction indices                  */
} hx_op_stats;

hx_status hx_op_get_stats(hx_op op, hx_op_stats *stats);

void hx_op_destroy(hx_op op);

/* ------------------------------------------------------------------------ */
/* Solves                                                                    */
/* ------------------------------------------------------------------------ */

enum { HX_PC_NONE = 0, HX_PC_JACOBI = 1, HX_PC_CHEBYSHEV = 2, HX_PC_MLP = 3, HX_PC_PMG = 4 };

/* p-multigrid hierarchy (declared below) */
typedef struct hx_pmg_s *hx_pmg;
enum { HX_SOLVE_FP64 = 0, HX_SOLVE_IR = 1, HX_SOLVE_MIXED = 2 };

typedef struct {
  int mode;            /* HX_SOLVE_FP64: FP64 PCG. HX_SOLVE_IR: FP64 iterative
                          refinement around an FP32 inner PCG (each restart
                          discards the Krylov space). HX_SOLVE_MIXED: one FP32
                          PCG whose residual is replaced by the FP64 residual
                          b - A x (x accumulated in FP64) whenever it has fallen
                          by reliable_delta since the last replacement, keeping
                          the search direction (reliable updates, van der Vorst
                          and Ye 2000); converged on the FP64 residual        */
  int precond;         /* HX_PC_*                                            */
  double rtol;         /* stop when ||b - A x||_2 <= rtol ||b||_2 (free nodes) */
  int maxit;           /* iteration cap (outer cap for IR)                    */
  int check_every;     /* host convergence check period (>= 1)               */
  int use_x0;          /* 1: x holds the initial guess; 0: start from x = 0   */
  int cheb_degree;     /* Chebyshev steps per application (>= 1)             */
  double cheb_ratio;   /* lam_lo = lam_hi / cheb_ratio                        */
  int cheb_prec;       /* operator precision in the Chebyshev polynomial:
                          HX_FP64, HX_FP32, HX_BF16 or HX_BF16_SPLIT          */
  int lanczos_steps;   /* steps of the lam_max estimate (>= 2)               */
  double inner_rtol;   /* IR: inner FP32 solve tolerance (relative to the outer
                          residual; loosened to 0.5 rtol ||b|| / ||r|| when that
                          is larger, at most 0.5)                              */
  int inner_maxit;     /* IR: inner iteration cap per outer step (a restart
                          loses the Krylov space: keep it above the iterations
                          one inner solve needs)                               */
  int inner_qdata;     /* IR and MIXED: HX_FP64 or HX_FP32 geometric factors of
                          the FP32 operator                                    */
  int flexible;        /* 1: flexible CG (Polak-Ribiere beta) for preconditioners
                          that are not exactly linear or symmetric (the bf16
                          Chebyshev forms); 0: plain PCG                         */
  hx_mlp mlp;          /* HX_PC_MLP: the trained network (flexible CG is used)  */
  int fallback;        /* HX_PC_MLP: HX_PC_JACOBI or HX_PC_CHEBYSHEV, run from the
                          current iterate when the learned solve breaks down or
                          stalls                                               */
  int stall_window;    /* HX_PC_MLP: stall = the residual fell by less than     */
  double stall_factor; /* stall_factor over the last stall_window iterations   */
  int mlp_mode;        /* HX_PC_MLP: 0: z = network correction; 1: z = D^-1 r plus
                          the network correction (trained on targets e - D^-1 r);
                          2: cheb_degree Chebyshev steps on M A e = M r with M
                          the mode-1 map as the base (lam_max of M A from
                          lanczos_steps power iterations; FP64 operator)        */
  int graph;           /* 1: from the second iteration on, replay each PCG
                          iteration as a HIP graph captured once per solve, on a
                          stream the operator owns (results identical to 0; on
                          MI355X measured no faster: the per-iteration floor is
                          the kernels' own boundaries, not their submission).
                          Used when the operator needs no zero-fill of its output
                          and the preconditioner is not HX_PC_MLP. 0: launch every
                          kernel on the caller's stream                         */
  hx_pmg pmg;          /* HX_PC_PMG: the hierarchy, whose finest operator is the
                          solved one; one V-cycle per iteration, flexible CG    */
  int scatter;         /* the FP64 operator of the CG iteration itself:
                          HX_SCATTER_COLORS: the colored atomic-free scatter (one
                          launch per element or strip color);
                          HX_SCATTER_GATHER: the element kernel writes the E-vector
                          in one launch and a node gather (the transpose of the
                          element restriction, each node's contributions summed in a
                          fixed order) forms A p with p'Ap fused: two launches, for
                          small problems where each launch's fixed cost dominates;
                          the E-vector (nelem*ncomp*(p+1)^3 doubles) and the
                          transpose (nelem*(p+1)^3 + nnodes + 1 ints) are kept by the
                          operator and its mesh. Results differ from
                          HX_SCATTER_COLORS in the last bits (summation order) and
                          are deterministic                                        */
  double reliable_delta; /* HX_SOLVE_MIXED: replace the FP32 residual by the FP64
                          one when its norm has fallen below reliable_delta
                          times the norm at the last replacement (checked every
                          check_every iterations), 0 < reliable_delta < 1     */
} hx_solve_opts;

enum { HX_SCATTER_COLORS = 0, HX_SCATTER_GATHER = 1 };

typedef struct {
  int iterations;        /* PCG iterations (sum of inner iterations for IR)  */
  int outer_iterations;  /* IR refinement steps (0 for FP64 PCG)             */
  int operator_applies;  /* applies of A in any precision (HX_PC_PMG: with the
                            V-cycles' applies of this operator, not those of
                            the coarser levels)                               */
  double rel_residual;   /* recurrence residual at exit                      */
  double true_rel_residual; /* ||b - A x|| / ||b|| recomputed in FP64 at exit */
  double lam_max;        /* Chebyshev: estimated lambda_max of D^-1 A (of M A
                            for the learned Chebyshev form, mlp_mode 2)       */
  double setup_seconds;  /* Chebyshev lambda estimate, diagonal               */
  double solve_seconds;  /* wall time of the iteration                        */
  int fallback_used;     /* HX_PC_MLP: 1 if the fallback solve ran            */
  int fallback_iterations; /* iterations of the fallback solve                */
  int fallback_reason;   /* HX_PC_MLP: 0 none, 1 breakdown (r'z <= 0, p'Ap <= 0
                            or non-finite), 2 stall, 3 maxit                   */
} hx_solve_info;

/* Fill opts with defaults: FP64 Jacobi PCG, rtol 1e-8, maxit 10000,
 * check_every 10, degree 4, ratio 30, FP32 Chebyshev, 20 Lanczos steps,
 * inner_rtol 1e-4, inner_maxit 10000, FP64 inner qdata, flexible 0, no network,
 * fallback Jacobi, stall window 20 iterations, stall factor 0.1, mlp_mode 1,
 * graph 0, no hierarchy, HX_SCATTER_COLORS, reliable_delta 0.25. */
void hx_solve_opts_default(hx_solve_opts *opts);

/* Solve A_II x_I = b_I with x = 0 on Dirichlet nodes (Benchmarks section:
 * homogeneous Dirichlet conditions; CG), preconditioned as opts says.
 *   b, x: device FP64 L-vectors (nnodes*ncomp); b's constrained entries are
 *         ignored; x is overwritten (constrained entries set to 0).
 * Synchronous: returns once x is final; the host reads 8 bytes every
 * check_every iterations. Uses work vectors owned by op (allocated on first
 * use: 10 vectors of nnodes*ncomp doubles, and 10 of floats for the FP32 forms).
 * Errors: HX_EINVAL, HX_ENOCONV (maxit reached; info filled),
 * HX_EBREAKDOWN, HX_ENOMEM, HX_EHIP. */
hx_status hx_pcg_solve(hx_op op, const double *b, double *x, const hx_solve_opts *opts,
                       hx_solve_info *info, hx_stream s);

/* Largest nnodes*ncomp that hx_pcg_solve_noalloc accepts. */
#define HX_NOALLOC_MAX_DOFS 1048576

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the FP64 Jacobi-preconditioned (or
 * unpreconditioned) solve of hx_pcg_solve with every work vector, reduction
 * partial and device scalar in one array of about 56 MiB that the library
 * holds in static device memory, one copy per device, until the process ends.
 * No hipMalloc, hipFree, pinned-host allocation or allocating library call is
 * made; the caller passes b and x as for hx_pcg_solve, and the result is the
 * same, bit for bit, as hx_pcg_solve's with the same opts.
 *   opts: mode HX_SOLVE_FP64, precond HX_PC_NONE or HX_PC_JACOBI, scatter
 *         HX_SCATTER_COLORS, graph 0 (other values: HX_EUNSUPPORTED).
 *   op:   nnodes*ncomp <= HX_NOALLOC_MAX_DOFS (else HX_EINVAL, with the sizes
 *         in hx_last_error()); its device must be the current one.
 * The diagonal is the one an earlier hx_pcg_solve cached in op, else it is
 * computed into the array on every call. Every call on one device shares that
 * device's array and starts by clearing what it reads before writing: two
 * calls that overlap on one device (two host threads, or two streams) race and
 * give wrong results; serialise them. Synchronous, like hx_pcg_solve.
 * Errors: HX_EINVAL, HX_EUNSUPPORTED, HX_ENOCONV (info filled), HX_EBREAKDOWN,
 * HX_EHIP. */
hx_status hx_pcg_solve_noalloc(hx_op op, const double *b, double *x, const hx_solve_opts *opts,
                               hx_solve_info *info, hx_stream s);

/* ------------------------------------------------------------------------ */
/* Two-layer network (learned element preconditioner; not in the paper)      */
/* ------------------------------------------------------------------------ */

/* y = W2 tanh(W1 x + b1) + b2, FP32 parameters on the device. Parameter vector
 * layout (hx_mlp_set_params / get_params / loss_grad): W1 [n_hidden][n_in],
 * b1 [n_hidden], W2 [n_out][n_hidden], b2 [n_out], row-major, FP32. */

/* Weights uniform(-1, 1)/sqrt(fan_in) from a seeded generator, zero biases.
 * Errors: HX_EINVAL (sizes), HX_ENOMEM, HX_EHIP. */
hx_status hx_mlp_create(int n_in, int n_hidden, int n_out, uint64_t seed, hx_mlp *out);
hx_status hx_mlp_get_shape(hx_mlp net, int *n_in, int *n_hidden, int *n_out);
/* host arrays of n_hidden*(n_in+1) + n_out*(n_hidden+1) floats */
hx_status hx_mlp_set_params(hx_mlp net, const float *params);
hx_status hx_mlp_get_params(hx_mlp net, float *params);

/* Y [batch][n_out] = net(X [batch][n_in]); device FP32 arrays. prec HX_FP32:
 * FP32 arithmetic; HX_BF16: operands rounded to bfloat16 on matrix cores, FP32
 * accumulation, bf16 hidden activations. Asynchronous. */
hx_status hx_mlp_forward(hx_mlp net, int prec, const float *X, int64_t batch, float *Y, hx_stream s);

/* Mean squared error over all batch*n_out entries and its gradient with respect
 * to every parameter (FP32 arithmetic). loss: host double (may be NULL); grads:
 * host array in the parameter layout (may be NULL). Synchronous. */
hx_status hx_mlp_loss_grad(hx_mlp net, const float *X, const float *T, int64_t batch, double *loss, float *grads,
                           hx_stream s);

typedef struct {
  int epochs;        /* passes over the samples                          */
  int batch;         /* rows per Adam step (the tail of an epoch is dropped) */
  double lr, beta1, beta2, eps;  /* Adam                                  */
  uint64_t seed;     /* minibatch shuffling                               */
} hx_train_opts;

typedef struct {
  int64_t steps;
  double first_loss;  /* loss of the last batch of the first epoch        */
  double final_loss;  /* loss of the last batch of the last epoch         */
  double seconds;
} hx_train_info;

/* Defaults: 200 epochs, batch 256, lr 1e-3, betas 0.9/0.999, eps 1e-8, seed 7. */
void hx_train_opts_default(hx_train_opts *opts);

/* Adam on the GPU over X [nsamples][n_in], T [nsamples][n_out] (device FP32).
 * Synchronous. Errors: HX_EINVAL, HX_ENOMEM, HX_EHIP. */
hx_status hx_mlp_train(hx_mlp net, const float *X, const float *T, int64_t nsamples, const hx_train_opts *opts,
                       hx_train_info *info, hx_stream s);

/* Learned element preconditioner on a scalar diffusion operator (see the
 * HX_PC_MLP solve), in Jacobi-scaled variables: with D the assembled diagonal and
 * r~ = D^-1/2 r (0 on constrained nodes), element e's network input is
 * [r~_e/|r~_e|, f_e] (2 (p+1)^3 values), f_e = log kappa_e - mean(log kappa_e) at
 * the element's nodes with the value 3 on constrained nodes, and the correction is
 * z = D^-1/2 G^T (w * |r~_e| * net(input)), w = 1 over the node's multiplicity
 * (0 on constrained nodes).
 *   hx_op_mlp_features: X [nelem][2 (p+1)^3] and rnorm = |r~_e| [nelem] (device
 *     FP32, caller element order), the inputs for a residual r (FP64 L-vector).
 *   hx_op_mlp_targets: T [nelem][(p+1)^3] (device FP32, caller order): the
 *     training targets D^1/2 err_e / |r~_e| for an error vector err (FP64).
 *   hx_op_mlp_precond: the map of the HX_PC_MLP solve for r (device FP64; z must
 *     not alias r), on bf16 matrix cores: mode 0 z = the correction; mode 1
 *     z = D^-1 r + the correction (D^-1 r is 0 on constrained nodes).
 * Asynchronous. Errors: HX_EINVAL (shapes), HX_EUNSUPPORTED (not scalar
 * diffusion), HX_ENOMEM, HX_EHIP. */
hx_status hx_op_mlp_features(hx_op op, const double *r, float *X, float *rnorm, hx_stream s);
hx_status hx_op_mlp_targets(hx_op op, const double *err, const float *rnorm, float *T, hx_stream s);
hx_status hx_op_mlp_precond(hx_op op, hx_mlp net, int mode, const double *r, double *z, hx_stream s);

/* ------------------------------------------------------------------------ */
/* p-multigrid                                                               */
/* ------------------------------------------------------------------------ */

/* A V-cycle over polynomial degrees on one mesh (the preconditioning section:
 * multigrid over a hierarchy of degrees with matrix-free smoothers). Level 0 is
 * the finest. P_l, the prolongation from level l+1 to level l, evaluates a
 * coarse function (its values at the coarse GLL nodes of each element) at the
 * fine GLL nodes: a fine node shared by several elements takes its value from
 * one of them (all give the same value up to rounding). The restriction is P_l^T.
 * One V-cycle z = V_0 r:
 *   level l < L-1: z = S_l r (Chebyshev smoothing from 0: smooth_degree steps on
 *     D_l^-1 A_l over [lam_hi / smooth_ratio, lam_hi], lam_hi = 1.1 lam_max(D_l^-1 A_l));
 *     z += P_l V_{l+1}(P_l^T (r - A_l z)); z += S_l (r - A_l z);
 *   level L-1: Jacobi-PCG from 0 on A_{L-1} e = r.
 * Residuals, corrections and results are zero at constrained nodes. */
typedef struct {
  int smooth_degree;   /* Chebyshev steps per smoothing (>= 1)                 */
  double smooth_ratio; /* > 1                                                  */
  int lanczos_steps;   /* steps of each level's lam_max estimate (>= 2)       */
  int coarse_maxit;    /* Jacobi-PCG iteration cap on the coarsest level (>= 1) */
  double coarse_rtol;  /* coarse PCG tolerance relative to its right-hand side;
                          0: exactly coarse_maxit iterations (a fixed map)       */
  int prec;            /* HX_FP64, or HX_FP32: the V-cycle's vectors, operators
                          (FP32 copies of the geometric factors, made at
                          creation) and smoothers in FP32, the transfers'
                          contractions and every reduction in FP64; the
                          V-cycle's input and output stay FP64. HX_BF16 or
                          HX_BF16_SPLIT: as HX_FP32, with the finest level's
                          operator on the bf16 matrix cores (hx_op_apply_bf16;
                          scalar diffusion, p+1 <= 8, q <= 8)                   */
  hx_mlp smoother_mlp; /* NULL: every smoother is Chebyshev on D_l^-1 A_l. A
                          trained network (learned element preconditioner, see
                          hx_op_mlp_precond): the finest level's smoother is
                          the same Chebyshev polynomial with the mode-1 learned
                          map M r = D^-1 r + correction in place of D^-1, on
                          [lam_hi / smooth_ratio, lam_hi], lam_hi = 1.1 lam_max(M A)
                          from lanczos_steps power iterations; prec HX_FP64 and
                          scalar diffusion only (not in the paper: the learned
                          map as a smoother inside the multigrid cycle)        */
  int cycles;          /* V-cycles per application (>= 1): z = V r, then
                          z += V (r - A_0 z) cycles - 1 times (an approximate
                          inverse of A_0 that tightens with cycles; > 1 in FP64
                          hierarchies only)                                    */
} hx_pmg_opts;

/* Defaults: smooth_degree 3, smooth_ratio 15, 20 Lanczos steps, coarse_maxit 30,
 * coarse_rtol 0.1 (the coarse PCG checks its residual every 10 iterations), HX_FP64,
 * no learned smoother, one cycle. */
void hx_pmg_opts_default(hx_pmg_opts *opts);

/* Builds the hierarchy over ops[0..nlevels-1] (not owned; they must outlive it):
 * 2 <= nlevels <= 8, every operator of one kind and one ncomp (the transfers act on
 * each interleaved component; the coarse PCG is one CG on all of them), degrees
 * strictly decreasing, meshes with the same elements in the same caller order and
 * the same corner positions (element e of every level is the same hexahedron in
 * the same local orientation), every node in some element. Computes each level's
 * diagonal and lam_max on s and returns after they are done. The hierarchy keeps
 * work vectors per level: calls that use one hierarchy (V-cycles, solves) must not
 * overlap. Errors: HX_EINVAL (arguments, mismatched levels), HX_ENOMEM, HX_EHIP,
 * HX_EBREAKDOWN (a lam_max estimate failed). */
hx_status hx_pmg_create(const hx_op *ops, int nlevels, const hx_pmg_opts *opts, hx_stream s, hx_pmg *out);
int hx_pmg_levels(hx_pmg mg);
/* lam_max of D_l^-1 A_l as estimated at creation (0 for the coarsest level; of M A
 * on level 0 with a learned smoother). */
hx_status hx_pmg_lambda_max(hx_pmg mg, int level, double *lam_max);
/* z = V_0 r (device FP64 L-vectors of level 0; z must not alias r). Synchronises s
 * at the coarse solve's convergence checks: once with coarse_rtol 0, otherwise at
 * most 2 + coarse_maxit / 10 times. */
hx_status hx_pmg_vcycle(hx_pmg mg, const double *r, double *z, hx_stream s);
/* y_l = P_l x_{l+1} and y_{l+1} = P_l^T r_l, 0 <= level < nlevels-1 (device FP64
 * L-vectors of the two levels; no masking). Asynchronous. */
hx_status hx_pmg_prolong(hx_pmg mg, int level, const double *x_coarse, double *y_fine, hx_stream s);
hx_status hx_pmg_restrict(hx_pmg mg, int level, const double *r_fine, double *y_coarse, hx_stream s);
void hx_pmg_destroy(hx_pmg mg);

/* Checkpoint: 8-byte magic "HXMLP1", int32 n_in, n_hidden, n_out, 0, then the FP32
 * parameters in the layout above. */
hx_status hx_mlp_save(hx_mlp net, const char *path);
hx_status hx_mlp_load(const char *path, hx_mlp *out);
void hx_mlp_destroy(hx_mlp net);

#ifdef __cplusplus
}
#endif
#endif /* HEXPA_H */
