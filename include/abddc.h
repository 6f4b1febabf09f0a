/*
 * abddc.h -- C ABI of the MI355X (gfx950) adaptive BDDC library.
 *
 * Method: Peng, Shu, Wang, Zhong, "A BDDC method with an adaptive coarse
 * space for three-dimensional advection-diffusion problems", arXiv 2501.01676.
 *
 *   problem      Section 2, eq. (model-AD-equation) and (stab-var-pb): GLS
 *                stabilised advection-diffusion, a(.,.) = b(.,.) + z(.,.)
 *   system       Section 3, eq. (Schur-complex-sys): the interface Schur
 *                complement system Rt^T St Rt u = Rt^T gt
 *   precond.     Section 3: M^{-1} = Rt^T Dt St^{-1} Dt^T Rt, deluxe scaling,
 *                vertex constraints, adaptive face constraints (eq. equ-4-8,
 *                primal-constraints-F) and the edge constraints of the new
 *                edge eigenproblem (eq. equ-5-21, equ-5-22, and the Remark
 *                after it on the SVD/QR change of basis)
 *   solver       Section 4: GMRES stopped at a residual of 1e-8 or 300 steps
 *
 * Discretisation here: a box grid on a tensor-product box partition, with
 * trilinear (Q1) boxes or the paper's linear tetrahedra (six per box), zero
 * or lifted Dirichlet data (abddc_problem below).
 *
 * Conventions (every entry point):
 *  - Return value: ABDDC_OK (0) on success, a positive warning code when the
 *    result is valid but flagged, a negative error code otherwise.  The
 *    message of the last error on the calling thread is abddc_last_error().
 *    No C++ exception crosses this boundary.
 *  - Call order: abddc_assemble -> abddc_setup_coarse_space -> any number of
 *    abddc_apply_bddc / abddc_apply_schur / abddc_gmres_solve.  Out of order
 *    calls return ABDDC_ESTATE.  One context must not be used by two host
 *    threads at once; different contexts are independent.
 *  - Problem arrays (abddc_problem nu, f_nodal, a_nodal, u_dirichlet) are HOST pointers, or
 *    DEVICE pointers of the context's device when arrays_on_device is set;
 *    either way abddc_assemble copies them and the caller keeps ownership.
 *    The width arrays are always host pointers.
 *  - Vectors passed to apply/solve (r, z, x, y, u) are DEVICE pointers of
 *    the context's device, read and written in stream order on the stream
 *    given at assemble time; the caller owns them.
 *  - All other device memory belongs to the library (allocated at assemble,
 *    setup and solve, released by abddc_destroy), taken from the caller's
 *    allocation hooks when abddc_device provides them.
 *  - Vector layouts: the interface vector (length n_gamma) lists all faces,
 *    then all edges, then all vertices; objects of one kind by increasing
 *    smallest grid-node id; the nodes of an object by increasing node id.
 *    Grid node id = ix + (nx+1)(iy + (ny+1) iz).  The full solution u
 *    (length n_dof) lists the free (non-Dirichlet) grid nodes by node id.
 *    Subdomain id = sx + Nx (sy + Ny sz).
 */
#ifndef ABDDC_H
#define ABDDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abddc_ctx abddc_ctx; /* opaque, owned by the library */

enum {
  ABDDC_OK = 0,
  ABDDC_NOT_CONVERGED = 1, /* gmres_solve: maxit reached; last iterate returned */
  ABDDC_EINVAL = -1,       /* invalid argument (sizes, coefficients, options)   */
  ABDDC_ENOMEM = -2,       /* device allocation failed                          */
  ABDDC_ESINGULAR = -3,    /* zero or non-finite pivot in a factorisation       */
  ABDDC_EEIG = -4,         /* eigensolver failure (metric not positive definite)*/
  ABDDC_EDEVICE = -5,      /* HIP runtime error                                 */
  ABDDC_ESTATE = -6        /* entry point called out of order                   */
};

/* Device binding: which GPU, which HIP stream (hipStream_t) to use, and
 * optionally the caller's device memory.  stream may be NULL for the default
 * stream.  alloc / free / user: when alloc is set, every device allocation
 * the library makes for the context (or network) created with this binding
 * -- its persistent buffers and the temporaries of each call -- is
 * alloc(bytes, user) and is returned by free(p, user); alloc and free must
 * both be set or both be NULL (NULL: the library's own caching allocator).
 * alloc must return memory of the binding's device, aligned to 256 bytes,
 * usable by work queued on the stream after it returns (NULL for failure:
 * the call then fails with ABDDC_ENOMEM).  free is called once the last
 * work using p has been queued on the stream; the allocator may hand p out
 * again for work queued later on that stream (stream-ordered reuse, as a
 * caching allocator that tags blocks with their stream does).  Both are
 * called on the thread of the entry point, never concurrently for one
 * context.  Pinned host memory (descriptor and upload rings) and the
 * primitive test hooks' work space still come from the library. */
typedef struct {
  int32_t device;
  void* stream;
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* p, void* user);
  void* user;
} abddc_device;

/* The model problem of Section 2 on a box grid split into box subdomains.
 * Coefficients: nu > 0 piecewise constant per element; velocity affine,
 * a(x) = beta0 + beta1 x (beta1 row-major 3x3), or given at the grid nodes;
 * constant reaction c; source f constant (f_nodal == NULL) or interpolated
 * from nodal values; Dirichlet data zero or given at the grid nodes.
 *
 * element selects the finite elements (Section 2's stabilised form on either):
 *   ABDDC_ELEM_Q1: trilinear boxes; nu has one value per box.
 *   ABDDC_ELEM_P1: the linear tetrahedra of Section 2 and of Section 4's
 *     example: every box split into six (the corner paths from its lowest
 *     to its highest corner, one per ordering of the axes: xyz, xzy, yxz,
 *     yzx, zxy, zyx); nu has six values per box in that order; the velocity
 *     is interpolated linearly on each tetrahedron from its nodal values
 *     (a_nodal, or the affine field at the nodes), so |a|_K is the largest
 *     vertex speed and div a is constant on K.
 * u_dirichlet lifts nonzero Dirichlet data (Section 4's example): the
 * computed u is then the free-node part of u_h = u_0 + w, u_0 the data on
 * the boundary nodes; boundary entries keep their data.
 *
 * part gives a general partition (Section 4's irregular subdomains), every
 * subdomain a union of grid boxes.  Interface objects then follow from the
 * sharing sets n(x) of the free nodes: nodes with one set split into pieces
 * connected through common boxes; a piece is a face when |n(x)| = 2, an edge
 * when |n(x)| >= 3 and it has two or more nodes, else a vertex.  (On box
 * partitions this is the box rule except that an edge of a single node is
 * a vertex.)  Limits of the kernels: faces of at most 512 dofs (above 128
 * the face eigenproblems and parallel sums take a global-memory variant,
 * and a parallel sum whose LU test fails has no pseudo-inverse fallback
 * there: ESINGULAR), edge eigenproblems of at most 128 unknowns, edges of at
 * most 32 dofs shared by at most 8 subdomains; larger objects return
 * EINVAL. */
enum { ABDDC_ELEM_Q1 = 0, ABDDC_ELEM_P1 = 1 };
typedef struct {
  int32_t nsub[3];          /* subdomains per axis                              */
  const int32_t* width[3];  /* elements per subdomain along each axis (>= 2)   */
  double length[3];         /* box edge lengths (> 0)                           */
  const double* nu;         /* per box (x-fastest), six per box for P1: len
                               prod_a sum(width[a]), times 6 for P1            */
  double beta0[3];
  double beta1[9];
  double c;
  const double* f_nodal;    /* NULL, or per grid node (x-fastest)               */
  double f_const;
  double tau;               /* GLS constant tau of C(x) (0.7 in the paper)      */
  int32_t arrays_on_device; /* nonzero: nu / f_nodal / a_nodal / u_dirichlet are device pointers */
  int32_t element;          /* ABDDC_ELEM_Q1 or ABDDC_ELEM_P1                    */
  double origin[3];         /* coordinates of grid node (0, 0, 0)                */
  const double* a_nodal;    /* NULL (affine beta0 + beta1 x), or 3 per grid node
                               (x, y, z), node-id order; ABDDC_ELEM_P1 only      */
  const double* u_dirichlet;/* NULL (zero data), or one per grid node; only the
                               boundary nodes' values are read                   */
  const int32_t* part;      /* NULL (the tensor-product box partition of nsub and
                               width), or a general partition: the subdomain id
                               in [0, n_parts) of every box (x-fastest); nsub must
                               then be {1, 1, 1} (width gives the grid) and every
                               part hold a box.  Always a HOST array.           */
  int32_t n_parts;          /* number of subdomains of part                     */
} abddc_problem;

enum { ABDDC_PREC_FP64 = 0, ABDDC_PREC_MIXED = 1 };
enum { ABDDC_EDGE_NEW = 0, ABDDC_EDGE_OLD = 1 };
enum { ABDDC_H_SHARED = 0, ABDDC_H_SEPARATE = 1 };
enum { ABDDC_DELUXE_S = 0, ABDDC_DELUXE_B = 1 };
enum { ABDDC_CONSTRAINTS_EXACT = 0, ABDDC_CONSTRAINTS_MLP = 1 };

/* Adaptive coarse-space options (Section 3 thresholds; Section 4 values
 * are Theta_F = 1 + log m, Theta_E = 10). */
typedef struct {
  double theta_face;        /* Theta_F >= 0: select lambda >= Theta_F           */
  double theta_edge;        /* Theta_E >= 0                                      */
  int32_t edge_variant;     /* ABDDC_EDGE_NEW (eq. equ-5-21) or ABDDC_EDGE_OLD,
                               the earlier edge eigenproblem (eq. equ-4-8-E:
                               B_E over ordered member pairs, parallel sum of
                               the members' Schur complements onto the edge,
                               one constraint per selected eigenvector; edges
                               of 2..4 members and <= 16 dofs; exact
                               constraints only)                              */
  int32_t edge_h_mode;      /* prior-selected primal unknowns shared / separate */
  int32_t deluxe_source;    /* deluxe weights from S^(i) (default) or B^(i)     */
  double pinv_rtol;         /* pseudo-inverse eigenvalue cut (1e-10)            */
  double svd_rtol;          /* edge SVD rank cut relative to sigma_1 (1e-8)     */
  double tie_rtol;          /* |lambda - Theta| <= tie_rtol Theta: near tie     */
  int32_t precision;        /* ABDDC_PREC_FP64 or ABDDC_PREC_MIXED             */
  int32_t constraint_source;/* exact GEP, or learned edge constraints          */
  const struct abddc_mlp* mlp; /* trained network for ABDDC_CONSTRAINTS_MLP     */
  int32_t judge_iters;      /* learned constraints only: reference iteration
                               count of the exact method (0: no judge); a
                               gmres_solve that fails or needs more than
                               judge_ratio * judge_iters iterations redoes
                               the setup with exact edge constraints and
                               solves again                                  */
  double judge_ratio;       /* > 0, or 0 for the default 1.2                   */
} abddc_options;

typedef struct {
  int32_t n_vertex, pnum_face, pnum_edge, n_primal, n_near_ties;
} abddc_counts;

typedef struct {
  int32_t iters;            /* preconditioned Arnoldi steps                      */
  int32_t restarts;
  double relres_true;       /* ||ghat - Shat u|| / ||ghat|| at exit              */
  double t_setup_s;         /* assemble + setup wall time (stream-synchronised) */
  double t_iter_s;          /* gmres_solve wall time incl. interior recovery     */
  double* resid_history;    /* HOST array or NULL; Arnoldi estimates / ||ghat|| */
  int32_t resid_cap;        /* capacity of resid_history                         */
  int32_t redone;           /* 1: the judge replaced learned edge constraints
                               by exact ones and the solve was repeated (the
                               fields above describe the repeated solve;
                               t_iter_s covers the whole call)                */
  int32_t first_iters;      /* iterations of the first solve                   */
} abddc_solve_info;

/* Section 3 (local matrices A^(i), f^(i) of a_i and g; Schur complements
 * S^(i) = A_BB - A_BI A_II^{-1} A_IB, g^(i) = f_B - A_BI A_II^{-1} f_I;
 * B^(i) = sym(S^(i))).  Builds the topology, assembles every subdomain on
 * the GPU and forms S^(i), g^(i), B^(i) and ghat = sum R_i^T g^(i).
 * EINVAL on bad sizes / non-positive or non-finite nu / tau <= 0 / an
 * unknown element / a_nodal with ABDDC_ELEM_Q1 / non-finite a_nodal or
 * u_dirichlet values (host arrays). */
int abddc_assemble(const abddc_problem* prob, const abddc_device* dev, abddc_ctx** out);

/* Section 3: deluxe weights, face eigenproblems (eq. equ-4-8), new edge
 * eigenproblems (eq. equ-5-21) with the SVD/QR edge basis (or the earlier
 * ones, eq. equ-4-8-E, with edge_variant = ABDDC_EDGE_OLD), change of basis,
 * local constrained factorisations and the coarse matrix.  Fills counts
 * (may be NULL).  opts may be NULL (defaults: Theta_F = Theta_E = 10,
 * shared H, deluxe from S, FP64). */
int abddc_setup_coarse_space(abddc_ctx* ctx, const abddc_options* opts, abddc_counts* counts);

/* z = M^{-1} r (Section 3, M_BDDC^{-1}); r, z device vectors of length
 * n_gamma (may not alias). */
int abddc_apply_bddc(abddc_ctx* ctx, const double* r, double* z);

/* z = M^{-1} r as abddc_apply_bddc (same kernels, same result), for callers
 * that cannot allocate device memory during the call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The work
 * vectors (sum_i (n_B,i + n_Pi,i) + 2 n_Pi doubles, each part rounded up to
 * 32) live in a fixed device array of ABDDC_NOALLOC_SCRATCH_DOUBLES doubles
 * (16 MiB) per GPU, held from the first call on that GPU until the process
 * ends; the call makes no allocation, no host-device copy and records no
 * event.  Every call on one GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (two host threads, or two streams whose work
 * runs concurrently) race and give undefined results; calls ordered on one
 * stream are safe.  Returns ABDDC_EINVAL when the work vectors do not fit,
 * ABDDC_ESTATE before setup. */
#define ABDDC_NOALLOC_SCRATCH_DOUBLES (1 << 21)
int abddc_apply_bddc_noalloc(abddc_ctx* ctx, const double* r, double* z);

/* y = Shat x = sum_i R_i^T S^(i) R_i x (the operator of eq.
 * Schur-complex-sys); device vectors of length n_gamma (may not alias). */
int abddc_apply_schur(abddc_ctx* ctx, const double* x, double* y);

/* Copies ghat (device, length n_gamma) into g. */
int abddc_get_rhs(abddc_ctx* ctx, double* g);

/* Right-preconditioned restarted GMRES(restart) on the Schur system from
 * u = 0 (Section 4 stopping rule: ||ghat - Shat u|| <= rtol ||ghat|| or maxit
 * Arnoldi steps), then interior recovery u_I = A_II^{-1}(f_I - A_IB u_B).
 * u: device vector of length n_dof (full solution).  info may be NULL.
 * restart must be in [1, 63].  Returns ABDDC_NOT_CONVERGED when maxit is
 * reached first. */
int abddc_gmres_solve(abddc_ctx* ctx, int32_t restart, double rtol, int32_t maxit,
                      double* u, abddc_solve_info* info);

/* Sizes of an assembled context; any pointer may be NULL. */
int abddc_query(const abddc_ctx* ctx, int64_t* n_dof, int64_t* n_gamma, int32_t* n_sub,
                int32_t* n_face, int32_t* n_edge);

/* Parity hook: copies an intermediate into the HOST buffer buf (capacity
 * cap doubles).  Returns the number of doubles of the item (>= 0; nothing
 * is written when it exceeds cap) or a negative error code.
 *   ABDDC_STAGE_SCHUR      S^(index), n_B x n_B row-major
 *   ABDDC_STAGE_LOCAL_RHS  g^(index)
 *   ABDDC_STAGE_FACE_EIG   mu = 1/lambda of face index (ascending)
 *   ABDDC_STAGE_EDGE_EIG   mu = 1/lambda of edge index (ascending; (m-1) n_E
 *                          values for the new eigenproblem, n_E for the old)
 *   ABDDC_STAGE_FACE_BASIS [Q_F | Q_F^perp] of face index, n_F x n_F row-major
 *   ABDDC_STAGE_EDGE_BASIS [Q_E | Q_E^perp] of edge index, n_E x n_E row-major
 *   ABDDC_STAGE_COUNTS     per face p_F then per edge r_E (as doubles)
 *   ABDDC_STAGE_DELUXE     D of object index/8, member index%8 of n(X)
 *   ABDDC_STAGE_SUB_SIZES  n_I, n_B, n_Pi of subdomain index (interior,
 *                          interface and primal unknowns; n_Pi is 0 before
 *                          the coarse-space setup) */
enum {
  ABDDC_STAGE_SCHUR = 0,
  ABDDC_STAGE_LOCAL_RHS = 1,
  ABDDC_STAGE_FACE_EIG = 2,
  ABDDC_STAGE_EDGE_EIG = 3,
  ABDDC_STAGE_FACE_BASIS = 4,
  ABDDC_STAGE_EDGE_BASIS = 5,
  ABDDC_STAGE_COUNTS = 6,
  ABDDC_STAGE_DELUXE = 7,
  ABDDC_STAGE_SUB_SIZES = 8
};
int64_t abddc_get_stage(abddc_ctx* ctx, int32_t stage, int32_t index, double* buf, int64_t cap);

/* Per-phase device times of the last setup / solve in seconds (HIP events
 * on the context stream): [0] assemble, [1] local Schur, [2] deluxe,
 * [3] face stage, [4] edge stage, [5] change of basis + local factors,
 * [6] coarse, [7] GMRES iterations, [8] recovery.  n <= 16. */
int abddc_phase_times(const abddc_ctx* ctx, double* t, int32_t n);

/* Live per-kernel statistics accumulated over the context's lifetime from
 * HIP events recorded around each launch on the context stream:
 *   ABDDC_KSTAT_PLU_UPDATE  final trailing Schur product of the blocked
 *                           partial LU on MFMA (work = algorithmic flops,
 *                           2 m n k)
 *   ABDDC_KSTAT_GEMV        batched GEMV of M^{-1} and Shat (work =
 *                           algorithmic bytes: matrix + gathered input + output)
 *   ABDDC_KSTAT_PLU_LEAD    per-group MFMA update of the still-to-be-factored
 *                           rows and columns of the blocked partial LU
 *                           (work = algorithmic flops, 2 m n depth)
 *   ABDDC_KSTAT_PLU_DIAG    LU of the 64 x 64 diagonal blocks with their
 *                           lookahead update (work = 2/3 b^3 + 2 b^2 depth)
 *   ABDDC_KSTAT_PLU_TRSM    triangular solves of each panel's row and column
 *                           strips (work = algorithmic bytes: every strip
 *                           entry read and written once, 16 b per strip row /
 *                           column, plus the two b x b inverses read)
 *   ABDDC_KSTAT_PLU_BAND    update of the next panel's strips inside a panel
 *                           group (work = algorithmic flops, 2 m n depth)
 * Any output pointer may be NULL. */
enum {
  ABDDC_KSTAT_PLU_UPDATE = 0,
  ABDDC_KSTAT_GEMV = 1,
  ABDDC_KSTAT_PLU_LEAD = 2,
  ABDDC_KSTAT_PLU_DIAG = 3,
  ABDDC_KSTAT_PLU_TRSM = 4,
  ABDDC_KSTAT_PLU_BAND = 5
};
int abddc_kernel_stats(abddc_ctx* ctx, int32_t kernel, double* seconds, int64_t* launches, double* work);

/* Which of the classes above are timed, process-wide: bit k (1 << k) times
 * class k on every context from the next launch on; returns the previous
 * mask (bits beyond the last class are ignored).  Default: every class.  A
 * timed launch carries its start and stop events, which adds a few
 * microseconds between it and the next kernel on the stream, so a caller
 * that needs no statistics clears the mask; untimed classes report no
 * launches. */
uint32_t abddc_set_kernel_stats(uint32_t mask);

void abddc_destroy(abddc_ctx* ctx);

/* Allocations the library's own caching device allocator has served on a
 * device since the process started (count and bytes requested), for
 * checking that a binding with allocation hooks routes every allocation
 * through them.  Either pointer may be NULL; EINVAL for device < 0 or
 * >= 64. */
int abddc_cache_stats(int32_t device, int64_t* allocations, int64_t* bytes);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* abddc_last_error(void);

/* ---- Learned edge constraints (library extension of the edge
 * eigenproblem, eq. equ-5-21 and equ-5-22) ----
 * A network predicts, for every edge of n_E = 7 dofs, the projector
 * P = Q_E Q_E^T onto the span of the primal constraint vectors the exact
 * edge eigenproblem would select (Q_E: first r_E columns of the edge basis).
 * Features (ABDDC_MLP_FEATURES per edge, float): log10 nu on the 4 x 4 x 8
 * element tube around the edge in the edge frame (along-axis bins x first
 * transverse axis x second transverse axis, transverse axes in cyclic order
 * after the edge axis, element ranges resampled to 8 bins along the edge),
 * asinh of the velocity at the edge midpoint in that frame (transverse,
 * transverse, along), log10 of the mean and the maximum element Peclet
 * number h_max |a| / nu over the tube.
 * Network: 133 -> 128 (ReLU) -> 128 (ReLU) -> 28; bfloat16 weights and
 * layer inputs on MFMA with FP32 accumulation, FP32 biases.  Outputs: the
 * upper triangle of P-hat, row-major with the diagonal.  Parameters (FP32,
 * ABDDC_MLP_PARAMS): W1 (128 x 133 row-major), b1, W2 (128 x 128), b2,
 * W3 (28 x 128), b3.  Loss: mean over the batch of ||P-hat - P||_F^2;
 * optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 weights.
 * Gate (setup with ABDDC_CONSTRAINTS_MLP): an edge is solved exactly when
 * n_E != 7, when an eigenvalue of P-hat lies in [0.3, 0.7], or when one of
 * its features lies outside the training range widened by 10 % on each
 * side; otherwise its constraint basis is the eigenvectors of P-hat with
 * eigenvalue > 1/2, completed by QR.  A network is tied to the device of
 * its creation; it is not thread-safe. */
#define ABDDC_MLP_FEATURES 133
#define ABDDC_MLP_OUTPUTS 28
#define ABDDC_MLP_PARAMS 37276
typedef struct abddc_mlp abddc_mlp;

/* Network with the given FP32 parameters (HOST array of ABDDC_MLP_PARAMS),
 * Adam moments zero.  EINVAL on a wrong count or null pointers. */
int abddc_mlp_create(const float* params, int32_t n_params, const abddc_device* dev, abddc_mlp** out);
/* Copies the FP32 parameters to a HOST array. */
int abddc_mlp_get_params(abddc_mlp* mlp, float* params, int32_t n_params);
/* Y (n x 28) = network(X (n x 133)); DEVICE pointers, stream-ordered on
 * the network's stream (returns after the launch). */
int abddc_mlp_forward(abddc_mlp* mlp, const float* X, int32_t n, float* Y);
/* Loss (HOST scalar) and gradient (DEVICE array in the parameter layout) of
 * the batch (X n x 133, targets T n x 28, DEVICE); synchronises. */
int abddc_mlp_loss_grad(abddc_mlp* mlp, const float* X, const float* T, int32_t n, float* grad, float* loss);
/* One Adam step on the batch; loss (HOST, may be NULL) before the step.
 * Synchronises only when loss is requested. */
int abddc_mlp_train_step(abddc_mlp* mlp, const float* X, const float* T, int32_t n, float lr, float* loss);
/* Records the per-feature [min, max] of the training features X (DEVICE,
 * n x 133) for the gate. */
int abddc_mlp_set_ranges(abddc_mlp* mlp, const float* X, int32_t n);
void abddc_mlp_destroy(abddc_mlp* mlp);

/* Features of every edge of the context (edge kind order) into X (DEVICE,
 * n_edge x 133); eligible (DEVICE int32 per edge, may be NULL) is 1 for
 * edges of n_E = 7 dofs (features of other edges are still written).
 * Trilinear boxes on box partitions only (EINVAL for ABDDC_ELEM_P1 or a
 * general partition); so is constraint_source = ABDDC_CONSTRAINTS_MLP in
 * abddc_setup_coarse_space. */
int abddc_edge_features(abddc_ctx* ctx, float* X, int32_t* eligible);
/* Training targets after a setup: the projector upper triangles of the
 * context's edge bases (DEVICE, n_edge x 28; zeros for n_E != 7). */
int abddc_edge_projectors(abddc_ctx* ctx, float* Y);
/* Edges of the last setup whose constraints came from the network / from
 * the exact eigenproblem. */
int abddc_learned_stats(const abddc_ctx* ctx, int32_t* n_predicted, int32_t* n_exact);

/* ---- Primitive test hooks (batched kernels the setup is built from) ----
 * Batched partial LU without pivoting, in place, on row-major matrices that
 * live in one DEVICE buffer: matrix b starts at buf + off[b] (host array),
 * has nrow[b] rows, ncol[b] columns, leading dimension ld[b], and its first
 * k[b] pivots are eliminated, leaving the Schur complement
 * A22 - A21 A11^{-1} A12 in rows/cols >= k[b], U/L factors in front.
 * precision: 0 = FP64 (buf is double*), 1 = FP32 (buf is float*).
 * Returns ABDDC_ESINGULAR on a zero or non-finite pivot. */
int abddc_test_partial_lu(int32_t batch, void* buf, const int64_t* off, const int32_t* nrow,
                          const int32_t* ncol, const int32_t* ld, const int32_t* k,
                          int32_t precision, void* stream);

/* Batched C_b = alpha op(A_b) op(B_b) + beta C_b on row-major FP64 DEVICE
 * matrices inside one buffer; offsets in doubles (host arrays); trans*
 * nonzero means the transpose.  Used to test the MFMA tile kernel. */
int abddc_test_gemm(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                    const int64_t* offC, const int32_t* m, const int32_t* n, const int32_t* k,
                    const int32_t* lda, const int32_t* ldb, const int32_t* ldc, int32_t transA,
                    int32_t transB, double alpha, double beta, void* stream);

/* Batched symmetric-definite generalized eigenproblem A y = mu B y with B
 * SPD, n x n row-major FP64 DEVICE matrices in one buffer (A at offA[b], B
 * at offB[b], ld = n[b]); writes mu ascending to buf + offW[b] and X = L Y
 * (B = L L^T, Y orthonormal eigenvectors of L^{-1} A L^{-T}) to
 * buf + offX[b].  Returns ABDDC_EEIG if B is not positive definite. */
int abddc_test_sygv(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                    const int64_t* offW, const int64_t* offX, const int32_t* n, void* stream);

/* As abddc_test_sygv, but only the columns of X whose eigenvalue is
 * <= sel are written (the rest of X is left as it was): the solver the face
 * and edge eigenproblems of eq. equ-4-8 and equ-5-21 use, which need only
 * those eigenvectors.  Tridiagonalisation, bisection, inverse iteration. */
int abddc_test_sygv_select(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                           const int64_t* offW, const int64_t* offX, const int32_t* n, double sel,
                           void* stream);

/* Batched Schur complement with a pseudo-inverse, in place: for each
 * nv[b] x nv[b] row-major FP64 DEVICE matrix M at buf + off[b] (ld nv[b]),
 * the trailing block becomes M22 - M21 (sym M11)^+ M12, M11 the leading
 * k[b] x k[b] block, the pseudo-inverse dropping eigenvalues <= rtol
 * lambda_max (the eliminations of the face and edge operators, Section 3,
 * whose eliminated blocks may be singular).  Leading rows/columns are
 * scratch afterwards.  Returns ABDDC_ESINGULAR when a block with
 * k[b] > 128 is not positive definite and well conditioned. */
int abddc_test_schur_pinv(int32_t batch, double* buf, const int64_t* off, const int32_t* nv, const int32_t* k,
                          double rtol, void* stream);

/* Batched parallel sum of the face operators (Section 3, face part):
 * out_b = sym(A_b (A_b + B_b)^+ B_b), the pseudo-inverse dropping
 * eigenvalues <= rtol lambda_max of sym(A_b + B_b).  n x n row-major FP64
 * DEVICE matrices in one buffer (A at offA[b], B at offB[b], out at
 * offOut[b], ld = n[b], 1 <= n[b] <= 128).  A well-conditioned A + B takes
 * an LU path, the rest an eigenvalue path; both give the definition. */
int abddc_test_parallel_sum(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                            const int64_t* offOut, const int32_t* n, double rtol, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ABDDC_H */
