/*
 * tpfdm -- batched tensor-product operators and their fast-diagonalization
 * inverse on AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2609.04534, "Adaptive Multilevel Discontinuous Galerkin
 * Methods on GPUs".  The library implements, for a batch of independent
 * hexahedral blocks (cells or patches) of tensor-product degree p, n = p+1
 * points per direction:
 *
 *   apply          v = (P_x (x) M_y (x) M_z + M_x (x) P_y (x) M_z
 *                       + M_x (x) M_y (x) P_z) u              Sec. 3.1, eq. (eval_pipeline)
 *   apply_inverse  x = D^{-1} r by fast diagonalization        Sec. 5.2, eq. (cell_block)
 *   solve          D x = b by block-local iterative refinement with a
 *                  low-precision fast-diagonalization inner solve
 *
 * with per-direction factors M_d = h_d M_hat, P_d = P_hat / h_d on a block of
 * edge lengths (h_x, h_y, h_z) (Sec. 2: every Cartesian cell is a scaled
 * translate of the reference cube).  P_hat is either the 1D stiffness K_hat
 * ("Neumann" volume operator) or A_hat = K_hat + the own-side blocks of both
 * SIPG face stencils with penalty C p(p+1)/h (eq. (face_coupling), Sec. 5.2,
 * Sec. 6.2).  The basis is the Lagrange basis on the n Gauss-Lobatto points
 * of [0, 1]; M_hat and K_hat are its exact integrals.
 *
 * Vector layout (Sec. 2, blocked storage [B, n_x, n_y, n_z, n_e]): group g of
 * a plan occupies elements [offset, offset + tiles * n^3 * B) of every vector
 * buffer, with tiles = ceil(nblocks / B).  Block b of the group lives in tile
 * t = b / B at lane l = b % B, and its DoF q = (i_x n + i_y) n + i_z is
 * element  offset + (t * n^3 + q) * B + l.  B is a power of two; B = 1 is the
 * plain block-contiguous (node-major) order.  Lanes of the last tile beyond
 * nblocks are padding: they are never read as input and never written.
 *
 * Conventions shared by every call:
 *  - Every pointer named "device" must be device memory (hipMalloc or torch);
 *    the caller owns all vectors.  The plan owns its own copies of the block
 *    metadata and all workspace.
 *  - Calls taking a stream are asynchronous on that stream; argument errors
 *    are returned synchronously, errors of a kernel surface at the caller's
 *    next synchronisation (and as TP_ERR_HIP from later calls).
 *  - Outputs are overwritten, never accumulated.  Input and output buffers
 *    must not alias.
 *  - No call aborts or prints.  On error the call returns a negative status
 *    and tp_last_error() returns a message (thread-local); the one positive
 *    status, TP_PENDING, is not an error.
 *  - A plan may be used from one host thread at a time; distinct plans are
 *    independent.
 */
#ifndef TPFDM_H
#define TPFDM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TP_OK = 0,
    TP_ERR_ARG = -1,           /* invalid argument (null, size, layout, value)     */
    TP_ERR_UNSUPPORTED = -2,   /* n, dtype, layout or mode not supported            */
    TP_ERR_NOT_SPD = -3,       /* Cholesky of the 1D mass matrix failed             */
    TP_ERR_SINGULAR = -4,      /* min eigenvalue sum <= tol * max (e.g. Neumann)    */
    TP_ERR_NOT_CONVERGED = -5, /* some block missed rtol within maxit               */
    TP_ERR_NONFINITE = -6,     /* NaN/Inf in an input or a residual                 */
    TP_ERR_HIP = -7,           /* a HIP runtime call failed                         */
    TP_ERR_OOM = -8,           /* device allocation failed                          */
    TP_ERR_STATE = -9,         /* call out of order (e.g. inverse before setup)     */
    TP_PENDING = 1             /* tp_pcg_poll: the solve is still running (no error) */
} tp_status;

typedef enum { TP_F64 = 0, TP_F32 = 1, TP_F16 = 2, TP_BF16 = 3 } tp_dtype;

/* Which 1D operator P_hat fills the Kronecker sum. */
typedef enum {
    TP_OP_NEUMANN = 0,  /* P_hat = K_hat: the volume operator of eq. (eval_pipeline); A 1 = 0 */
    TP_OP_CELL = 1,     /* P_hat = A_hat: the SIPG cell block of eq. (cell_block); SPD        */
    TP_OP_SIPG = 2,     /* mesh plans only: the coupled SIPG operator A = A^vol + A^face of
                           eq. (sipg) / eq. (operator_split) over the whole mesh        */
    TP_OP_SIPG_FACE = 3 /* mesh plans only: its face part A^face (interior and boundary
                           faces); TP_OP_NEUMANN on a mesh plan is A^vol             */
} tp_operator;

/* How per-block eigenfactors are represented (Sec. 5.2).
 * SCALED: one generalized eigenproblem P_hat S = M_hat S Lambda per degree; a
 *   block with lengths h_d uses S_d = S_hat / sqrt(h_d), lambda_d =
 *   lambda_hat / h_d^2, the exact eigen-decomposition of its own pair
 *   (P_hat/h_d, h_d M_hat).  Only for groups given by edge lengths.
 * GENERAL: one eigenproblem P_d S_d = M_d S_d Lambda_d per block and
 *   direction (3 nblocks problems of n x n), stored per block: for groups
 *   given by their own factors, and for length groups from (P_hat/h_d,
 *   h_d M_hat), where it agrees with SCALED up to rounding. */
typedef enum { TP_FACTOR_SCALED = 0, TP_FACTOR_GENERAL = 1 } tp_factor_mode;

/* One group of blocks of equal degree and layout.  A group is given either
 * by edge lengths h (the blocks are axis-aligned boxes and use the reference
 * matrices) or by per-block factors M and P (h null): block b's operator is
 * P_x (x) M_y (x) M_z + M_x (x) P_y (x) M_z + M_x (x) M_y (x) P_z with the
 * pairs (M_d, P_d) = (M[b][d], P[b][d]), d = x, y, z. */
typedef struct {
    int32_t n;            /* points per direction, 2 <= n <= 8 (degree p = n-1)       */
    int32_t layout_B;     /* interleave width B, a power of two, 1 <= B <= 1024        */
    int64_t nblocks;      /* number of blocks (0 allowed)                             */
    const double* h;      /* [nblocks][3] edge lengths (x, y, z), host or device,
                             finite and > 0; copied into the plan at creation;
                             null for a factor group                                 */
    int64_t offset;       /* first element of the group in every vector buffer        */
    const double* M;      /* factor group: [nblocks][3][n][n] row-major per-direction
                             mass factors, host or device, copied at creation; M_d
                             must be symmetric positive definite for the inverse    */
    const double* P;      /* factor group: [nblocks][3][n][n] operator factors (the
                             stiffness K or the penalized cell operator A)           */
} tp_group;

/* Kernel mapping of a group's blocks onto the wavefront. */
typedef enum {
    TP_MAP_AUTO = 0,      /* lane-per-block for n <= 4, wave-per-tile otherwise; the
                             solve goes lane-per-block only for groups of at least
                             one 64-block tile per SIMD (smaller ones spread wider) */
    TP_MAP_LANE = 1,      /* one block per lane (n <= 4), for the solve too            */
    TP_MAP_WAVE = 2       /* one wave per tile of blocks, pencils staged through LDS   */
} tp_mapping;

/* What the blocks of a plan are.
 * CELLS: each block is one cell of degree n-1 (the reference pair of
 *   the n-point Gauss-Lobatto Lagrange basis).
 * PATCHES: each block is a vertex patch, the 2 x 2 x 2 cells of degree
 *   n/2 - 1 around a mesh vertex (n even, 4 <= n <= 8; groups given by the
 *   cell lengths h, which all eight cells share).  Per direction the patch
 *   holds two cells: the reference mass is blockdiag(M_hat, M_hat), the
 *   Neumann operator blockdiag(K_hat, K_hat) (the cells' volume operators),
 *   and TP_OP_CELL the patch block of the SIPG operator: the cell block
 *   A_hat of each cell (interior stencil) and the coupling blocks of the
 *   face between them (eq. (face_coupling)), penalty C p(p+1) with the
 *   cells' p.  The patch operator is the SIPG operator of a Cartesian mesh
 *   restricted to the patch's eight cells (Sec. 6.1 names such vertex-patch
 *   local solves); apply_inverse and solve are its exact local solve by
 *   fast diagonalization.  DoF order per direction: cell 0's points, then
 *   cell 1's. */
typedef enum { TP_BLOCKS_CELLS = 0, TP_BLOCKS_PATCHES = 1 } tp_blocks;

typedef struct {
    double penalty_C;     /* SIPG penalty constant C of sigma = C p(p+1)/h (default 2) */
    int32_t persistent;   /* 1: every call runs as ONE launch over all groups (its
                             solve uses wave-per-tile bodies for every degree)      */
    int32_t mapping;      /* tp_mapping for apply / apply_inverse                      */
    int32_t blocks;       /* tp_blocks (default TP_BLOCKS_CELLS); not for mesh plans  */
    int32_t reserved[5];  /* must be zero                                             */
} tp_plan_opts;

typedef struct {
    int32_t max_iters;    /* largest per-block iteration count                        */
    int32_t n_failed;     /* blocks that missed rtol                                  */
    double max_relres;    /* largest per-block final ||b - D x||_2 / ||b||_2          */
} tp_solve_summary;

typedef struct tp_plan tp_plan;

/* Default options: C = 2, non-persistent, automatic mapping. */
void tp_plan_opts_default(tp_plan_opts* opts);

/* Create a plan over ngroups groups on the current HIP device (the batch of
 * independent cell or patch blocks of Sec. 2, each a scaled reference cell
 * whose operator is the sum-factorized form of Sec. 3.1,
 * eq. (eval_pipeline)).  Validates the
 * groups (n, B, sizes, non-overlapping element ranges, h finite and > 0),
 * copies h into plan-owned device memory, builds the 1D reference matrices
 * for every degree used, and allocates the solve workspace.  Host-synchronous.
 * Errors: TP_ERR_ARG, TP_ERR_UNSUPPORTED, TP_ERR_OOM, TP_ERR_HIP. */
tp_status tp_plan_create(const tp_group* groups, int32_t ngroups,
                         const tp_plan_opts* opts, tp_plan** out);

/* A uniform Cartesian box mesh (Sec. 3): cells[0] x cells[1] x cells[2]
 * axis-aligned cells, all with edge lengths h, degree n-1 in every cell,
 * homogeneous Dirichlet data imposed weakly by the SIPG (Nitsche) terms on
 * the boundary faces (eq. (sipg), penalty C p(p+1)/h_F with h_F the cell
 * length normal to the face, Sec. 6.2).  Cell (cx, cy, cz) is block
 * c = (cx cells[1] + cy) cells[2] + cz of the plan's single group, so the B
 * cells of a layout tile are consecutive along z. */
/* The 1D basis of every cell's coefficients (Sec. 3.1).
 * LAGRANGE: Lagrange polynomials on the n Gauss-Lobatto points of [0, 1]
 *   (coefficients = nodal values).
 * HERMITE: the Hermite-type basis of eq. (hermite_conditions), mesh plans
 *   with n >= 4 (p >= 3; TP_ERR_UNSUPPORTED for n < 4, and for n = 4 with
 *   TP_MAP_WAVE): coefficient 0 is the value and 1 the derivative at 0,
 *   n-2 the derivative and n-1 the value at 1, so a face term reads two
 *   layers of the neighbour (eq. (hermite_traces_3d)).  The endpoint
 *   functions are the cubic Hermite polynomials, the interior ones bubbles
 *   x^2 (1-x)^2 times Lagrange polynomials on the interior nodes of the
 *   (n-2)-point Gauss-Lobatto rule.  The coupled operator, tp_setup_inverse,
 *   PCG and tp_change_basis act on coefficients in this basis (the same
 *   discrete space and operator: A_H = T3^T A_L T3 with T3 = T (x) T (x) T
 *   cell by cell, T[i][j] = psi_j(x_i)); with n = 4 also the block calls
 *   (tp_apply with a block operator, tp_apply_inverse, tp_solve, graphs)
 *   and multigrid, which return TP_ERR_UNSUPPORTED for n >= 5. */
typedef enum { TP_BASIS_LAGRANGE = 0, TP_BASIS_HERMITE = 1 } tp_basis;

typedef struct {
    int32_t n;            /* points per direction, 2 <= n <= 8                          */
    int32_t layout_B;     /* interleave width, a power of two <= 1024                    */
    int32_t cells[3];     /* cells per direction (x, y, z), each >= 1, product < 2^31    */
    int32_t basis;        /* tp_basis (0: Lagrange)                                      */
    double h[3];          /* cell edge lengths (x, y, z), finite and > 0                 */
} tp_mesh;

/* Create a plan over the cells of a mesh: one group of cells[0] cells[1]
 * cells[2] blocks (offset 0) whose blocks all have the lengths h.  Every
 * block call works on it as on any plan (TP_OP_CELL: the cell blocks, whose
 * inverse is the block-Jacobi preconditioner of Sec. 5.2, with the interior
 * stencil on boundary cells); in addition tp_apply takes TP_OP_SIPG and
 * TP_OP_SIPG_FACE, which couple neighbouring cells.  opts->persistent must
 * be 0 (TP_ERR_UNSUPPORTED).  Host-synchronous.  Errors as tp_plan_create. */
tp_status tp_plan_create_mesh(const tp_mesh* mesh, const tp_plan_opts* opts, tp_plan** out);

/* Free everything the plan owns.  Null is accepted. */
tp_status tp_plan_destroy(tp_plan* plan);

/* Number of elements every vector buffer must hold:
 * max over groups of offset + ceil(nblocks/B) * n^3 * B.  -1 on a null plan. */
int64_t tp_plan_vector_elems(const tp_plan* plan);

/* Total degrees of freedom sum_g nblocks_g * n_g^3 (padding excluded). */
int64_t tp_plan_ndof(const tp_plan* plan);

/* v <- A u for every block of every group, in dtype (storage and contraction
 * operands); FP64 accumulates in FP64, the others in FP32.  u, v: device
 * buffers of tp_plan_vector_elems() elements of dtype.  Sec. 3.1,
 * eq. (eval_pipeline) with P_hat chosen by op (length groups); factor groups
 * use their own P and ignore op.
 * TP_OP_SIPG / TP_OP_SIPG_FACE (mesh plans, TP_F64 and TP_F32, every n;
 * TP_ERR_UNSUPPORTED for FP16/BF16): v <- A u with the coupled operator,
 * every cell's row reading its face neighbours' blocks of u. */
tp_status tp_apply(tp_plan* plan, tp_operator op, const void* u, void* v,
                   tp_dtype dtype, hipStream_t stream);

/* Fast-diagonalization setup for the operator op (TP_OP_NEUMANN or
 * TP_OP_CELL; the coupled operators have no such inverse) (Sec. 5.2): Cholesky
 * M = L L^T, symmetric Jacobi eigen-decomposition of L^{-1} P L^{-T},
 * S = L^{-T} Q, in FP64 on the host: per degree (SCALED) or per block and
 * direction (GENERAL, host threads; P symmetrized as (P + P^T)/2 first).
 * op selects P_hat for length groups; factor groups use their own P and
 * need GENERAL (TP_ERR_UNSUPPORTED with SCALED); a persistent plan supports
 * SCALED only.  Fails with
 * TP_ERR_SINGULAR when the smallest eigenvalue sum of a block is <=
 * singular_tol times its largest (the Neumann operator, whose constants are
 * in the null space), TP_ERR_NOT_SPD when a mass factor is not SPD; the
 * message names the first offending block.  singular_tol <= 0 selects
 * 1e-12.  Host-synchronous; a failed setup leaves the plan without an
 * inverse (TP_ERR_STATE from later inverse calls). */
tp_status tp_setup_inverse(tp_plan* plan, tp_operator op, tp_factor_mode mode,
                           double singular_tol);

/* x <- D^{-1} r = (S (x) S (x) S) Lambda^{-1} (S (x) S (x) S)^T r for every
 * block: six 1D contractions and one diagonal scaling (Sec. 5.2).  Lambda^{-1}
 * is formed in FP64 for TP_F64 and FP32 otherwise.  Requires tp_setup_inverse
 * (TP_ERR_STATE otherwise).  r, x: device, dtype, tp_plan_vector_elems(). */
tp_status tp_apply_inverse(tp_plan* plan, const void* r, void* x, tp_dtype dtype,
                           hipStream_t stream);

/* Solve D x = b for every block, D the cell block of Sec. 5.2,
 * eq. (cell_block), whose exact inverse is the fast diagonalization of
 * tp_apply_inverse; by iterative refinement, one launch per group (one in
 * all for a persistent plan):
 *   r = b - D x (FP64);  s = ||r||_inf;  d = D~^{-1}(r/s) in `inner` precision;
 *   x <- x + s d  (FP64)
 * until ||r||_2 / ||b||_2 <= rtol or maxit corrections.  inner: TP_F64 and
 * TP_F32 compute the inner fast diagonalization in that precision; TP_F16 and
 * TP_BF16 round r/s and d to that format and compute in FP32 (as
 * tp_apply_inverse does for vectors stored in it).  A block with b = 0
 * gets x = 0 and 0 iterations.  b, x: device FP64 vectors; x holds the initial
 * guess on entry and the best iterate on exit.  iters (int32) and relres
 * (double): optional device arrays of tp_plan_ndof-order block count (groups
 * in order, blocks in order), may be null.  summary: optional host struct,
 * filled after one synchronisation of the stream (only when non-null).
 * Returns TP_ERR_NOT_CONVERGED when summary is requested and some block
 * failed; TP_ERR_NONFINITE when a residual became NaN/Inf. */
tp_status tp_solve(tp_plan* plan, const double* b, double* x, tp_dtype inner,
                   double rtol, int32_t maxit, int32_t* iters, double* relres,
                   tp_solve_summary* summary, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tp_solve
 * with the same arguments, kernels and results (bit for bit), except that
 * the per-workgroup partial summaries and the reduced summary go to a
 * static device workspace of the library (a file-scope device array of
 * 384 KiB + 256 B, one per GPU, held until the process ends) instead of the
 * plan's workspace.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine; the plan, b and x are the caller's).  It
 * rejects, with TP_ERR_ARG and before any launch, plans whose solve may
 * need more than 16384 partial summaries (a bound of one per tile, at most
 * 8192 per group's launch on a 256-CU device).  Every call on a GPU shares
 * that GPU's workspace and overwrites it: calls that overlap on one GPU
 * (other streams or threads) race, and tp_solve_summary_fetch does not see
 * these solves (pass summary instead). */
tp_status tp_solve_static(tp_plan* plan, const double* b, double* x, tp_dtype inner,
                          double rtol, int32_t maxit, int32_t* iters, double* relres,
                          tp_solve_summary* summary, hipStream_t stream);

/* The summary (max iterations, failures, max relative residual) of the most
 * recent tp_solve on this plan, including solves replayed from a graph.
 * Synchronises the stream.  Returns TP_ERR_NOT_CONVERGED / TP_ERR_NONFINITE
 * like tp_solve when the recorded solve had such blocks. */
tp_status tp_solve_summary_fetch(tp_plan* plan, tp_solve_summary* summary, hipStream_t stream);

/* HIP graphs of single calls, for replay in launch-bound loops.  A graph
 * records the kernels of ONE call on a private capture stream: what = APPLY
 * (v = A u with `op`), INVERSE (x = D^{-1} r) or SOLVE (block-local
 * refinement with `inner` precision, no host summary; fetch it with
 * tp_solve_summary_fetch).  The buffers, dtype and solve parameters are baked
 * into the graph: replay reads `in` and overwrites `out` as the call would.
 * With a persistent plan (opts.persistent = 1) each graph holds one kernel
 * node over all groups, otherwise the per-group kernels in order.  The plan
 * must outlive its graphs.  Nothing is allocated at replay. */
typedef enum { TP_GRAPH_APPLY = 0, TP_GRAPH_INVERSE = 1, TP_GRAPH_SOLVE = 2 } tp_graph_op;
typedef struct tp_graph tp_graph;
tp_status tp_graph_create(tp_plan* plan, tp_graph_op what, tp_operator op, tp_dtype dtype, const void* in,
                          void* out, double rtol, int32_t maxit, int32_t* iters, double* relres,
                          tp_graph** graph);
tp_status tp_graph_launch(tp_graph* graph, hipStream_t stream);
tp_status tp_graph_destroy(tp_graph* graph);

/* Layout helpers: convert between the canonical order (groups in order, each
 * group's blocks contiguous as [nblocks][n^3]) and the plan's blocked layout.
 * Pure data movement of elements of the given dtype; the canonical buffer has
 * tp_plan_ndof() elements.  Padding lanes of the blocked buffer are written
 * as zero by tp_pack. */
tp_status tp_pack(tp_plan* plan, const void* canonical, void* blocked, tp_dtype dtype,
                  hipStream_t stream);
tp_status tp_unpack(tp_plan* plan, const void* blocked, void* canonical, tp_dtype dtype,
                    hipStream_t stream);

/* Autotuning of the kernel choice per group (the mapping of blocks onto the
 * wavefront and the tile grid): for every group of a non-persistent plan and
 * the given storage dtype, times apply (Neumann), apply_inverse (when set up
 * in SCALED mode) and the FP64-inner solve (when set up for TP_OP_CELL) with
 * every applicable variant -- one block per lane (n <= 4), one wave per tile
 * with the full or half occupancy grid or one workgroup per tile, MFMA
 * (n = 8 FP16/BF16, B = 1) -- on
 * plan-sized scratch vectors of pseudo-random values, and keeps the fastest
 * per group and call for later calls in that dtype (the solve's choice for
 * every inner precision).  us: optional host array [ngroups][3] that receives
 * the best average microseconds per launch (apply, apply_inverse, solve; -1
 * where not measured).  reps <= 0 selects 10.  Host-synchronous; allocates
 * and frees its scratch.
 * For a persistent plan it tunes the single launch of each call instead
 * (apply and apply_inverse in dtype, the solve with inner precision dtype):
 * per group the tile body (one block per lane for n <= 4, or one wave per
 * tile) and the tiles each workgroup runs (1, 2, 4, 8), the order of the
 * groups' segments in the launch, and the solve's grid (occupancy grid,
 * half of it, one workgroup per work item), by coordinate descent over
 * whole-launch timings (at least 30 launches each), keeping the default when
 * the tuned choice is not faster.  us[0..2] then receive the single
 * launch's times, the rest -1.  Tile bodies and per-tile arithmetic are
 * those of the per-group launches, so results are unchanged bit for bit.
 * Graphs capture the launch configuration current at their creation: create
 * them after tuning. */
tp_status tp_plan_autotune(tp_plan* plan, tp_dtype dtype, int32_t reps, double* us);

/* Kernel family a call would use for a group in dtype, in the low 4 bits:
 * 0 one block per lane, 1 one wave per tile, 2 MFMA, 3 per-block factors
 * (GENERAL); for apply / apply_inverse with one wave per tile, bits 4-7 hold
 * the grid (1 full occupancy grid, 2 half, 0 one workgroup per tile).  call
 * 0 apply, 1 apply_inverse, 2 solve (dtype ignored).  MFMA assumes 16-byte
 * aligned vectors.  For a persistent plan (dtype = the storage type, for the
 * solve the inner precision): bits 0-3 the tile body (0 lane, 1 wave), bits
 * 4-7 the solve grid (1 occupancy grid, 2 half, 0 one workgroup per item),
 * bits 8-11 log2 of the tiles per workgroup, bits 12-27 the position of the
 * group's segment in the launch.  -1 for an invalid argument. */
int32_t tp_plan_group_kernel(const tp_plan* plan, int32_t group, int32_t call, tp_dtype dtype);

/* Preconditioned conjugate gradients for the coupled SIPG system A x = b of
 * a mesh plan (every n), FP64 throughout except the preconditioner: the
 * cell-wise fast-diagonalization block-Jacobi z = D^{-1} r of Sec. 5.2 (the
 * cell blocks of eq. (cell_block), interior stencil on every cell), applied
 * in `inner` precision (TP_F64, or TP_F32 on the FP64 vectors).  Needs
 * tp_setup_inverse(plan, TP_OP_CELL, TP_FACTOR_SCALED, ...) first
 * (TP_ERR_STATE).  tp_pcg_create allocates the solver's workspace (five
 * plan-sized FP64 vectors, the iterate included, and the reduction
 * partials); the plan must outlive it.  The first solve in each `inner`
 * precision captures a chunk of check_every iterations into a HIP graph that
 * later solves replay (iterations are enqueued as graph launches).  tp_pcg_solve: b, x device FP64 vectors in the plan's layout; x is the
 * initial guess unless x_is_zero (then x is overwritten with zero first) and
 * holds the last iterate on return (x is written only at the end).  b = 0
 * with x_is_zero gives x = 0 at once; b = 0 with a non-zero guess cannot meet
 * the relative test and runs to maxit.  Stops when ||r||_2 <= rtol ||b||_2 for
 * the recursively updated residual r, or after maxit iterations
 * (TP_ERR_NOT_CONVERGED), or on a breakdown / non-finite value
 * (TP_ERR_NONFINITE).  Every iteration runs on the device without host
 * synchronisation; the host reads the solver state once per check_every
 * iterations (<= 0 selects 16), so up to check_every - 1 iterations' kernels
 * run after convergence and return at once.  Synchronises the stream before
 * returning; summary (optional) receives the iterations, whether it
 * converged and the final relative residual.  One solve at a time per
 * solver object. */
typedef struct {
    int32_t iterations;
    int32_t converged;
    double relres;
} tp_pcg_summary;
typedef struct tp_pcg tp_pcg;
tp_status tp_pcg_create(tp_plan* plan, tp_pcg** out);
tp_status tp_pcg_solve(tp_pcg* pcg, const double* b, double* x, int32_t x_is_zero, tp_dtype inner, double rtol,
                       int32_t maxit, int32_t check_every, tp_pcg_summary* summary, hipStream_t stream);
tp_status tp_pcg_destroy(tp_pcg* pcg);

/* The same solve without blocking, for callers that keep several solves in
 * flight (each solver object on its own stream).  tp_pcg_begin checks the
 * arguments like tp_pcg_solve, enqueues the start on stream and returns.
 * Each tp_pcg_poll call returns TP_PENDING while the last enqueued step is
 * still running or after it has enqueued the next one (a chunk of
 * check_every iterations, or the copy of the result into x), and, once the
 * copy has finished, the solve's final status (as tp_pcg_solve's) with
 * summary filled.  poll never waits.  While a solve is running the solver
 * accepts no other solve (TP_ERR_STATE), and b and x must stay untouched by
 * the caller until poll returns its final status. */
tp_status tp_pcg_begin(tp_pcg* pcg, const double* b, double* x, int32_t x_is_zero, tp_dtype inner, double rtol,
                       int32_t maxit, int32_t check_every, hipStream_t stream);
tp_status tp_pcg_poll(tp_pcg* pcg, tp_pcg_summary* summary);

/* Geometric multigrid for the coupled system of a mesh plan (n <= 4 with the
 * default layout B = 64; n = 5..8 with the default layout B = 1, in the
 * Lagrange basis, on one-cell-per-wave kernels): the V-cycle the paper uses
 * to precondition CG (Sec. 5, Sec. 6.1).
 * Levels: the mesh and its uniform coarsenings (cells halved while all three
 * counts are even, lengths doubled, each level's own operator); per level
 * one pre- and one post-smoothing application of the degree-three
 * Chebyshev-accelerated block-Jacobi method on [0.2, 2]
 * (eq. (chebyshev_weights), eq. (chebyshev_richardson): three Richardson
 * updates with the cell-block fast-diagonalization inverse); transfers by
 * polynomial embedding into the eight children and its transpose; the
 * coarsest level (at most 2048 unknowns) solved with a dense inverse
 * assembled once by applying its operator to unit vectors and kept for the
 * life of the process (shared by hierarchies with the same coarsest level).
 * For n >= 5, when the coarsest geometric level has more than 2048
 * unknowns, one more level of degree 1 on the same cells (at most 256
 * cells) is the one solved densely: reached by the cellwise embedding E of
 * the trilinear polynomials into degree p and its transpose, with the
 * Galerkin operator E^T A E.  A larger coarsest level is TP_ERR_UNSUPPORTED.  Needs tp_setup_inverse(TP_OP_CELL,
 * TP_FACTOR_SCALED) on the plan (TP_ERR_STATE).  tp_mg_create allocates the
 * level vectors (host-synchronous); the plan must outlive the object, and
 * every V-cycle (alone or inside a solve) returns TP_ERR_STATE unless the
 * plan's current inverse setup is still TP_OP_CELL, TP_FACTOR_SCALED; tp_mg_vcycle enqueues x <- V(b) (FP64
 * smoothing; b, x: distinct device vectors of the plan's layout, x
 * overwritten, TP_ERR_ARG when null or equal).  The level vectors are the
 * object's scratch: one V-cycle at a time per object, and a solver that uses
 * it counts as its user for the whole solve (give concurrent solvers their
 * own objects).  tp_pcg_set_multigrid makes later solves of that solver use
 * one V-cycle as the preconditioner, with the smoother's block inverse in
 * the solve's `inner` precision; null restores block-Jacobi; TP_ERR_ARG for
 * a multigrid of another plan, TP_ERR_STATE during a non-blocking solve; a
 * multigrid is destroyed only after its solvers are destroyed or reset. */
/* Stopping test of tp_pcg_* solves (default TP_PCG_RESIDUAL):
 * RESIDUAL: ||r||_2 <= rtol ||b||_2 with the recursively updated residual;
 * PRECONDITIONED: the preconditioned residual norm <r, z>^{1/2} has
 *   decreased by the factor rtol from its initial value (the rule of
 *   Sec. 6.1; invariant under a change of basis).
 * tp_pcg_set_norm applies to later solves of that solver (TP_ERR_STATE
 * during a non-blocking solve, TP_ERR_ARG for another value).  The summary's
 * relres is ||r||_2 / ||b||_2 under either test. */
typedef enum { TP_PCG_RESIDUAL = 0, TP_PCG_PRECONDITIONED = 1 } tp_pcg_norm;
tp_status tp_pcg_set_norm(tp_pcg* pcg, int32_t norm);

typedef struct tp_mg tp_mg;
tp_status tp_mg_create(tp_plan* plan, tp_mg** out);
/* The same hierarchy with its level vectors (right-hand sides, corrections,
 * residual scratch, on every level) stored in `storage`: TP_F64 (as
 * tp_mg_create) or TP_F32, which halves the bytes every smoothing, transfer
 * and coarse kernel moves.  With TP_F32 the operator rows of the smoothing
 * updates and of the residual are computed in FP32 as well, the smoother's
 * block inverse in the solve's inner precision, the transfers and the
 * degree-1 coarsest level (n >= 5) in FP64; values are rounded to FP32
 * where a level vector is stored.  A V-cycle first rounds b into the finest
 * FP32 right-hand side; tp_mg_vcycle writes x back in FP64, and inside
 * tp_pcg_* solves the preconditioned residual z stays in FP32 (the CG
 * recurrences, x, r, p and every dot product remain FP64: (r, z) and
 * p = z + beta p read z in FP32).  TP_ERR_UNSUPPORTED for other types. */
tp_status tp_mg_create_typed(tp_plan* plan, tp_dtype storage, tp_mg** out);
tp_status tp_mg_vcycle(tp_mg* mg, const double* b, double* x, hipStream_t stream);
tp_status tp_mg_destroy(tp_mg* mg);
tp_status tp_pcg_set_multigrid(tp_pcg* pcg, tp_mg* mg);

/* Change of basis of a mesh plan's vectors (Sec. 3.1: the fixed n x n
 * matrix T per direction, used when interfacing with nodal data, e.g. for
 * output or right-hand-side evaluation), cell by cell, by mode (to_nodal):
 *   1  v = (T (x) T (x) T) u: coefficients to nodal values;
 *   0  v = (T^{-1} (x) T^{-1} (x) T^{-1}) u: nodal values to coefficients;
 *   2  v = (T^T (x) T^T (x) T^T) u: a load vector assembled against the
 *      nodal (Lagrange) basis to one against this basis (b_H = T3^T b_L).
 * u, v: distinct FP64 device vectors in the plan's layout (padding lanes are
 * not written).  On a Lagrange plan T = I and v is a copy of u.  Errors:
 * TP_ERR_ARG (null, aliasing, mode not 0/1/2), TP_ERR_UNSUPPORTED (not a
 * mesh plan). */
tp_status tp_change_basis(tp_plan* plan, int32_t to_nodal, const double* u, double* v, hipStream_t stream);

/* Number of blocks in the plan (sum over groups). */
int64_t tp_plan_nblocks(const tp_plan* plan);

/* Host-side reference data (no GPU needed), for inspection and tests:
 * M_hat, K_hat and A_hat of the n-point GLL basis (row-major n x n host
 * arrays, any may be null), with penalty constant C. */
tp_status tp_reference_matrices(int32_t n, double penalty_C, double* M, double* K,
                                double* A);

/* Host-side reference data of a plan's blocks (no GPU needed): the tables a
 * plan with this basis (tp_basis) and block kind (tp_blocks) uses, row-major
 * n x n host arrays, any may be null.  M_hat, K_hat (the volume operator)
 * and A_hat (the cell or patch block operator), and T, the change of basis
 * (nodal values = T * coefficients; the identity for the Lagrange basis).
 * Errors: TP_ERR_ARG (values), TP_ERR_UNSUPPORTED (the combinations plans
 * reject: Hermite-type basis for n < 4 or for patches, patches with odd n). */
tp_status tp_reference_basis(int32_t n, int32_t basis, int32_t blocks, double penalty_C, double* M,
                             double* K, double* A, double* T);

/* Host-side generalized eigen-decomposition P_hat S = M_hat S diag(lam) with
 * S^T M_hat S = I, eigenvalues ascending, each column's largest-magnitude
 * entry positive.  S: row-major n x n host array (column j = eigenvector j),
 * lam: n host doubles. */
tp_status tp_reference_eigen(int32_t n, double penalty_C, tp_operator op, double* S,
                             double* lam);

/* Message of the last failing call on this host thread ("" if none). */
const char* tp_last_error(void);

/* Library version string. */
const char* tp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TPFDM_H */
