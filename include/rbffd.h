/*
 * rbffd.h -- C ABI of the MI355X (gfx950) staggered-node PHS+poly RBF-FD
 * Navier-Stokes library.
 *
 * Method: Chu & Schmidt, "RBF-FD discretization of the Navier-Stokes
 * equations on scattered but staggered nodes".  The library generates local
 * RBF-FD stencil weights (Sec. 2.1-2.2), stores them as fixed-width ELL
 * sparse operators, and applies them every time step of the semi-implicit
 * fractional-step scheme of Sec. 3 (AB2 advection, Crank-Nicolson viscous
 * step, pressure projection with Kim-Moin intermediate boundary values).
 *
 * Conventions (all calls):
 *  - Every call returns rbf_status: RBF_OK (0) or a negative error code and
 *    never aborts; rbf_last_error() returns a message for the calling thread,
 *    valid until that thread's next call.
 *  - Pointers documented as "device" are HIP device allocations (for example
 *    torch tensors on a ROCm device); "host" pointers are ordinary memory.
 *    The caller owns every buffer it passes; the library never frees or
 *    reallocates caller memory.  A solver handle owns only its internal
 *    copies and workspace, released by rbf_solver_destroy().
 *  - Node coordinates are structure-of-arrays: x[2][n] holds all x first,
 *    then all y (FP64).
 *  - ELL operators are slot-major: entry s of row r is at [s * rows + r];
 *    idx is int32 (column index into the source node set), weights FP64
 *    (or FP32 where stated).  Sizes are int64.
 *  - rbf_stream is a hipStream_t passed as an opaque pointer (NULL = the
 *    default stream).  All device work of a call is ordered on that stream;
 *    calls do not synchronise the device except where stated (setup calls
 *    that read back a few scalars, and the solver calls that read back
 *    convergence flags).
 *  - Operator codes (bit mask, outputs in increasing bit order):
 *    RBF_OP_ID = 1 (interpolation, L = identity), RBF_OP_DX = 2 (d/dx),
 *    RBF_OP_DY = 4 (d/dy), RBF_OP_LAP = 8 (Laplacian).
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rbf_status;
#define RBF_OK 0
#define RBF_E_ARG (-1)      /* invalid argument (sizes, pointers, parameters) */
#define RBF_E_SINGULAR (-2) /* a local saddle-point system is singular        */
#define RBF_E_NOCONV (-3)   /* Krylov solve hit its iteration cap             */
#define RBF_E_DEVICE (-4)   /* HIP runtime error                              */
#define RBF_E_NOMEM (-5)    /* device allocation failed                       */
#define RBF_E_NAN (-6)      /* non-finite value in a Krylov solve             */

#define RBF_OP_ID 1u
#define RBF_OP_DX 2u
#define RBF_OP_DY 4u
#define RBF_OP_LAP 8u

#define RBF_ABI_VERSION 5

typedef void *rbf_stream;

/* Message describing the last error on the calling thread ("" if none). */
const char *rbf_last_error(void);

/* RBF_ABI_VERSION of the loaded library. */
int32_t rbf_abi_version(void);

/*
 * rbf_build_nodes -- seeded staggered node sets (host only, no device work).
 *
 * Stand-in for the DistMesh grids of Sec. 3.  kind 0: lid-driven cavity on
 * the unit square with the paper's staggering: P-nodes are the vertices
 * (i/K, j/K), i, j = 0..K, of a triangulation whose interior vertices are
 * jittered by U(-jitter/K, jitter/K) per coordinate, V-nodes are the
 * midpoints of all triangle edges (cell diagonals alternate in a checkerboard);
 * N = 3K^2 + 2K, M = (K+1)^2.  kind 1: operator-bench square, N = M = K^2,
 * V on jittered cell centres ((i+1/2)/K, (j+1/2)/K), P on jittered vertices
 * (i/K, j/K), i, j = 0..K-1, no walls.  kind 2: lid-driven cavity on a
 * near-equilateral triangulation (the kind of grid DistMesh produces): P rows
 * y_j = j/R, j = 0..R, R = floor(2K/sqrt(3) + 1/2); walls at rows 0 and R
 * (x = i/K) and at the ends of every row; even interior rows x = i/K,
 * i = 1..K-1, odd ones x = (i+1/2)/K, i = 0..K-1; interior vertices at least
 * 1.5/K from every wall (unjittered position) jittered by
 * U(-jitter/K, jitter/K) per coordinate; edges: each row's horizontal edges
 * and, between consecutive rows, the strip triangulation that merges the two
 * rows in order of unjittered x (ties advance the lower row); V-nodes on the
 * edge midpoints, ordered by row (horizontal edges, then that row's strip
 * edges in merge order); N/M about 3; jitter <= 0.4.
 * Random numbers: SplitMix64 as a
 * counter-based generator (draw c of stream g uses counter (g << 40) | c;
 * stream 0 = V, 1 = P; draws 2n and 2n+1 jitter node n).
 *
 * Two-call pattern: pass NULL for every array to obtain *n_v and *n_p, then
 * call again with host arrays of that size:
 *   xv [2][n_v], v_tag [n_v] (0 interior, 1 wall, 2 lid = top wall),
 *   xp [2][n_p], p_tag [n_p] (0 interior, 1 wall),
 *   p_normal [2][n_p] (outward unit normal of wall P-nodes, 0 elsewhere).
 * Errors: RBF_E_ARG for an unknown kind, K < 2 (cavities) or K < 1 (square),
 * jitter outside [0, 0.45] (kind 2: [0, 0.4]), or a partial set of NULL
 * arrays.
 */
rbf_status rbf_build_nodes(int32_t kind, int32_t K, double jitter, uint64_t seed,
                           int64_t *n_v, double *xv, int8_t *v_tag,
                           int64_t *n_p, double *xp, int8_t *p_tag, double *p_normal);

/*
 * rbf_knn -- n-nearest-neighbour stencils (Sec. 2.2: row r of D^(alpha,beta)
 * uses the k nearest beta-nodes of the alpha-node r; Sec. 4 uses k = 28).
 *
 * xq: device [2][nq] query (alpha) nodes; xs: device [2][ns] source (beta)
 * nodes; idx: device int32 [k][nq], slot-major output.  The stencil is the
 * first k source nodes in the order of the key (d^2, index), with
 * d^2 = dx*dx + dy*dy in FP64 with separately rounded products (no fused
 * multiply-add), so ties are broken by the lower index and the result is a
 * unique function of the inputs.  When alpha = beta and nodes are distinct,
 * slot 0 is the node itself.  Synchronises the stream twice (bounding box,
 * end of the search).  Device scratch (cell grid, about 34 bytes per source)
 * is allocated and freed inside the call.
 * Errors: RBF_E_ARG if k < 1, k > 64, k > ns, nq < 0, ns < 1, a NULL
 * pointer with a non-zero size, or a NaN or infinite coordinate in either
 * node set (checked before any search, so no stencil is written);
 * RBF_E_NOMEM / RBF_E_DEVICE for allocation or device failures.
 */
rbf_status rbf_knn(const double *xq, int64_t nq, const double *xs, int64_t ns, int32_t k,
                   int32_t *idx, rbf_stream st);

/*
 * rbf_knn_noalloc -- rbf_knn for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as rbf_knn; the cell grid
 * lives in a fixed per-device scratch array of 64 MiB (held by each device
 * the library runs on until the process ends), so no allocation or
 * deallocation happens in the call.  Capacity: about 30 bytes per source
 * node, i.e. at most about 2.2 million sources; larger ns is refused with
 * RBF_E_ARG (message naming the limit) before any search.  Every call on a
 * device shares that device's array: calls that overlap on one GPU (two
 * host threads, or two streams) race and must be serialised by the caller.
 * Synchronises the stream twice, like rbf_knn.
 */
rbf_status rbf_knn_noalloc(const double *xq, int64_t nq, const double *xs, int64_t ns, int32_t k,
                           int32_t *idx, rbf_stream st);

/*
 * rbf_assemble_weights -- local PHS+poly RBF-FD weights (Sec. 2.1, eqs. (3)-(9)).
 *
 * For each query node r, solves the augmented saddle-point system
 *   [A P; P^T 0] [w; c] = [L phi; L P]
 * with A_ij = ||x_i - x_j||^m (m odd), P the (q+1)(q+2)/2 monomials of degree
 * <= q (graded order 1; x, y; x^2, xy, y^2; ...), and right-hand sides L
 * applied to phi(||x - x_j||) and to the monomials at x = x_r, for every
 * operator in op_mask at once; w (the first k unknowns) is kept, c is
 * discarded.  Coordinates are shifted to x_r and divided by the power of two
 * s = 2^e with 1/4 <= max_j |x_j - x_r|^2 / s^2 < 1 (exact); weights are
 * returned in physical units (local weights times s^-order).  Each system is
 * solved by LU with partial pivoting in FP64 followed by one step of
 * iterative refinement with a double-FP64 residual.
 *
 * xq: device [2][nq]; xs: device [2][ns]; idx: device int32 [k][nq] (from
 * rbf_knn); w: device FP64 [popcount(op_mask)][k][nq], operators in
 * increasing bit order.  cond_est: NULL, or device FP64 [nq] that receives
 * an estimate of the 1-norm condition number ||A_aug||_1 ||A_aug^-1||_1 of
 * each local system in the shifted and scaled coordinates it is solved in
 * (the conditioning studied in Sec. 4): ||A_aug||_1 exactly, times Hager's
 * lower estimate of ||A_aug^-1||_1 with Higham's safeguards (LAPACK xLACON's
 * method; usually exact, never above the true value up to rounding, and
 * within a factor of a few in practice), computed from the same LU factors
 * with at most 11 extra triangular solves per row; NaN for rows reported
 * bad.  bad_row: host, set to the lowest row whose system was numerically
 * singular or non-finite, -1 if none (synchronises the stream to read it
 * back).
 * Limits: 1 <= k, k + (q+1)(q+2)/2 <= 64, q in [-1, 5] (-1: no polynomials),
 * m odd in [1, 11] (m >= 3 for derivative operators), and
 * k >= (q+1)(q+2) (stability rule of Sec. 4) unless op_mask has bit 31 set.
 * Errors: RBF_E_ARG for violated limits or an empty op_mask;
 * RBF_E_SINGULAR if any row failed: a numerically singular or non-finite
 * system, or a stencil index outside [0, ns) (tested before any load
 * through it); the weights of such a row are NaN.
 */
#define RBF_FORCE_SMALL_STENCIL 0x80000000u
rbf_status rbf_assemble_weights(const double *xq, int64_t nq, const double *xs, int64_t ns,
                                const int32_t *idx, int32_t k, int32_t m, int32_t q,
                                uint32_t op_mask, double *w, double *cond_est, int64_t *bad_row,
                                rbf_stream st);

/*
 * rbf_ell_apply -- y = D x for one ELL operator (eq. (10) applied to a vector).
 *
 * rows: number of rows; k: entries per row; idx: device int32 [k][rows];
 * w: device [k][rows]; x: device vector indexed by idx; y: device [rows].
 * dtype 0: w, x, y FP64, FP64 accumulation; dtype 1: w, x, y FP32, FP32
 * accumulation.  Launch shape: the one rbf_ell_autotune recorded for this
 * (dtype, k, rows), else the default.  No synchronisation.  Errors:
 * RBF_E_ARG for bad sizes/dtype.
 */
rbf_status rbf_ell_apply(int64_t rows, int32_t k, const int32_t *idx, const void *w,
                         const void *x, void *y, int32_t dtype, rbf_stream st);

/*
 * rbf_ell_autotune -- choose the launch shape of rbf_ell_apply for one
 * operator size by timing (for the 28-wide operators of Sec. 4; other
 * widths keep the default shape).  Shapes: block size 64, 128, 256 or
 * 512 threads (one row per thread) x blocks remapped to one contiguous row
 * range per XCD or not x operator loads non-temporal or not; shape 0 is the
 * default (256, remapped, non-temporal).  Every shape sums each row in the
 * same order, so results are bit-identical across shapes.  Each shape runs
 * once untimed and `reps` times timed with HIP events on `st`; the fastest
 * (the lower shape on ties) is recorded for (dtype, k, rows) in a
 * process-wide table that later rbf_ell_apply calls of that size use.
 * Arguments as rbf_ell_apply (y is overwritten); shape: host, the chosen
 * shape; ms: NULL or host [16], the mean time per application of each
 * shape (-1 where not timed).  Synchronises the stream.  Errors: RBF_E_ARG
 * (sizes, dtype, reps outside [1, 10000], NULL), RBF_E_DEVICE.
 */
rbf_status rbf_ell_autotune(int64_t rows, int32_t k, const int32_t *idx, const void *w,
                            const void *x, void *y, int32_t dtype, int32_t reps, int32_t *shape,
                            float *ms, rbf_stream st);

/*
 * rbf_cast_f32 -- dst[i] = (float)src[i] (round to nearest) for i < n; used
 * to build FP32-stored copies of ELL weights and vectors.  src: device FP64
 * [n]; dst: device FP32 [n].  No synchronisation.  Errors: RBF_E_ARG.
 */
rbf_status rbf_cast_f32(const double *src, float *dst, int64_t n, rbf_stream st);

/*
 * rbf_ell_transpose -- column structure of D^T for one ELL operator, the
 * transposed product that adjoints of the steps of Sec. 3 apply (the rows of
 * D^T are the columns of eq. (10)'s matrix: z_c = sum of w_{r,s} y_r over
 * the entries (s, r) with idx[s][r] == c).
 *
 * rows, k, idx: the ELL operator as for rbf_ell_apply (device int32
 * [k][rows]); ncols: number of columns (every idx must lie in [0, ncols)).
 * Outputs (device, caller-allocated): colptr int64 [ncols + 1] (column c
 * holds entries colptr[c] .. colptr[c+1]-1); src int32 [k * rows] (source
 * row r of each entry) and slot int32 [k * rows] (its slot s), ordered by
 * increasing (r, s) inside each column.  Every ELL entry appears once,
 * zero weights included, so the structure serves every weight array of the
 * same idx (FP64 or FP32, permuted by rbf_ell_transpose_weights).
 * bad_entry: host; -1, or the lowest ELL position s * rows + r whose index
 * is outside [0, ncols).  Synchronises the stream twice (the range and
 * column-length check, and the end of the build) and allocates a workspace
 * of ncols ints for the duration of the call.  Limits: k in [1, 64],
 * rows * k < 2^31, ncols < 2^31, at most 4096 entries per column.
 * Errors: RBF_E_ARG for violated limits or an index out of range (outputs
 * then undefined); RBF_E_NOMEM / RBF_E_DEVICE from the runtime.
 */
rbf_status rbf_ell_transpose(int64_t rows, int32_t k, const int32_t *idx, int64_t ncols,
                             int64_t *colptr, int32_t *src, int32_t *slot, int64_t *bad_entry,
                             rbf_stream st);

/*
 * rbf_ell_transpose_weights -- one weight array of the operator in the
 * column order of rbf_ell_transpose: wt[e] = w[slot[e]][src[e]] for
 * e < k * rows (a gather, once per weight array, so that transposed
 * products read their weights contiguously).
 *
 * rows, k: the ELL operator; src, slot: from rbf_ell_transpose (device
 * int32 [k * rows]); w: device [k][rows]; wt: device [k * rows], caller-
 * allocated.  dtype 0: FP64 w and wt; 1: FP32.  No synchronisation.
 * Errors: RBF_E_ARG for bad sizes, dtype or NULL pointers.
 */
rbf_status rbf_ell_transpose_weights(int64_t rows, int32_t k, const int32_t *src,
                                     const int32_t *slot, const void *w, void *wt, int32_t dtype,
                                     rbf_stream st);

/*
 * rbf_ell_apply_transpose -- z = D^T y: z_c = sum over the entries e of
 * column c (colptr[c] <= e < colptr[c+1], from rbf_ell_transpose) of
 * wt[e] * y[src[e]] (wt from rbf_ell_transpose_weights).  One wavefront
 * per 64 consecutive columns walks their contiguous entries in chunks with
 * coalesced loads, stages the products wt[e] * y[src[e]] in LDS, and each
 * lane adds its column's products in entry order; no atomics, so results
 * are reproducible bit for bit.
 *
 * y: device [rows] of the operator; z: device [ncols] (columns without
 * entries get 0); src, wt and y may be NULL for an operator without rows.
 * dtype 0: FP64 wt, y, z; 1: FP32 (FP32 accumulation).
 * No synchronisation.  Errors: RBF_E_ARG for bad sizes, dtype or NULL
 * pointers.
 */
rbf_status rbf_ell_apply_transpose(int64_t ncols, const int64_t *colptr, const int32_t *src,
                                   const void *wt, const void *y, void *z, int32_t dtype,
                                   rbf_stream st);

/* ---------------------------------------------------------------------------
 * Fractional-step solver (Sec. 3).
 * ------------------------------------------------------------------------- */

/* V-node tags with a boundary condition other than Dirichlet values (the
 * channel of Sec. 5.2; every boundary row enters u** through the Kim-Moin
 * form of eq. (21), u** = u_bc^{j+1} + dt D^VP p~_j, with u_bc^{j+1}):
 *   RBF_VTAG_OUTFLOW   convective outflow dq/dt + u_conv dq/dx = 0 for
 *                      q = u, v, explicit Euler from step j:
 *                      q_bc = q_j - dt u_conv (D_x^VV q_j);
 *   RBF_VTAG_SYMMETRY  v_bc = 0 and u_bc from du/dy = 0: the node's own
 *                      D_y^VV row solved for its value with the neighbours'
 *                      values at step j.
 * Any other non-zero tag is a Dirichlet row with the values u_bc, v_bc
 * given to rbf_solver_create (inflow, no slip, a moving lid). */
#define RBF_VTAG_OUTFLOW 4
#define RBF_VTAG_SYMMETRY 5

/* Node sets and boundary data, all device memory. */
typedef struct {
    int64_t n_v, n_p;
    const double *xv;       /* [2][n_v]                                      */
    const double *xp;       /* [2][n_p]                                      */
    const int8_t *v_tag;    /* [n_v]: 0 interior, RBF_VTAG_OUTFLOW,
                               RBF_VTAG_SYMMETRY, other != 0 Dirichlet     */
    const int8_t *p_tag;    /* [n_p]: 0 interior, != 0 wall (Neumann)        */
    const double *p_normal; /* [2][n_p] outward unit normal at wall P-nodes  */
} rbf_grid;

/* The eight operators of Sec. 4 plus D_x, D_y on (P,P) for the pressure
 * boundary rows; device memory, slot-major [k][rows].  The solver copies
 * them at creation, so the caller may free them afterwards. */
typedef struct {
    int32_t k;
    const int32_t *idx_vv; const double *vv_dx, *vv_dy, *vv_lap; /* rows n_v, cols n_v */
    const int32_t *idx_pv; const double *pv_dx, *pv_dy;          /* rows n_p, cols n_v */
    const int32_t *idx_pp; const double *pp_dx, *pp_dy, *pp_lap; /* rows n_p, cols n_p */
    const int32_t *idx_vp; const double *vp_dx, *vp_dy;          /* rows n_v, cols n_p */
} rbf_ops;

typedef struct {
    double re;        /* Reynolds number                                     */
    double dt;        /* time step                                           */
    double rtol_h;    /* relative residual tolerance, Helmholtz solves       */
    double rtol_p;    /* relative residual tolerance, pressure Poisson solve */
    int32_t maxit_h;  /* iteration caps                                      */
    int32_t maxit_p;
    int32_t precision;/* RBF_PRECISION_*                                     */
    int32_t precond;  /* pressure-solve preconditioner, RBF_PRECOND_*        */
    double u_conv;    /* convection velocity of RBF_VTAG_OUTFLOW rows        */
} rbf_params;

/* rbf_params.precision:
 * FP64   every stage in FP64;
 * MIXED  with the lattice preconditioner: its transforms and tridiagonal
 *        solves stored in FP32 (FP32 matrix cores), everything else FP64;
 *        with the auxiliary-lattice preconditioner: FP32 inside FP64
 *        iterative refinement -- each restart cycle of the pressure solve
 *        forms the residual b - A x in FP64 from the FP64 weights, runs
 *        flexible GMRES on FP32-stored weights, vectors and transforms (FP64
 *        dot products) until the residual drops by 1e-4 or the cycle ends,
 *        and adds the correction to the FP64 iterate.  The viscous solve,
 *        when H's Jacobi bound is at most 0.25 (rbf_solver_query), is FP32
 *        inside FP64 refinement too: each outer step forms b - H x in FP64,
 *        runs two FP32 Jacobi sweeps on FP32-stored weights for the
 *        correction and adds it to the FP64 iterate; otherwise it stays
 *        FP64.  The weights, the outer residuals, the projection and the
 *        tolerances stay FP64, so the fields differ from FP64 runs at the
 *        tolerance level. */
#define RBF_PRECISION_FP64 0
#define RBF_PRECISION_MIXED 1

/* rbf_params.precond:
 * AUTO     the lattice preconditioner when the P-nodes form a jittered
 *          (K+1)^2 lattice of the unit square (the cavity layout of
 *          rbf_build_nodes kind 0) with K <= 513; else the auxiliary-lattice
 *          preconditioner when the P-nodes' bounding box is a square;
 *          none otherwise;
 * NONE     unpreconditioned BiCGSTAB on the row-scaled system;
 * LATTICE  the lattice preconditioner, RBF_E_ARG if the P-nodes are not
 *          such a lattice or K > 513;
 * AUX      the auxiliary-lattice preconditioner, RBF_E_ARG if the bounding
 *          box is not a square.
 * The lattice preconditioner is the 5-point Laplacian of the unjittered
 * lattice with one-sided Neumann rows, inverted exactly by a fast Poisson
 * solve (DCT-II along x as dense products on the matrix cores, tridiagonal
 * solves along y), followed by bilinear interpolation to the node
 * positions; BiCGSTAB iterates with it.
 * The auxiliary-lattice preconditioner (any node set in a square) is a
 * two-level method: an l1-Jacobi sweep (damping 2) on the stored Poisson
 * rows, the
 * residual restricted (normalised bilinear weights, interior nodes to
 * interior lattice points) to a lattice of about one node spacing per cell
 * and solved there by the same fast Poisson solve with homogeneous Neumann
 * rows, interpolated back with the border's constant, and a second sweep;
 * flexible GMRES (restart 30) iterates with it.  Neither changes the
 * system solved. */
#define RBF_PRECOND_AUTO 0
#define RBF_PRECOND_NONE 1
#define RBF_PRECOND_LATTICE 2
#define RBF_PRECOND_AUX 3

/* Solver state at step j, device memory owned by the caller. */
typedef struct {
    double *u, *v;             /* [n_v] velocity                             */
    double *p_tilde, *p;       /* [n_p] pressure correction and pressure     */
    double *cu_prev, *cv_prev; /* [n_v] advection terms C_{j-1} (AB2)        */
    int64_t step;              /* j; the AB2 start uses C_{-1} = C_0 at j=0 */
} rbf_state;

typedef struct {
    int32_t iterations;    /* BiCGSTAB iterations (or Jacobi sweeps)        */
    int32_t converged;     /* 1 if the tolerance was met                    */
    double rel_residual;   /* ||b - A x|| / ||b|| recomputed at the end     */
    int32_t restarts;      /* restarts after a BiCGSTAB breakdown           */
    int32_t final_flag;    /* 0 running, 1 converged, -1 non-finite, 2 breakdown */
} rbf_solve_stats;

typedef struct {
    int32_t steps_done;            /* steps committed by this call          */
    int32_t status;                /* status of the last step attempted     */
    int64_t helmholtz_iters;       /* summed over steps (both components)   */
    int64_t poisson_iters;         /* summed over steps                     */
    rbf_solve_stats last_helmholtz_u, last_helmholtz_v, last_poisson;
} rbf_step_stats;

typedef struct rbf_solver rbf_solver;

/*
 * rbf_solver_create -- build the implicit system matrices of Sec. 3.
 *
 * Helmholtz (eq. (16)): H = I - a D_Lap^(V,V), a = dt/(2 Re), on interior
 * V rows, identity on wall rows (which carry the Kim-Moin values of
 * eq. (21)).  When the Jacobi iteration matrix I - D^-1 H (D = diag H) has
 * infinity norm <= 0.25 (small a, as at the paper's time steps on fine
 * grids), H is solved by Jacobi sweeps, whose residual test uses the true
 * residual; otherwise by Jacobi-preconditioned BiCGSTAB.
 * Pressure Poisson (eq. (18)): D_Lap^(P,P) on interior P rows and
 * homogeneous Neumann rows n_x D_x^(P,P) + n_y D_y^(P,P) on wall rows.  The
 * paper states no pressure boundary condition; with Neumann rows the
 * constants are a null vector and F/dt is in general not compatible, so the
 * system is bordered: a uniform source lam on interior rows absorbs the
 * incompatibility and p~ has zero mean.  It is solved as
 * (A0 + u1 v^T) x = b with the rank-one border, then p~ = x - mean(x); the
 * operator is stored row-scaled (interior rows by -1/||row||_2, wall rows by
 * +1/||row||_2) and iterated by BiCGSTAB, right-preconditioned as chosen by
 * prm->precond; the Poisson tolerance applies to the row-scaled system.
 * u_bc, v_bc: device [n_v] boundary velocities (read on wall rows; copied).
 * The solver keeps `st` for all of its work.
 * Errors: RBF_E_ARG (NULL pointers, sizes, dt/re <= 0, unknown precision,
 * unknown precond, RBF_PRECOND_LATTICE on a non-lattice P-grid, a stencil
 * index outside its source node range (checked on the device before any
 * other use; the message names the array, slot, row and value), a self
 * index missing from a (V,V) or (P,P) stencil, no interior P node),
 * RBF_E_NOMEM, RBF_E_DEVICE.
 */
rbf_status rbf_solver_create(rbf_solver **out, const rbf_grid *grid, const rbf_ops *ops,
                             const double *u_bc, const double *v_bc, const rbf_params *prm,
                             rbf_stream st);

/*
 * rbf_step -- advance `state` by nsteps steps of Sec. 3, eqs. (14)-(21).
 *
 * Transactional: each step is computed in solver workspace and committed
 * only if every solve converged and stayed finite; on error `state` holds the
 * last committed step and stats (host, nullable) says where it stopped.
 * Reads back a convergence flag every few Krylov iterations (synchronises).
 * Errors: RBF_E_ARG, RBF_E_NOCONV, RBF_E_NAN, RBF_E_DEVICE.
 */
rbf_status rbf_step(rbf_solver *s, int32_t nsteps, rbf_state *state, rbf_step_stats *stats);

/*
 * rbf_step_batch -- advance `count` independent instances (solvers[b] with
 * states[b]) by nsteps steps each, concurrently.  The method is that of
 * rbf_step, per instance; the instances run on nthreads host threads
 * (nthreads <= 0: 8; never more than count), each taking the next instance
 * in order and driving rbf_step on the stream its solver was created with,
 * so that the work of instances on distinct streams overlaps on the device.
 * Results are those of calling rbf_step on each instance alone.
 * solvers: host [count] distinct handles; states: host [count];
 * stats (nullable): host [count]; statuses (nullable): host [count], each
 * instance's rbf_step status.  Every instance is attempted; a failed one
 * keeps its last committed step (rbf_step is transactional).
 * Returns RBF_OK, or the status of the lowest-numbered failed instance, whose
 * message rbf_last_error reports on the calling thread.
 * Errors: RBF_E_ARG (NULL or repeated handle, count or nsteps < 0), and
 * those of rbf_step.
 */
rbf_status rbf_step_batch(rbf_solver *const *solvers, int32_t count, int32_t nsteps,
                          rbf_state *states, rbf_step_stats *stats, rbf_status *statuses,
                          int32_t nthreads);

/*
 * rbf_solve_pressure -- solve the bordered pressure-Poisson system of
 * eq. (18) described at rbf_solver_create: D_Lap^PP p~ + lam = rhs on
 * interior rows, n . grad p~ = rhs on wall rows, mean(p~) = 0.  rhs: device
 * [n_p]; p_tilde: device [n_p], initial guess in, zero-mean solution out.
 * stats nullable.  Synchronises.  Errors: RBF_E_ARG, RBF_E_NOCONV, RBF_E_NAN.
 */
rbf_status rbf_solve_pressure(rbf_solver *s, const double *rhs, double *p_tilde,
                              rbf_solve_stats *stats);

/*
 * rbf_solver_apply_precond -- apply the pressure preconditioner once, z =
 * P^-1 y: the lattice preconditioner J (L5 + chi c 1^T)^-1 D^-1, or the
 * auxiliary-lattice two-level preconditioner (both described at
 * rbf_params.precond; D: the row scale of the stored Poisson rows).  For
 * tests and diagnostics.  y, z: device [n_p], distinct.  Synchronises the
 * solver's stream.  Errors: RBF_E_ARG (NULL, no preconditioner, or the
 * auxiliary-lattice preconditioner of a mixed-precision solver).
 */
rbf_status rbf_solver_apply_precond(rbf_solver *s, const double *y, double *z);

/*
 * rbf_solver_profile -- sample kernel durations of the pressure solve on the
 * solver's stream:
 *   RBF_PROF_GEMM    the first transform of the lattice preconditioner or of
 *                    the auxiliary lattice (k_pc_gemm<0>, an n x n x n FP64
 *                    or FP32 product, n = cells per side - 1);
 *   RBF_PROF_SPMV    the Krylov product with the Poisson matrix (k_pc_av with
 *                    the lattice preconditioner, k_kry_a without one, k_fg_av2
 *                    in FGMRES (k_fg_av for stencils other than 28 nodes): the
 *                    product plus the Gram-Schmidt dots);
 *   RBF_PROF_SMOOTH  the post-smoothing product of the auxiliary-lattice
 *                    preconditioner (k_aux_post2; k_aux_post for stencils
 *                    other than 28 nodes);
 *   RBF_PROF_GS      the Gram-Schmidt update of FGMRES (k_fg_gs<2>).
 * A sampled launch goes through hipExtLaunchKernelGGL with an event pair
 * that records the kernel's own start and end; the pairs are read at the
 * solver's next stream synchronisation (no extra synchronisation).
 * Returns in avg_ms[q] and count[q] (nullable host arrays of RBF_PROF_N) the
 * average duration per launch and the number of launches timed so far;
 * then, if sample_every >= 0, resets the counters and samples every
 * sample_every-th iteration from now on (0 disables sampling).
 * Errors: RBF_E_ARG (NULL solver), RBF_E_DEVICE.
 */
#define RBF_PROF_GEMM 0
#define RBF_PROF_SPMV 1
#define RBF_PROF_SMOOTH 2
#define RBF_PROF_GS 3
#define RBF_PROF_N 4
rbf_status rbf_solver_profile(rbf_solver *s, int32_t sample_every, double *avg_ms,
                              int64_t *count);

/*
 * rbf_solver_query -- how the solver runs its solves (host struct, filled):
 * viscous_jacobi 1 when the viscous solve uses Jacobi sweeps (see
 * rbf_solver_create), jacobi_bound the infinity norm of I - D^-1 H that
 * decided it, lattice_precond 1 when the pressure solve uses the lattice
 * preconditioner, viscous_mixed 1 when the viscous solve runs FP32 sweeps
 * inside FP64 iterative refinement (RBF_PRECISION_MIXED with
 * viscous_jacobi set), aux_smooth_weight the weight of the second sweep of
 * each smoothing pair of the auxiliary-lattice preconditioner relative to
 * the first (in [1, 1.6], chosen at creation from the largest eigenvalue of
 * the smoother's operator).  Errors: RBF_E_ARG (NULL argument).
 */
typedef struct {
    int32_t viscous_jacobi;
    int32_t lattice_precond;
    double jacobi_bound;
    int32_t aux_precond;   /* 1: auxiliary-lattice preconditioner with FGMRES */
    int32_t aux_cells;     /* its lattice cells per side (0 if unused)       */
    int32_t viscous_mixed; /* 1: FP32 viscous sweeps inside FP64 refinement  */
    double aux_smooth_weight; /* weight of the second smoothing sweep of each
                                 pair relative to the first (0 if unused)   */
} rbf_solver_info;
rbf_status rbf_solver_query(rbf_solver *s, rbf_solver_info *info);

/*
 * rbf_solver_diagnostics -- per-step health figures of a state (host struct,
 * filled; for logging and for spotting a diverging run):
 *   div_max, div_rms   max and root mean square over interior P-nodes of
 *                      F = D_x^PV u + D_y^PV v (eq. (17) applied to u, v);
 *   kinetic_energy     (1/2) mean over V-nodes of u^2 + v^2 (unweighted);
 *   speed_max          max over V-nodes of sqrt(u^2 + v^2);
 *   cfl                dt * max over V-nodes of sqrt(u^2 + v^2) / d_r, d_r
 *                      the distance to the nearest other node of the node's
 *                      (V,V) stencil.
 * Non-finite velocities give NaN maxima.  state: device u, v [n_v] (the other
 * fields are not read).  Reductions run in a fixed order (repeatable bit for
 * bit).  Synchronises the solver's stream.  Errors: RBF_E_ARG (NULL).
 */
typedef struct {
    double div_max, div_rms, kinetic_energy, speed_max, cfl;
} rbf_diagnostics;
rbf_status rbf_solver_diagnostics(rbf_solver *s, const rbf_state *state, rbf_diagnostics *out);

/*
 * rbf_solver_forces -- force on a circular body (Sec. 5.2: drag and lift of
 * the cylinder): F = closed integral over the body of
 * (-p I + (1/Re)(grad U + grad U^T)) n ds, n the unit normal pointing out of
 * the body, the pressure p of the state (eq. (19)) taken at the P-nodes
 * tagged `tag`, the velocity gradients (D_x^VV, D_y^VV rows) at the V-nodes
 * tagged `tag`; each set is ordered by its angle about (cx, cy) in
 * [0, 2 pi) and integrated by the periodic composite Simpson's rule (4/3
 * and 2/3 of the angle step, 2/3 at the first node, times `radius`), so
 * both counts must be even and the nodes equally spaced in angle.
 * C_D = 2 F_x / (rho U^2 D) and C_L likewise.  grid: the solver's node sets
 * (device; read at the first call and when tag or circle change); state:
 * device u, v, p.  force: host [2] = (F_x, F_y).  Synchronises the solver's
 * stream.  Errors: RBF_E_ARG (NULL argument, sizes differing from the
 * solver's, tag 0, a non-finite circle, odd or zero counts).
 */
rbf_status rbf_solver_forces(rbf_solver *s, const rbf_grid *grid, const rbf_state *state,
                             int32_t tag, double cx, double cy, double radius, double *force);

/*
 * rbf_adjoint_step -- reverse-mode derivative of one rbf_step (the stages of
 * Sec. 3, eqs. (14)-(21), transposed in reverse order), for gradients of an
 * objective of a rollout with respect to the viscosity nu = 1/Re and the
 * wall velocities.
 *
 * fwd: the forward state at step j (device arrays as in rbf_step; read
 * only; fwd->step says whether the AB2 start C_{-1} = C_0 applies).  The
 * call recomputes the forward step j -> j+1 from it (the same solves as
 * rbf_step), so a rollout needs only checkpointed states.
 * adj (in/out): on entry the adjoints of the state at j+1 -- u, v, p_tilde
 * the adjoints of u_{j+1}, v_{j+1}, p~_{j+1}, and cu_prev, cv_prev the
 * adjoints of C_j (which the next step reads as its C_{j-1}); on return the
 * adjoints of the state at j (p and step are not used).
 * grad_bc: device [2][n_v], accumulated: the adjoints of u_bc and v_bc from
 * this step (wall rows; the Kim-Moin values of eq. (21) use them).
 * dnu: host, accumulated: the derivative with respect to nu (through
 * H = I - (dt nu / 2) D_Lap and the right-hand side of eq. (16)).
 * The transposed solves: the viscous matrix by Jacobi-scaled BiCGSTAB on
 * H^T, the bordered pressure system by BiCGSTAB on (A_s + u1 c 1^T)^T (the
 * transpose of the zero-mean bordered solve), with the solver's tolerances
 * (pressure: a tenth of rtol_p).  The first call builds the transposed
 * operators (rbf_ell_transpose).  Synchronises.
 * Errors: RBF_E_ARG (NULL arguments), RBF_E_NOCONV, RBF_E_NAN, those of
 * rbf_step for the recomputed forward step.
 */
rbf_status rbf_adjoint_step(rbf_solver *s, const rbf_state *fwd, rbf_state *adj, double *grad_bc,
                            double *dnu);

/* Release a solver (NULL is ignored). */
void rbf_solver_destroy(rbf_solver *s);

#ifdef __cplusplus
}
#endif

#endif /* RBFFD_H */
