/*
 * lsqr_mi355x.h — C ABI of the MI355X (gfx950) damped, smoothing-regularised
 * LSQR library.
 *
 * Problem.  The paper (pDSurfTomo, arXiv 2604.11920) reduces each inversion
 * step to the sparse overdetermined system Delta d = G Delta m (its eq. (6)),
 * solved in the least-squares sense by a Krylov solver (its section "Solver for
 * the Large-scale Linear System", which names LSQR of Paige & Saunders 1982 and
 * LSMR; the unknown ordering is its eq. (7), depth fastest).  This library
 * solves the regularised form
 *
 *     dm = argmin |G dm - dt|^2 + w^2 |L dm|^2 + lambda^2 |dm|^2
 *
 * where w = smooth_weight, lambda = damp and L is the 3-D 7-point Laplacian on
 * the (nx, ny, nz) model grid in index space (off-grid neighbours dropped,
 * centre = -(number of in-grid neighbours), so L 1 = 0).  LSQR runs on the
 * explicit block operator Abar = [G; w L; lambda I] times an optional column
 * scaling D (x = D y), with right-hand side bbar = [dt; 0; 0].
 *
 * Conventions for every function:
 *   - Returns an lsqr_status; never throws, aborts or exits.  After a failure a
 *     message is available from lsqr_last_error().
 *   - The caller owns every pointer it passes; pointers need to stay valid only
 *     for the duration of the call.  Device pointers are HIP device addresses
 *     on the device that was current when the context was created.
 *   - Work is issued on opts.stream (a hipStream_t, NULL = default stream).
 *     lsqr_solve and lsqr_solve_batched return after the stream has finished
 *     the solve (they read back the stop state); the operator entry points
 *     lsqr_apply / lsqr_apply_t only enqueue work.
 *   - A context is not thread-safe; separate contexts may be used concurrently.
 */
#ifndef LSQR_MI355X_H
#define LSQR_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSQR_OK = 0,
    LSQR_E_INVALID_ARG = -1,   /* null pointer, bad size, negative damp, ...       */
    LSQR_E_BAD_CSR = -2,       /* row_ptr not monotone, column out of range,        */
                               /* columns unsorted or duplicated within a row       */
    LSQR_E_NONFINITE = -3,     /* NaN/Inf in G, dt or a scale; or a solver scalar    */
    LSQR_E_DEVICE = -4,        /* a HIP call failed (message names it)              */
    LSQR_E_OOM = -5,           /* allocation failed                                 */
    LSQR_E_UNSUPPORTED = -6    /* valid request this build does not provide         */
} lsqr_status;

typedef enum { LSQR_MEM_HOST = 0, LSQR_MEM_DEVICE = 1 } lsqr_mem;

/* Storage/arithmetic of the sparse products.  FP64: FP64 values, vectors and
 * accumulation.  FP32: FP32 values, vectors and accumulation; LSQR scalars,
 * norms and x, w stay FP64.  BF16/FP16: each data row i is stored as a
 * power-of-two FP32 scale sigma_i times 16-bit codes q_ij = RNE(g_ij/sigma_i)
 * (rounded once, directly from FP64); the inner LSQR runs on these with FP32
 * vectors and accumulation and FP64 scalars, inside an FP64 iterative
 * refinement whose residuals use the FP64 operator (see lsqr_solve).  The
 * smoothing and damping rows are never quantised. */
typedef enum { LSQR_FP64 = 0, LSQR_FP32 = 1, LSQR_BF16 = 2, LSQR_FP16 = 3 } lsqr_precision;

/* Column scaling D.  NONE: D = I.  JACOBI: d_j = 1 / |column j of Abar|
 * (data, smoothing and damping entries).  USER: d_j = col_scale[j]. */
typedef enum { LSQR_PRECOND_NONE = 0, LSQR_PRECOND_JACOBI = 1, LSQR_PRECOND_USER = 2 } lsqr_precond;

/* The data block G in CSR form (smoothing and damping rows are implicit). */
typedef struct {
    int64_t m, n, nnz;          /* rows, columns, stored entries; n == nx*ny*nz        */
    int32_t nx, ny, nz;         /* grid; column l = (iy*nx + ix)*nz + iz               */
    const int64_t *row_ptr;     /* [m+1]; row_ptr[0] = 0, non-decreasing, [m] = nnz    */
    const int32_t *col_idx;     /* [nnz]; strictly increasing within a row, in [0, n)  */
    const double *val;          /* [nnz]; finite                                       */
    lsqr_mem mem;               /* where row_ptr/col_idx/val live                      */
} lsqr_csr;

/* Optional device allocator (e.g. PyTorch's caching allocator).  When alloc is
 * NULL the library calls hipMalloc/hipFree itself. */
typedef void *(*lsqr_alloc_fn)(size_t bytes, void *user);
typedef void (*lsqr_free_fn)(void *ptr, size_t bytes, void *user);

#define LSQR_FLAG_TIMING 1u     /* record HIP events around the sparse kernels  */
#define LSQR_FLAG_NO_GRAPH 2u   /* launch iterations one by one, no hipGraph     */
                                /* (other bits: INVALID_ARG)                     */

typedef struct {
    lsqr_precision precision;
    lsqr_precond precond;
    const double *col_scale;    /* host [n], > 0 and finite, when precond == USER      */
    int refine_sweeps;          /* mixed precision: maximum refinement sweeps (>= 1)   */
    int check_every;            /* iterations per device-side convergence block (>= 1) */
    void *stream;               /* hipStream_t                                         */
    lsqr_alloc_fn alloc;
    lsqr_free_fn dealloc;
    void *alloc_user;
    uint32_t flags;             /* LSQR_FLAG_*                                         */
    int lanes_per_row;          /* 0 = auto; else 4, 8, 16, 32 or 64 lanes per row    */
    int lanes_per_col;          /* 0 = auto; same choices for the transposed product   */
    int row_format;             /* data rows of the forward product: 0 = auto (row    */
                                /* groups for rows of >= 384 entries on average when  */
                                /* the groups' column lists hold at most nnz / 2      */
                                /* columns, else plain CSR), 1 = plain CSR,           */
                                /* 4 = row groups (CSR values; consecutive rows       */
                                /* grouped while their columns number at most the    */
                                /* longest row rounded up to 1024; per group its      */
                                /* sorted column list, per entry a 16-bit position in */
                                /* it; the group's part of D v is staged in LDS; rows */
                                /* of more than 7168 entries: UNSUPPORTED)            */
    int col_format;             /* data block of the transposed product: 0 = auto     */
                                /* (node runs in the depth-pair layout when the       */
                                /* matrix fits the format, else CSC), 1 = CSC, 2 =    */
                                /* node runs (per node, the rows reaching it with     */
                                /* their stretch of consecutive depths; needs nz <=   */
                                /* 64, nnz < 2^32), 4 = node runs in the depth-pair   */
                                /* layout (each run stored from an even position with */
                                /* a zero before an odd first depth and after an odd  */
                                /* end, so two depths load as one aligned word; FP32  */
                                /* values four and 16-bit codes eight depths to a     */
                                /* word; a second, padded copy of the node-run        */
                                /* values); other values: INVALID_ARG                 */
    double refine_inner_tol;    /* mixed precision: relative eta each inner solve     */
                                /* reaches before the FP64 correction (0 = 1e-2); a   */
                                /* sweep cannot gain more than the quantisation error */
                                /* allows (about 1e-2 for BF16), so tighter inner     */
                                /* solves mostly add restarted work                   */
    int method;                 /* 0 = LSQR (Paige & Saunders 1982); 1 = LSMR (Fong &  */
                                /* Saunders 2011, the solver the paper's "Solver for  */
                                /* the Large-scale Linear System" section says        */
                                /* DSurfTomo adopts): same products, MINRES on the    */
                                /* normal equations, |r| and |A^T r| both monotone.   */
                                /* LSMR's eta is the scaled-variable normal residual  */
                                /* |A_D^T r| / |A_D^T bbar| (equal to the original    */
                                /* variables' for D = I); the batched entry point     */
                                /* runs LSQR                                          */
    int fallback_iters;         /* precond USER with tol > 0: when the solve has not  */
                                /* reached tol after this many iterations (total      */
                                /* inner iterations for BF16/FP16, or a refinement    */
                                /* sweep that stalls: refine_stall_ratio), the Jacobi */
                                /* scale replaces the user scale and the solve        */
                                /* continues                                          */
                                /* from its current dm (info.fallback_used = 1; the   */
                                /* history is the continuation's); a                  */
                                /* natural choice is twice Jacobi's count on the      */
                                /* system.  0 = no fallback.  The context keeps the   */
                                /* user scale for later solves.                        */
    double refine_stall_ratio;  /* mixed precision: a sweep stalls when it leaves eta  */
                                /* above this times the previous sweep's (0 = 0.5;    */
                                /* [0, 1], else INVALID_ARG).  On the first stall the */
                                /* remaining inner solves run on FP32 copies of the   */
                                /* FP64 values (row groups or CSR and the CSC, built  */
                                /* then, 8 bytes per entry more) and info.inner_fp32  */
                                /* is set; a stall after that ends the solve, istop 4 */
                                /* (with a user scale and fallback_iters, the Jacobi  */
                                /* fallback comes first)                              */
} lsqr_opts;

/* Stop reasons (info.istop):
 *   0  bbar = 0 or Abar^T bbar = 0; dm = 0
 *   1  eta_k <= tol, with eta_k = |Abar^T rbar_k| / |Abar^T bbar| estimated from
 *      the bidiagonalisation (LSQR's |A^T r| estimate times |D^-1 v_{k+1}|)
 *   2  iteration limit reached
 *   3  exact breakdown (alpha or beta exactly 0): dm is the least-squares
 *      solution over the Krylov space reached
 *   4  mixed-precision refinement stalled (eta did not fall below
 *      opts.refine_stall_ratio times the previous sweep's), with FP32 inner
 *      solves already tried  */
typedef struct {
    int istop;
    int iters;                  /* iterations done (total inner iterations if mixed;  */
                                /* with a fallback, the user-scale attempt included)  */
    int sweeps;                 /* refinement sweeps done (mixed forms), else 0        */
    int fallback_used;          /* 1 if user scales were rejected for Jacobi, at      */
                                /* creation (not finite and > 0) or by the solve      */
                                /* (opts.fallback_iters)                              */
    double eta;                 /* final eta estimate (LSMR: scaled variables)         */
    double phibar;              /* final |bbar - Abar dm| estimate                     */
    double eta_final_fp64;      /* eta of the returned dm recomputed at exit with the  */
                                /* FP64 operator, |Abar^T (bbar - Abar dm)| /          */
                                /* |Abar^T bbar| in the original variables (every     */
                                /* form and method), when tol > 0; NaN for fixed      */
                                /* iteration counts (tol = 0)                          */
    int inner_fp32;             /* 1 if the refinement stalled and its later inner     */
                                /* solves ran on FP32 values (BF16 / FP16 forms)       */
} lsqr_info;

typedef struct lsqr_ctx lsqr_ctx;

/* Kernel timing (LSQR_FLAG_TIMING): totals over the last solve. */
typedef struct {
    double fwd_ms;              /* forward products Abar D v                          */
    double adj_ms;              /* transposed products D Abar^T u                      */
    int fwd_launches;
    int adj_launches;
    double fwd_bytes;           /* algorithmic bytes of one forward launch            */
    double adj_bytes;           /* algorithmic bytes of one transposed launch         */
    int row_format;             /* format the solver's forward product reads: 1 CSR,  */
                                /* 4 row groups                                       */
    int col_format;             /* transposed product: 1 CSC, 2 node runs, 4 node     */
                                /* runs in the depth-pair (four-depth) layout         */
    int fwd_entries_per_load;   /* row groups: entries a lane reads per load (1; 2:    */
                                /* aligned pairs, 4: quads, 8: octets of 16-bit codes; */
                                /* k_fwd_lcol_pair)                                    */
    int adj_depths_per_word;    /* node-run layouts: depths per lane and load (1 plain */
                                /* runs, 2 depth pairs, 4 four-depth words)            */
    int64_t groups;             /* row groups of the forward product (0 otherwise)     */
    int64_t staged_cols;        /* columns staged in LDS per forward product, summed   */
                                /* over the groups                                     */
    int64_t padded_values;      /* zeros the transposed layout adds to the stored      */
                                /* values (depth pairs, four-depth words)              */
} lsqr_kstats;

/*
 * lsqr_create — validate G (the data block of eq. (6), columns ordered as in
 * eq. (7)), copy it to the device, build its transpose (CSC, a stable device
 * sort by column so rows stay ascending within a column), the stored formats
 * opts.row_format / opts.col_format select (by default, where the matrix fits
 * them, row groups for the forward product and node runs in the depth-pair
 * layout for the transposed product, both built from the CSR structure on
 * the host) and the column scaling.  damp >= 0 and smooth_weight >= 0 (damp > 0 is required by
 * the mixed forms, whose refinement folds the FP64 correction into the damping
 * block).  opts may be NULL (FP64, no scaling, default stream, hipMalloc).
 * On success *out owns every derived buffer; free it with lsqr_destroy.
 * Errors: INVALID_ARG, BAD_CSR, NONFINITE, DEVICE, OOM, UNSUPPORTED.
 */
lsqr_status lsqr_create(const lsqr_csr *G, double damp, double smooth_weight,
                        const lsqr_opts *opts, lsqr_ctx **out);

/*
 * Device-side assembly of G from the rays (the data block of eq. (6); rows
 * per (path, period) as in eq. (1), columns ordered as in eq. (7)).  Input:
 * per path, the lateral nodes it crosses with the length of its path
 * integral against each node's bilinear hat function; per period, the phase
 * velocity and a depth kernel (weights on a contiguous range of depth nodes).
 * Row (p, t) exists when keep[p nper + t] != 0; rows are ordered path-major
 * (path p, then period t ascending), a row's entries node by node (in the
 * path's node order) and depth by depth.  Entry (node a of path p, depth
 * j0[t] + b) of row (p, t): column node_k[a] nz + j0[t] + b, value
 * (-node_len[a] / cvel[t]) w[w_ptr[t] + b] (the traveltime sensitivity of
 * the synthetic generator, evaluated in this order in FP64).  All inputs are
 * host arrays (they are small next to G) except node_k and node_len, which
 * may be device arrays (node_mem, e.g. from lsqr_split_polylines); outputs
 * are device arrays.
 */
typedef struct {
    int64_t npairs;             /* paths                                                 */
    int32_t nper;               /* periods (>= 1)                                         */
    int32_t nz;                 /* depth nodes per lateral node                           */
    const int64_t *node_ptr;    /* [npairs+1] path p's nodes: node_ptr[p] .. node_ptr[p+1]-1 */
    const int32_t *node_k;      /* [node_ptr[npairs]] lateral node index (>= 0)           */
    const double *node_len;     /* [node_ptr[npairs]] path length against the node (finite) */
    const double *cvel;         /* [nper] phase velocity (finite, != 0)                   */
    const int32_t *j0;          /* [nper] first depth of the period's kernel              */
    const int32_t *nj;          /* [nper] depths of the kernel; 0 <= j0, j0 + nj <= nz    */
    const int64_t *w_ptr;       /* [nper+1] w_ptr[t+1] - w_ptr[t] == nj[t]                */
    const double *w;            /* [w_ptr[nper]] depth weights (finite)                   */
    const uint8_t *keep;        /* [npairs*nper] row (p, t) exists when nonzero           */
    lsqr_mem node_mem;          /* where node_k and node_len live (LSQR_MEM_HOST = 0,     */
                                /* the zero default, or LSQR_MEM_DEVICE: lsqr_rays_size  */
                                /* does not read them; lsqr_assemble_rays checks them on */
                                /* the device: nodes >= 0, lengths finite, columns below */
                                /* 2^31)                                                 */
} lsqr_rays;

/*
 * Ray polylines on the lateral grid, as a ray tracer hands them over (the
 * rays of the travel-time step): per path its points and the length of each
 * piece between consecutive points.  Node (ix, iy) sits at (ix h, iy h),
 * k = iy nx + ix.  A piece may cross at most one grid line of each
 * direction (|dx| < h and |dy| < h).
 */
typedef struct {
    int64_t npaths;             /* paths                                                 */
    int32_t nx, ny;             /* lateral nodes (>= 2 each)                             */
    double h;                   /* node spacing (degrees, > 0)                           */
    double km_per_deg;          /* length unit of the results (> 0)                      */
    const int64_t *pt_ptr;      /* [npaths+1] path p owns points pt_ptr[p] .. pt_ptr[p+1]-1 */
    const double *px, *py;      /* [pt_ptr[npaths]] point coordinates (degrees, finite)  */
    const double *plen;         /* [pt_ptr[npaths]] length of the piece from point i to  */
                                /* i + 1 (degrees, finite, >= 0); unused at a path's     */
                                /* last point                                            */
} lsqr_polylines;

/*
 * lsqr_split_polylines — the bilinear split of every path on the device
 * (eq. (1)'s interpolation coefficients): each piece is cut where it crosses
 * grid lines, the four bilinear corner weights are integrated exactly along
 * every sub-piece (Simpson's rule; they are quadratic along it) and summed
 * per node in the order the sub-pieces occur along the path; nodes with a
 * positive integral are kept, ascending, with their lengths in km (length in
 * degrees times km_per_deg).  The same arithmetic as the synthetic
 * generator's split, so the result equals it to the bit.  One workgroup per
 * path; at most 4096 corner records per path (4 per sub-piece) and 129
 * contributions per node, else UNSUPPORTED.
 *   node_ptr  host [npaths+1], always written: path p's nodes are
 *             node_ptr[p] .. node_ptr[p+1]-1
 *   node_k, node_len  NULL (sizes only), or device arrays of node_ptr[npaths]
 *             entries (int32 node index, FP64 km), e.g. sized by a first call
 * Inputs are staged in temporary device buffers from alloc (hipMalloc when
 * alloc is NULL), returned before the call returns; work runs on `stream`.
 * Errors: INVALID_ARG, NONFINITE, UNSUPPORTED, DEVICE, OOM.
 */
lsqr_status lsqr_split_polylines(const lsqr_polylines *poly, void *stream, lsqr_alloc_fn alloc,
                                 lsqr_free_fn dealloc, void *alloc_user, int64_t *node_ptr,
                                 int32_t *node_k, double *node_len);

/* lsqr_rays_size — rows m and stored entries nnz of the assembled G (host
 * work only; validates the rays).  Errors: INVALID_ARG, NONFINITE (node_len
 * or w), UNSUPPORTED (m or a column >= 2^31). */
lsqr_status lsqr_rays_size(const lsqr_rays *rays, int64_t *m, int64_t *nnz);

/* lsqr_assemble_rays — write G as CSR into caller-owned device arrays
 * row_ptr [m+1], col_idx [nnz], val [nnz] (sizes from lsqr_rays_size), on
 * `stream` (a hipStream_t, NULL = default); returns after the arrays are
 * complete.  The result can be passed to lsqr_create with mem = DEVICE.
 * The ray arrays are staged in temporary device buffers taken from alloc
 * (hipMalloc when alloc is NULL) and returned through dealloc before the
 * call returns.
 * Errors: INVALID_ARG, NONFINITE, UNSUPPORTED, DEVICE, OOM. */
lsqr_status lsqr_assemble_rays(const lsqr_rays *rays, void *stream, lsqr_alloc_fn alloc,
                               lsqr_free_fn dealloc, void *alloc_user, int64_t *row_ptr,
                               int32_t *col_idx, double *val);

/*
 * lsqr_solve — run LSQR (Paige & Saunders) on bbar = [dt; 0; 0] from x0 = 0.
 * BF16/FP16 forms: each refinement sweep forms rbar = bbar - Abar dm and
 * Abar^T rbar in FP64 (FP64 values of G), the exact eta = |Abar^T rbar| /
 * |Abar^T bbar|, then runs the inner LSQR on [Ghat; w L; lambda I] D with
 * right-hand side [0; 0; (Abar^T rbar)/lambda] (whose image under the inner
 * operator's transpose is Abar^T rbar exactly, and which, unlike rbar,
 * vanishes at the solution, so its FP32 rounding does not bound eta) to the
 * relative eta opts.refine_inner_tol (default 1e-2), and adds
 * the correction; the solve stops when eta <= tol (istop 1) or after
 * opts.refine_sweeps sweeps (istop 2).  A sweep that leaves eta above
 * opts.refine_stall_ratio (default 0.5) times the previous one switches the
 * remaining inner solves to FP32 values (info.inner_fp32 = 1); a second
 * stall ends the solve (istop 4).
 *   dt        [m]   data right-hand side (vec_mem says host or device), finite
 *   iters     >= 0  iteration limit K (forward products after the start)
 *   tol       >= 0  stop when eta_k <= tol (0: run exactly K iterations)
 *   dm        [n]   output solution (vec_mem)
 *   res_hist  host [3*(K+1)] or NULL: row k = (phibar_{k+1} = |rbar_k| estimate,
 *                   psi_k = |A_D^T rbar_k| estimate, eta_k); row 0 is the start
 *                   (beta_1, alpha_1*beta_1, 1); rows past info.iters are NaN.
 *                   LSMR: (|rbar_k| from its third rotation chain,
 *                   |A_D^T rbar_k| = |zetabar_{k+1}|, that over alpha_1 beta_1)
 *   info      output, may be NULL
 * For the mixed forms (precision BF16/FP16) dm is refined in FP64 until
 * eta <= tol (tol must be > 0) or opts.refine_sweeps sweeps; iters then caps
 * each inner solve and res_hist receives the inner history of the last sweep.
 * Errors: INVALID_ARG, NONFINITE (dt or a solver scalar), DEVICE, OOM.
 */
lsqr_status lsqr_solve(lsqr_ctx *ctx, const double *dt, lsqr_mem vec_mem, int iters, double tol,
                       double *dm, double *res_hist, lsqr_info *info);

/*
 * lsqr_solve_x0 — lsqr_solve started from an initial solution x0 (warm start),
 * for the outer iterations of the inversion (the theoretical-framework section:
 * the system of eq. (6) is solved again after each model update and
 * re-linearisation) and for restarts and regularisation sweeps.  Plain forms:
 * the solver runs on the correction problem A_D y ~ r0 = bbar - Abar x0 and
 * returns dm = x0 + D y; its stopping ratio is rescaled so that eta keeps its
 * meaning, |Abar^T (bbar - Abar dm)| / |Abar^T bbar| (LSMR: the D-scaled
 * norms), in the history's eta column and info.eta as well (when
 * Abar^T bbar = 0, eta is relative to |Abar^T r0|).  When x0 already satisfies
 * the normal equations (Abar^T r0 = 0) nothing runs: dm = x0, istop 1, iters 0.
 * BF16/FP16 forms: the FP64 refinement starts from x0 instead of 0.
 *   x0   [n] initial solution (vec_mem), finite; may be the same device buffer
 *        as dm.  Other arguments, outputs and errors as for lsqr_solve
 *        (NONFINITE also for x0).
 */
lsqr_status lsqr_solve_x0(lsqr_ctx *ctx, const double *dt, const double *x0, lsqr_mem vec_mem,
                          int iters, double tol, double *dm, double *res_hist, lsqr_info *info);

/*
 * lsqr_solve_batched — LSQR for nrhs right-hand sides of each of nsys systems,
 * advanced together: sparse products read each system's matrix once per
 * right-hand-side tile (FP32 values and vectors, FP64 per-RHS scalars), and
 * every system's iterations are captured in one hipGraph and replayed.
 *   ctxs      [nsys] contexts (any precision; the batch reads FP32 copies of G)
 *   nrhs      1..32 (padded internally to a power of two with zero columns)
 *   dt        [nsys] pointers to [m_s][nrhs] row-major right-hand sides (vec_mem)
 *   iters     iteration limit; tol >= 0 as in lsqr_solve, applied per RHS (a
 *             converged right-hand side is frozen while the others continue)
 *   dm        [nsys] pointers to [n_s][nrhs] row-major outputs (vec_mem)
 *   res_hist  NULL, or [nsys] host pointers (each NULL or [iters+1][nrhs][3])
 *   info      NULL or [nsys*nrhs] per right-hand side (system-major)
 * Work runs on ctxs[0]'s stream (other contexts' streams are synchronised
 * first).  The schedule (RHS tile, workgroups) is each context's configuration:
 * the default, lsqr_set_batch_config or lsqr_autotune_batched.
 * Errors: INVALID_ARG, NONFINITE, DEVICE, OOM.
 */
lsqr_status lsqr_solve_batched(lsqr_ctx *const *ctxs, int nsys, int nrhs, const double *const *dt,
                               lsqr_mem vec_mem, int iters, double tol, double *const *dm,
                               double *const *res_hist, lsqr_info *info);

/*
 * lsqr_solve_batched_refined — the batched solve with iterative refinement
 * per right-hand side, so that the FP32 values and vectors of the batch
 * still reach the FP64 solution.  Each sweep computes, for every right-hand
 * side that has not stopped, in FP64 with the FP64 operator: the residual
 * rbar = bbar - Abar x, Abar^T rbar and eta = |Abar^T rbar| / |Abar^T bbar|;
 * it stops that right-hand side when eta <= tol (istop 1), after `sweeps`
 * sweeps (istop 2) or when eta fails to halve between sweeps (istop 4).  The
 * others are then solved together by the batched LSQR (at most `iters`
 * iterations, relative tolerance inner_tol, every system in one captured
 * graph) on the right-hand side f = [0; 0; (Abar^T rbar) / damp], whose
 * Ahat^T f equals Abar^T rbar for the FP32 values Ghat the batch reads, so
 * the refinement's fixed point is the FP64 least-squares solution; x += D y.
 * (The solver section of the paper; the problem of eq. (6) with the
 * smoothing and damping blocks.)
 *   arguments as lsqr_solve_batched, plus
 *   tol        > 0, the FP64 stopping ratio of every right-hand side
 *   inner_tol  in [0, 1): relative tolerance of each sweep's batched solve
 *   sweeps     >= 1: most refinement sweeps
 *   info       NULL or [nsys*nrhs]: istop as above (0: Abar^T bbar = 0),
 *              iters = inner iterations over all sweeps, sweeps, eta and
 *              eta_final_fp64 = the FP64 eta of the returned dm, phibar =
 *              |rbar| of the returned dm
 * Errors: as lsqr_solve_batched; INVALID_ARG for tol <= 0, inner_tol or
 * sweeps out of range; UNSUPPORTED when a system has damp = 0.
 */
lsqr_status lsqr_solve_batched_refined(lsqr_ctx *const *ctxs, int nsys, int nrhs,
                                       const double *const *dt, lsqr_mem vec_mem, int iters,
                                       double tol, double inner_tol, int sweeps,
                                       double *const *dm, lsqr_info *info);

/*
 * lsqr_apply_block / lsqr_apply_t_block — the batched kernels as plain
 * products on nrhs (a power of two <= 32) row-major FP32 blocks of device
 * vectors: Y [m+2n][nrhs] = Abar D X [n][nrhs]; X = D Abar^T Y.  Enqueued only.
 * For nrhs >= 4 the transposed product reads rows of Y as 16-byte vectors:
 * y must then be 16-byte aligned (LSQR_E_INVALID_ARG otherwise).
 */
lsqr_status lsqr_apply_block(lsqr_ctx *ctx, int nrhs, const float *x, float *y);
lsqr_status lsqr_apply_t_block(lsqr_ctx *ctx, int nrhs, const float *y, float *x);

/* Schedule of the batched kernels: right-hand sides per kernel pass (8, 16 or
 * 32; smaller tiles re-read the matrix, larger ones gather wider rows of the
 * vector blocks; with node runs, 32-wide tiles run both products on the
 * matrix cores, per lateral node: the forward product as per-run partial rows
 * then per-row sums, the transposed product reduced over the node's runs) and
 * the cap on workgroups per launch. */
typedef struct {
    int rhs_tile;
    int grid;
    double ms_per_iter;         /* measured by the autotuner (output only)           */
} lsqr_batch_cfg;

/* lsqr_set_batch_config — use this schedule for ctx's batched solves. */
lsqr_status lsqr_set_batch_config(lsqr_ctx *ctx, const lsqr_batch_cfg *cfg);

/*
 * lsqr_autotune_batched — time every schedule (RHS tile in {8,16,32} not above
 * the padded nrhs, grid in {256,512,1024,2048}) on ctx's system for
 * probe_iters batched iterations (median of 5 repeats, HIP events on ctx's
 * stream), keep the fastest for ctx and return it in *best.
 */
lsqr_status lsqr_autotune_batched(lsqr_ctx *ctx, int nrhs, int probe_iters, lsqr_batch_cfg *best);

/*
 * lsqr_apply — y = Abar D x on the device: y[0:m] = G (D x),
 * y[m:m+n] = w L (D x), y[m+n:m+2n] = lambda (D x).  x [n], y [m+2n], FP64,
 * device pointers.  Uses the same kernel as the solver's forward product.
 */
lsqr_status lsqr_apply(lsqr_ctx *ctx, const double *x, double *y);

/*
 * lsqr_apply_t — x = D Abar^T y = D (G^T y[0:m] + w L y[m:m+n] + lambda y[m+n:]),
 * device pointers, FP64.  Uses the FP64 transposed format of the solver (the
 * CSC, or the node runs when opts.col_format selected them; no atomics).
 */
lsqr_status lsqr_apply_t(lsqr_ctx *ctx, const double *y, double *x);

/*
 * lsqr_apply_stored / lsqr_apply_t_stored — the solver's own sparse products
 * as plain operator applications: the stored format and value type its
 * iterations read (FP64 or FP32 values, or for BF16/FP16 the row scales
 * sigma times the 16-bit codes Q; the forward product of eq. (6) and its
 * transpose), without the column scaling, for inspection and testing:
 *   y = [Ghat z; w L z; lambda z],  Ghat = G in the solver's value type, or
 *                                   diag(sigma) Q for the 16-bit forms;
 *   q = Ghat^T y_G + w L y_L + lambda y_D, where the data block reads tg
 *       instead of y_G when tg != NULL: the 16-bit forms' transposed product
 *       gathers tg = sigma * y_G (the row scale applied to the gathered
 *       vector, as in the solver) and computes Q^T tg.
 * Vectors are device arrays of the solver's vector type (double for FP64,
 * float for the other forms): z [n], y [m+2n], tg [m], q [n].  Enqueued
 * only.  Errors: INVALID_ARG.
 */
lsqr_status lsqr_apply_stored(lsqr_ctx *ctx, const void *z, void *y);
lsqr_status lsqr_apply_t_stored(lsqr_ctx *ctx, const void *y, const void *tg, void *q);

/*
 * lsqr_set_scale — replace the column scaling D (x = D y) by host d [n],
 * finite and > 0 (else INVALID_ARG and D unchanged).  Any d leaves the
 * regularised least-squares solution unchanged (only the iteration count
 * moves), so a learned scale can be tried on a context without rebuilding it.
 * The captured iteration graphs read D from the same buffer and stay valid.
 */
lsqr_status lsqr_set_scale(lsqr_ctx *ctx, const double *d);

/*
 * lsqr_get_scale — copy the column scaling d [n] (host buffer).
 * lsqr_get_transpose — copy the device-built CSC of G to host buffers
 * col_ptr [n+1], row_idx [nnz], val [nnz] (any may be NULL).
 */
lsqr_status lsqr_get_scale(const lsqr_ctx *ctx, double *d);
lsqr_status lsqr_get_transpose(const lsqr_ctx *ctx, int64_t *col_ptr, int32_t *row_idx, double *val);

/*
 * lsqr_get_quantised — the BF16/FP16 forms' stored values, for inspection:
 * row_scale [m] (FP32 powers of two), q_rows [nnz] (16-bit codes in CSR order)
 * and q_cols [nnz] (the same codes in CSC order); host buffers, any may be
 * NULL.  Entry (i, j) of the quantised G is row_scale[i] * q.  UNSUPPORTED for
 * the FP64/FP32 forms.
 */
lsqr_status lsqr_get_quantised(const lsqr_ctx *ctx, float *row_scale, uint16_t *q_rows,
                               uint16_t *q_cols);

/* ---------------------------------------------------------------------------
 * Learned column scaling.  A small MLP maps six per-column features to a
 * multiplier of the Jacobi scale, d_j = d_j^Jacobi * softplus(z_j), to cut the
 * iterations LSQR needs; any d > 0 leaves the solution unchanged, and Jacobi
 * (opts.precond = JACOBI) stays the fallback (lsqr_create falls back to it for
 * USER scales that are not finite and positive).
 * Features of column j of Abar (FP32, [n][6] row-major):
 *   f1 log10 |column j of Abar|   f2 log(1 + rows of G hitting j)
 *   f3 iz / (nz - 1)              f4, f5 |g|-weighted mean and standard
 *   deviation, over the rows hitting j, of each row's depth centroid
 *   sum_j |g_ij| iz(j) / sum_j |g_ij| / (nz - 1)
 *   f6 log(1 + mean of f2's counts over the in-grid 7-point neighbours)
 * Parameters: one flat FP32 vector W1[64][6], b1[64], W2[64][64], b2[64],
 * W3[64], b3 (LSQR_MLP_NPARAMS values); hidden layers use the exact (erf) GELU.
 * ------------------------------------------------------------------------- */
#define LSQR_MLP_NPARAMS 4673

/* lsqr_column_features — feat (device [n][6]) for ctx's system. */
lsqr_status lsqr_column_features(lsqr_ctx *ctx, float *feat);

/*
 * lsqr_mlp_scale — inference: d (device [n], FP64) = Jacobi scale times
 * softplus(MLP((feat - mean) / std)), with weights and activations rounded to
 * BF16 (nearest even) and FP32 sums.  params: device [LSQR_MLP_NPARAMS];
 * mean, std: host [6] standardisation of the training features (std > 0);
 * centre: bit f set = feature f is centred on this system's own mean over its
 * columns (computed here, FP64, fixed order) instead of mean[f], for
 * features whose level shifts with the survey size (coverage, norms).
 */
lsqr_status lsqr_mlp_scale(lsqr_ctx *ctx, const float *params, const float *mean, const float *std,
                           unsigned centre, const float *feat, double *d);

/*
 * lsqr_mlp_scale_noalloc — for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same operation, arguments and result as lsqr_mlp_scale
 * (the same kernels, so d is bitwise the same), with its temporary (the
 * Jacobi scale and the feature means, n + 6 doubles) in a static device
 * array of LSQR_NOALLOC_MAX_COLS + 6 doubles (8 MiB) that the library holds
 * on each device it runs on until the process ends, instead of an
 * allocation.  It calls no device allocator.
 * Errors: LSQR_E_INVALID_ARG as lsqr_mlp_scale, and when ctx's system has
 * more than LSQR_NOALLOC_MAX_COLS unknowns; LSQR_E_DEVICE if the array's
 * device address cannot be obtained.
 * All calls on one device share the array: calls that overlap on one device
 * (different host threads, or different streams without ordering between
 * them) race on it and must be serialised by the caller.  Every element a
 * call reads is written earlier in the same call, so nothing carries over.
 */
#define LSQR_NOALLOC_MAX_COLS 1048576
lsqr_status lsqr_mlp_scale_noalloc(lsqr_ctx *ctx, const float *params, const float *mean,
                                   const float *std, unsigned centre, const float *feat,
                                   double *d);

/* Training state (FP32 parameters and Adam moments on the device). */
typedef struct lsqr_trainer lsqr_trainer;

/* lsqr_trainer_create — params: host [LSQR_MLP_NPARAMS] initial values;
 * max_batch: largest minibatch; stream: hipStream_t for all its work;
 * alloc/dealloc/alloc_user: device allocator of its buffers (NULL alloc:
 * hipMalloc), released by lsqr_trainer_destroy. */
lsqr_status lsqr_trainer_create(int max_batch, const float *params, void *stream,
                                lsqr_alloc_fn alloc, lsqr_free_fn dealloc, void *alloc_user,
                                lsqr_trainer **out);

/*
 * lsqr_trainer_grad — loss = mean over the batch of (log softplus(z_b) -
 * target_b)^2 and its gradient (FP32 forward/backward per sample, per-parameter
 * sums over the batch in sample order).  x: device [batch][6] standardised
 * features; target: device [batch] log multipliers; grad: device
 * [LSQR_MLP_NPARAMS] or NULL; loss: host or NULL.
 */
lsqr_status lsqr_trainer_grad(lsqr_trainer *t, int batch, const float *x, const float *target,
                              float *grad, double *loss);

/* lsqr_trainer_step — the same gradient, then one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8, learning rate lr). */
lsqr_status lsqr_trainer_step(lsqr_trainer *t, int batch, const float *x, const float *target,
                              float lr, double *loss);

/* lsqr_trainer_params — copy the current parameters to a host and/or a device
 * buffer ([LSQR_MLP_NPARAMS]; either may be NULL, not both). */
lsqr_status lsqr_trainer_params(const lsqr_trainer *t, float *params, float *params_device);

/* lsqr_trainer_destroy — free t (NULL is a no-op). */
void lsqr_trainer_destroy(lsqr_trainer *t);

/* lsqr_kernel_stats — kernel timing of the last solve (LSQR_FLAG_TIMING; for
 * the BF16/FP16 forms, the inner products of all refinement sweeps), the
 * algorithmic bytes of one launch of each sparse kernel and the formats they
 * read.  Timing records events around every launch, so timed solves run
 * without hipGraph replay. */
lsqr_status lsqr_kernel_stats(const lsqr_ctx *ctx, lsqr_kstats *out);

/* lsqr_destroy — free every buffer of ctx (NULL is a no-op). */
void lsqr_destroy(lsqr_ctx *ctx);

/* lsqr_status_string — static text for a status code. */
const char *lsqr_status_string(lsqr_status s);

/* lsqr_last_error — message of the last failure on ctx; ctx == NULL gives the
 * calling thread's message from a failed lsqr_create. */
const char *lsqr_last_error(const lsqr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LSQR_MI355X_H */
