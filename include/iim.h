/*
 * iim.h -- C ABI of the MI355X immersed-interface Poisson library.
 *
 * The library solves  div(beta grad u) = f  on a uniform vertex-centred grid
 * of [lo, hi]^dim (dim = 2 or 3, n intervals per axis, h = (hi - lo)/n) with
 * an immersed boundary or interface Gamma given by an analytic level set
 * (Gabbard, Paris & van Rees, "A high order multigrid-preconditioned immersed
 * interface solver for the Poisson equation with boundary and interface
 * conditions", JCP 2025):
 *   - boundary problems (Sec. 2.1): u = ubar (Dirichlet) or beta dn u = qbar
 *     (Neumann) on Gamma, the solved region Omega^+ being the interior or the
 *     exterior of the body; box faces bounding the domain carry Dirichlet data;
 *   - interface problems (Sec. 2.2): Omega^- = {phi <= 0}, Omega^+ = {phi > 0},
 *     [u] = u^+ - u^- = j0 and [beta dn u] = j1 on Gamma, Dirichlet box.
 * The normal n at a control point points from Omega^- into Omega^+ (into the
 * solved region for boundary problems).
 *
 * The discretisation is the (n, k) = (4, 5) immersed-interface method, or the
 * (6, 7) one (Sec. 2.1-2.3): dimension-split central differences of order n
 * with least-squares ghost values (degree k - 1) at every crossing of a grid
 * line with Gamma.  The system L_Omega u + L_Gamma u_Gamma = f is solved
 * matrix-free by right-preconditioned FGMRES(restart) (Sec. 4.1) with one
 * Shortley-Weller multigrid cycle (V, or W) as preconditioner (Sec. 3.1,
 * 3.3).  The operator, the Krylov basis, dot products and least-squares fits
 * are FP64; the cycle runs in FP64, FP32, or FP32 with FP16 storage of its
 * iterates.  A solution can be post-processed into its gradient and the
 * boundary quantity its condition leaves open (Sec. 2.4).
 *
 * Conventions for every call:
 *   - return 0 on success, IIM_NOT_CONVERGED (> 0) when a solve stopped at
 *     max_iters (outputs still valid), a negative IIM_E_* code on error; the
 *     message of the last error of the calling thread is iim_last_error();
 *   - no C++ exception crosses this interface;
 *   - "full-grid array": (n+1)^dim values, x fastest: node (i, j, k) at
 *     i + (n+1) j + (n+1)^2 k;
 *   - the caller owns every buffer it passes; the library owns the handle and
 *     all device memory it allocated (released by iim_destroy);
 *   - device pointers must be on the device that was current at iim_create;
 *     work is ordered on the stream given at creation.
 */
#ifndef IIM_H
#define IIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IIM_OK 0
#define IIM_NOT_CONVERGED 1
#define IIM_E_INVALID_ARG (-1)
#define IIM_E_GEOMETRY_UNRESOLVED (-2)
#define IIM_E_BUDGET (-3)
#define IIM_E_DEVICE (-4)
#define IIM_E_BREAKDOWN (-5)
#define IIM_E_INTERNAL (-6)

/* geometry kinds (params layout in brackets) */
#define IIM_GEOM_SPHERE 0       /* circle / sphere [c_1..c_dim, r]                 */
#define IIM_GEOM_STAR2D 1       /* star r(t)=r0+eps cos(L t) [cx, cy, r0, eps, L]   */
#define IIM_GEOM_SPHERE_UNION 2 /* union [count, (c_1..c_dim, r) x count]          */
#define IIM_GEOM_GYROID 3       /* 3D: phi = cos(k1 x) sin(k2 y) + cos(k2 y) sin(k3 z)
                                   + cos(k3 z) sin(k1 x) - alpha  [k1, k2, k3, alpha]
                                   (Sec. 4.4.1; the body is phi < 0)              */

/* which side is solved */
#define IIM_SIDE_INTERIOR 0  /* Omega^+ = {phi < 0}                          */
#define IIM_SIDE_EXTERIOR 1  /* Omega^+ = {phi > 0}, Dirichlet box faces       */
#define IIM_SIDE_INTERFACE 2 /* Omega^- = {phi <= 0}, Omega^+ = {phi > 0}     */

/* condition on Gamma */
#define IIM_BC_DIRICHLET 0
#define IIM_BC_NEUMANN 1
#define IIM_BC_JUMP 2

/* V-cycle precision */
#define IIM_PREC_FP64 0
#define IIM_PREC_MIXED32 1 /* FP32 V-cycle                                   */
#define IIM_PREC_MIXED16 2 /* FP32 V-cycle arithmetic, FP16 iterate storage  */

/* memory kinds of caller buffers */
#define IIM_MEM_HOST 0
#define IIM_MEM_DEVICE 1

typedef struct iim_grid {
    int32_t dim;  /* 2 or 3 */
    int32_t n;    /* intervals per axis, >= 8 */
    double lo;    /* domain [lo, hi]^dim */
    double hi;
    int32_t periodic; /* 1: periodic in every direction (Sec. 2.3, 4.4.1): no box faces; node n
                         of a full-grid array is the image of node 0 and never an unknown (NaN in
                         u).  n must halve exactly down to the coarsest level, n >= 32; the
                         (4,5) scheme; no gradient post-processing.  A periodic problem whose
                         immersed condition is Neumann or a jump is singular (bordered). */
    int32_t reserved;
} iim_grid;

typedef struct iim_geometry {
    int32_t kind;    /* IIM_GEOM_* */
    int32_t side;    /* IIM_SIDE_* */
    int32_t bc;      /* IIM_BC_* (IIM_BC_JUMP iff side == IIM_SIDE_INTERFACE) */
    int32_t nparams; /* number of doubles in params */
    const double* params; /* host pointer, copied at creation */
} iim_geometry;

typedef struct iim_options {
    int32_t order_n;    /* interior order n: 4 (default), or 6 (Sec. 2.1: the (6,7) scheme) */
    int32_t order_k;    /* least-squares order k, n + 1: 5 (default) or 7 with n = 6; in 3D
                           the degree-6 fits (84 columns) run on the global-memory QR path */
    double beta_plus;   /* coefficient in Omega^+ */
    double beta_minus;  /* coefficient in Omega^- (interfaces) */
    double rtol;        /* stop when ||b - L u||_2 / ||b||_2 <= rtol */
    int32_t max_iters;  /* total FGMRES iterations */
    int32_t restart;    /* FGMRES restart length (1..11) */
    int32_t nu_pre;     /* red-black Gauss-Seidel sweeps before / after */
    int32_t nu_post;    /*   the coarse-grid correction                 */
    int32_t coarsest_n; /* direct solve once n_level <= coarsest_n */
    int32_t precision;  /* IIM_PREC_* */
    double ls_axis_t;   /* least-squares half-ellipse semi-axes in units of h */
    double ls_axis_n;   /*   (0 = defaults k and k - 1/2) */
    int32_t use_graph;  /* launching of the FGMRES iterations: 2 (default) eager launches, iteration
                           j+1 queued before the host reads column j; 1 the same with each
                           iteration replayed as a captured HIP graph; 0 eager, one iteration at
                           a time, with the per-phase GPU times of iim_stats filled in */
    int32_t tail_nodes; /* levels whose storage box has at most this many nodes run in one
                           single-workgroup kernel (0 = library default; < 0 = coarse solve only) */
    int32_t fused_smoothing; /* 1: LDS-tiled kernels fuse each level's smoothing with its
                                transfer (2D); 0: one kernel per half-sweep and transfer */
    int32_t colour_split;    /* 1: 3D multigrid levels above the single-workgroup kernel keep
                                their vectors split by red-black colour (contiguous rows per
                                colour); 0: storage-box order.  Results are identical. */
    int32_t orthogonalisation; /* Arnoldi step of FGMRES (Sec. 4.1): 1 (default) classical
                                Gram-Schmidt, one pass, with a second pass only when the first
                                leaves less than 1e-2 of |w| (the decision is taken on the
                                device); 0 two passes every iteration (CGS2) */
    int32_t cycle_gamma;     /* multigrid cycle of the preconditioner (Sec. 3.3): 1 (default)
                                V-cycle; 2 W-cycle (each coarser level visited twice per visit
                                of the level above, the second visit from the first one's
                                iterate).  The W-cycle runs one kernel per half-sweep and
                                transfer on every level (no fused legs, coarse solve alone in
                                the one-workgroup kernel). */
} iim_options;

typedef struct iim_stats {
    int32_t status;        /* return code of the solve */
    int32_t iterations;    /* FGMRES iterations performed */
    int32_t cycles;        /* restart cycles */
    int32_t hist_len;      /* entries written to the history */
    double final_rel_residual; /* true ||b - L u|| / ||b|| at exit */
    double t_solve_ms;     /* wall time of the solve (host clock) */
    double t_apply_ms;     /* GPU time in the high-order operator (use_graph = 0 only) */
    double t_vcycle_ms;    /* GPU time in the preconditioner (use_graph = 0 only) */
    double t_krylov_ms;    /* GPU time in orthogonalisation and updates (use_graph = 0);
                              otherwise the GPU time of the whole restart cycles */
    int32_t second_passes; /* Arnoldi steps that took a second Gram-Schmidt pass */
    int32_t bordered;      /* 1: a singular pure-Neumann problem, solved as the bordered
                              system (Sec. 2.3); 0 otherwise */
    double shift_alpha;    /* bordered solves: the shift alpha that moves b into the range
                              of L (the discrete integrability defect); 0 otherwise */
} iim_stats;

typedef struct iim_info {
    int32_t dim, n, levels, sides;
    int64_t n_unknowns;       /* active degrees of freedom */
    int64_t n_control_points;
    int64_t n_ls_entries;     /* sum of least-squares set sizes over control points and sides */
    int64_t n_irregular;      /* nodes whose high-order stencil uses ghost or box values */
    int64_t box_lo[3], box_dims[3]; /* padded level-0 storage box (node indices) */
    int64_t device_bytes;     /* device memory held by the handle */
    double t_setup_ms;        /* wall time of iim_create */
} iim_info;

typedef struct iim_problem iim_problem;

/* Defaults: (4,5), beta = 1, rtol 1e-10, restart 10, V(2,2), coarsest 8, FP64. */
int iim_default_options(iim_options* opt);

/* Builds everything a solve needs on the device (Sec. 2.1 and 3.1-3.3):
 * node labels, control points, least-squares fits (FP64), irregular-node
 * records, and the Shortley-Weller hierarchy with its coarse inverse.
 * stream: a hipStream_t (NULL = default stream).  Fails with
 * IIM_E_GEOMETRY_UNRESOLVED if |kappa h| >= 1/4 at a control point or a fit
 * stays rank deficient, IIM_E_INVALID_ARG for unsupported options. */
int iim_create(const iim_grid* grid, const iim_geometry* geom, const iim_options* opt,
               void* stream, iim_problem** out);

/* Waits for the handle's stream, then releases all its device memory (NULL is
 * ignored).  Device memory comes from the device's default stream-ordered
 * memory pool; released blocks stay cached in the process for later handles on
 * the same device (iim_server_destroy hands idle blocks back to the device, and
 * an allocation that finds the device full does so before it fails). */
void iim_destroy(iim_problem* p);

/* Thread-local message of the last failing call ("" if none). */
const char* iim_last_error(void);

int iim_get_info(const iim_problem* p, iim_info* info);

/* Control points x_c (Sec. 2.1) in the library's order: by axis, then by the
 * flat index of the segment's lower node.  Call with xyz = normal = NULL to get
 * the count.  xyz, normal: host arrays of count*dim doubles. */
int iim_control_points(const iim_problem* p, int64_t* count, double* xyz, double* normal);

/* Node labels on the full grid (host array of (n+1)^dim bytes):
 * 0 inactive, 1 Omega^+ unknown, 2 Omega^- unknown, 3 box face with known value. */
int iim_node_labels(const iim_problem* p, uint8_t* labels);

/* Boundary data u_Gamma (Sec. 2.3): cp_data holds one value per control point
 * (ubar or qbar) or two (j0, j1) for interfaces; box_data is a full-grid array
 * of which only box-face nodes are read (NULL if no face bounds the domain).
 * Both live in memory of kind mem_kind; they are copied. */
int iim_set_boundary_data(iim_problem* p, const double* cp_data, const double* box_data,
                          int32_t mem_kind);

/* iim_set_boundary_data for callers that cannot allocate device memory (code
 * that must not call hipMalloc, such as tight serving loops or harnesses that
 * forbid allocation): the same operation with no device allocation.  The box
 * data are staged in a library-wide static device array of
 * IIM_NOALLOC_MAX_NODES doubles (32 MiB, one copy per device, held until the
 * process ends) instead of a buffer allocated for the call; (n+1)^dim above
 * that limit fails with IIM_E_INVALID_ARG.  The handle's device must be the
 * current one.  All calls on one device share its array: calls that overlap
 * on one device (from several host threads) race and must be serialised by
 * the caller; each call has finished with the array when it returns. */
#define IIM_NOALLOC_MAX_NODES (1 << 22)
int iim_set_boundary_data_noalloc(iim_problem* p, const double* cp_data, const double* box_data,
                                  int32_t mem_kind);

/* Source term f (full-grid array, read at the unknowns); builds the right-hand
 * side b = f - L_Gamma u_Gamma with the current boundary data. */
int iim_set_rhs(iim_problem* p, const double* f, int32_t mem_kind);

/* FGMRES solve.  u: device full-grid array receiving the solution (NaN at nodes
 * that are not unknowns).  x0: device full-grid initial guess or NULL (zero).
 * hist: host array of hist_cap doubles receiving the relative residual estimate
 * after every iteration (may be NULL).  st: may be NULL.
 * Singular problems (Sec. 2.3): an interior domain (IIM_SIDE_INTERIOR) with a
 * Neumann boundary never reaches the box faces, so L 1 = 0 and u is fixed only
 * up to a constant.  The solver then works on the bordered system
 * [L 1; 1^T 0] [u; alpha] = [b; 0]: the returned unknowns sum to zero, the
 * residual is that of the bordered system, st->shift_alpha receives alpha and
 * st->bordered is 1.  The multigrid preconditioner borders its coarsest
 * Shortley-Weller matrix the same way and passes alpha through unchanged. */
int iim_solve(iim_problem* p, double* u, const double* x0, double* hist, int32_t hist_cap,
              iim_stats* st);

/* y = L_Omega x (with_data = 0) or y = L_Omega x + L_Gamma u_Gamma (with_data = 1)
 * at the unknowns, 0 elsewhere.  x, y: device full-grid arrays. */
int iim_apply(iim_problem* p, const double* x, double* y, int32_t with_data);

/* z = M^{-1} v, one multigrid cycle (V, or W if cycle_gamma = 2) with zero
 * initial guess on Lap z = v / beta (Sec. 3.3), in the handle's precision.
 * v, z: device full-grid arrays. */
int iim_vcycle(iim_problem* p, const double* v, double* z);

/* Post-processing of a solution (Sec. 2.4), with the boundary data last given
 * by iim_set_boundary_data.  u: device full-grid array (values read at the
 * unknowns only).
 * grad: device array of dim * (n+1)^dim doubles, component d at offset
 * d * (n+1)^dim: du/dx_d at every unknown by the order-n central first
 * derivative over the same extended function as the operator (ghost values
 * from the fits, box data and extrapolation past box faces), NaN elsewhere. */
int iim_gradient(iim_problem* p, const double* u, double* grad);

/* q: device array of n_control_points doubles (control-point order of
 * iim_control_points): the boundary quantity the condition leaves open, by the
 * normal-derivative row of each fit: du/dn for Dirichlet, u for Neumann
 * (the closure), du+/dn for interfaces (u+ at x_c from the closure); n is the
 * control point's unit normal from Omega^- into Omega^+.  Dirichlet fits carry
 * no such row: the first call fits every control point once more with it
 * (device memory then held by the handle). */
int iim_boundary_quantity(iim_problem* p, const double* u, double* q);

/* Wall derivatives of a solution at every control point (Sec. 2.1 fits,
 * evaluated as in the potential-flow application of Sec. 4.4.2, which
 * recovers the wall velocity and the pressure coefficient from them), with the
 * boundary data last given by iim_set_boundary_data.  u: device full-grid
 * array (read at the unknowns).
 * grad: device array of n_control_points * dim doubles (control point c's
 * components at c * dim + d, control-point order of iim_control_points): the
 * gradient at x_c of the solved side's least-squares polynomial (the Omega^+
 * one for interfaces), whose value at x_c is ubar (Dirichlet), the Neumann
 * closure, or u+ from the interface closure.  For a Neumann condition its
 * normal component is qbar / beta.
 * u_inf, cp: both NULL, or a host array of dim doubles (a free stream U, not
 * zero) and a device array of n_control_points doubles receiving the pressure
 * coefficient C_p = 1 - |grad + U|^2 / |U|^2 of the wall velocity grad + U
 * (u the disturbance potential of a potential flow).
 * The first call fits every control point once more with the derivative rows
 * (device memory then held by the handle). */
int iim_wall_gradient(iim_problem* p, const double* u, double* grad, const double* u_inf, double* cp);

/* Least-squares stencil of control point cp on side (1 = Omega^+, 2 = Omega^-):
 * m grid points (full-grid flat indices in idx) and the (m+1) x r weights in
 * weights[row * r + col] (row 0 multiplies u(x_c); columns: ghosts 1..w, then
 * the normal derivative for Neumann and interface problems).  Host buffers of capacity cap rows;
 * returns the sizes in *m and *r. */
int iim_ls_stencil(const iim_problem* p, int64_t cp, int32_t side, int32_t* m, int32_t* r,
                   int64_t* idx, double* weights, int32_t cap);

/* Multigrid level access for tests: number of intervals of a level, its labels
 * (host full-level array) and one operation on device full-level FP64 arrays:
 *   op 0: out = A_l in1 (Shortley-Weller operator, unscaled)
 *   op 1: in-place red-black sweep on out with right-hand side in1
 *   op 2: out(level+1) = half-weighting of in1 restricted to unknowns
 *   op 3: out(level-1) = prolongation of in1 (level) onto the finer unknowns
 *   op 4: out = coarse direct solve of in1 (coarsest level only)
 * All in the handle's V-cycle precision. */
int iim_level_info(const iim_problem* p, int32_t level, int32_t* n, int64_t* n_unknowns);
int iim_level_labels(const iim_problem* p, int32_t level, uint8_t* labels);
int iim_level_op(iim_problem* p, int32_t level, int32_t op, const double* in1, double* out);

/* Kernel timing for measurement: launches one hot-path kernel `reps` times in
 * its production launch configuration on the handle's stream, bracketed by two
 * HIP events on that stream, and returns the average duration per launch in
 * *avg_ms.  The operands are the handle's own work vectors (contents are
 * overwritten).  kernel: 0 = high-order stencil apply kernel (level 0; in 3D
 * the regular nodes, 11 = the 3D irregular-node kernel), 1 = ghost values,
 * 2 = one red-black sweep on level 0 (both colours, two launches),
 * 3 = residual + restriction 0 -> 1, 4 = prolongation 1 -> 0,
 * 5 = orthogonalisation update + dots over 6 basis vectors (the streaming
 * first stage; the one-block second stage is not included),
 * 6 = one whole V-cycle, 7 = one whole operator apply (ghosts + stencil),
 * 8 = fused pre-smoothing + residual + restriction leg 0 -> 1 and
 * 9 = fused prolongation + post-smoothing leg 1 -> 0 (the LDS-tiled legs the
 * V-cycle uses in 2D; IIM_E_INVALID_ARG where they do not apply). */
int iim_time_kernel(iim_problem* p, int32_t kernel, int32_t reps, double* avg_ms);

/* Synthetic manufactured data for benchmarks and serving, computed on the
 * device at the library's own control points and nodes: kind 1 is
 * u = sin(2 pi x) cos(2 pi y) in 2D and u = sin(pi x) sin(pi y) sin(pi z) in 3D,
 * giving Dirichlet data u(x_c), box values u, and f = beta Lap(u) (Dirichlet
 * boundary problems only).  Replaces the boundary data and the right-hand side. */
int iim_set_synthetic_data(iim_problem* p, int32_t kind);

/* max |u - u_exact| over the unknowns for a solution u (device full-grid array)
 * of a problem whose data came from iim_set_synthetic_data(kind).  For a singular
 * (bordered) problem, whose u is fixed only up to a constant, the mean of
 * u - u_exact over the unknowns is removed first (Sec. 2.3 compares singular
 * solutions mean-free). */
int iim_synthetic_error(iim_problem* p, int32_t kind, const double* u, double* max_err);

/* ---- serving: continuous batching of independent solves on one device ----
 * A server owns max_slots worker threads.  Each worker solves one request at a
 * time on its own non-blocking HIP stream, so the device work of concurrent
 * requests overlaps.  Requests are admitted in arrival (FIFO) order when a slot
 * is free and their estimated device memory fits in what is left of
 * budget_bytes; a request whose estimate alone exceeds the budget fails with
 * IIM_E_BUDGET without blocking the queue.  Every request keeps its level
 * hierarchy and Krylov basis resident on the device until it completes.
 * With batch_tails (iim_server_create_ex), the small coarse levels of the
 * V-cycles (Sec. 3.3: the levels below the finest ones, coarse solve included,
 * which one workgroup handles) of the requests that reach them together run as
 * one batched launch, one workgroup per request; each request's result is bit
 * for bit the one it gets alone.  Batching couples the requests' streams (a
 * batch waits for every member's finer levels), so it is off by default. */
typedef struct iim_server iim_server;

typedef struct iim_request {
    iim_grid grid;
    iim_geometry geom;   /* params are copied at submission */
    iim_options opt;
    int32_t data_kind;   /* 0: the caller's data (f, cp_data, box_data below);
                            1: synthetic family 1 (see iim_set_synthetic_data) */
    int32_t mem_kind;    /* IIM_MEM_* of f, cp_data and box_data */
    double* u_out;       /* optional device full-grid array receiving u (NULL: not copied);
                            must stay valid until the request completes */
    /* data_kind 0 (Sec. 2.1-2.3; read when the request starts, so they must stay
       valid until it completes): */
    const double* f;        /* full-grid source term, read at the unknowns */
    const double* cp_data;  /* one value per control point (two, j0 then j1, for interfaces), in
                               the order of iim_control_points for the same grid and geometry */
    const double* box_data; /* full-grid box-face values, or NULL (no face bounds the domain) */
    int64_t n_cp_data;      /* doubles in cp_data; the request fails with IIM_E_INVALID_ARG
                               unless it matches the problem's control points */
    double* hist;           /* optional host array of hist_cap doubles receiving the relative
                               residual estimate after every iteration; valid until completion */
    int32_t hist_cap;
    int32_t reserved;
} iim_request;

typedef struct iim_result {
    int32_t done;        /* 1 once finished (successfully or not) */
    int32_t status;      /* IIM_OK, IIM_NOT_CONVERGED or a negative error code */
    int32_t iterations;
    int32_t hist_len;    /* entries written to the request's hist */
    double rel_residual; /* final true relative residual */
    double max_error;    /* synthetic data: max |u - u_exact| over the unknowns (mean-free for
                            singular problems); caller data: 0 */
    double t_submit, t_start, t_finish; /* seconds on the server's steady clock */
    int64_t n_unknowns;
    int64_t device_bytes;   /* device memory the request held */
    int64_t estimated_bytes;
    double shift_alpha;     /* singular (bordered) problems: alpha; 0 otherwise */
} iim_result;

typedef struct iim_server_stats {
    int64_t submitted, completed, failed, running, queued;
    int64_t bytes_reserved, bytes_budget, peak_bytes_reserved;
    int64_t tail_batches;   /* batched coarse-level launches */
    int64_t tail_jobs;      /* V-cycle tails they ran (tail_jobs / tail_batches = mean batch size) */
} iim_server_stats;

typedef struct iim_server_options {
    int32_t batch_tails;     /* 1: batch the V-cycle tails of requests solving together;
                                0 (default): every request launches its own */
    int32_t batch_window_us; /* longest wait of the first tail of a batch for the other solving
                                requests to reach theirs (default 0: a batch holds the tails
                                that arrive while its first one is being launched) */
} iim_server_options;

/* budget_bytes: device memory the server may reserve for running requests;
 * max_slots: requests solved concurrently (1..64).  iim_server_create uses the
 * default options. */
int iim_server_create(int64_t budget_bytes, int32_t max_slots, iim_server** out);
int iim_server_create_ex(int64_t budget_bytes, int32_t max_slots, const iim_server_options* opt,
                         iim_server** out);
/* Enqueues a request; returns at once with its ticket. */
int iim_server_submit(iim_server* s, const iim_request* req, uint64_t* ticket);
/* Copies the request's result (done = 0 while queued or running). */
int iim_server_poll(iim_server* s, uint64_t ticket, iim_result* res);
/* Blocks until the request is done, then copies its result. */
int iim_server_wait(iim_server* s, uint64_t ticket, iim_result* res);
int iim_server_stats_get(iim_server* s, iim_server_stats* st);
/* Seconds on the server's clock (the time base of iim_result). */
double iim_server_clock(iim_server* s);
/* Finishes every queued and running request, then frees the server. */
void iim_server_destroy(iim_server* s);

#ifdef __cplusplus
}
#endif
#endif /* IIM_H */
