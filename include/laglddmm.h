/*
 * laglddmm.h - C ABI of the MI355X (gfx950) Lagrangian Gauss-Newton-Krylov
 * registration hot path.
 *
 * The library implements, on one GPU, the operations of Mang & Ruthotto,
 * "A Lagrangian Gauss-Newton-Krylov solver for mass- and intensity-
 * preserving diffeomorphic image registration" (SIAM J. Sci. Comput. 2017):
 * RK4 characteristics of a stationary or time-dependent velocity
 * (Algorithm 1), the transport solve (eq. rhoEndIR) and the particle push-
 * forward (eq. rhoEndOMT), the Jacobian products of the final state with
 * respect to the velocity (Sec. 3.2), the Gauss-Newton Hessian matvec
 * (Sec. 3.2) and the spectral preconditioner (Sec. 3.2, PCG paragraph).
 *
 * Conventions (all calls):
 *  - Grids are cell-centred and periodic on the box [0, extent_0) x ... ;
 *    sizes are given x first; unused axes (dim = 2) have size 1.
 *  - All arrays are float32, contiguous, x fastest:
 *      image-shaped   : [m_z][m_y][m_x]                       (n_points floats)
 *      velocity-shaped: [nt_nodes][dim][m_z][m_y][m_x]       (n_unknowns floats)
 *                       component 0 is the x component
 *      phi            : [dim][n_points], the displacement of each
 *                       characteristic's end point from its start cell centre
 *                       (not wrapped; periodic wrap happens inside
 *                       interpolation).
 *  - Every pointer argument except the plan and `stream` is a DEVICE pointer
 *    unless stated otherwise.  The caller allocates and owns every buffer;
 *    the plan owns only its workspace.  Outputs must not alias inputs.
 *  - `stream` is a hipStream_t (NULL = the default stream).  The hot-path
 *    calls are asynchronous on that stream and allocate nothing (the
 *    Gauss-Newton step, and the solvers built on it, may grow the assembled
 *    Jacobian's storage: see lag_gn_step).  Plan
 *    creation/destruction allocate/free and synchronise the device; the
 *    profiling reads, lag_pcg and lag_gn_solve synchronise (documented at
 *    each).
 *  - A plan is used by one stream at a time (it owns scratch buffers).
 *  - Return value: LAG_OK (0) or one of the LAG_E* codes; no exception ever
 *    crosses the ABI.  lag_strerror() names a code.  After LAG_EHIP the HIP
 *    error string is available from lag_last_hip_error().
 */
#ifndef LAGLDDMM_H
#define LAGLDDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LAG_OK = 0,
    LAG_EINVAL = 1,        /* bad argument: null pointer, bad size/model/dir  */
    LAG_EUNSUPPORTED = 2,  /* valid request this build does not implement     */
    LAG_EHIP = 3,          /* a HIP runtime call or kernel launch failed      */
    LAG_ENOMEM = 4,        /* device allocation failed (allocating calls only)*/
    LAG_EBREAKDOWN = 5,    /* PCG met p^T H p <= 0                            */
    LAG_ELINESEARCH = 6,   /* Armijo line search found no acceptable step     */
    LAG_ETOOLARGE = 7      /* problem exceeds a fixed-size scratch buffer     */
};

enum { LAG_TRANSPORT = 0, LAG_CONTINUITY = 1 };   /* eq. transport / eq. continuity */
enum { LAG_DIFFUSION = 0, LAG_CURVATURE = 1 };    /* H1 / H2 seminorm regulariser (Sec. 2.1) */

/* One registration problem.  The discrete velocity has
 * n_unknowns = nt_nodes * dim * prod(vel_m) entries (Sec. 3: n = (n_t+1) d m^d),
 * stored at the velocity-grid cell centres and, when nt_nodes > 1, at the
 * time nodes t_j = j / (nt_nodes - 1).  Characteristics start at every image
 * cell centre (n_points = prod(img_m)). */
typedef struct lag_problem {
    int32_t dim;          /* 2 or 3                                            */
    int32_t img_m[3];     /* image cells per axis (x, y, z); >= 2 on used axes */
    int32_t vel_m[3];     /* velocity cells per axis; >= 2 on used axes        */
    double  extent[3];    /* domain edge lengths, > 0                          */
    int32_t nt_nodes;     /* 1 = stationary velocity, else n_t + 1 >= 2        */
    int32_t model;        /* LAG_TRANSPORT or LAG_CONTINUITY                   */
    int32_t reg;          /* LAG_DIFFUSION or LAG_CURVATURE                    */
    int32_t nsteps;       /* N >= 1 RK4 steps over the unit time interval      */
    double  alpha;        /* regularisation weight, >= 0                       */
    double  gamma;        /* Hessian shift gamma I (Sec. 3.2), >= 0            */
    int32_t jac_blocks;   /* capacity of the assembled Jacobian, in velocity-
                             cell blocks per characteristic (0 = no assembled
                             Jacobian; used only by the transport model with
                             a stationary velocity; <= 255).  lag_gn_step
                             raises it when an assembly overflows (see
                             there); lag_jacobian_assemble never does.         */
} lag_problem;

typedef struct lag_plan_s* lag_plan;

/* ---- host-only helpers (no GPU needed) -------------------------------- */

/* Validate a problem description.  Host only; touches no device. */
int lag_problem_check(const lag_problem* prob);

/* Sizes of a valid problem: characteristics (= image cells) and unknowns.
 * Host pointers; either output may be NULL. */
int lag_problem_sizes(const lag_problem* prob, int64_t* n_points, int64_t* n_unknowns);

const char* lag_strerror(int status);

/* Text of the last HIP error seen by this library in the calling thread
 * (empty string if none).  The returned pointer stays valid until the next
 * library call in that thread. */
const char* lag_last_hip_error(void);

/* ---- plans ------------------------------------------------------------- */

/* Create a plan for `prob` on the current HIP device: validates the problem,
 * allocates the workspace (packed velocity copies, RK4 stage-time tables,
 * FFT twiddles, scratch) and uploads host-computed tables.  This is the
 * allocating call; it synchronises the device.  *out receives the plan.
 * LAG_EUNSUPPORTED if the 64-bit accumulation tile of one brick (8 bytes
 * per velocity node of the tile and field) does not fit the device's LDS
 * per block (only for very many time nodes). */
int lag_plan_create(const lag_problem* prob, lag_plan* out);

/* lag_plan_create with a chosen brick shape: brick_target[a] image cells per
 * brick along axis a (a < dim; 1..1024; NULL = the default 16 x 16 x 12 in
 * 3-D, 16 x 16 in 2-D).  A wave's 64 lanes cover a 4 x 4 x 4 or 8 x 4 x 2
 * lattice of velocity cells in 3-D (the one that divides the shape), 8 x 8
 * in 2-D.  The shape is rounded to whole wave lattices and shrunk until the
 * LDS tile fits 64 KB, as for the default.  Bricks change
 * only the order of floating-point sums: results agree to rounding. */
int lag_plan_create_tuned(const lag_problem* prob, const int32_t* brick_target, lag_plan* out);

/* Release a plan and its workspace (synchronises the device).  NULL is OK. */
int lag_plan_destroy(lag_plan plan);

/* Copy of the plan's problem (host pointer). */
int lag_plan_problem(lag_plan plan, lag_problem* out);

/* Status bits the adjoint kernels (lag_vjp, gn_hessmat, the gradient, the
 * Jacobian assembly) accumulate in the plan, read into *flags (host) after
 * `stream` has finished; clear != 0 resets them.  Synchronises `stream`.
 *   bit 0 (1): some characteristic's RK4 step Jacobians were close to
 *              singular (product of their condition numbers above 100), so
 *              its adjoint took the reverse sweep with recomputed step start
 *              points instead of forward recovery (Sec. 3.2's derivative
 *              recursion run backward; no matrix is inverted).  Informational:
 *              the results are exact either way.
 *   bit 1 (2): forward recovery met an exactly singular step Jacobian and
 *              used the identity for it.  The guard above routes such
 *              characteristics to the recomputed sweep first, so this bit
 *              signals an internal error.
 *   bit 2 (4): a matrix-free adjoint value fell outside the accumulation
 *              tile that the characteristic's forward cells had been checked
 *              against, and was added by a float atomic (correct, but not
 *              reproducible bit for bit).  Not expected: the reverse sweep
 *              samples the cells of the forward pass. */
int lag_plan_flags(lag_plan plan, int32_t* flags, int32_t clear, void* stream);

/* Work counters of the last matrix-free adjoint product (lag_vjp,
 * gn_hessmat, lag_gradient on the plan's stream): *deferred = number of
 * characteristics whose samples left their brick's accumulation tile (summed
 * apart in 64-bit fixed point), *redone = number of bricks whose first pass
 * was redone at the exact fixed-point unit.  Either pointer may be NULL.
 * Synchronises `stream`. */
int lag_adjoint_stats(lag_plan plan, int32_t* deferred, int32_t* redone, void* stream);

/* Kernel timing for measurement: when enabled, every launch of the
 * Gauss-Newton matvec's main kernel carries a pair of HIP events that the
 * dispatch on its stream stamps at the kernel's start and end (so the time
 * excludes the gap before the dispatch; up to 256 launches between reads).  Enabling
 * creates the events (host call, once per plan).  lag_profile_read
 * synchronises on the recorded events, returns the summed kernel time in
 * milliseconds and the number of timed launches (host pointers), and resets
 * the count. */
int lag_profile_enable(lag_plan plan, int32_t enable);
int lag_profile_read(lag_plan plan, double* ms_total, int32_t* launches);

/* ---- the hot path ------------------------------------------------------- */

/* Characteristics by RK4 with N equal steps (Algorithm 1 without the
 * derivative; classical fourth stage at y + dt*v3).  dir = -1 traces from
 * t = 1 back to t = 0, giving y(v, x_c, 1, 0) (transport); dir = +1 traces
 * from 0 to 1, giving y(v, x_c, 0, 1) (continuity).
 * v: velocity-shaped.  phi: [dim][n_points] output displacements. */
int lag_trace(lag_plan plan, const float* v, int32_t dir, float* phi, void* stream);

/* Transport solve u1(x_c) = T(y(v, x_c, 1, 0)) (eq. rhoEndIR): periodic
 * (bi/tri)linear interpolation of the image T at x_c + phi.
 * T, u: image-shaped; phi: [dim][n_points]. */
int lag_transport(lag_plan plan, const float* T, const float* phi, float* u, void* stream);

/* Particle push-forward u1 = F(y(v, x_c, 0, 1)) T (eq. rhoEndOMT) with hat
 * width equal to the image cell size, i.e. F is the transpose of linear
 * interpolation at the end points x_c + phi (mass preserving by
 * construction).  Deterministic: particles are binned by cell and every
 * cell sums its contributions in a fixed order (no float atomics).
 * T, u: image-shaped; phi: [dim][n_points]. */
int lag_pushforward(lag_plan plan, const float* T, const float* phi, float* u, void* stream);

/* Jacobian-vector product Jdv = (d_v u1) dv of the plan's model (Sec. 3.2,
 * derivative of u1; Algorithm 1's derivative recursion applied to dv).
 * v, dv: velocity-shaped; T, Jdv: image-shaped.  For the transport model
 * Jdv[i] = grad T(y_i) . (d_v y_i) dv; for continuity
 * Jdv = sum_j T_j grad_y F(y_j) (d_v y_j) dv (deterministic binned sum). */
int lag_jvp(lag_plan plan, const float* v, const float* T, const float* dv,
            float* Jdv, void* stream);

/* Vector-Jacobian product JTw = (d_v u1)^T w (the data part of the gradient,
 * Sec. 3.2).  v, JTw: velocity-shaped; T, w: image-shaped.  Characteristics
 * are recomputed, never stored (memory independent of N).  Reproducible bit
 * for bit: every velocity-grid sum is taken in integer fixed point (32-bit
 * per brick tile, 64-bit for characteristics that leave their tile), whose
 * value does not depend on the order of the additions, and the tiles are
 * combined in a fixed order. */
int lag_vjp(lag_plan plan, const float* v, const float* T, const float* w,
            float* JTw, void* stream);

/* Gauss-Newton Hessian matvec (Sec. 3.2):
 *   Hp = h^d J^T (W (J p)) + alpha h_v^d sum_j w_j A p_j + gamma p,
 * h^d = image cell volume, h_v^d = velocity cell volume, w_j the
 * trapezoidal time weights of the velocity nodes (1 if stationary),
 * A = -Laplace_h (diffusion) or Laplace_h^2 (curvature), periodic.
 * wvox: image-shaped voxel weights W, or NULL for W = 1.
 * v, p, Hp: velocity-shaped; T image-shaped.  Transport: one fused pass per
 * characteristic; continuity: J p on the image grid, then J^T.  Reproducible
 * bit for bit (the sums of lag_vjp). */
int gn_hessmat(lag_plan plan, const float* v, const float* T, const float* wvox,
               const float* p, float* Hp, void* stream);

/* Spectral preconditioner (Sec. 3.2, PCG paragraph): per velocity component
 * and time node j, z = F^-1[ F(r) / mu_j(k) ] with
 * mu_j(k) = alpha h_v^d w_j lambda_A(k) + gamma, the symbol of the
 * regulariser block of H on the periodic grid (DFT, hand-written radix-2/3/5
 * FFT).  If mu_j(0) = 0 (gamma = 0) the constant mode is divided by the
 * smallest nonzero mu_j instead (pseudo-inverse made SPD).
 * r, z: velocity-shaped.  Supported sizes: every vel_m[a] <= 1024 whose
 * prime factors are 2, 3 and 5; other sizes return LAG_EUNSUPPORTED.
 * alpha = gamma = 0 (no regulariser block to invert) returns LAG_EINVAL. */
int spectral_precond_apply(lag_plan plan, const float* r, float* z, void* stream);

/* ---- allocation-free variant ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * push-forward as lag_pushforward, without a plan.  Its binning scratch is a
 * file-scope device array of LAG_NOALLOC_SCRATCH_BYTES that the loader
 * places on every GPU the library runs on and that stays there until the
 * process ends; the call itself allocates nothing and needs no plan.  The
 * scratch holds 36 bytes per image cell in 2-D and 52 in 3-D (plus
 * alignment), so problems up to about 1.8 M cells (2-D) or 1.2 M cells (3-D)
 * fit; larger ones return LAG_ETOOLARGE.  All calls on one GPU share that
 * GPU's scratch: calls that overlap on one GPU (concurrent streams or host
 * threads) race and must be serialised by the caller.  The result is
 * bitwise that of lag_pushforward.  T, u: image-shaped; phi: [dim][n_points]
 * (device pointers); prob: host pointer. */
#define LAG_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int lag_pushforward_noalloc(const lag_problem* prob, const float* T, const float* phi, float* u,
                            void* stream);

/* ---- assembled Jacobian (transport model, stationary velocity) ----------
 * The paper notes that the sparse derivative can be built explicitly to
 * speed up matrix-vector products (Sec. 1.1; Sec. 3.3).  Row i of
 * J = d u1/d v, grad T(y_i)^T d y_i/d v, is stored as one block of
 * 2^d x dim values per velocity cell the characteristic's RK4 samples visit
 * (plan capacity: jac_blocks blocks per characteristic).  Assembly costs
 * about one lag_vjp; each following product streams the stored blocks. */

/* Assemble J(v) for the plan's template T.  Synchronises `stream`.
 * *stored (host) is set to 1 if every row fit the plan's capacity (the
 * assembled calls below may then be used until the next assembly), else 0
 * (callers use the matrix-free calls).  LAG_EUNSUPPORTED if the plan has no
 * Jacobian storage (jac_blocks = 0, continuity, or a time-dependent
 * velocity). */
int lag_jacobian_assemble(lag_plan plan, const float* v, const float* T, int32_t* stored,
                          void* stream);

/* Size of the last assembly (host pointers): stored blocks (0 if none is
 * stored), the largest block count of any characteristic (may exceed the
 * capacity, which is why an assembly was not stored; above 255 if a block
 * lay beyond the packed cell offset's reach of 512 cells, which no capacity
 * can store), and the bytes one block occupies (values plus packed cell). */
int lag_jacobian_info(lag_plan plan, int64_t* blocks, int32_t* max_blocks, int32_t* bytes_per_block);

/* gn_hessmat with the assembled J of the last successful assembly:
 * Hp = h^d J^T (W (J p)) + alpha h_v^d A p + gamma p.  LAG_EINVAL if no
 * assembly is stored. */
int gn_hessmat_assembled(lag_plan plan, const float* wvox, const float* p, float* Hp,
                         void* stream);

/* J^T w with the assembled J (w image-shaped, JTw velocity-shaped). */
int lag_vjp_assembled(lag_plan plan, const float* w, float* JTw, void* stream);

/* ---- compositions used by the Gauss-Newton driver ----------------------- */

/* Regulariser part of H: out = alpha h_v^d w_j A p_j + gamma p. */
int lag_reg_apply(lag_plan plan, const float* p, float* out, void* stream);

/* Objective J(v) = D + alpha S (eq. discOpti, eq. SSD, Sec. 2.1).
 * u (image-shaped, may be NULL) receives u1(v); out3 (device, 3 doubles)
 * receives {J, D, S}. */
int lag_objective(lag_plan plan, const float* v, const float* T, const float* R,
                  float* u, double* out3, void* stream);

/* Gradient g = J^T (h^d (u1 - R)) + alpha h_v^d w_j A v (Sec. 3.2) and the
 * objective (out3 as in lag_objective; may be NULL). */
int lag_gradient(lag_plan plan, const float* v, const float* T, const float* R,
                 float* g, double* out3, void* stream);

/* lag_gradient at v = 0 without tracing: the RK4 map of a zero field is the
 * identity, so the characteristics stay at the cell centres and the adjoint
 * sweep reduces to the sum of the RK4 stage weights at the start points
 * (Sec. 3.1 with v = 0; both models, stationary or time-dependent).  Same
 * result as lag_gradient with v = 0 up to float rounding; used by
 * lag_gn_solve for the reference norm |g(0)| of its stopping test.  g
 * velocity-shaped output; out3 as in lag_gradient (may be NULL). */
int lag_gradient_at_zero(lag_plan plan, const float* T, const float* R, float* g, double* out3,
                         void* stream);

/* Dot product of two n-vectors with float64 accumulation, deterministic
 * order; result written to out (device, 1 double). n <= 2^31. */
int lag_dot(lag_plan plan, int64_t n, const float* x, const float* y, double* out,
            void* stream);

typedef struct lag_pcg_info {
    int32_t iters;        /* PCG iterations taken                           */
    int32_t matvecs;      /* gn_hessmat calls                               */
    int32_t breakdown;    /* 1 if p^T H p <= 0 stopped the iteration        */
    double  relres;       /* final |r| / |b|                                */
} lag_pcg_info;

/* lag_gradient whose data term J^T (h^d res) uses the assembled J; v and T
 * must be the ones passed to the last successful lag_jacobian_assemble. */
int lag_gradient_assembled(lag_plan plan, const float* v, const float* T, const float* R,
                           float* g, double* out3, void* stream);

/* Preconditioned CG for H(v) x = b (Sec. 3.2, eq. solveGN), x0 = 0,
 * stopping when |r|_2 <= tol |b|_2 or after maxit iterations.  H is
 * gn_hessmat with voxel weights wvox (NULL = 1); the preconditioner is
 * spectral_precond_apply.  Runs on `stream` and synchronises it once per
 * iteration to read the residual (host-side control flow).  info: host
 * pointer, may be NULL.  Returns LAG_EBREAKDOWN if p^T H p <= 0 (x then
 * holds the last iterate). */
int lag_pcg(lag_plan plan, const float* v, const float* T, const float* wvox,
            const float* b, float* x, double tol, int32_t maxit,
            lag_pcg_info* info, void* stream);

/* lag_pcg with the assembled Gauss-Newton operator (gn_hessmat_assembled). */
int lag_pcg_assembled(lag_plan plan, const float* wvox, const float* b, float* x, double tol,
                      int32_t maxit, lag_pcg_info* info, void* stream);

/* lag_pcg with the stopping test on the device, so the iteration can run as
 * a captured HIP graph: `iters_per_graph` (1..64) iterations are captured
 * once per plan and argument set (v, T, wvox, b, x) and replayed; a device
 * flag set by the residual test (or the iteration cap, or a breakdown)
 * makes every kernel of the remaining captured iterations return at entry.
 * The host reads the flag once per replay instead of once per iteration.
 * Same iterates as lag_pcg.  Allocating on first use (a control block, a
 * private capture stream, the graph); a cached graph is rebuilt when the
 * arguments change and freed with the plan.  A plan's graph serves one
 * stream at a time, like the plan. */
int lag_pcg_graph(lag_plan plan, const float* v, const float* T, const float* wvox,
                  const float* b, float* x, double tol, int32_t maxit, int32_t iters_per_graph,
                  lag_pcg_info* info, void* stream);

/* lag_pcg_graph with the assembled Gauss-Newton operator. */
int lag_pcg_assembled_graph(lag_plan plan, const float* wvox, const float* b, float* x, double tol,
                            int32_t maxit, int32_t iters_per_graph, lag_pcg_info* info, void* stream);

typedef struct lag_gn_options {
    double  gtol;           /* stop when |g| <= gtol |g(v=0)|   (1e-2)        */
    int32_t max_gn;         /* Gauss-Newton iteration cap         (50)        */
    double  pcg_tol;        /* PCG relative residual               (0.1)      */
    int32_t pcg_maxit;      /* PCG iteration cap                   (50)       */
    double  armijo_c1;      /* sufficient decrease constant        (1e-4)     */
    int32_t max_halvings;   /* line-search step halvings           (10)       */
    int32_t graph_iters;    /* 0: host-driven PCG; k in 1..64: PCG with the
                               stopping test on the device, k iterations per
                               captured-graph replay (lag_pcg_graph)   (0) */
} lag_gn_options;

typedef struct lag_gn_info {
    int32_t iters;          /* Gauss-Newton iterations (search directions)    */
    int32_t pcg_iters;      /* total PCG iterations                           */
    int32_t matvecs;        /* total gn_hessmat calls                          */
    int32_t converged;      /* 1 if the gradient tolerance was met            */
    double  J0, J;          /* objective at the start and at the end          */
    double  g0, gnorm;      /* |g(v=0)| and final |g|                         */
} lag_gn_info;

/* Default options (host pointer). */
void lag_gn_default_options(lag_gn_options* opt);

typedef struct lag_gn_step_info {
    int32_t assembled;      /* 1 if the step used the assembled Jacobian       */
    int32_t pcg_iters;      /* PCG iterations                                 */
    int32_t matvecs;        /* Gauss-Newton matvecs                            */
    int32_t halvings;       /* line-search step halvings                       */
    int32_t stopped;        /* 1 if |g| <= gstop and no step was taken         */
    int32_t accepted;       /* 1 if the line search found a step               */
    double  J, gnorm;       /* objective and gradient norm at v                */
    double  J_next, mu;     /* objective at v_next and the step length         */
} lag_gn_step_info;

/* One inexact Gauss-Newton iteration (Sec. 3.2, eq. solveGN): gradient at v,
 * PCG for H(v) dv = -g (assembled Jacobian when the plan has one and it
 * fits, else matrix-free), Armijo backtracking, v_next = v + mu dv.  When
 * the assembly overflows the plan's capacity, the step reallocates the
 * Jacobian storage once for the longest row seen plus a quarter (at most
 * 255 blocks; only if the new arrays fit in half of the free device memory)
 * and assembles again; the larger capacity stays with the plan.  If
 * |g| <= gstop, no step is taken and v_next = v.  v and v_next are distinct
 * velocity-shaped device buffers.  Synchronises `stream`.  Returns
 * LAG_ELINESEARCH if no acceptable step was found (v_next = v). */
int lag_gn_step(lag_plan plan, const float* T, const float* R, const float* v, float* v_next,
                const lag_gn_options* opt, double gstop, lag_gn_step_info* info, void* stream);

/* Inexact Gauss-Newton-Krylov solve of min_v J(v) (Sec. 3.2): search
 * direction from lag_pcg, Armijo backtracking by halving.  v is the start
 * value on entry and the solution on exit (velocity-shaped, device).
 * opt: host pointer or NULL for defaults; info: host pointer or NULL.
 * Each iteration is lag_gn_step.  The stopping test is
 * |g| <= gtol |g(v = 0)|: the reference comes from lag_gradient_at_zero, or,
 * when v is zero on entry, from the first step's own gradient.  Synchronises
 * `stream` to read scalars.  Returns LAG_ELINESEARCH if the line search
 * fails (v then holds the last accepted iterate). */
int lag_gn_solve(lag_plan plan, const float* T, const float* R, float* v,
                 const lag_gn_options* opt, lag_gn_info* info, void* stream);

/* ---- multilevel continuation (Sec. 3.2, last paragraph) -----------------
 * Level l+1 has half the image and velocity cells of level l along every
 * axis (all sizes even and >= 4 on every level but the coarsest). */

/* Restrict an image of the plan's image grid to the grid with half the cells
 * per axis: each coarse value is the mean of its 2^d fine cells.  f: image-
 * shaped for the plan; coarse: (prod img_m / 2^d) floats. */
int lag_restrict_image(lag_plan plan, const float* f, float* coarse, void* stream);

/* Refine a velocity from the grid with half the cells per axis to the plan's
 * velocity grid by cell-centred periodic (bi/tri)linear interpolation (axis
 * weights 3/4 and 1/4), per component and time node.  v_coarse:
 * n_unknowns / 2^d floats; v_fine: velocity-shaped for the plan. */
int lag_prolong_velocity(lag_plan plan, const float* v_coarse, float* v_fine, void* stream);

/* Average an image of the plan's image grid over the cells of the plan's
 * velocity grid: each output value is the integral of the piecewise-constant
 * image over a velocity cell divided by the cell's volume (per axis, fine
 * cell i weighs its overlap with the coarse cell; any ratio img_m / vel_m
 * >= 1, also a non-integer one such as 224 / 64).  For a ratio of 2 this is
 * lag_restrict_image.  It feeds images to the warm-start network below.
 * f: image-shaped; out: prod(vel_m) floats.  LAG_EINVAL if some
 * img_m[a] < vel_m[a]. */
int lag_resample_to_velocity_grid(lag_plan plan, const float* f, float* out, void* stream);

/* Coarse-to-fine Gauss-Newton: `levels` levels (1..8; level 0 = `finest`),
 * T and R restricted level by level, lag_gn_solve on each level starting
 * from the refined solution of the level below (zero on the coarsest).  v
 * (velocity-shaped for `finest`) receives the finest solution; its input is
 * the start value only when levels = 1.  infos: host array of `levels`
 * entries (coarsest first) or NULL.  Allocating: creates one plan and the
 * restricted images per level and frees them before returning; synchronises
 * `stream`.  A coarse level whose line search stalls hands its last
 * accepted iterate to the next level; LAG_ELINESEARCH is returned only if
 * the finest level's line search fails. */
int lag_multilevel_solve(const lag_problem* finest, int32_t levels, const float* T, const float* R,
                         float* v, const lag_gn_options* opt, lag_gn_info* infos, void* stream);

/* ---- many problems at once -------------------------------------------------
 * For batches of independent registrations of uneven sizes (2-D and 3-D,
 * transport and continuity): a brick-shape autotuner and a batched driver.
 * Not in the paper; for callers with many small problems, where a single
 * solve cannot fill the GPU. */

/* Time the Gauss-Newton matvec of `prob` (assembled when prob->jac_blocks >
 * 0 and the model is transport, matrix-free otherwise) at a smooth synthetic
 * velocity with about two cells of displacement, for a fixed list of brick
 * shapes (3-D: 16x16x12, 16x16x8, 8x16x8, 16x16x16, 8x8x8, 32x16x8, 16x8x8; 2-D: 16x16,
 * 32x16, 32x32, 64x32, 16x8, 64x64), and return the fastest shape in
 * best_target[3] (for lag_plan_create_tuned) and its time per matvec in
 * *best_ms (may be NULL).  Allocating (one plan per shape, freed) and
 * synchronising `stream`. */
int lag_autotune_bricks(const lag_problem* prob, int32_t* best_target, double* best_ms, void* stream);

/* Solve npairs independent problems: pair i is (probs[i], T[i], R[i]) with v[i]
 * the start value and the solution (device pointers of each problem's
 * sizes).  `workers` (1..16) host threads, each with its own HIP stream and a
 * plan per distinct problem, take pairs largest first and run lag_gn_solve
 * with `opt` (graph_iters > 0 keeps the PCG loops on the device).  Brick
 * shapes: `bricks` (host, npairs x 3, e.g. from lag_autotune_bricks; the
 * first pair of each distinct problem decides) or, if NULL and `autotune`
 * is non-zero, lag_autotune_bricks per distinct problem, else the default.
 * infos (host array of npairs, may be NULL) and status (host array of
 * npairs) receive each solve's info and return code.  Allocating and
 * synchronising; returns the first status that is neither LAG_OK nor
 * LAG_ELINESEARCH, else LAG_OK.  The T, R, v buffers of different pairs must
 * not overlap. */
int lag_batch_solve(int32_t npairs, const lag_problem* probs, const float* const* T, const float* const* R,
                    float* const* v, const lag_gn_options* opt, int32_t workers, const int32_t* bricks,
                    int32_t autotune, lag_gn_info* infos, int32_t* status);

/* The batch in lockstep from one host thread, with the PCG iterations of all
 * pairs in one captured HIP graph.  Every pair has its own plan (brick
 * shape from `bricks`, host npairs x 3, or the default if NULL).  Each
 * Gauss-Newton iteration (Sec. 3.2, as lag_gn_step) takes the gradients of
 * all running pairs on four HIP streams, starts their PCG solves, replays
 * the batch graph (opt->graph_iters PCG iterations of every pair per
 * replay, 4 if 0) until every pair's device-side stopping test has halted
 * it, then runs the Armijo line search of all pairs round by round (one
 * synchronisation per halving round).  A pair that has stopped keeps its
 * place in the graph with its PCG halted (its kernels return at entry).
 * The graph is captured again only when some running pair changes its
 * operator (assembled or matrix-free) or its Jacobian storage grows.  The
 * stopping test and its reference |g(v = 0)| are those of lag_gn_solve;
 * infos (host, npairs, may be NULL) and status (host, npairs: LAG_OK or
 * LAG_ELINESEARCH) as in lag_batch_solve.  Allocating and synchronising. */
int lag_batch_solve_graph(int32_t npairs, const lag_problem* probs, const float* const* T, const float* const* R,
                          float* const* v, const lag_gn_options* opt, const int32_t* bricks, lag_gn_info* infos,
                          int32_t* status);

/* ---- learned warm start: a 3-D U-Net on the MFMA units --------------------
 * Maps the template and reference, resampled to a cubic grid of side `size`
 * (the velocity grid), to a stationary velocity [3][size^3] that starts the
 * Gauss-Newton solve.  Four levels (size, size/2, size/4, size/8), channels
 * channels[0..3] in {16, 32, 64}, 3x3x3 periodic convolutions with ReLU,
 * 2x average pooling, nearest-neighbour upsampling with skip
 * concatenation, and a 1x1 output head scaled by out_scale.  Convolutions
 * run as implicit GEMMs on bf16 MFMA with float32 accumulation; weights are
 * kept in float32 for Adam and copied to bf16 by the first pass after they
 * change (creation, lag_cnn_set_params, lag_cnn_adam_step).  Parameters
 * are stored flat, layer by layer (e0a e0b e1a e1b e2a e2b ma mb d2 d1 d0
 * head), each as W[taps][cin][cout] followed by b[cout] (taps = 27, 1 for
 * the head; the first layer has cin = 2). */
typedef struct lag_cnn_config {
    int32_t size;          /* grid side, a multiple of 32 in [32, 256]        */
    int32_t channels[4];   /* per level, each 16, 32 or 64                    */
    float   in_scale;      /* multiplies T and R on input                     */
    float   out_scale;     /* multiplies the head's output                    */
    uint64_t seed;         /* He-normal initialisation                        */
} lag_cnn_config;

typedef struct lag_cnn_s* lag_cnn;

void lag_cnn_default_config(lag_cnn_config* cfg);
/* Allocating: parameters, Adam moments and activation buffers. */
int lag_cnn_create(const lag_cnn_config* cfg, lag_cnn* out);
int lag_cnn_destroy(lag_cnn net);
int lag_cnn_param_count(lag_cnn net, int64_t* count);
/* Host copies of the flat parameters / of the gradients of the last
 * lag_cnn_backward (synchronising). */
int lag_cnn_get_params(lag_cnn net, float* host);
int lag_cnn_set_params(lag_cnn net, const float* host);
int lag_cnn_get_grads(lag_cnn net, float* host);
/* Inference: T, R are size^3 images (x fastest); v receives [3][size^3]. */
int lag_cnn_forward(lag_cnn net, const float* T, const float* R, float* v, void* stream);
/* Forward, loss = 1/2 mean (v - target)^2 written to *loss (device double),
 * and the gradient of every parameter (kept in the net).  Every gradient sum
 * runs in a fixed order, so repeated calls give the same bits. */
int lag_cnn_backward(lag_cnn net, const float* T, const float* R, const float* target, float* v,
                     double* loss, void* stream);
/* One Adam update of the parameters with the last gradients. */
int lag_cnn_adam_step(lag_cnn net, float lr, float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LAGLDDMM_H */
