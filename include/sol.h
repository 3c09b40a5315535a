/*
 * sol.h -- C ABI of the MI355X solidification / macro-segregation step library.
 *
 * One time step is the fully decoupled operator-splitting scheme of
 * arXiv 2303.10783 (Algorithm 1): momentum predictor (eq. 3.3), pressure
 * correction (eq. 3.4) and projection (eq. 3.5), matrix-based solute
 * transport (eq. 3.10), split energy equation (eqs. 3.11-3.12) and the
 * lever-rule phase / concentration update (eqs. 3.13-3.18), on a uniform
 * staggered grid (Section 3, spatial discretization) with the systems
 * assembled term-wise (Section 4): constant-coefficient terms (transient,
 * diffusion, wall terms, the pressure Laplacian) once at creation, upwind
 * convection, Carman-Kozeny drag and the right-hand sides every step.
 * Linear systems: CG preconditioned by a multigrid V-cycle (pressure;
 * Jacobi on request) and BiCGSTAB preconditioned by one or two Jacobi
 * sweeps (momentum, solute, energy), stopped on the true residual
 * ||b - A x||_2 <= tol ||b||_2.  Every step of the path runs in HIP kernels
 * on one gfx950 device; the library never computes a step on the host.
 *
 * Conventions
 *  - All functions return an int status (SOL_OK or a negative SOL_E* code);
 *    sol_last_error() returns a thread-local message owned by the library.
 *  - Every argument is validated before any device work; on an error nothing
 *    partial is visible (state stays at the last completed step).
 *  - Layouts: FP64, lexicographic, x fastest (Section 4, eq. 4.2).
 *      cells  : nx*ny*nz, index i + nx*(j + ny*k)            (p, T, C, gl, Cl, Cs)
 *      u faces: interior x-faces, (nx-1)*ny*nz, index (i-1) + (nx-1)*(j + ny*k), i = 1..nx-1
 *      v faces: interior y-faces, nx*(ny-1)*nz
 *      w faces: interior z-faces, nx*ny*(nz-1) (3D only; 2D has none)
 *    Wall faces are impermeable and carry no unknown.  In 2D nz = 1, gravity
 *    acts along -y; in 3D along -z.
 *  - Ownership: a handle owns all device memory of its case, allocated with
 *    ctx->alloc (e.g. a framework's caching allocator) when given, else
 *    hipMalloc; work is queued on ctx->stream (default stream when NULL).
 *    Host buffers are always caller-owned.
 *  - Threading: a handle is not thread-safe; distinct handles may be used
 *    from distinct threads on distinct streams.
 */
#ifndef SOL_H
#define SOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOL_OK          0
#define SOL_EINVAL     -1   /* invalid argument                                  */
#define SOL_ENOMEM     -2   /* device allocation failed                          */
#define SOL_ENOCONV    -3   /* a Krylov solve reached max_iter; state rolled back */
#define SOL_ENONFINITE -4   /* non-finite input field or solver breakdown         */
#define SOL_EDEVICE    -5   /* HIP runtime error                                  */
#define SOL_EBUSY      -6   /* handle is part of a live batch                     */

/* systems (matrix rows); also the order of per-system statistics */
#define SOL_SYS_U 0
#define SOL_SYS_V 1
#define SOL_SYS_W 2
#define SOL_SYS_P 3   /* pressure correction phi (eq. 3.4), cells          */
#define SOL_SYS_C 4   /* solute C^{n+1} (eq. 3.10), cells                   */
#define SOL_SYS_T 5   /* intermediate temperature T* (eq. 3.11), cells      */

/* field mask bits; host_src / host_dst arrays are indexed by bit position */
#define SOL_F_U      (1u << 0)
#define SOL_F_V      (1u << 1)
#define SOL_F_W      (1u << 2)
#define SOL_F_P      (1u << 3)
#define SOL_F_T      (1u << 4)
#define SOL_F_C      (1u << 5)
#define SOL_F_GL     (1u << 6)
#define SOL_F_CL     (1u << 7)
#define SOL_F_CS     (1u << 8)
/* read-only intermediates of the last completed step */
#define SOL_F_USTAR  (1u << 9)    /* u* (face layout of u)  */
#define SOL_F_VSTAR  (1u << 10)
#define SOL_F_WSTAR  (1u << 11)
#define SOL_F_PHI    (1u << 12)   /* zero-mean pressure correction (cells) */
#define SOL_F_TSTAR  (1u << 13)   /* T* before the latent correction (cells) */
#define SOL_NFIELDS  14

#define SOL_THERMAL_ADIABATIC 0
#define SOL_THERMAL_ROBIN     1   /* q = h (T - T_ext), film in series with the half cell */
#define SOL_THERMAL_DIRICHLET 2   /* wall temperature T(t) = T0 - b t                     */
#define SOL_VELOCITY_NOSLIP   0
#define SOL_VELOCITY_FREESLIP 1

#define SOL_PRECISION_FP64  0
#define SOL_PRECISION_MIXED 1     /* FP32 Krylov inside FP64 iterative refinement */

typedef struct sol_handle sol_handle;
typedef struct sol_batch sol_batch;

typedef struct { int32_t dim, nx, ny, nz; double lx, ly, lz; } sol_grid;  /* dim 2|3; 2D: nz=1 */

/* Alloy and model constants (SI units, K, wt%).  Phase diagram: liquidus
   T = T_m + m_sp C_l (eq. 2.20), partition k_p (eq. 2.19), eutectic C_e.
   Boussinesq reference state T_ref, C_ref (eq. 2.9).  Carman-Kozeny drag
   with secondary arm spacing lambda2 and g^3 regularised by darcy_eps
   (eq. 2.8).  D_l >= 0: liquid solute diffusivity of eq. (3.7) (0: no
   diffusion, the minimal model's eq. 3.6). */
typedef struct {
    double rho, mu, cp, k, latent, beta_T, beta_C, lambda2;
    double T_m, m_sp, k_p, C_e, T_ref, C_ref, g, D_l, darcy_eps;
} sol_alloy;

typedef struct {
    int32_t thermal;            /* SOL_THERMAL_*                    */
    double h, T_ext, T0, b;     /* Robin: h, T_ext; Dirichlet: T0, b */
    int32_t velocity;           /* SOL_VELOCITY_*                   */
} sol_face_bc;

typedef struct { sol_face_bc face[6]; } sol_bcs;   /* W E S N B T; 2D uses the first four */

typedef struct {
    double dt, tol_p, tol_t;    /* time step; relative tolerances (pressure, transport) */
    int32_t max_iter;           /* per solve                                            */
    int32_t precision;          /* SOL_PRECISION_*                                       */
} sol_numerics;

typedef struct {
    void *stream;                          /* hipStream_t or NULL          */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} sol_device_ctx;

typedef struct {
    int32_t iters[6];            /* Krylov iterations per system, last step      */
    int64_t iters_total[6];      /* summed over the steps of this call            */
    double rel_resid[6];         /* final true ||b - A x|| / ||b|| per system      */
    double sum_resid[6];         /* sum of the final true residual vector          */
    double sum_C;                /* sum over cells of C^{n+1}                      */
    double sum_H;                /* sum over cells of T + (L/c_p) g_l at n+1       */
    double wall_flux;            /* sum over cooled-wall cells of U/(rho c_p h)(T* - T_wall) */
    double div_star;             /* ||D u*||_2                                     */
    double div_new;              /* ||D u^{n+1}||_2                                */
    int64_t step;                /* completed steps of the handle                  */
    int64_t redone;              /* steps of the handle run twice: the momentum and
                                    pressure solves hand over before their true-
                                    residual check; when a check asks for a restart
                                    the step is discarded before its commit and run
                                    again with every check in order (cumulative)   */
} sol_step_stats;

/* Create a case.  Defined by the problem statement of Algorithm 1 (given the
   initial fields and the boundary conditions, advance the scheme), the alloy
   properties of Table 1 and the wall conditions of Section 5 (convective
   cooling q = h (T - T_ext), adiabatic, rigid no-slip and free-slip walls,
   prescribed wall temperature T0 - b t), on the staggered grid of Section 3
   (spatial discretization).
   Validates every argument (e.g. nx < 2, dt <= 0, k_p outside (0,1),
   m_sp >= 0, D_l < 0 -> SOL_EINVAL), allocates device memory, builds the
   constant-coefficient systems of the term-wise split of Section 4
   (transient, diffusion, wall terms, pressure Laplacian) on the device, and
   sets the initial state u = v = w = p = 0, C = C_ref, g_l = 1,
   C_l = C_ref, C_s = 0, T = T_ref.  ctx may be NULL (hipMalloc and the
   default stream).  *out receives the handle; on an error *out is set to
   NULL and nothing stays allocated. */
int sol_create(const sol_grid *grid, const sol_alloy *alloy, const sol_bcs *bcs,
               const sol_numerics *num, const sol_device_ctx *ctx, sol_handle **out);
void sol_destroy(sol_handle *h);

/* Write the level-n state of the scheme: the velocity and pressure of the
   momentum step (eqs. 3.3-3.5), the temperature and liquid fraction of the
   split energy step (eqs. 3.11-3.12), the mixture concentration of the
   solute step (eq. 3.10) and the phase concentrations of eqs. 3.17-3.18
   (initial state or restart).  Copies host fields (SOL_F_U..SOL_F_CS bits
   only) into the handle; host_src is an array of SOL_NFIELDS pointers
   indexed by bit position (layouts above), entries for unset bits are
   ignored; the caller keeps ownership.  Non-finite values ->
   SOL_ENONFINITE, a NULL pointer for a set bit or a bit outside
   SOL_F_U..SOL_F_CS -> SOL_EINVAL (nothing written in either case).
   Synchronous with respect to the caller's buffers.  Resets the time
   extrapolation of the initial guesses. */
int sol_write_fields(sol_handle *h, uint32_t mask, const double *const *host_src);

/* Read the fields the scheme produces: u, v, w, p (eqs. 3.3-3.5), T and g_l
   (eqs. 3.11-3.16), C (eq. 3.10), C_l and C_s (eqs. 3.17-3.18), and the
   intermediates u* (eq. 3.3), the pressure correction phi = p^{n+1} - p^n
   (eq. 3.4, zero mean) and T* (eq. 3.11).  Copies to caller-owned host
   buffers sized from the grid (layouts above), synchronously.  Intermediates
   (SOL_F_USTAR .. SOL_F_TSTAR) are those of the last completed step or
   sol_assemble call.  A NULL pointer for a set bit -> SOL_EINVAL. */
int sol_read_fields(sol_handle *h, uint32_t mask, double *const *host_dst);

/* Number of rows and structural nonzeros of a system: the 5- / 7-point
   pattern of the staggered-grid stencils (Section 4, the matrix picture of
   eq. 4.2), in-domain neighbours only.  Unknown system -> SOL_EINVAL. */
int sol_system_size(const sol_handle *h, int32_t system, int32_t *rows, int32_t *nnz);

/* Assemble, for the current state, the systems in system_mask (bit s =
   SOL_SYS_s) without solving: Section 4's matrix assembly (eqs. 4.1-4.4:
   upwind convection rows, diffusion rows, transient diagonal) with the
   term-wise split (constant terms built once at sol_create, convection,
   Carman-Kozeny drag of eq. 2.8, Boussinesq force of eq. 2.9 and the
   right-hand sides per call), for the momentum predictor (eq. 3.3), the
   pressure correction (eq. 3.4), the solute system with its A_g scaling
   (eqs. 3.9-3.10) and the energy system (eq. 3.11).  The momentum systems
   use the level-n fields; the pressure system takes the current velocity
   as u*; the solute and energy systems take the current velocity as the
   advecting field and the next time level for prescribed wall
   temperatures.  Bits beyond SOL_SYS_T -> SOL_EINVAL; SOL_EBUSY while the
   handle belongs to a batch. */
int sol_assemble(sol_handle *h, uint32_t system_mask);

/* Export the last assembled system (sol_assemble) as CSR: the matrix and
   right-hand side of Section 4 (eqs. 4.1-4.4) in the row order of eq. 4.2.
   Caller-owned host buffers sized from sol_system_size: int32
   row_ptr[rows+1], col_idx[nnz] ascending per row, val[nnz], rhs[rows].
   The values are those of the system's last assembly, by sol_assemble or
   by the last step (the solute and energy systems of a step are assembled
   with u^{n+1}).  The CSR pattern is built on the device at the first
   export of a system (device memory held by the handle).  Unknown system
   or a NULL buffer -> SOL_EINVAL. */
int sol_read_matrix(sol_handle *h, int32_t system, int32_t *row_ptr, int32_t *col_idx,
                    double *val, double *rhs);

/* Allocation-free variant of sol_read_matrix, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc).  Same arguments, output and
   errors as sol_read_matrix, but it allocates nothing: the CSR row counts,
   row pointers, columns and values are staged in a fixed device array of
   SOL_NOALLOC_SCRATCH_BYTES held by each GPU the library runs on until the
   process ends, the columns and values in blocks of rows that fit it.  A
   system whose row counts and row pointers (8 (rows + 1) bytes, about 4.19
   million rows) do not fit the array -> SOL_EINVAL.  Every call on a GPU
   shares that GPU's array: calls that overlap on one GPU (from other
   threads or streams) race.  Synchronous; the handle's device must be
   current. */
#define SOL_NOALLOC_SCRATCH_BYTES (32u << 20)
int sol_read_matrix_noalloc(sol_handle *h, int32_t system, int32_t *row_ptr, int32_t *col_idx, double *val,
                            double *rhs);

/* Advance nsteps time steps of Algorithm 1: momentum predictor (eq. 3.3),
   pressure correction (eq. 3.4), projection (eq. 3.5), solute (eq. 3.10),
   liquidus (eq. 3.13), energy (eqs. 3.11-3.12), phase update (eqs.
   3.14-3.16 and the eutectic rule after eq. 3.16), C_l and C_s (eqs.
   3.17-3.18).  stats may be NULL.  On SOL_ENOCONV / SOL_ENONFINITE the
   handle stays at the last completed step.  nsteps < 0 -> SOL_EINVAL;
   SOL_EBUSY while the handle belongs to a batch. */
int sol_step(sol_handle *h, int32_t nsteps, sol_step_stats *stats);

/* Device bytes sol_create would allocate for a case of this grid and
   precision (the state of Algorithm 1 on the grid of Section 3, the
   systems of Section 4 and the solver work space): admission control of
   served requests.  Invalid grid -> SOL_EINVAL. */
int sol_footprint_bytes(const sol_grid *grid, const sol_numerics *num, size_t *out);

/* Batches: n handles advanced together by Algorithm 1 (each case its own
   scheme, as sol_step), every kernel of the step launched
   once for all cases (uneven sizes allowed).  The handles keep their state
   and may not be stepped alone while the batch lives (SOL_EBUSY).  All
   handles must share one stream.  nsteps_per_case[i] steps for case i (a
   case with 0 sits out); per-case stats optional (array of n). */
int sol_batch_create(sol_handle *const *cases, int32_t n, sol_batch **out);
int sol_batch_step(sol_batch *b, const int32_t *nsteps_per_case, sol_step_stats *stats);
void sol_batch_destroy(sol_batch *b);

/* Kernel timing for roofline reports.  When enabled, HIP events on the
   handle's stream bracket windows of 16 consecutive CG launches (one event
   pair per window, starting every 32nd iteration), every single launch of
   the BiCGSTAB and multigrid kernels (events stamped by the dispatch itself)
   and every assembly / phase launch.  Every launch counts, also one queued
   after its solves converged (it exits at once: time, no bytes); samples of
   a solve that restarted are dropped.  sol_get_timing returns the number of
   timed launches, their summed duration and the algorithmic bytes those
   launches move (matrix values + vectors read and written once, per row of
   the systems that were iterating; FP32 values count 4 bytes).  Enabling or
   disabling resets the counters. */
#define SOL_KCLASS_CG        0   /* CG iteration (one kernel): p, s, x, r, w = A M r, (r,Mr), (w,Mr) */
#define SOL_KCLASS_BICG_A    1   /* BiCGSTAB: x, r update; p, v = A M p; (rh,v), (r,r) */
#define SOL_KCLASS_BICG_B    2   /* BiCGSTAB: s, t = A M s; (t,s), (t,t), (rh,s), (rh,t) */
#define SOL_KCLASS_BICG_C    3   /* unused (the x, r update rides in SOL_KCLASS_BICG_A); never launched */
#define SOL_KCLASS_ASM_MOM   4   /* momentum assembly                           */
#define SOL_KCLASS_ASM_TRN   5   /* solute + energy assembly                    */
#define SOL_KCLASS_PHASE     6   /* phase update + commit                       */
#define SOL_KCLASS_MG_PQ     7   /* multigrid CG: p = z + beta p, q = A p, (p,q) */
#define SOL_KCLASS_MG_DOWN0  8   /* multigrid CG: x, r update, (r,r), level-0 pre-smoothing + restriction */
#define SOL_KCLASS_MG_UP0    9   /* multigrid CG: level-0 prolongation + post-smoothing -> z, (r,z) */
#define SOL_KCLASS_MG_COARSE 10  /* multigrid CG: levels >= 1 (time only, bytes 0) */
#define SOL_NKCLASS          11
int sol_set_timing(sol_handle *h, int32_t enable);
int sol_get_timing(sol_handle *h, int32_t kclass, int64_t *launches, double *total_ms,
                   double *bytes);

/* Number of device work items the library has queued in this process, over
   all handles and batches: kernel dispatches (each node of a replayed graph
   counts) and device-to-host copies of solver state; monotonic.  The
   difference over a run of sol_step calls, divided by the steps, is the
   launches per time step.  NULL -> SOL_EINVAL. */
int sol_dispatch_count(int64_t *count);

/* Options.  SOL_OPT_GRAPH (0/1): replay chunks of 16 Krylov iterations as
   instantiated HIP graphs (the iteration index comes from a device counter
   the graph advances) instead of launching each kernel; batches follow the
   option of their first handle.  Results are bit-identical either way. */
#define SOL_OPT_GRAPH 1
/* SOL_OPT_PRECOND: preconditioner of the pressure-correction CG (eq. 3.4).
   SOL_PRECOND_MG (default): one V-cycle of an aggregation multigrid
   hierarchy of the constant Neumann Laplacian (Galerkin coarse operators,
   damped-Jacobi smoothing, built once at sol_create); SOL_PRECOND_JACOBI:
   the inverse diagonal.  Both stop at the same relative residual.  Not
   allowed while the handle is part of a batch (SOL_EBUSY); the handles of
   one batch must share it (SOL_EINVAL at sol_batch_create). */
#define SOL_OPT_PRECOND 2
#define SOL_PRECOND_JACOBI 0
#define SOL_PRECOND_MG     1
/* SOL_OPT_TPRECOND: preconditioner of the BiCGSTAB solves of the momentum
   (eq. 3.3), solute (eq. 3.10) and energy (eq. 3.11) systems.
   SOL_TPRECOND_JACOBI: the inverse diagonal.  SOL_TPRECOND_JACOBI2: two
   Jacobi sweeps from a zero start, M f = D^-1 (f - (A - D) D^-1 f), D the
   diagonal of A: about half the iterations of one sweep on these systems,
   each product A M f reaching two stencil steps.  SOL_TPRECOND_AUTO
   (default): two sweeps on 2D (5-point) systems, one on 3D (7-point)
   systems, the faster choice for each on gfx950.  All stop at the same
   relative residual of the unpreconditioned system.  Not allowed while the
   handle is part of a batch (SOL_EBUSY); the handles of one batch must
   share it (SOL_EINVAL at sol_batch_create). */
#define SOL_OPT_TPRECOND 3
#define SOL_TPRECOND_JACOBI  0
#define SOL_TPRECOND_JACOBI2 1
#define SOL_TPRECOND_AUTO    2
/* SOL_OPT_ASSEMBLY: route of the per-step assembly of the momentum
   (eq. 3.3), solute (eqs. 3.7-3.10) and energy (eq. 3.11) systems.
   SOL_ASSEMBLY_STENCIL (default): each row's coefficients from the
   closed-form stencil rows (eq. 4.4, diffusion eq. 3.26).
   SOL_ASSEMBLY_FORWARD: the forward method of Section 4 (eqs. 4.5-4.7): the
   step-varying part of each discrete equation is evaluated as a residual
   Eq(phi) = A phi - b, b = -Eq(0), and the entries are the responses to the
   9 (2D) / 27 (3D) colour probes; the constant part of the term-wise split
   is the same offline assembly.  Both give the same systems up to rounding
   (a few ulp of the row scale).  Not allowed while the handle is part of a
   batch (SOL_EBUSY); the handles of one batch must share it (SOL_EINVAL at
   sol_batch_create). */
#define SOL_OPT_ASSEMBLY 4
#define SOL_ASSEMBLY_STENCIL 0
#define SOL_ASSEMBLY_FORWARD 1
/* SOL_OPT_MOMENTUM: the momentum equation the predictor (eq. 3.3)
   discretises.  SOL_MOMENTUM_PLAIN (default): eq. (2.7), the form of the
   scheme.  SOL_MOMENTUM_MINIMAL: eq. (2.6), the minimal model's form, whose
   advecting velocity is u/g_l and whose pressure gradient, Carman-Kozeny
   drag (eq. 2.8) and force carry a factor g_l; the two coincide where
   g_l = 1 (fully liquid melt), bit for bit.  g_l of a velocity face is the
   mean of its two cells; 1/g_l and the g_l of the drag use
   max(g_l, darcy_eps^(1/3)), so that the advecting velocity stays finite
   and the drag large in solid cells; the pressure correction and the
   projection (eqs. 3.4-3.5) are unchanged.  A per-case property: the cases
   of a batch may differ.  Not allowed while the handle is part of a batch
   (SOL_EBUSY). */
#define SOL_OPT_MOMENTUM 5
#define SOL_MOMENTUM_PLAIN   0
#define SOL_MOMENTUM_MINIMAL 1
/* SOL_OPT_MG_FUSE (0/1, default 1): run two consecutive coarse levels of the
   multigrid V-cycle (both smoothed, above the exactly solved level) in one
   launch each way, each workgroup recomputing in local memory the halo its
   results depend on; with 0 every level is its own launch.  The two give
   the same results; the option exists to time them against each other.
   Not allowed while the handle is part of a batch (SOL_EBUSY); a batch
   follows its first handle. */
#define SOL_OPT_MG_FUSE 6
int sol_set_option(sol_handle *h, int32_t option, int64_t value);

/* Tile-size autotuner: times iterations of this case's pressure solve
   (FP32 inner solve under mixed precision) for candidate tile sizes and
   keeps the fastest for the case's size class (stencil width, floor(log2
   rows), preconditioner).  Jacobi: 256, 512, 1024, 2048, 4096 rows per
   workgroup; multigrid: 256, 512, 1024, 2048 level-1 cells per workgroup of
   the level-0 kernels (each cell covers 4 rows in 2D, 8 in 3D).  The choice is
   process-wide and applies to every later solve of that class, alone or in
   a batch (tile size changes the summation order, so tune before creating
   the cases to be compared).  The state of the case is not changed.
   *rows_per_tile (nullable) receives the choice. */
int sol_autotune(sol_handle *h, int32_t *rows_per_tile);

const char *sol_last_error(void);
const char *sol_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SOL_H */
