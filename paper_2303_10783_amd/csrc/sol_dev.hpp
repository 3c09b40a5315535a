// Internal descriptors shared by the kernels and the host engine of the
// solidification step library (gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sol {

constexpr int TILE = 256;          // rows per workgroup (4 wave64)
constexpr int NXCD = 8;            // MI355X: 8 XCDs, workgroups dealt round-robin

enum System { SU = 0, SV = 1, SW = 2, SP = 3, SC = 4, ST = 5, NSYS = 6 };

// Krylov status codes (KState::status)
enum KStatus {
    K_RUNNING = 0, K_CONVERGED = 1, K_FAILED = 2, K_RESTART = 3, K_DONE = 4,
    K_ZERO = 5,      // ||b|| = 0: x = 0 by definition
    K_IDLE = 6,      // not part of the current solve
    K_NONFINITE = 7
};

enum KKind { K_CG = 0, K_BICGSTAB = 1, K_MGCG = 2 };

// Multigrid hierarchy of the pressure system (levels 0 = the system itself,
// 1, 2, ... down to a single cell).  Level l+1 aggregates 2 x 2 (x 2) cells
// of level l (1 along a direction whose level-l count is odd at its upper
// end, or is 1); a level-l cell is then an aligned block of up to 2^l
// level-0 cells per axis.  Its operator is the Galerkin product P^T A_l P
// with the aggregation P: for the Neumann Laplacian (constant 1/h_a^2 per
// axis) the coupling of two neighbouring level-l cells across an a-face is
// 1/h_a^2 times the number of level-0 faces in it, the product of the block
// extents along the other axes, and the diagonal is the sum of the
// couplings (rows sum to zero).  The kernels apply it in this closed form.
// The first level at or below MG_EXACT_MAX cells is solved exactly.  A grid
// of at least MG_LARGE_CELLS cells stepped alone solves the first level at
// or below MG_EXACT_MAX_LARGE exactly instead: that saves the launches of
// the levels below it and some iterations (500x300: 18 -> 17, 128x128x64:
// 26 -> 23), for a dense product of n^2 FP32 values per iteration (23 MB at
// 2394 cells), a gain for a case whose iterations are launch bound, a loss
// in a batch, where every case would read its own.
constexpr int MG_EXACT_MAX = 1024;
constexpr int MG_EXACT_MAX_LARGE = 2600;
constexpr int MG_LARGE_CELLS = 131072;
constexpr int MG_XROWS = TILE / 64; // rows of the exact solve per workgroup (one per wave)
// Set-up of the exact level's dense inverse: Gauss-Jordan elimination in
// blocks of MG_GJB pivots; its scratch holds the block's transformed pivot
// rows (MG_GJB x n), the previous pivot columns (n x MG_GJB), the inverse of
// the diagonal block and the shift c.
constexpr int MG_GJB = 16;
__host__ __device__ inline size_t mg_gj_work(int n) { return 2 * (size_t)MG_GJB * n + MG_GJB * MG_GJB + 1; }
constexpr int MG_MAXLEV = 32;
struct MLevel {
    int32_t n, nx, ny, nz;        // cells of this level and their counts per axis
    int32_t cn, cnx, cny, cnz;    // the next coarser level (cn = 0 at the coarsest)
    int32_t cpt;                  // coarse cells per tile of the kernels that work on this level
    int32_t ntile;                // tiles of those kernels: ceil(cn / cpt)
    int32_t sc;                   // 2^l: block extent of a level-l cell in level-0 cells
    int32_t n0[3];                // level-0 cell counts per axis
    double ih2[3];                // 1 / h_a^2 of level 0
    const void *minv;             // Jacobi inverse of the diagonal (levels above the exact one)
    void *b, *e;                  // right-hand side and correction (levels >= 1)
    void *xs;                     // levels >= 1, and level 0 in 2D: the pre-smoothed value, read back by the post-smoothing
    const void *pinv;             // exact level: dense n x n inverse of A + c 1 1^T (symmetric), FP32
};

// Per-solve device state.  Iteration kernels read it at their start; only
// workgroup 0 of a solve writes it, and only fields no other workgroup of
// the same kernel reads (alpha is double-buffered by iteration parity;
// status changes are taken by every workgroup from the same reduced
// partials, so all of them stop together).
struct KState {
    double bb;                 // ||b||^2 of the current solve
    double rr;                 // ||r||^2 at the last convergence test
    double tr2, tsum, xsum;    // true residual ||b - A x||^2, sum(b - A x), sum(x)
    double bmean;              // mean of the pressure rhs (removed before the solve)
    double tol2;               // tol^2
    double alpha[2];           // CG step length of iterations of parity 0 / 1
    double gamma[2];           // CG (r, M r) of iterations of parity 0 / 1
    int32_t status;            // KStatus
    int32_t it;                // iterations done (valid once not RUNNING)
    int32_t it_base;           // iterations done before the current (re)start
    int32_t k0;                // host iteration index of the current (re)start
    int32_t max_iter, restarts;
    int32_t outer;             // mixed precision: refinement sweeps done
    int32_t inner_total;       // mixed precision: inner iterations summed
    int32_t half;              // BiCGSTAB: the last iteration stopped at its half step (x += alpha M p)
};

// Partial-sum slots of a solve: part[(par * NSLOT + slot) * ntile + tile],
// par = parity of the iteration that produced them.
enum PSlot { PS_Q = 0, PS_TS = 1, PS_TT = 2, PS_RHO = 3, PS_RR = 4, PS_BB = 5, PS_RHS = 6, PS_RHT = 7, PS_SS = 8,
             NSLOT = 9 };

// Physical / geometric constants of one case (immutable after create).
struct Phys {
    int32_t dim, nx, ny, nz;
    int32_t ncell;
    int32_t nsys[NSYS];
    int32_t sdim[NSYS][3];
    double h[3], ih[3], ih2[3];
    double rho, mu, nu, dt, idt, alpha, lam, kp, Tm, msp, Ce, Tref, Cref;
    double grav, betaT, betaC, lambda2, eps, rcp, kcond;
    double Dl;                // liquid solute diffusivity (eq. 3.7); 0 = minimal model
    double gfloor;            // darcy_eps^(1/3): lower bound of g_l in 1/g_l and the drag of form (2.6)
    int32_t mom1;             // momentum predictor in the form of eq. (2.6) instead of eq. (2.7)
    int32_t thermal[6], slip[6];
    double hc[6], Text[6], Tw0[6], Tramp[6];
};

// Device pointers of one case.
struct CaseDev {
    Phys ph;
    // level-n state (updated in place by the commit at the end of a step)
    double *u, *v, *w, *p, *T, *C, *gl, *Cl, *Cs;
    // step intermediates
    double *us[3];            // u* (momentum predictor)
    double *usprev[3], *usprev2[3];   // u* of the two previous steps (momentum initial guesses)
    double *un[3];            // u^{n+1} (projected), committed to u, v, w
    double *phi, *Cnew, *Tstar;
    // systems, DIA storage: A[s][slot*n + row], slot order -sxy,-sx,-1,0,+1,+sx,+sxy
    double *A[NSYS], *b[NSYS], *minv[NSYS];
    double *Ac[NSYS];         // constant (offline) parts of U, V, W, T; P uses A[SP]
    // mixed precision copies (FP32) of matrices and inverse diagonals
    float *A32[NSYS], *minv32[NSYS];
    int64_t *step;            // completed steps (device counter)
    int64_t *hist;            // step at which the solution history below was last reset
    // previous solutions of the energy (T*) and pressure-correction (phi)
    // solves, x^(n-1) and x^(n-2); the latest, x^n, is in Tstar / phi
    double *Tprev, *phiprev, *Tprev2, *phiprev2;
    KState *ks;               // [NSYS] solver states of this case
    double *red;              // [16] per-case reduction results
    double *red_part;         // [ntile_cell * 4] reduction partials
    uint32_t *red_cnt;        // [2] arrival counters
    int32_t ntile_cell;
};

// Reduction result slots in CaseDev::red
enum RedSlot { R_SUMB = 0, R_DIVSTAR = 1, R_SUMC = 2, R_SUMH = 3, R_WALL = 4, R_DIVNEW = 5 };

// One linear solve.  Vector and matrix pointers are FP64 for the plain
// solves and the refinement (outer) solves, FP32 for the inner solves of the
// mixed-precision form; partial sums and scalars are always FP64.
// Work-vector roles: BiCGSTAB r, rh, p0/p1, v0/v1, t; CG (one kernel per
// iteration) r0/r1 = r/rh, s0/s1 = p0/p1, w0/w1 = v0/v1, p = t; multigrid
// CG r0/r1 = r/rh, p0/p1, z = v0, q = v1.
struct KJob {
    int32_t n, sx, sxy;
    int32_t rpt;              // rows per tile (multiple of TILE)
    int32_t ntile;            // tiles of this solve
    int32_t kind;             // KKind
    const void *A, *b, *minv;
    void *x;
    const void *x0;           // initial guess copied into x on a fresh start (NULL: x = 0)
    void *r, *rh, *p0, *p1, *v0, *v1, *t;
    void *r1;                 // BiCGSTAB: residual of odd iterations (r holds the even ones)
    void *aux;                // refinement: FP32 residual (the inner rhs)
    double *part;             // [2 * NSLOT * ntile]
    KState *st;
    KState *partner;          // refinement: its inner solve; inner solve: its refinement
    int32_t role;             // KRole
    int32_t nlev;             // multigrid: levels (0 for the other solves)
    const MLevel *lev;        // multigrid: level table (device), vectors of type T
    int32_t nglob;            // multigrid: the exactly solved level (levels 0..nglob-1 are smoothed)
    int32_t staged;           // BiCGSTAB, FP64: the tile's neighbourhood goes through LDS (two sweeps on a
                              // 5-point system, one sweep on a 7-point system)
};

enum KRole { ROLE_PLAIN = 0, ROLE_REFINE = 1, ROLE_INNER = 2 };

// Tile of a per-row kernel: case, system (or component), tile within it.
struct Tile { int32_t c, s, t, pad; };
// Tile of a Krylov kernel: job, tile within it, multigrid level it works on.
struct JTile { int32_t j, t, lv, pad; };

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Two-sweep BiCGSTAB on a 5-point system with its tile staged in LDS: values
// held per tile of rpt rows on a grid of row stride sx (rows within two
// stencil steps, then within one); a tile is staged when they fit
// STAGE2_LDS_MAX bytes.
__host__ __device__ inline int stage2_values(int rpt, int sx) { return 2 * rpt + 6 * sx + 6; }
constexpr int STAGE2_LDS_MAX = 60 * 1024;
// One-sweep BiCGSTAB on a 7-point system staged in LDS: the tile's rows and
// one grid row on either side (the same budget)
__host__ __device__ inline int stage1_values(int rpt, int sx) { return rpt + 2 * sx; }

}  // namespace sol
