// Multigrid-preconditioned conjugate gradients for the pressure-correction
// system of eq. (3.4).  The paper leaves the solver of this constant,
// symmetric Neumann Laplacian open; Jacobi-PCG needs O(n^(1/d)) iterations
// per solve, a V-cycle preconditioner a few tens at any size.
//
// Hierarchy: level l+1 aggregates 2 x 2 (x 2) cells of level l; its operator
// is the Galerkin product P^T A_l P with the piecewise-constant aggregation
// P.  For the pressure Laplacian that product has a closed form (coupling =
// 1/h_a^2 x level-0 faces between two blocks, diagonal = sum of couplings,
// rows sum to zero: the constant null space is kept), so every level is
// applied matrix-free: no kernel of the cycle loads matrix coefficients.
// Only the inverse diagonals of the coarse levels are stored (built once).
//
// Preconditioner z = M r: one V-cycle from a zero initial guess.
//   levels 0 .. nglob-1: damped-Jacobi sweeps before and after the
//     coarse correction (two on every level of a 2D grid, one in 3D), the
//     correction scaled by mg_og (aggregation under-estimates smooth error;
//     the scaling restores most of the rate);
//   level nglob (the first with at most MG_EXACT_MAX cells, or
//     MG_EXACT_MAX_LARGE on large grids): solved exactly
//     with a dense inverse of A + c 1 1^T (c = mean diagonal / n), built once
//     per case; for a mean-free right-hand side that is the minimum-norm
//     solution, and a constant part is removed with the mean of z anyway.
// Every piece is linear and the pre- and post-smoothers are the same
// symmetric operator, so M is symmetric; the scalings are chosen so that it
// stays positive definite on the grids of the workloads (checked by the
// solve itself: a non-positive (r, z) or (p, A p) restarts it).  The
// operator is singular (constants); a right-hand side is mean-free only to
// rounding (FP32 inner solves: ~1e-7), and the V-cycle maps a constant into
// z with a large gain, so z is used with its mean removed, z - mean(z): the
// search directions then stay in the mean-free subspace where A is definite.
//
// One PCG iteration k (Hestenes-Stiefel form) is the launch sequence
//   pq(k):     zbar = mean(z_k), gamma_k = (r_k, z_k - zbar) and ||r_k||^2
//              from the partials of the previous up0 / down0; convergence
//              test; beta; p_k = z_k - zbar + beta p_(k-1); q = A p_k;
//              partials (p_k, q)
//   down0(k):  alpha = gamma_k / (p_k, q); x += alpha p_k;
//              r_(k+1) = r_k - alpha q; partial ||r_(k+1)||^2; pre-smooth
//              on level 0 (2D: two sweeps, the result kept) and restrict
//              the residual to level 1
//   down(l):   pre-smooth level l (2D: two sweeps, the result kept),
//              restrict to level l+1                       (l = 1 .. nglob-1)
//   exact:     e = P^-1 b on level nglob (dense product, one wave per row)
//   up(l):     prolong onto the pre-smoothed value, post-smooth level l
//              (2D: two sweeps)                            (l = nglob-1 .. 1)
//   up0(k):    prolong, post-smooth level 0 (2D: two sweeps) -> z_(k+1);
//              partials (r, z), sum(z), sum(r)
// Kernels work on coarse cells of the next level: a thread takes one coarse
// cell and its 2^d children, so a restriction needs no cross-thread sum.
// The level-0 kernels first load every value their children's stencils
// reach into a register window, once per thread (3D, one sweep: the 8
// children and their 24 face neighbours, 23.5 -> 16.9 us per down0 launch
// at 128x128x64, pq 15.9 -> 12.7, up0 15.2 -> 10.7; 2D: the 24 cells within
// two steps of the 4 children for the two sweeps of down0 and up0, the 12
// within one for pq).
// Values a stencil needs at neighbour rows are recomputed there from
// vectors the same kernel does not write (r and p are ping-ponged by
// iteration parity), as in the other Krylov kernels.
#include "sol_dev.hpp"
#include "kcommon.hpp"
#include "kernels.hpp"

namespace sol {

// damped-Jacobi weight and coarse-correction scaling per dimension, chosen
// by the PCG iteration count of the V-cycle over grid sizes of the
// workloads.  2D (50x30 .. 800x480, two sweeps per level): 0.8 / 2.0 needs
// 9 iterations at every size, 0.8 / 1.8 needs 9 - 12 (11 at 500x300), 1.9
// and 2.1 lie between, 0.75 and 0.85 lose one.  3D (24x20x16 .. 160x160x80,
// one sweep): 0.9 / 1.65 needs 26 iterations at 128x128x64 where the 2D
// pair of one sweep (0.8 / 1.8) needs 31, and 29 instead of 35 at
// 160x160x80; 1.8 - 2.0 lose two to five.  Both weights stay below 1, and
// the spectrum of D^-1 A lies in [0, 2] on every level (diagonally dominant,
// zero row sums), so the smoother converges in the A-norm.  The V-cycle
// stays positive definite for any positive scaling: its error operator is
// the smoother's, S^v (I - og P B_c P^T A) S^v, and the correction term is
// non-negative in the A-inner product (B_c, the coarse cycle, is itself
// positive definite), so every eigenvalue stays below that of S^(2v), below
// 1 off the constants.
template <int DIM> constexpr double mg_w() { return DIM == 3 ? 0.9 : 0.8; }
template <int DIM> constexpr double mg_og() { return DIM == 3 ? 1.65 : 2.0; }

// floor(i / d) for 0 <= i < 2^31, 1 <= d, from the double reciprocal inv = 1/d
__device__ __forceinline__ int fdiv(int i, int d, double inv)
{
    int q = (int)((double)i * inv);
    if ((long long)q * d > i) --q;
    else if ((long long)(q + 1) * d <= i) ++q;
    return q;
}

// A coarse cell and its children on the finer level of an MLevel
template <int DIM>
struct Agg {
    int I;           // coarse index
    int c[3];        // coarse coordinates
    int w[3];        // children per axis (1 or 2)
    int i0;          // first child (fine index)
};

template <int DIM>
__device__ __forceinline__ Agg<DIM> agg_of(const MLevel &L, int I, double icnx, double icnxy)
{
    Agg<DIM> a;
    a.I = I;
    int rem = I;
    if (DIM == 3) {
        a.c[2] = fdiv(I, L.cnx * L.cny, icnxy);
        rem = I - a.c[2] * L.cnx * L.cny;
    } else {
        a.c[2] = 0;
    }
    a.c[1] = fdiv(rem, L.cnx, icnx);
    a.c[0] = rem - a.c[1] * L.cnx;
    const int n3[3] = {L.nx, L.ny, L.nz};
#pragma unroll
    for (int d = 0; d < 3; ++d) a.w[d] = min(2, n3[d] - 2 * a.c[d]);
    a.i0 = 2 * a.c[0] + L.nx * (2 * a.c[1] + L.ny * 2 * a.c[2]);
    return a;
}

// coarse cell holding the in-domain neighbour of child cx along axis ax in
// direction dir (0: the child itself): the neighbour aggregate when the step
// leaves the aggregate, else the child's own
template <int DIM>
__device__ __forceinline__ int agg_nb(const MLevel &L, const Agg<DIM> &a, const int *cx, int ax, int dir)
{
    if (dir == 0) return a.I;
    const int cs = ax == 0 ? 1 : (ax == 1 ? L.cnx : L.cnx * L.cny);
    if (dir < 0) return cx[ax] == 0 ? a.I - cs : a.I;
    return cx[ax] == 1 ? a.I + cs : a.I;
}

// visit the children of aggregate a: f(i, cx, q) with cx the position in
// the aggregate and q the fine coordinates
template <int DIM, class F>
__device__ __forceinline__ void for_children(const MLevel &L, const Agg<DIM> &a, F f)
{
    const int sxy = L.nx * L.ny;
#pragma unroll
    for (int cz = 0; cz < (DIM == 3 ? 2 : 1); ++cz) {
        if (cz >= a.w[2]) continue;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            if (cy >= a.w[1]) continue;
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                if (cx >= a.w[0]) continue;
                const int c3[3] = {cx, cy, cz};
                const int q[3] = {2 * a.c[0] + cx, 2 * a.c[1] + cy, 2 * a.c[2] + cz};
                f(a.i0 + cx + L.nx * cy + sxy * cz, c3, q);
            }
        }
    }
}

// a solve whose multigrid stages run at iteration index k: RUNNING, or its
// (re)start whose first iteration is k + 1 (the start cycle runs at k0 - 1)
__device__ __forceinline__ bool mg_live(const KJob &J, int k)
{
    const int s = wg_status(J.st);
    return s == K_RUNNING || ((s == K_RESTART) && J.st->k0 == k + 1);
}

__device__ __forceinline__ int kidx(const int *kbase, int koff) { return (kbase ? *kbase : 0) + koff; }

// ------------------------------------------------- 2D level 0, two sweeps
// A thread of the level-0 kernels of a 2D grid holds the window of its
// aggregate: the 2 x 2 children at window positions (u, v) = (2..3, 2..3)
// and every cell within two stencil steps of them, inside the 6 x 6 square
// whose corner (0, 0) is the fine cell (2 cx - 2, 2 cy - 2).  A window cell
// beyond the grid is loaded from the nearest grid cell; it enters no result,
// since the coupling across a boundary face is 0.
constexpr int W2 = 6;
__host__ __device__ constexpr int wdist(int u, int v)
{
    return (u < 2 ? 2 - u : (u > 3 ? u - 3 : 0)) + (v < 2 ? 2 - v : (v > 3 ? v - 3 : 0));
}

__device__ __forceinline__ int win_idx(const MLevel &L, int gx, int gy)
{
    return min(max(gx, 0), L.nx - 1) + L.nx * min(max(gy, 0), L.ny - 1);
}

// (A f) at window cell (u, v) of a cell within one step of the children:
// level 0 couples neighbours across a face with 1/h_a^2
template <class T>
__device__ __forceinline__ T win_op(const MLevel &L, int gx, int gy, int u, int v, const T (&f)[W2][W2], T c0, T c1)
{
    const T fc = f[v][u];
    return (gx > 0 ? c0 : T(0)) * (fc - f[v][u - 1]) + (gx + 1 < L.nx ? c0 : T(0)) * (fc - f[v][u + 1]) +
           (gy > 0 ? c1 : T(0)) * (fc - f[v - 1][u]) + (gy + 1 < L.ny ? c1 : T(0)) * (fc - f[v + 1][u]);
}

// 3D level 0: a thread holds the 2 x 2 x 2 children of its aggregate at
// window positions (1..2)^3 and their face neighbours (one stencil step
// from the block) in the 4 x 4 x 4 window whose corner (0, 0, 0) is the fine
// cell (2 cx - 1, 2 cy - 1, 2 cz - 1): each value a child's stencil needs is
// loaded once per thread instead of once per child that reaches it.  Window
// cells beyond the grid are handled as in 2D.
constexpr int W3 = 4;
__host__ __device__ constexpr int wdist3(int u, int v, int w)
{
    return (u < 1 ? 1 - u : (u > 2 ? u - 2 : 0)) + (v < 1 ? 1 - v : (v > 2 ? v - 2 : 0)) +
           (w < 1 ? 1 - w : (w > 2 ? w - 2 : 0));
}

__device__ __forceinline__ int win3_idx(const MLevel &L, int gx, int gy, int gz)
{
    return min(max(gx, 0), L.nx - 1) + L.nx * (min(max(gy, 0), L.ny - 1) + L.ny * min(max(gz, 0), L.nz - 1));
}

// (A f) at a child (u, v, w) of the window, in the order of apply_op
template <class T>
__device__ __forceinline__ T win3_op(const MLevel &L, int gx, int gy, int gz, int u, int v, int w,
                                     const T (&f)[W3][W3][W3], T c0, T c1, T c2)
{
    const T fc = f[w][v][u];
    T acc = T(0);
    acc += (gx > 0 ? c0 : T(0)) * (fc - f[w][v][u - 1]) + (gx + 1 < L.nx ? c0 : T(0)) * (fc - f[w][v][u + 1]);
    acc += (gy > 0 ? c1 : T(0)) * (fc - f[w][v - 1][u]) + (gy + 1 < L.ny ? c1 : T(0)) * (fc - f[w][v + 1][u]);
    acc += (gz > 0 ? c2 : T(0)) * (fc - f[w - 1][v][u]) + (gz + 1 < L.nz ? c2 : T(0)) * (fc - f[w + 1][v][u]);
    return acc;
}

// Jacobi inverse of the level-0 (pressure) diagonal.  The assembled row of a
// cell adds 1/h_a^2 once per face it has inside the grid, axis by axis (low
// face, then high face), and the stored inverse is 1 / that sum (1 for a cell
// without neighbours).  The sum depends only on the number of such faces per
// axis (0, 1 or 2), so the level-0 smoothers take the inverse from a
// workgroup table of the 3^d values, formed by the same additions in the same
// order (the stored values, bit for bit), instead of loading it for every
// window cell.  Entry kx + 3 ky + 9 kz; written before the workgroup's first
// barrier, read after it.
template <int DIM>
__device__ __forceinline__ void write_minv0(const MLevel &L, double *tab)
{
    const int t = threadIdx.x;
    if (t < (DIM == 3 ? 27 : 9)) {
        const int k[3] = {t % 3, (t / 3) % 3, t / 9};
        double d = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (k[a] >= 1) d += L.ih2[a];
            if (k[a] == 2) d += L.ih2[a];
        }
        tab[t] = d > 0.0 ? 1.0 / d : 1.0;
    }
}

// faces inside the grid along one axis of n cells of the cell at g, clamped
// into [0, n) as the window's loads are
__device__ __forceinline__ int faces_in(int g, int n)
{
    const int c = min(max(g, 0), n - 1);
    return (c > 0 ? 1 : 0) + (c + 1 < n ? 1 : 0);
}

// ------------------------------------------------------------- operator

// couplings of the level-l cell with coordinates q to its neighbours along
// each axis: 1/h_a^2 times the product of its block extents (in level-0
// cells) along the other axes
template <int DIM, class T>
__device__ __forceinline__ void couplings(const MLevel &L, const int *q, T *co)
{
    int e[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) e[b] = min(L.sc, L.n0[b] - q[b] * L.sc);
    if (DIM == 2) {
        co[0] = (T)L.ih2[0] * (T)e[1];
        co[1] = (T)L.ih2[1] * (T)e[0];
    } else {
        co[0] = (T)L.ih2[0] * (T)(e[1] * e[2]);
        co[1] = (T)L.ih2[1] * (T)(e[0] * e[2]);
        co[2] = (T)L.ih2[2] * (T)(e[0] * e[1]);
    }
}

// diagonal of the level operator at q (0 for a cell without neighbours)
template <int DIM, class T>
__device__ __forceinline__ T op_diag(const MLevel &L, const int *q)
{
    T co[3];
    couplings<DIM, T>(L, q, co);
    const int nn[3] = {L.nx, L.ny, L.nz};
    T d = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (q[a] > 0) d += co[a];
        if (q[a] + 1 < nn[a]) d += co[a];
    }
    return d;
}

// (A f)_i = sum over in-domain neighbours j of c_a (f_i - f_j), with
// f(j, axis, direction) (direction 0: the cell itself).  Branch-free: a
// missing neighbour is replaced by the cell itself with a zero coupling, so
// every value is loaded unconditionally and the loads can be issued together.
// NOFMA: the sum without contraction into fused multiply-adds (the coarse
// levels, whose fused and per-level kernels must round alike).
template <int DIM, class T, bool NOFMA = false, class F>
__device__ __forceinline__ T apply_op(const MLevel &L, int i, const int *q, F f)
{
    T co[3];
    couplings<DIM, T>(L, q, co);
    const int st[3] = {1, L.nx, L.nx * L.ny};
    const int nn[3] = {L.nx, L.ny, L.nz};
    const T fi = f(i, 0, 0);
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const bool lo = q[a] > 0, hi = q[a] + 1 < nn[a];
        const T vlo = f(lo ? i - st[a] : i, a, lo ? -1 : 0);
        const T vhi = f(hi ? i + st[a] : i, a, hi ? 1 : 0);
        if constexpr (NOFMA) {
#pragma clang fp contract(off)
            acc += (lo ? co[a] : T(0)) * (fi - vlo) + (hi ? co[a] : T(0)) * (fi - vhi);
        } else {
            acc += (lo ? co[a] : T(0)) * (fi - vlo) + (hi ? co[a] : T(0)) * (fi - vhi);
        }
    }
    return acc;
}

// coordinates of cell i on a level with counts (nx, ny)
template <int DIM>
__device__ __forceinline__ void cell_coords(int i, int nx, int ny, double inx, double inxy, int *q)
{
    int rem = i;
    q[2] = 0;
    if (DIM == 3) {
        q[2] = fdiv(i, nx * ny, inxy);
        rem = i - q[2] * nx * ny;
    }
    q[1] = fdiv(rem, nx, inx);
    q[0] = rem - q[1] * nx;
}

// inverse diagonal of level l >= 1 (FP64, and FP32 when requested)
template <int DIM>
__global__ __launch_bounds__(TILE) void k_mg_minv(const MLevel *__restrict__ lev, int l, double *mi, float *mi32)
{
    const MLevel &L = lev[l];
    const int i = blockIdx.x * TILE + threadIdx.x;
    if (i >= L.n) return;
    int q[3];
    cell_coords<DIM>(i, L.nx, L.ny, 1.0 / L.nx, 1.0 / ((double)L.nx * L.ny), q);
    const double d = op_diag<DIM, double>(L, q);
    const double m = d > 0.0 ? 1.0 / d : 0.0;
    mi[i] = m;
    if (mi32) mi32[i] = (float)m;
}

void launch_mg_minv(int dim, const MLevel *lev, int l, int n, double *mi, float *mi32, hipStream_t s)
{
    if (n <= 0) return;
    const dim3 g(ceil_div(n, TILE)), b(TILE);
    if (dim == 2) SOL_LAUNCH(k_mg_minv<2>, g, b, 0, s, lev, l, mi, mi32);
    else SOL_LAUNCH(k_mg_minv<3>, g, b, 0, s, lev, l, mi, mi32);
}

// ------------------------------------------------------------- start

// start at iteration index k (mode 0: every solve, x = x0 or 0; mode 1:
// solves in K_RESTART, keep x): r_k = b - A x, p_(k-1) = 0; partial (b, b)
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_init(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k,
                                                  int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RESTART) return;
    if (outer_idle(J)) return;
    const int pk = k & 1;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    auto b = G<T>(J.b);
    auto x = G<T>(J.x), x0 = G<T>(J.x0);
    auto r = G<T>(pk ? J.rh : J.r), pz = G<T>(pk ? J.p0 : J.p1);
    const bool from_x0 = mode == 0 && J.x0;
    const bool keep_x = mode == 1;
    double bb = 0.0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *, const int *q) {
            const T bi = b[i];
            T ri = bi;
            if (from_x0 || keep_x) {
                auto src = from_x0 ? x0 : x;
                ri = bi - apply_op<DIM, T>(L, i, q, [&](int j, int, int) { return src[j]; });
            }
            if (from_x0) {
                if (J.x0 != J.x) x[i] = x0[i];            // a guess written into x stays
            } else if (!keep_x) {
                x[i] = T(0);
            }
            r[i] = ri;
            pz[i] = T(0);
            bb += (double)bi * bi;
        });
    }
    double v[1] = {bb};
    const int off[1] = {poff(J, pk, PS_BB)};
    put_partials<1>(v, J.part, off, tl.t);
    mark_start(tl, J.st, k, mode);
}

// ------------------------------------------------------------- finish

// The true residual b - A x of the converged solves (totalled by k_kdecide)
// and the FP64 residual sweep of a refinement (mode 0: x = x0 or 0; mode 1:
// keep x; its FP32 copy into aux, totalled by k_ir_decide), the operator
// from its closed form instead of the stored diagonals k_kfinish and
// k_ir_resid read: the same rows, 16 instead of 72 bytes each; partials in
// the same slots.
template <int DIM>
__global__ __launch_bounds__(TILE) void k_mg_finish(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    const int status = J.st->status;
    if (status != K_CONVERGED && status != K_ZERO) return;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    auto b = G<double>(J.b);
    auto x = G<double>(J.x);
    double v[3] = {0.0, 0.0, 0.0};
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *, const int *q) {
            if (status == K_ZERO) {
                x[i] = 0.0;
                return;
            }
            const double rt = b[i] - apply_op<DIM, double>(L, i, q, [&](int j, int, int) { return x[j]; });
            v[0] += rt * rt;
            v[1] += rt;
            v[2] += x[i];
        });
    }
    const int off[3] = {poff(J, 0, PS_Q), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    put_partials<3>(v, J.part, off, tl.t);
}

template <int DIM>
__global__ __launch_bounds__(TILE) void k_mg_ir_resid(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                      int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RUNNING) return;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    auto b = G<double>(J.b);
    auto x = G<double>(J.x), x0 = G<double>(J.x0);
    auto r32 = G<float>(J.aux);
    const bool zero = mode == 0 && !J.x0;
    const auto src = mode == 0 ? x0 : x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *, const int *q) {
            const double bi = b[i];
            double ri = bi, xi = 0.0;
            if (zero) {
                x[i] = 0.0;
            } else {
                ri = bi - apply_op<DIM, double>(L, i, q, [&](int j, int, int) { return src[j]; });
                xi = src[i];
                if (mode == 0 && J.x0 != J.x) x[i] = xi;     // a guess written into x stays
            }
            r32[i] = (float)ri;
            v[0] += ri * ri;
            v[1] += bi * bi;
            v[2] += ri;
            v[3] += xi;
        });
    }
    const int off[4] = {poff(J, 0, PS_RR), poff(J, 0, PS_BB), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    put_partials<4>(v, J.part, off, tl.t);
}

// ------------------------------------------------------------- iteration

// pq(k).  On a grid with an even x count the two children of a window row
// come in one 16-byte (FP32: 8-byte) load.
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_pq(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                const int *kbase, int koff)
{
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (!active(J, k) || outer_idle(J)) return;
    KState *st = J.st;
    const int pk = k & 1, pm = (k + 1) & 1;
    const bool first = k == st->k0;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const void *zb = J.v0, *pb = pm ? J.p1 : J.p0;
    auto z = R<T>(zb);
    auto q = G<T>(J.v1);
    auto po = R<T>(pb);
    auto pn = G<T>(pk ? J.p1 : J.p0);
    const bool pairs = (L.nx & 1) == 0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    int I = I0 + threadIdx.x;
    // raw window values: zr = z, pr = p_(k-1) on the window cells
    constexpr int WN = DIM == 2 ? W2 : W3;
    T zr[DIM == 3 ? W3 : 1][WN][WN], pr[DIM == 3 ? W3 : 1][WN][WN];
    auto load_window = [&](int Ia) {
        const Agg<DIM> ag = agg_of<DIM>(L, Ia, icx, icxy);
        if constexpr (DIM == 2) {
            // the 12 cells within one step of the 2 x 2 children (positions 1..4)
            const int X0 = 2 * ag.c[0] - 2, Y0 = 2 * ag.c[1] - 2;
#pragma unroll
            for (int vy = 1; vy < W2 - 1; ++vy) {
                const int row = L.nx * min(max(Y0 + vy, 0), L.ny - 1);
                if (pairs && 2 * ag.c[0] + 1 < L.nx) {
                    const Pair<T> zz = load_pair<T>(zb, row + 2 * ag.c[0]), pp = load_pair<T>(pb, row + 2 * ag.c[0]);
                    zr[0][vy][2] = zz.x; zr[0][vy][3] = zz.y; pr[0][vy][2] = pp.x; pr[0][vy][3] = pp.y;
                } else {
#pragma unroll
                    for (int ux = 2; ux < 4; ++ux) {
                        const int j = win_idx(L, X0 + ux, Y0 + vy);
                        zr[0][vy][ux] = z[j]; pr[0][vy][ux] = po[j];
                    }
                }
                if (vy == 2 || vy == 3) {
                    const int jm = win_idx(L, X0 + 1, Y0 + vy), jp = win_idx(L, X0 + 4, Y0 + vy);
                    zr[0][vy][1] = z[jm]; pr[0][vy][1] = po[jm];
                    zr[0][vy][4] = z[jp]; pr[0][vy][4] = po[jp];
                }
            }
        } else {
            // the 8 children and their 24 face neighbours (positions 0..3)
            const int X0 = 2 * ag.c[0] - 1, Y0 = 2 * ag.c[1] - 1, Z0 = 2 * ag.c[2] - 1;
#pragma unroll
            for (int w = 0; w < W3; ++w)
#pragma unroll
                for (int v2 = 0; v2 < W3; ++v2) {
                    if (wdist3(1, v2, w) > 1) continue;
                    const int row = L.nx * (min(max(Y0 + v2, 0), L.ny - 1) + L.ny * min(max(Z0 + w, 0), L.nz - 1));
                    if (pairs && 2 * ag.c[0] + 1 < L.nx) {
                        const Pair<T> zz = load_pair<T>(zb, row + 2 * ag.c[0]), pp = load_pair<T>(pb, row + 2 * ag.c[0]);
                        zr[w][v2][1] = zz.x; zr[w][v2][2] = zz.y; pr[w][v2][1] = pp.x; pr[w][v2][2] = pp.y;
                    } else {
#pragma unroll
                        for (int u = 1; u < 3; ++u) {
                            const int j = win3_idx(L, X0 + u, Y0 + v2, Z0 + w);
                            zr[w][v2][u] = z[j]; pr[w][v2][u] = po[j];
                        }
                    }
                    if (wdist3(0, v2, w) <= 1) {
                        const int jm = win3_idx(L, X0, Y0 + v2, Z0 + w), jp = win3_idx(L, X0 + 3, Y0 + v2, Z0 + w);
                        zr[w][v2][0] = z[jm]; pr[w][v2][0] = po[jm];
                        zr[w][v2][3] = z[jp]; pr[w][v2][3] = po[jp];
                    }
                }
        }
    };
    double s5[5];
    {
        const int off[5] = {poff(J, pk, PS_RHO), poff(J, pk, PS_RR), poff(J, pk, PS_BB), poff(J, pk, PS_Q),
                            poff(J, pk, PS_TT)};
        sum_partials<5>(J.part, off, J.ntile, s5);
    }
    if (!keep_going(J, tl, k, s5[1], s5[2])) return;
    const double zbar = s5[3] / J.n;
    const double gam = s5[0] - zbar * s5[4];
    if (!(gam > 0.0) || !finite(gam)) {
        set_status(tl, st, finite(gam) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0), s5[1]);
        return;
    }
    const double beta = first ? 0.0 : gam / st->gamma[pm];
    if (tl.t == 0 && threadIdx.x == 0) st->gamma[pk] = gam;
    const T tb = (T)beta, tz = (T)zbar;
    double v = 0.0;
    for (; I < I1; I += TILE) {
        load_window(I);
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        if constexpr (DIM == 2) {
            // p on the children and their neighbours, then q = A p at the children
            const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1];
            const int X0 = 2 * a.c[0] - 2, Y0 = 2 * a.c[1] - 2;
            T f[W2][W2];
#pragma unroll
            for (int vy = 1; vy < W2 - 1; ++vy)
#pragma unroll
                for (int ux = 1; ux < W2 - 1; ++ux) {
                    if (wdist(ux, vy) > 1) continue;
                    f[vy][ux] = (zr[0][vy][ux] - tz) + tb * pr[0][vy][ux];
                }
#pragma unroll
            for (int vy = 2; vy < 4; ++vy)
#pragma unroll
                for (int ux = 2; ux < 4; ++ux) {
                    const int gx = X0 + ux, gy = Y0 + vy;
                    if (gx >= L.nx || gy >= L.ny) continue;
                    const int i = gx + L.nx * gy;
                    const T qv = win_op(L, gx, gy, ux, vy, f, c0, c1);
                    pn[i] = f[vy][ux];
                    q[i] = qv;
                    v += (double)f[vy][ux] * qv;
                }
        } else {
            const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1], c2 = (T)L.ih2[2];
            const int X0 = 2 * a.c[0] - 1, Y0 = 2 * a.c[1] - 1, Z0 = 2 * a.c[2] - 1;
            T f[W3][W3][W3];
#pragma unroll
            for (int w = 0; w < W3; ++w)
#pragma unroll
                for (int v2 = 0; v2 < W3; ++v2)
#pragma unroll
                    for (int u = 0; u < W3; ++u) {
                        if (wdist3(u, v2, w) > 1) continue;
                        f[w][v2][u] = (zr[w][v2][u] - tz) + tb * pr[w][v2][u];
                    }
#pragma unroll
            for (int w = 1; w < 3; ++w)
#pragma unroll
                for (int v2 = 1; v2 < 3; ++v2)
#pragma unroll
                    for (int u = 1; u < 3; ++u) {
                        const int gx = X0 + u, gy = Y0 + v2, gz = Z0 + w;
                        if (gx >= L.nx || gy >= L.ny || gz >= L.nz) continue;
                        const int i = gx + L.nx * (gy + L.ny * gz);
                        const T qv = win3_op(L, gx, gy, gz, u, v2, w, f, c0, c1, c2);
                        pn[i] = f[w][v2][u];
                        q[i] = qv;
                        v += (double)f[w][v2][u] * qv;
                    }
        }
    }
    double vv[1] = {v};
    const int off[1] = {poff(J, pk, PS_TS)};
    put_partials<1>(vv, J.part, off, tl.t);
}

// level 0, pre-smoothing and restriction; INIT: the start cycle (r_(k+1) is
// the start residual, no update)
template <int DIM, class T, bool INIT>
__global__ __launch_bounds__(TILE) void k_mg_down0(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                   const int *kbase, int koff)
{
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J)) return;
    __shared__ double tab[27];
    write_minv0<DIM>(J.lev[0], tab);
    KState *st = J.st;
    if (INIT ? !mg_live(J, k) : wg_status(st) != K_RUNNING) return;
    const int pk = k & 1, pn1 = (k + 1) & 1;
    double alpha = 0.0;
    if (!INIT) {
        double s1[1];
        const int off[1] = {poff(J, pk, PS_TS)};
        sum_partials<1>(J.part, off, J.ntile, s1);
        alpha = st->gamma[pk] / s1[0];
        if (!(alpha > 0.0) || !finite(alpha)) {
            set_status(tl, st, finite(alpha) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0), st->rr);
            return;
        }
        if (tl.t == 0 && threadIdx.x == 0) st->alpha[pk] = alpha;
    }
    const T ta = (T)alpha, w = (T)mg_w<DIM>();
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    auto x = G<T>(J.x);
    auto p = R<T>(pk ? J.p1 : J.p0);
    auto q = R<T>(J.v1);
    const void *rcb = pk ? J.rh : J.r;
    void *rnb = pn1 ? J.rh : J.r;
    auto rc = R<T>(rcb);
    auto rn = G<T>(rnb);
    auto bc = G<T>(J.lev[1].b);
    const bool pairs = (L.nx & 1) == 0;
    double rr = 0.0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    if constexpr (DIM == 2) {
        // x1 = w D^-1 r on the window, x2 = x1 + w D^-1 (r - A x1) within
        // one step of the children, then their residual r - A x2
        auto xs = G<T>(L.xs);
        const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1];
        for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
            const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
            const int X0 = 2 * a.c[0] - 2, Y0 = 2 * a.c[1] - 2;
            int kx[W2], ky[W2];
#pragma unroll
            for (int u = 0; u < W2; ++u) {
                kx[u] = faces_in(X0 + u, L.nx);
                ky[u] = 3 * faces_in(Y0 + u, L.ny);
            }
            T rw[W2][W2], mw[W2][W2], f1[W2][W2], f2[W2][W2];
#pragma unroll
            for (int v = 0; v < W2; ++v)
#pragma unroll
                for (int u = 0; u < W2; ++u) {
                    if (wdist(u, v) > 2) continue;
                    const int j = win_idx(L, X0 + u, Y0 + v);
                    rw[v][u] = INIT ? rn[j] : rc[j] - ta * q[j];
                    mw[v][u] = (T)tab[kx[u] + ky[v]];
                }
#pragma unroll
            for (int v = 0; v < W2; ++v)
#pragma unroll
                for (int u = 0; u < W2; ++u)
                    if (wdist(u, v) <= 2) f1[v][u] = w * mw[v][u] * rw[v][u];
#pragma unroll
            for (int v = 1; v < W2 - 1; ++v)
#pragma unroll
                for (int u = 1; u < W2 - 1; ++u)
                    if (wdist(u, v) <= 1)
                        f2[v][u] = f1[v][u] + w * mw[v][u] * (rw[v][u] - win_op(L, X0 + u, Y0 + v, u, v, f1, c0, c1));
            T bsum = T(0);
#pragma unroll
            for (int v = 2; v < 4; ++v)
#pragma unroll
                for (int u = 2; u < 4; ++u) {
                    const int gx = X0 + u, gy = Y0 + v;
                    if (gx >= L.nx || gy >= L.ny) continue;
                    const int i = gx + L.nx * gy;
                    bsum += rw[v][u] - win_op(L, gx, gy, u, v, f2, c0, c1);
                    xs[i] = f2[v][u];
                    if (!INIT) {
                        rn[i] = rw[v][u];
                        x[i] = x[i] + ta * p[i];
                    }
                    rr += (double)rw[v][u] * rw[v][u];
                }
            bc[I] = bsum;
        }
    } else {
        // x1 = w D^-1 r on the window, then the children's residual r - A x1
        const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1], c2 = (T)L.ih2[2];
        for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
            const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
            const int X0 = 2 * a.c[0] - 1, Y0 = 2 * a.c[1] - 1, Z0 = 2 * a.c[2] - 1;
            int kx[W3], kyz[W3][W3];
#pragma unroll
            for (int u = 0; u < W3; ++u) kx[u] = faces_in(X0 + u, L.nx);
#pragma unroll
            for (int wz = 0; wz < W3; ++wz)
#pragma unroll
                for (int vy = 0; vy < W3; ++vy) kyz[wz][vy] = 3 * faces_in(Y0 + vy, L.ny) + 9 * faces_in(Z0 + wz, L.nz);
            T rw[W3][W3][W3], f1[W3][W3][W3];
            auto cell = [&](int wz, int vy, int ux, T rv, T qv) {
                const T rj = INIT ? rv : rv - ta * qv;
                const T mv = (T)tab[kx[ux] + kyz[wz][vy]];
                rw[wz][vy][ux] = rj;
                f1[wz][vy][ux] = w * mv * rj;
            };
#pragma unroll
            for (int wz = 0; wz < W3; ++wz)
#pragma unroll
                for (int vy = 0; vy < W3; ++vy) {
                    if (wdist3(1, vy, wz) > 1) continue;
                    if (pairs && 2 * a.c[0] + 1 < L.nx) {
                        // the window row's two children in one load per vector
                        const int j = L.nx * (min(max(Y0 + vy, 0), L.ny - 1) + L.ny * min(max(Z0 + wz, 0), L.nz - 1)) +
                                      2 * a.c[0];
                        const Pair<T> rr2 = load_pair<T>(INIT ? (const void *)rnb : rcb, j);
                        const Pair<T> qq2 = INIT ? Pair<T>{T(0), T(0)} : load_pair<T>(J.v1, j);
                        cell(wz, vy, 1, rr2.x, qq2.x);
                        cell(wz, vy, 2, rr2.y, qq2.y);
                    } else {
#pragma unroll
                        for (int ux = 1; ux < 3; ++ux) {
                            const int j = win3_idx(L, X0 + ux, Y0 + vy, Z0 + wz);
                            cell(wz, vy, ux, INIT ? rn[j] : rc[j], INIT ? T(0) : q[j]);
                        }
                    }
                    if (wdist3(0, vy, wz) <= 1) {
#pragma unroll
                        for (int ux = 0; ux < W3; ux += 3) {
                            const int j = win3_idx(L, X0 + ux, Y0 + vy, Z0 + wz);
                            cell(wz, vy, ux, INIT ? rn[j] : rc[j], INIT ? T(0) : q[j]);
                        }
                    }
                }
            T bsum = T(0);
#pragma unroll
            for (int wz = 1; wz < 3; ++wz)
#pragma unroll
                for (int vy = 1; vy < 3; ++vy)
#pragma unroll
                    for (int ux = 1; ux < 3; ++ux) {
                        const int gx = X0 + ux, gy = Y0 + vy, gz = Z0 + wz;
                        if (gx >= L.nx || gy >= L.ny || gz >= L.nz) continue;
                        const int i = gx + L.nx * (gy + L.ny * gz);
                        const T ri = rw[wz][vy][ux];
                        if (!INIT) {
                            rn[i] = ri;
                            x[i] = x[i] + ta * p[i];
                        }
                        rr += (double)ri * ri;
                        bsum += ri - win3_op(L, gx, gy, gz, ux, vy, wz, f1, c0, c1, c2);
                    }
            bc[I] = bsum;
        }
    }
    double vv[1] = {rr};
    const int off[1] = {poff(J, pn1, PS_RR)};
    put_partials<1>(vv, J.part, off, tl.t);
}

// Levels l >= 1 carry no partial sums, so their kernels take one thread per
// child: tile t covers the coarse cells t*cpt .. t*cpt+cpt-1 with cpt =
// TILE / 2^d, thread = (coarse cell, child); a child beyond an odd upper end
// does nothing.
template <int DIM>
__device__ __forceinline__ bool child_of(const MLevel &L, int t, double icx, double icxy, Agg<DIM> &a, int *cx, int *q,
                                         int &i, int &I)
{
    constexpr int NC = 1 << DIM;
    const int c = threadIdx.x & (NC - 1);
    I = t * L.cpt + (int)(threadIdx.x >> DIM);
    if (I >= L.cn) return false;
    a = agg_of<DIM>(L, I, icx, icxy);
    cx[0] = c & 1;
    cx[1] = (c >> 1) & 1;
    cx[2] = DIM == 3 ? (c >> 2) & 1 : 0;
    if (cx[0] >= a.w[0] || cx[1] >= a.w[1] || cx[2] >= a.w[2]) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) q[d] = 2 * a.c[d] + cx[d];
    i = a.i0 + cx[0] + L.nx * cx[1] + L.nx * L.ny * cx[2];
    return true;
}

// coarse index (on the next level) of the level-l cell with coordinates q
__device__ __forceinline__ int agg_index(const MLevel &L, const int *q)
{
    return (q[0] >> 1) + L.cnx * ((q[1] >> 1) + L.cny * (q[2] >> 1));
}

// coordinates of the cell apply_op reached from q along axis ax in
// direction dir (0: q itself)
__device__ __forceinline__ void step_q(const int *q, int ax, int dir, int *qj)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) qj[d] = q[d] + (d == ax ? dir : 0);
}

// In 2D, every level smooths with two damped-Jacobi sweeps before and
// after the coarse correction: in a study of the V-cycle-PCG two sweeps on
// the coarse levels cut the iterations from 17 to 14 at 500x300 (measured
// 13.5 -> 11.5 per step), two on level 0 as well from 14 to 11 (measured
// 11.5 -> 8.6), and these kernels are bound by launch latency, not by the
// loads the second sweep adds.  The pre-smoothed value x2 is stored (xs)
// for the post-smoothing; each sweep's value at a neighbour is recomputed
// there, so a kernel reaches two stencil steps.  3D keeps one sweep: at
// 128x128x64 the 25-cell reach on the 131072-cell first level cost more
// than the 2.3 iterations per step it saved (282 -> 265 M
// cell-updates/s).

// level l >= 1 (launch level): pre-smooth from zero, x1 = w D^-1 b (3D),
// or two sweeps, x2 = x1 + w D^-1 (b - A x1), stored (2D); restrict the
// residual
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_down(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                  const int *kbase, int koff)
{
#pragma clang fp contract(off)
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    const MLevel &L = J.lev[tl.lv];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const T w = (T)mg_w<DIM>();
    auto mi = G<T>(L.minv);
    auto b = G<T>(L.b);
    Agg<DIM> a;
    int cx[3], q[3], i, I;
    T v = T(0);
    if (child_of<DIM>(L, tl.t, icx, icxy, a, cx, q, i, I)) {
        auto x1 = [&](int j, int, int) { return w * mi[j] * b[j]; };
        if constexpr (DIM == 2) {
            auto x2 = [&](int j, const int *qj) {
                return x1(j, 0, 0) + w * mi[j] * (b[j] - apply_op<DIM, T, true>(L, j, qj, x1));
            };
            const T x2i = x2(i, q);
            const T ax = apply_op<DIM, T, true>(L, i, q, [&](int j, int ax_, int dir) {
                int qj[3];
                step_q(q, ax_, dir, qj);
                return x2(j, qj);
            });
            G<T>(L.xs)[i] = x2i;
            v = b[i] - ax;
        } else {
            v = b[i] - apply_op<DIM, T, true>(L, i, q, x1);
        }
    }
    // sum over the 2^d children (consecutive lanes), fixed order
#pragma unroll
    for (int o = 1; o < (1 << DIM); o <<= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & ((1 << DIM) - 1)) == 0) {
        const int Iw = tl.t * L.cpt + (int)(threadIdx.x >> DIM);
        if (Iw < L.cn) G<T>(J.lev[tl.lv + 1].b)[Iw] = v;
    }
}

// level l >= 1 (launch level): e = x + mg_og P e_c on the pre-smoothed x,
// then one sweep (3D) or two (2D), e1 = e + w D^-1 (b - A e),
// e2 = e1 + w D^-1 (b - A e1)
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_up(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                const int *kbase, int koff)
{
#pragma clang fp contract(off)
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    const MLevel &L = J.lev[tl.lv];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const T w = (T)mg_w<DIM>(), og = (T)mg_og<DIM>();
    auto mi = G<T>(L.minv);
    auto b = G<T>(L.b);
    auto e = G<T>(L.e);
    auto xs = G<T>(L.xs);
    auto ec = G<T>(J.lev[tl.lv + 1].e);
    Agg<DIM> a;
    int cx[3], q[3], i, I;
    if (!child_of<DIM>(L, tl.t, icx, icxy, a, cx, q, i, I)) return;
    if constexpr (DIM == 3) {
        const T ax = apply_op<DIM, T, true>(L, i, q, [&](int j, int ax_, int dir) {
            return w * mi[j] * b[j] + og * ec[agg_nb<DIM>(L, a, cx, ax_, dir)];
        });
        const T xi = w * mi[i] * b[i] + og * ec[I];
        e[i] = xi + w * mi[i] * (b[i] - ax);
        return;
    }
    auto e0 = [&](int j, const int *qj) { return xs[j] + og * ec[agg_index(L, qj)]; };
    auto e1 = [&](int j, const int *qj) {
        const T aj = apply_op<DIM, T, true>(L, j, qj, [&](int jj, int ax_, int dir) {
            int qjj[3];
            step_q(qj, ax_, dir, qjj);
            return e0(jj, qjj);
        });
        return e0(j, qj) + w * mi[j] * (b[j] - aj);
    };
    const T ax = apply_op<DIM, T, true>(L, i, q, [&](int j, int ax_, int dir) {
        int qj[3];
        step_q(q, ax_, dir, qj);
        return e1(j, qj);
    });
    e[i] = e1(i, q) + w * mi[i] * (b[i] - ax);
}

// level 0: prolong, post-smooth -> z_(k+1); partials (r_(k+1), z_(k+1)),
// sum(z_(k+1)), sum(r_(k+1))
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_up0(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                 const int *kbase, int koff)
{
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J)) return;
    __shared__ double tab[27];
    write_minv0<DIM>(J.lev[0], tab);
    if (!mg_live(J, k)) return;
    const int pn1 = (k + 1) & 1;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const T w = (T)mg_w<DIM>(), og = (T)mg_og<DIM>();
    auto r = R<T>(pn1 ? J.rh : J.r);
    auto z = G<T>(J.v0);
    auto ec = R<T>(J.lev[1].e);
    double vv[3] = {0.0, 0.0, 0.0};     // (r, z), sum z, sum r
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    if constexpr (DIM == 2) {
        // e0 = x2 + og P e_c on the window, e1 = e0 + w D^-1 (r - A e0)
        // within one step of the children, z = e1 + w D^-1 (r - A e1)
        auto xs = R<T>(L.xs);
        const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1];
        for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
            const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
            const int X0 = 2 * a.c[0] - 2, Y0 = 2 * a.c[1] - 2;
            // coarse corrections of the 3 x 3 aggregates the window meets
            T ew[3][3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    ew[b][c] = ec[min(max(a.c[0] - 1 + c, 0), L.cnx - 1) + L.cnx * min(max(a.c[1] - 1 + b, 0), L.cny - 1)];
            int kx[W2], ky[W2];
#pragma unroll
            for (int u = 0; u < W2; ++u) {
                kx[u] = faces_in(X0 + u, L.nx);
                ky[u] = 3 * faces_in(Y0 + u, L.ny);
            }
            T e0[W2][W2], e1[W2][W2], rw[W2][W2], mw[W2][W2];
#pragma unroll
            for (int v = 0; v < W2; ++v)
#pragma unroll
                for (int u = 0; u < W2; ++u) {
                    if (wdist(u, v) > 2) continue;
                    const int j = win_idx(L, X0 + u, Y0 + v);
                    e0[v][u] = xs[j] + og * ew[v >> 1][u >> 1];
                    if (wdist(u, v) <= 1) {
                        rw[v][u] = r[j];
                        mw[v][u] = (T)tab[kx[u] + ky[v]];
                    }
                }
#pragma unroll
            for (int v = 1; v < W2 - 1; ++v)
#pragma unroll
                for (int u = 1; u < W2 - 1; ++u)
                    if (wdist(u, v) <= 1)
                        e1[v][u] = e0[v][u] + w * mw[v][u] * (rw[v][u] - win_op(L, X0 + u, Y0 + v, u, v, e0, c0, c1));
#pragma unroll
            for (int v = 2; v < 4; ++v)
#pragma unroll
                for (int u = 2; u < 4; ++u) {
                    const int gx = X0 + u, gy = Y0 + v;
                    if (gx >= L.nx || gy >= L.ny) continue;
                    const T zi = e1[v][u] + w * mw[v][u] * (rw[v][u] - win_op(L, gx, gy, u, v, e1, c0, c1));
                    z[gx + L.nx * gy] = zi;
                    vv[0] += (double)rw[v][u] * zi;
                    vv[1] += (double)zi;
                    vv[2] += (double)rw[v][u];
                }
        }
    } else {
        // x = w D^-1 r + og P e_c on the window, z = x + w D^-1 (r - A x)
        // at the children
        const T c0 = (T)L.ih2[0], c1 = (T)L.ih2[1], c2 = (T)L.ih2[2];
        for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
            const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
            const int X0 = 2 * a.c[0] - 1, Y0 = 2 * a.c[1] - 1, Z0 = 2 * a.c[2] - 1;
            // coarse corrections of the aggregate and of its six face
            // neighbours (a window cell off the block lies in one of them)
            auto cix = [&](int dx, int dy, int dz) {
                return min(max(a.c[0] + dx, 0), L.cnx - 1) +
                       L.cnx * (min(max(a.c[1] + dy, 0), L.cny - 1) + L.cny * min(max(a.c[2] + dz, 0), L.cnz - 1));
            };
            const T e0 = ec[I], exm = ec[cix(-1, 0, 0)], exp_ = ec[cix(1, 0, 0)], eym = ec[cix(0, -1, 0)],
                    eyp = ec[cix(0, 1, 0)], ezm = ec[cix(0, 0, -1)], ezp = ec[cix(0, 0, 1)];
            int kx[W3], ky[W3], kz[W3];
#pragma unroll
            for (int u = 0; u < W3; ++u) {
                kx[u] = faces_in(X0 + u, L.nx);
                ky[u] = 3 * faces_in(Y0 + u, L.ny);
                kz[u] = 9 * faces_in(Z0 + u, L.nz);
            }
            T xw[W3][W3][W3], rw[W3][W3][W3], mw[W3][W3][W3];
#pragma unroll
            for (int wz = 0; wz < W3; ++wz)
#pragma unroll
                for (int vy = 0; vy < W3; ++vy)
#pragma unroll
                    for (int ux = 0; ux < W3; ++ux) {
                        if (wdist3(ux, vy, wz) > 1) continue;
                        const int j = win3_idx(L, X0 + ux, Y0 + vy, Z0 + wz);
                        const T e = ux == 0 ? exm : ux == 3 ? exp_ : vy == 0 ? eym : vy == 3 ? eyp
                                  : wz == 0 ? ezm : wz == 3 ? ezp : e0;
                        const T rj = r[j], mj = (T)tab[kx[ux] + ky[vy] + kz[wz]];
                        rw[wz][vy][ux] = rj;
                        mw[wz][vy][ux] = mj;
                        xw[wz][vy][ux] = w * mj * rj + og * e;
                    }
#pragma unroll
            for (int wz = 1; wz < 3; ++wz)
#pragma unroll
                for (int vy = 1; vy < 3; ++vy)
#pragma unroll
                    for (int ux = 1; ux < 3; ++ux) {
                        const int gx = X0 + ux, gy = Y0 + vy, gz = Z0 + wz;
                        if (gx >= L.nx || gy >= L.ny || gz >= L.nz) continue;
                        const T ri = rw[wz][vy][ux];
                        const T zi = xw[wz][vy][ux] +
                                     w * mw[wz][vy][ux] * (ri - win3_op(L, gx, gy, gz, ux, vy, wz, xw, c0, c1, c2));
                        z[gx + L.nx * (gy + L.ny * gz)] = zi;
                        vv[0] += (double)ri * zi;
                        vv[1] += (double)zi;
                        vv[2] += (double)ri;
                    }
        }
    }
    const int off[3] = {poff(J, pn1, PS_RHO), poff(J, pn1, PS_Q), poff(J, pn1, PS_TT)};
    put_partials<3>(vv, J.part, off, tl.t);
}

// ------------------------------------------------ fused coarse-level pairs
// Two consecutive coarse levels l, l+1 (both smoothed, l+1 < nglob) in one
// launch each way instead of two.  A workgroup owns a brick of level-(l+2)
// cells and recomputes, in LDS, every value its brick's results depend on
// within the stencil reach of the sweeps (a halo of the finer levels),
// instead of reading them back from memory after a launch boundary: the
// only grid-wide dependencies of the V-cycle are the exact level and
// level 0's partial sums.  Each value is formed by the expression of the
// per-level kernels above in the same order (region_op is apply_op on an
// LDS region), and contraction into fused multiply-adds is off in both (the
// compiler's choice of which product to fuse may differ between the two
// kernels), so the two paths give the same results bit for bit; values the
// owning workgroup does not own are recomputed by every workgroup whose
// halo holds them.
//
// Brick edge in level-(l+2) cells: 2 in 3D (8 cells: level l+1 owned 4^3,
// with its one-step halo 6^3, level l 12^3 plus its halo 14^3), 4 in 2D
// (level l+1 owned 8^2, two-sweep halo 12^2; level l 24^2, load halo 28^2).
constexpr int FZ3 = 2, FZ2 = 4;

__host__ __device__ constexpr int fused_brick(int dim) { return dim == 3 ? FZ3 : FZ2; }

// (A f) at the level cell with coordinates q whose value sits at o in an
// LDS region with row stride RX and plane stride RXY: apply_op's arithmetic
// (a missing neighbour enters through a zero coupling with the cell's own
// value); every read stays inside the region, because cells are only
// evaluated at least one step inside it
template <int DIM, class T, int RX, int RXY>
__device__ __forceinline__ T region_op(const MLevel &L, const int *q, const T *f, int o)
{
#pragma clang fp contract(off)
    T co[3];
    couplings<DIM, T>(L, q, co);
    const int st[3] = {1, RX, RXY};
    const int nn[3] = {L.nx, L.ny, L.nz};
    const T fi = f[o];
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const bool lo = q[a] > 0, hi = q[a] + 1 < nn[a];
        const T vlo = f[lo ? o - st[a] : o];
        const T vhi = f[hi ? o + st[a] : o];
        acc += (lo ? co[a] : T(0)) * (fi - vlo) + (hi ? co[a] : T(0)) * (fi - vhi);
    }
    return acc;
}

__device__ __forceinline__ bool in_level(const MLevel &L, int x, int y, int z)
{
    return x >= 0 && y >= 0 && z >= 0 && x < L.nx && y < L.ny && z < L.nz;
}

// brick coordinates of tile t over the level-(l+2) counts of M (= level l+1)
template <int DIM>
__device__ __forceinline__ void brick_of(const MLevel &M, int t, int *bq)
{
    constexpr int B = DIM == 3 ? FZ3 : FZ2;
    const int nbx = ceil_div(M.cnx, B), nby = ceil_div(M.cny, B);
    bq[2] = DIM == 3 ? t / (nbx * nby) : 0;
    const int rem = t - bq[2] * nbx * nby;
    bq[1] = rem / nbx;
    bq[0] = rem - bq[1] * nbx;
}

// level l+2 rhs of the owned children: lanes 2^d c .. 2^d c + 2^d - 1 hold
// the residuals of the children of brick cell c (zero for a child off the
// grid); summed in k_mg_down's order and written by the first lane
template <int DIM, class T>
__device__ __forceinline__ void restrict_owned(const MLevel &M, const KJob &J, int lv, const int *bq, T v)
{
    constexpr int B = DIM == 3 ? FZ3 : FZ2;
#pragma unroll
    for (int o = 1; o < (1 << DIM); o <<= 1) v += __shfl_xor(v, o, 64);
    const int a = (int)threadIdx.x >> DIM;
    if ((threadIdx.x & ((1 << DIM) - 1)) == 0 && a < (DIM == 3 ? B * B * B : B * B)) {
        const int ax = a % B, ay = (a / B) % B, az = DIM == 3 ? a / (B * B) : 0;
        const int X = B * bq[0] + ax, Y = B * bq[1] + ay, Z = B * bq[2] + az;
        if (X < M.cnx && Y < M.cny && Z < M.cnz) G<T>(J.lev[lv + 2].b)[X + M.cnx * (Y + M.cny * Z)] = v;
    }
}

// pre-smooth levels l and l+1 and restrict twice (3D: one sweep from zero
// per level, x1 = w D^-1 b).  Every global load of the launch is issued
// first, held in registers, so that they are in flight together: one round
// trip instead of one per pass over the region.  The loads are
// unconditional (a cell off the grid reads element 0, and its value is
// replaced by 0): a load under a branch made the compiler wait for all
// earlier loads before the branch, one round trip per cell again.
template <class T>
__global__ __launch_bounds__(TILE) void k_mg_down2_3(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                     const int *kbase, int koff)
{
#pragma clang fp contract(off)
    constexpr int R1 = 2 * FZ3 + 2, RR = 2 * R1, RL = RR + 2;
    constexpr int NL = RL * RL * RL, NIL = (NL + TILE - 1) / TILE, N1 = R1 * R1 * R1;
    static_assert(N1 <= TILE, "one level-(l+1) region cell per thread");
    __shared__ T X[NL];                  // level l: x1 on the load region
    __shared__ T Bv[RR * RR * RR];       // level l: b, then the residual, on the residual region
    __shared__ T Xc[N1];                 // level l+1: x1
    __shared__ T Bc[N1];                 // level l+1: b (the restricted residual)
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    // level tables by value: read once into registers (through a reference
    // the compiler reloads the counts inside the loops, a wait each time)
    const MLevel L = J.lev[tl.lv], M = J.lev[tl.lv + 1];
    const T w = (T)mg_w<3>();
    int bq[3];
    brick_of<3>(M, tl.t, bq);
    int o1[3], oR[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o1[a] = 2 * FZ3 * bq[a] - 1;      // level l+1 region origin
        oR[a] = 2 * o1[a];                // level l residual region origin (load region: oR - 1)
    }
    const int U = threadIdx.x % R1, V = (threadIdx.x / R1) % R1, W = threadIdx.x / (R1 * R1);
    const int g1[3] = {o1[0] + U, o1[1] + V, o1[2] + W};
    const bool c1 = (int)threadIdx.x < N1 && in_level(M, g1[0], g1[1], g1[2]);
    const int I1 = g1[0] + M.nx * (g1[1] + M.ny * g1[2]);
    T bl[NIL], ml[NIL], mc = T(0);
    {
        auto mi = G<T>(L.minv);
        auto b = G<T>(L.b);
#pragma unroll
        for (int it = 0; it < NIL; ++it) {
            const int id = threadIdx.x + it * TILE;
            const int u = id % RL, v = (id / RL) % RL, s = id / (RL * RL);
            const int gx = oR[0] - 1 + u, gy = oR[1] - 1 + v, gz = oR[2] - 1 + s;
            const bool ok = id < NL && in_level(L, gx, gy, gz);
            const int j = ok ? gx + L.nx * (gy + L.ny * gz) : 0;
            const T bv = b[j], mv = mi[j];
            bl[it] = ok ? bv : T(0);
            ml[it] = ok ? mv : T(0);
        }
        const T m1 = G<T>(M.minv)[c1 ? I1 : 0];
        mc = c1 ? m1 : T(0);
    }
#pragma unroll
    for (int it = 0; it < NIL; ++it) {
        const int id = threadIdx.x + it * TILE;
        if (id < NL) {
            const int u = id % RL, v = (id / RL) % RL, s = id / (RL * RL);
            X[id] = w * ml[it] * bl[it];
            if (u >= 1 && v >= 1 && s >= 1 && u <= RR && v <= RR && s <= RR)
                Bv[(u - 1) + RR * ((v - 1) + RR * (s - 1))] = bl[it];
        }
    }
    __syncthreads();
    for (int id = threadIdx.x; id < RR * RR * RR; id += TILE) {
        const int u = id % RR, v = (id / RR) % RR, s = id / (RR * RR);
        const int q[3] = {oR[0] + u, oR[1] + v, oR[2] + s};
        T r = T(0);
        if (in_level(L, q[0], q[1], q[2]))
            r = Bv[id] - region_op<3, T, RL, RL * RL>(L, q, X, (u + 1) + RL * ((v + 1) + RL * (s + 1)));
        Bv[id] = r;
    }
    __syncthreads();
    if ((int)threadIdx.x < N1) {
        T bc = T(0), xc = T(0);
        if (c1) {
            auto rr = [&](int cx, int cy, int cz) {
                return Bv[(2 * U + cx) + RR * ((2 * V + cy) + RR * (2 * W + cz))];
            };
            bc = ((rr(0, 0, 0) + rr(1, 0, 0)) + (rr(0, 1, 0) + rr(1, 1, 0))) +
                 ((rr(0, 0, 1) + rr(1, 0, 1)) + (rr(0, 1, 1) + rr(1, 1, 1)));
            if (U >= 1 && V >= 1 && W >= 1 && U < R1 - 1 && V < R1 - 1 && W < R1 - 1) G<T>(M.b)[I1] = bc;
            xc = w * mc * bc;
        }
        Bc[threadIdx.x] = bc;
        Xc[threadIdx.x] = xc;
    }
    __syncthreads();
    // owned level-(l+1) cells: 8 lanes per brick cell (threads 0..63)
    T v = T(0);
    {
        const int c = threadIdx.x & 7, a = (int)threadIdx.x >> 3;
        if (a < FZ3 * FZ3 * FZ3) {
            const int Uo = 1 + 2 * (a % FZ3) + (c & 1), Vo = 1 + 2 * ((a / FZ3) % FZ3) + ((c >> 1) & 1),
                      Wo = 1 + 2 * (a / (FZ3 * FZ3)) + ((c >> 2) & 1);
            const int q[3] = {o1[0] + Uo, o1[1] + Vo, o1[2] + Wo};
            if (in_level(M, q[0], q[1], q[2])) {
                const int o = Uo + R1 * (Vo + R1 * Wo);
                v = Bc[o] - region_op<3, T, R1, R1 * R1>(M, q, Xc, o);
            }
        }
    }
    restrict_owned<3, T>(M, J, tl.lv, bq, v);
}

// 2D: two sweeps per level, the pre-smoothed x2 stored for the
// post-smoothing (xs of levels l and l+1); loads first, as in 3D
template <class T>
__global__ __launch_bounds__(TILE) void k_mg_down2_2(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                     const int *kbase, int koff)
{
#pragma clang fp contract(off)
    constexpr int R1 = 2 * FZ2 + 4, RR = 2 * R1, RL = RR + 4;
    constexpr int NL = RL * RL, NIL = (NL + TILE - 1) / TILE, N1 = R1 * R1;
    static_assert(N1 <= TILE, "one level-(l+1) region cell per thread");
    __shared__ T X1[NL], X2[NL], Bl[NL], Ml[NL];           // level l on the load region
    __shared__ T Rr[RR * RR];                              // level l residual
    __shared__ T C1[N1], C2[N1], Bc[N1], Mc[N1];           // level l+1
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    // level tables by value: read once into registers (through a reference
    // the compiler reloads the counts inside the loops, a wait each time)
    const MLevel L = J.lev[tl.lv], M = J.lev[tl.lv + 1];
    const T w = (T)mg_w<2>();
    int bq[3];
    brick_of<2>(M, tl.t, bq);
    const int o1[2] = {2 * FZ2 * bq[0] - 2, 2 * FZ2 * bq[1] - 2};   // level l+1 region origin
    const int oL[2] = {2 * o1[0] - 2, 2 * o1[1] - 2};               // level l load region origin
    const int U = threadIdx.x % R1, V = threadIdx.x / R1;
    const int g1[2] = {o1[0] + U, o1[1] + V};
    const bool c1 = (int)threadIdx.x < N1 && in_level(M, g1[0], g1[1], 0);
    const int I1 = g1[0] + M.nx * g1[1];
    T bl[NIL], ml[NIL], mc = T(0);
    {
        auto mi = G<T>(L.minv);
        auto b = G<T>(L.b);
#pragma unroll
        for (int it = 0; it < NIL; ++it) {
            const int id = threadIdx.x + it * TILE;
            const int gx = oL[0] + id % RL, gy = oL[1] + id / RL;
            const bool ok = id < NL && in_level(L, gx, gy, 0);
            const int j = ok ? gx + L.nx * gy : 0;
            const T bv = b[j], mv = mi[j];
            bl[it] = ok ? bv : T(0);
            ml[it] = ok ? mv : T(0);
        }
        const T m1 = G<T>(M.minv)[c1 ? I1 : 0];
        mc = c1 ? m1 : T(0);
    }
#pragma unroll
    for (int it = 0; it < NIL; ++it) {
        const int id = threadIdx.x + it * TILE;
        if (id < NL) {
            Bl[id] = bl[it];
            Ml[id] = ml[it];
            X1[id] = w * ml[it] * bl[it];
        }
    }
    __syncthreads();
    for (int id = threadIdx.x; id < NL; id += TILE) {
        const int u = id % RL, v = id / RL;
        const int q[3] = {oL[0] + u, oL[1] + v, 0};
        T x2 = T(0);
        if (u >= 1 && v >= 1 && u < RL - 1 && v < RL - 1 && in_level(L, q[0], q[1], 0))
            x2 = X1[id] + w * Ml[id] * (Bl[id] - region_op<2, T, RL, RL * RL>(L, q, X1, id));
        X2[id] = x2;
    }
    __syncthreads();
    {
        auto xs = G<T>(L.xs);
        for (int id = threadIdx.x; id < RR * RR; id += TILE) {
            const int u = id % RR, v = id / RR;
            const int o = (u + 2) + RL * (v + 2);
            const int q[3] = {oL[0] + u + 2, oL[1] + v + 2, 0};
            T r = T(0);
            if (in_level(L, q[0], q[1], 0)) {
                r = Bl[o] - region_op<2, T, RL, RL * RL>(L, q, X2, o);
                if (u >= 4 && v >= 4 && u < RR - 4 && v < RR - 4) xs[q[0] + L.nx * q[1]] = X2[o];
            }
            Rr[id] = r;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < N1) {
        T bc = T(0), xc = T(0);
        if (c1) {
            bc = (Rr[2 * U + RR * (2 * V)] + Rr[2 * U + 1 + RR * (2 * V)]) +
                 (Rr[2 * U + RR * (2 * V + 1)] + Rr[2 * U + 1 + RR * (2 * V + 1)]);
            if (U >= 2 && V >= 2 && U < R1 - 2 && V < R1 - 2) G<T>(M.b)[I1] = bc;
            xc = w * mc * bc;
        }
        Bc[threadIdx.x] = bc;
        Mc[threadIdx.x] = mc;
        C1[threadIdx.x] = xc;
    }
    __syncthreads();
    if ((int)threadIdx.x < N1) {
        const int q[3] = {g1[0], g1[1], 0};
        T x2 = T(0);
        if (U >= 1 && V >= 1 && U < R1 - 1 && V < R1 - 1 && c1)
            x2 = C1[threadIdx.x] + w * Mc[threadIdx.x] * (Bc[threadIdx.x] -
                                                        region_op<2, T, R1, R1 * R1>(M, q, C1, threadIdx.x));
        C2[threadIdx.x] = x2;
    }
    __syncthreads();
    // owned level-(l+1) cells: 4 lanes per brick cell (threads 0..63)
    T v = T(0);
    {
        const int c = threadIdx.x & 3, a = (int)threadIdx.x >> 2;
        if (a < FZ2 * FZ2) {
            const int Uo = 2 + 2 * (a % FZ2) + (c & 1), Vo = 2 + 2 * (a / FZ2) + (c >> 1);
            const int q[3] = {o1[0] + Uo, o1[1] + Vo, 0};
            if (in_level(M, q[0], q[1], 0)) {
                const int o = Uo + R1 * Vo;
                v = Bc[o] - region_op<2, T, R1, R1 * R1>(M, q, C2, o);
                G<T>(M.xs)[q[0] + M.nx * q[1]] = C2[o];
            }
        }
    }
    restrict_owned<2, T>(M, J, tl.lv, bq, v);
}

// prolong onto and post-smooth levels l+1 and l (3D, one sweep per level):
// e = x + w D^-1 (b - A x), x = w D^-1 b + mg_og P e_c; the loads of both
// levels first
template <class T>
__global__ __launch_bounds__(TILE) void k_mg_up2_3(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                   const int *kbase, int koff)
{
#pragma clang fp contract(off)
    constexpr int RX1 = 2 * FZ3 + 4, RE = RX1 - 2;   // level l+1: x region 8^3, e region 6^3
    constexpr int RXL = 4 * FZ3 + 2;                 // level l: x region 10^3 (owned 8^3)
    constexpr int NC = RX1 * RX1 * RX1, NIC = (NC + TILE - 1) / TILE;
    constexpr int NLv = RXL * RXL * RXL, NIL = (NLv + TILE - 1) / TILE;
    __shared__ T Xc[NC], Bc[NC], Mc[NC];
    __shared__ T Ec[RE * RE * RE];
    __shared__ T Xl[NLv], Bl[NLv], Ml[NLv];
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    // level tables by value: read once into registers (through a reference
    // the compiler reloads the counts inside the loops, a wait each time)
    const MLevel L = J.lev[tl.lv], M = J.lev[tl.lv + 1];
    const T w = (T)mg_w<3>(), og = (T)mg_og<3>();
    int bq[3];
    brick_of<3>(M, tl.t, bq);
    int oX1[3], oE[3], oXL[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        oX1[a] = 2 * FZ3 * bq[a] - 2;    // level l+1 x region origin
        oE[a] = oX1[a] + 1;              // level l+1 e region origin
        oXL[a] = 4 * FZ3 * bq[a] - 1;    // level l x region origin
    }
    T bc[NIC], mc[NIC], ecv[NIC], bl[NIL], ml[NIL];
    {
        auto mi = G<T>(M.minv);
        auto b = G<T>(M.b);
        auto ec = G<T>(J.lev[tl.lv + 2].e);
#pragma unroll
        for (int it = 0; it < NIC; ++it) {
            const int id = threadIdx.x + it * TILE;
            const int q[3] = {oX1[0] + id % RX1, oX1[1] + (id / RX1) % RX1, oX1[2] + id / (RX1 * RX1)};
            const bool ok = id < NC && in_level(M, q[0], q[1], q[2]);
            const int j = ok ? q[0] + M.nx * (q[1] + M.ny * q[2]) : 0;
            const int je = ok ? agg_index(M, q) : 0;
            const T bv = b[j], mv = mi[j], ev = ec[je];
            bc[it] = ok ? bv : T(0);
            mc[it] = ok ? mv : T(0);
            ecv[it] = ok ? ev : T(0);
        }
        auto mil = G<T>(L.minv);
        auto bll = G<T>(L.b);
#pragma unroll
        for (int it = 0; it < NIL; ++it) {
            const int id = threadIdx.x + it * TILE;
            const int gx = oXL[0] + id % RXL, gy = oXL[1] + (id / RXL) % RXL, gz = oXL[2] + id / (RXL * RXL);
            const bool ok = id < NLv && in_level(L, gx, gy, gz);
            const int j = ok ? gx + L.nx * (gy + L.ny * gz) : 0;
            const T bv = bll[j], mv = mil[j];
            bl[it] = ok ? bv : T(0);
            ml[it] = ok ? mv : T(0);
        }
    }
#pragma unroll
    for (int it = 0; it < NIC; ++it) {
        const int id = threadIdx.x + it * TILE;
        if (id < NC) {
            Bc[id] = bc[it];
            Mc[id] = mc[it];
            Xc[id] = w * mc[it] * bc[it] + og * ecv[it];   // exactly 0 off the grid
        }
    }
    __syncthreads();
    for (int id = threadIdx.x; id < RE * RE * RE; id += TILE) {
        const int u = id % RE, v = (id / RE) % RE, s = id / (RE * RE);
        const int q[3] = {oE[0] + u, oE[1] + v, oE[2] + s};
        T e = T(0);
        if (in_level(M, q[0], q[1], q[2])) {
            const int o = (u + 1) + RX1 * ((v + 1) + RX1 * (s + 1));
            e = Xc[o] + w * Mc[o] * (Bc[o] - region_op<3, T, RX1, RX1 * RX1>(M, q, Xc, o));
        }
        Ec[id] = e;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIL; ++it) {
        const int id = threadIdx.x + it * TILE;
        if (id < NLv) {
            const int gx = oXL[0] + id % RXL, gy = oXL[1] + (id / RXL) % RXL, gz = oXL[2] + id / (RXL * RXL);
            T xv = T(0);
            if (in_level(L, gx, gy, gz)) {
                const int ce = ((gx >> 1) - oE[0]) + RE * (((gy >> 1) - oE[1]) + RE * ((gz >> 1) - oE[2]));
                xv = w * ml[it] * bl[it] + og * Ec[ce];
            }
            Bl[id] = bl[it];
            Ml[id] = ml[it];
            Xl[id] = xv;
        }
    }
    __syncthreads();
    auto e = G<T>(L.e);
    constexpr int RO = RXL - 2;
    for (int id = threadIdx.x; id < RO * RO * RO; id += TILE) {
        const int u = id % RO, v = (id / RO) % RO, s = id / (RO * RO);
        const int q[3] = {oXL[0] + 1 + u, oXL[1] + 1 + v, oXL[2] + 1 + s};
        if (!in_level(L, q[0], q[1], q[2])) continue;
        const int o = (u + 1) + RXL * ((v + 1) + RXL * (s + 1));
        e[q[0] + L.nx * (q[1] + L.ny * q[2])] =
            Xl[o] + w * Ml[o] * (Bl[o] - region_op<3, T, RXL, RXL * RXL>(L, q, Xl, o));
    }
}

// 2D: two post-sweeps per level from e0 = x2 + mg_og P e_c; loads first
template <class T>
__global__ __launch_bounds__(TILE) void k_mg_up2_2(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                   const int *kbase, int koff)
{
#pragma clang fp contract(off)
    constexpr int RC = 2 * FZ2 + 6;        // level l+1: e0 region 14 (e1 12, e 10)
    constexpr int RLX = 4 * FZ2 + 4;       // level l: e0 region 20 (e1 18, owned 16)
    constexpr int NC = RC * RC, NLv = RLX * RLX, NIL = (NLv + TILE - 1) / TILE;
    static_assert(NC <= TILE, "one level-(l+1) region cell per thread");
    __shared__ T E0c[NC], E1c[NC], Ec[NC], Bc[NC], Mc[NC];
    __shared__ T E0[NLv], E1[NLv], Bl[NLv], Ml[NLv];
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    // level tables by value: read once into registers (through a reference
    // the compiler reloads the counts inside the loops, a wait each time)
    const MLevel L = J.lev[tl.lv], M = J.lev[tl.lv + 1];
    const T w = (T)mg_w<2>(), og = (T)mg_og<2>();
    int bq[3];
    brick_of<2>(M, tl.t, bq);
    const int oC[2] = {2 * FZ2 * bq[0] - 3, 2 * FZ2 * bq[1] - 3};   // level l+1 region origin
    const int oL[2] = {4 * FZ2 * bq[0] - 2, 4 * FZ2 * bq[1] - 2};   // level l region origin
    const int Uc = threadIdx.x % RC, Vc = threadIdx.x / RC;
    const int qc[3] = {oC[0] + Uc, oC[1] + Vc, 0};
    const bool cc = (int)threadIdx.x < NC && in_level(M, qc[0], qc[1], 0);
    T bcv = T(0), mcv = T(0), xsc = T(0), ecv = T(0), bl[NIL], ml[NIL], xl[NIL];
    {
        {
            const int j = cc ? qc[0] + M.nx * qc[1] : 0;
            const int je = cc ? agg_index(M, qc) : 0;
            const T b1 = G<T>(M.b)[j], m1 = G<T>(M.minv)[j], x1 = G<T>(M.xs)[j], e1 = G<T>(J.lev[tl.lv + 2].e)[je];
            bcv = cc ? b1 : T(0);
            mcv = cc ? m1 : T(0);
            xsc = cc ? x1 : T(0);
            ecv = cc ? e1 : T(0);
        }
        auto mi = G<T>(L.minv);
        auto b = G<T>(L.b);
        auto xs = G<T>(L.xs);
#pragma unroll
        for (int it = 0; it < NIL; ++it) {
            const int id = threadIdx.x + it * TILE;
            const int gx = oL[0] + id % RLX, gy = oL[1] + id / RLX;
            const bool ok = id < NLv && in_level(L, gx, gy, 0);
            const int j = ok ? gx + L.nx * gy : 0;
            const T bv = b[j], mv = mi[j], xv = xs[j];
            bl[it] = ok ? bv : T(0);
            ml[it] = ok ? mv : T(0);
            xl[it] = ok ? xv : T(0);
        }
    }
    if ((int)threadIdx.x < NC) {
        Bc[threadIdx.x] = bcv;
        Mc[threadIdx.x] = mcv;
        E0c[threadIdx.x] = cc ? xsc + og * ecv : T(0);
    }
    __syncthreads();
    if ((int)threadIdx.x < NC) {
        T e1 = T(0);
        if (Uc >= 1 && Vc >= 1 && Uc < RC - 1 && Vc < RC - 1 && cc)
            e1 = E0c[threadIdx.x] + w * Mc[threadIdx.x] * (Bc[threadIdx.x] -
                                                          region_op<2, T, RC, RC * RC>(M, qc, E0c, threadIdx.x));
        E1c[threadIdx.x] = e1;
    }
    __syncthreads();
    if ((int)threadIdx.x < NC) {
        T ev = T(0);
        if (Uc >= 2 && Vc >= 2 && Uc < RC - 2 && Vc < RC - 2 && cc)
            ev = E1c[threadIdx.x] + w * Mc[threadIdx.x] * (Bc[threadIdx.x] -
                                                          region_op<2, T, RC, RC * RC>(M, qc, E1c, threadIdx.x));
        Ec[threadIdx.x] = ev;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIL; ++it) {
        const int id = threadIdx.x + it * TILE;
        if (id < NLv) {
            const int gx = oL[0] + id % RLX, gy = oL[1] + id / RLX;
            Bl[id] = bl[it];
            Ml[id] = ml[it];
            E0[id] = in_level(L, gx, gy, 0) ? xl[it] + og * Ec[((gx >> 1) - oC[0]) + RC * ((gy >> 1) - oC[1])]
                                            : T(0);
        }
    }
    __syncthreads();
    for (int id = threadIdx.x; id < NLv; id += TILE) {
        const int u = id % RLX, v = id / RLX;
        const int q[3] = {oL[0] + u, oL[1] + v, 0};
        T e1 = T(0);
        if (u >= 1 && v >= 1 && u < RLX - 1 && v < RLX - 1 && in_level(L, q[0], q[1], 0))
            e1 = E0[id] + w * Ml[id] * (Bl[id] - region_op<2, T, RLX, RLX * RLX>(L, q, E0, id));
        E1[id] = e1;
    }
    __syncthreads();
    auto e = G<T>(L.e);
    for (int id = threadIdx.x; id < NLv; id += TILE) {
        const int u = id % RLX, v = id / RLX;
        const int q[3] = {oL[0] + u, oL[1] + v, 0};
        if (u < 2 || v < 2 || u >= RLX - 2 || v >= RLX - 2 || !in_level(L, q[0], q[1], 0)) continue;
        e[q[0] + L.nx * q[1]] = E1[id] + w * Ml[id] * (Bl[id] - region_op<2, T, RLX, RLX * RLX>(L, q, E1, id));
    }
}

// ------------------------------------------------------------- exact level
// e = P^-1 b on level nglob, one wave per row: workgroup (job, t) takes rows
// 4t .. 4t+3.  P^-1 is symmetric, so the stored row is read: lane l sums
// columns l, l+64, ... with four accumulators (64 consecutive entries per
// load), the wave adds its lanes in the fixed DPP tree.  The entries are
// the FP32 rounding of the FP64 inverse at either precision (half the bytes
// of the product that dominates this kernel): still symmetric, and its
// relative perturbation (6e-8) is far below 1 / cond(A + c 1 1^T), so the
// preconditioner stays positive definite; the FP64 solve's residuals and
// updates stay FP64.
template <class T>
__global__ __launch_bounds__(TILE) void k_mg_exact(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                   const int *kbase, int koff)
{
    const int k = kidx(kbase, koff);
    const JTile tl = tiles[blockIdx.x];
    const KJob &J = jobs[tl.j];
    if (outer_idle(J) || !mg_live(J, k)) return;
    const MLevel &L = J.lev[tl.lv];
    const int n = L.n;
    const int row = tl.t * MG_XROWS + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= n) return;                       // whole waves
    auto P = G<float>(L.pinv) + (size_t)row * n;
    auto b = G<T>(L.b);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    int j = lane;
    for (; j + 192 < n; j += 256) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += (T)P[j + 64 * u] * b[j + 64 * u];
    }
    for (; j < n; j += 64) acc[0] += (T)P[j] * b[j];
    const double s = wave_sum((double)((acc[0] + acc[1]) + (acc[2] + acc[3])));
    if (lane == 0) G<T>(L.e)[row] = (T)s;
}

// setup: P^-1 of the exactly solved level l (n <= MG_EXACT_MAX_LARGE) by
// Gauss-Jordan elimination of the symmetric positive definite A + c 1 1^T in
// place (no pivoting needed), in blocks of MG_GJB pivots K, two launches per
// block: (a) every workgroup inverts the diagonal block D = P[K,K] in LDS;
// thread j forms the transformed pivot row X[:,j] = D^-1 P[K,j] and copies
// row j's pivot columns C[j,:] = P[j,K]; (b) P[K,K] = D^-1, P[K,j] = X[:,j],
// P[i,K] = -C[i,:] D^-1, and P[i,j] -= C[i,:] X[:,j] elsewhere.  Launch (b)
// reads only its own entry of P and the scratch (a) wrote.  Scratch layout
// (mg_gj_work): X at 0, C at MG_GJB n, D^-1 at 2 MG_GJB n, c last.

// dense operator from the closed form: -coupling for a neighbour, the
// diagonal for j = i (thread per entry)
template <int DIM>
__global__ __launch_bounds__(TILE) void k_mg_pdense(const MLevel *__restrict__ lev, int l, double *P)
{
    const MLevel &L = lev[l];
    const int n = L.n;
    const int idx = blockIdx.x * TILE + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx - i * n;
    int q[3];
    cell_coords<DIM>(i, L.nx, L.ny, 1.0 / L.nx, 1.0 / ((double)L.nx * L.ny), q);
    double co[3];
    couplings<DIM, double>(L, q, co);
    const int st[3] = {1, L.nx, L.nx * L.ny};
    const int nn[3] = {L.nx, L.ny, L.nz};
    double v = 0.0;
    if (j == i) v = op_diag<DIM, double>(L, q);
    for (int a = 0; a < DIM; ++a) {
        if (q[a] > 0 && j == i - st[a]) v = -co[a];
        if (q[a] + 1 < nn[a] && j == i + st[a]) v = -co[a];
    }
    P[idx] = v;
}

// c = (sum of the diagonal) / n^2 (1 for a zero operator); one workgroup
__global__ __launch_bounds__(TILE) void k_mg_pshift(const double *__restrict__ P, int n, double *work)
{
    double t[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += TILE) t[0] += P[(size_t)i * n + i];
    __shared__ double sh[4];
    block_sum<1>(t, sh);
    if (threadIdx.x == 0) work[mg_gj_work(n) - 1] = t[0] > 0.0 ? t[0] / ((double)n * n) : 1.0;
}

// P += c
__global__ __launch_bounds__(TILE) void k_mg_padd(double *P, int n, const double *work)
{
    const int idx = blockIdx.x * TILE + threadIdx.x;
    if (idx >= n * n) return;
    P[idx] += work[mg_gj_work(n) - 1];
}

// block K = [k0, k0 + bk), launch (a)
__global__ __launch_bounds__(TILE) void k_mg_pgj_a(const double *__restrict__ P, int n, int k0, int bk, double *work)
{
    constexpr int B = MG_GJB;
    __shared__ double Dm[2][B][B + 1];
    const int t = threadIdx.x, r = t / B, c = t % B;     // TILE == B * B
    if (r < bk && c < bk) Dm[0][r][c] = P[(size_t)(k0 + r) * n + k0 + c];
    __syncthreads();
    for (int p = 0; p < bk; ++p) {
        const int a = p & 1;
        if (r < bk && c < bk) {
            const double piv = Dm[a][p][p];
            const double rk = (c == p ? 1.0 : Dm[a][p][c]) / piv;
            const double ck = r == p ? 0.0 : Dm[a][r][p];
            Dm[a ^ 1][r][c] = r == p ? rk : (c == p ? 0.0 : Dm[a][r][c]) - ck * rk;
        }
        __syncthreads();
    }
    const int f = bk & 1;                                 // the buffer holding D^-1
    double *X = work, *Cp = work + (size_t)B * n, *Di = work + 2 * (size_t)B * n;
    if (blockIdx.x == 0 && r < bk && c < bk) Di[r * B + c] = Dm[f][r][c];
    const int j = blockIdx.x * TILE + t;
    if (j >= n) return;
    double pk[B];
#pragma unroll
    for (int q = 0; q < B; ++q) pk[q] = q < bk ? P[(size_t)(k0 + q) * n + j] : 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
        if (q >= bk) break;
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < B; ++w)
            if (w < bk) x += Dm[f][q][w] * pk[w];
        X[(size_t)q * n + j] = x;
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
        if (q < bk) Cp[(size_t)j * B + q] = P[(size_t)j * n + k0 + q];
}

// block K = [k0, k0 + bk), launch (b)
__global__ __launch_bounds__(TILE) void k_mg_pgj_b(double *P, int n, int k0, int bk, const double *__restrict__ work)
{
    constexpr int B = MG_GJB;
    const int idx = blockIdx.x * TILE + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx - i * n;
    const double *X = work, *Cp = work + (size_t)B * n, *Di = work + 2 * (size_t)B * n;
    const bool iK = i >= k0 && i < k0 + bk, jK = j >= k0 && j < k0 + bk;
    double v;
    if (iK && jK) {
        v = Di[(i - k0) * B + (j - k0)];
    } else if (iK) {
        v = X[(size_t)(i - k0) * n + j];
    } else if (jK) {
        v = 0.0;
        for (int q = 0; q < bk; ++q) v -= Cp[(size_t)i * B + q] * Di[q * B + (j - k0)];
    } else {
        v = P[idx];
        for (int q = 0; q < bk; ++q) v -= Cp[(size_t)i * B + q] * X[(size_t)q * n + j];
    }
    P[idx] = v;
}

__global__ __launch_bounds__(TILE) void k_mg_p32(const double *__restrict__ P, float *P32, int nn)
{
    const int idx = blockIdx.x * TILE + threadIdx.x;
    if (idx < nn) P32[idx] = (float)P[idx];
}

void launch_mg_pinv(int dim, const MLevel *lev, int l, int n, double *P, float *P32, double *work, hipStream_t s)
{
    if (n <= 0) return;
    const int nn = n * n;
    const dim3 g(ceil_div(nn, TILE)), b(TILE);
    if (dim == 2) SOL_LAUNCH(k_mg_pdense<2>, g, b, 0, s, lev, l, P);
    else SOL_LAUNCH(k_mg_pdense<3>, g, b, 0, s, lev, l, P);
    SOL_LAUNCH(k_mg_pshift, dim3(1), dim3(TILE), 0, s, (const double *)P, n, work);
    SOL_LAUNCH(k_mg_padd, g, b, 0, s, P, n, (const double *)work);
    static_assert(MG_GJB * MG_GJB == TILE, "one thread per entry of the diagonal block");
    for (int k0 = 0; k0 < n; k0 += MG_GJB) {
        const int bk = std::min(MG_GJB, n - k0);
        SOL_LAUNCH(k_mg_pgj_a, dim3(ceil_div(n, TILE)), b, 0, s, (const double *)P, n, k0, bk, work);
        SOL_LAUNCH(k_mg_pgj_b, g, b, 0, s, P, n, k0, bk, (const double *)work);
    }
    if (P32) SOL_LAUNCH(k_mg_p32, g, b, 0, s, (const double *)P, P32, nn);
}

// ------------------------------------------------------------- launchers

template <int DIM, class T>
static const void *mg_fn_t(int which)
{
    switch (which) {
    case KI_MG_PQ: return (const void *)&k_mg_pq<DIM, T>;
    case KI_MG_DOWN0: return (const void *)&k_mg_down0<DIM, T, false>;
    case KI_MG_DOWN0_INIT: return (const void *)&k_mg_down0<DIM, T, true>;
    case KI_MG_DOWN: return (const void *)&k_mg_down<DIM, T>;
    case KI_MG_EXACT: return (const void *)&k_mg_exact<T>;
    case KI_MG_UP: return (const void *)&k_mg_up<DIM, T>;
    case KI_MG_UP0: return (const void *)&k_mg_up0<DIM, T>;
    case KI_MG_DOWN2: return DIM == 3 ? (const void *)&k_mg_down2_3<T> : (const void *)&k_mg_down2_2<T>;
    case KI_MG_UP2: return DIM == 3 ? (const void *)&k_mg_up2_3<T> : (const void *)&k_mg_up2_2<T>;
    }
    return nullptr;
}

int mg_fused_bricks(int dim, const MLevel &M)
{
    const int B = fused_brick(dim);
    return ceil_div(M.cnx, B) * ceil_div(M.cny, B) * (dim == 3 ? ceil_div(M.cnz, B) : 1);
}

const void *mg_fn(int which, int nd, int fp32)
{
    if (nd == 5) return fp32 ? mg_fn_t<2, float>(which) : mg_fn_t<2, double>(which);
    return fp32 ? mg_fn_t<3, float>(which) : mg_fn_t<3, double>(which);
}

void launch_mg_finish(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    const dim3 g(nt), b(TILE);
    if (nd == 5) SOL_LAUNCH(k_mg_finish<2>, g, b, 0, s, j, t);
    else SOL_LAUNCH(k_mg_finish<3>, g, b, 0, s, j, t);
}

void launch_mg_ir_resid(int nd, const KJob *j, const JTile *t, int nt, int mode, hipStream_t s)
{
    if (nt <= 0) return;
    const dim3 g(nt), b(TILE);
    if (nd == 5) SOL_LAUNCH(k_mg_ir_resid<2>, g, b, 0, s, j, t, mode);
    else SOL_LAUNCH(k_mg_ir_resid<3>, g, b, 0, s, j, t, mode);
}

void launch_mg_init(int nd, int fp32, const KJob *j, const JTile *t, int nt, int k, int mode, hipStream_t s)
{
    if (nt <= 0) return;
    const dim3 g(nt), b(TILE);
    if (nd == 5) {
        if (fp32) SOL_LAUNCH((k_mg_init<2, float>), g, b, 0, s, j, t, k, mode);
        else SOL_LAUNCH((k_mg_init<2, double>), g, b, 0, s, j, t, k, mode);
    } else {
        if (fp32) SOL_LAUNCH((k_mg_init<3, float>), g, b, 0, s, j, t, k, mode);
        else SOL_LAUNCH((k_mg_init<3, double>), g, b, 0, s, j, t, k, mode);
    }
}

}  // namespace sol
