// Multigrid-preconditioned conjugate gradients for the pressure-correction
// system of eq. (3.4).  The paper leaves the solver of this constant,
// symmetric Neumann Laplacian open; Jacobi-PCG needs O(n^(1/d)) iterations
// per solve, a V-cycle preconditioner a few tens at any size.
//
// Hierarchy (built once per case, the operator never changes): level l+1
// aggregates 2 x 2 (x 2) cells of level l; its operator is the Galerkin
// product P^T A_l P with the piecewise-constant aggregation P.  For a
// 5- / 7-point operator that is again 5- / 7-point: coarse couplings are sums
// of the fine couplings across the aggregate faces, the diagonal collects the
// rest, and row sums stay zero (the constant null space is kept).
//
// Preconditioner z = M r: one V-cycle from a zero initial guess.
//   launch levels (0 .. nglob-1): one damped-Jacobi sweep before and after
//     the coarse correction, the correction scaled by MG_OG (aggregation
//     under-estimates smooth error; the scaling restores most of the rate);
//   LDS levels (nglob .. coarsest): one workgroup per solve runs a V(2,2)
//     cycle with correction scaling MG_OL in local memory; the single-cell
//     coarsest level has a zero operator and returns 0.
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
//              on level 0 and restrict the residual to level 1
//   down(l):   pre-smooth level l, restrict to level l+1     (l = 1 .. nglob-1)
//   lds:       levels nglob .. coarsest in one workgroup
//   up(l):     prolong, post-smooth level l                  (l = nglob-1 .. 1)
//   up0(k):    prolong, post-smooth level 0 -> z_(k+1); partials (r, z),
//              sum(z), sum(r)
// Kernels work on coarse cells of the next level: a thread takes one coarse
// cell and its 2^d children, so a restriction needs no cross-thread sum.
// Values a stencil needs at neighbour rows are recomputed there from
// vectors the same kernel does not write (r and p are ping-ponged by
// iteration parity), as in the other Krylov kernels.
#include "sol_dev.hpp"
#include "kcommon.hpp"
#include "kernels.hpp"

namespace sol {

constexpr double MG_W = 0.8;       // damped-Jacobi weight
constexpr double MG_OG = 1.8;      // coarse-correction scaling, launch levels
constexpr double MG_OL = 1.4;      // coarse-correction scaling, LDS levels
constexpr int MG_LPT = MG_LDS_MAX / TILE;   // LDS-level cells per thread

// floor(i / d) for 0 <= i < 2^31, 1 <= d, from the double reciprocal inv = 1/d
__device__ __forceinline__ int fdiv(int i, int d, double inv)
{
    int q = (int)((double)i * inv);
    if ((long long)q * d > i) --q;
    else if ((long long)(q + 1) * d <= i) ++q;
    return q;
}

// (axis, direction) of DIA slot s; the centre slot is DIM
template <int DIM>
__device__ __forceinline__ int slot_axis(int s) { return s < DIM ? DIM - 1 - s : s - DIM - 1; }

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

// coarse cell holding the level-l neighbour of child (cx) in slot s: the
// neighbour aggregate when the step leaves the aggregate inside the domain,
// else the cell's own (an out-of-domain neighbour has a zero coefficient)
template <int DIM>
__device__ __forceinline__ int agg_nb(const MLevel &L, const Agg<DIM> &a, const int *cx, int s)
{
    if (s == DIM) return a.I;
    const int ax = slot_axis<DIM>(s);
    const int cs = ax == 0 ? 1 : (ax == 1 ? L.cnx : L.cnx * L.cny);
    const int cn = ax == 0 ? L.cnx : (ax == 1 ? L.cny : L.cnz);
    if (s < DIM) return (cx[ax] == 0 && a.c[ax] > 0) ? a.I - cs : a.I;
    return (cx[ax] == 1 && a.c[ax] + 1 < cn) ? a.I + cs : a.I;
}

// visit the children of aggregate a: f(i, cx) with cx the child position
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
                f(a.i0 + cx + L.nx * cy + sxy * cz, c3);
            }
        }
    }
}

template <int ND>
__device__ __forceinline__ int nb_index(int i, int s, int n, int sx, int sxy)
{
    int j = i + slot_off<ND>(s, sx, sxy);
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// a solve whose multigrid stages run at iteration index k: RUNNING, or its
// (re)start whose first iteration is k + 1 (the start cycle runs at k0 - 1)
__device__ __forceinline__ bool mg_live(const KJob &J, int k)
{
    const int s = J.st->status;
    return s == K_RUNNING || ((s == K_RESTART) && J.st->k0 == k + 1);
}

__device__ __forceinline__ int kidx(const int *kbase, int koff) { return (kbase ? *kbase : 0) + koff; }

// ------------------------------------------------------------- hierarchy

// level l+1 operator from level l (Galerkin with aggregation), inverse
// diagonal (0 where the diagonal is 0: the single-cell coarsest level), and
// FP32 copies when requested; deterministic (fixed summation order)
template <int DIM>
__global__ __launch_bounds__(TILE) void k_mg_coarsen(const MLevel *__restrict__ lev, int l, double *Ac, double *mic,
                                                     float *Ac32, float *mic32)
{
    constexpr int ND = 2 * DIM + 1;
    const MLevel &L = lev[l];
    const int I = blockIdx.x * TILE + threadIdx.x;
    if (I >= L.cn) return;
    const Agg<DIM> a = agg_of<DIM>(L, I, 1.0 / L.cnx, 1.0 / ((double)L.cnx * L.cny));
    auto A = G<double>(L.A);
    double acc[ND];
#pragma unroll
    for (int s = 0; s < ND; ++s) acc[s] = 0.0;
    for_children<DIM>(L, a, [&](int i, const int *cx) {
#pragma unroll
        for (int s = 0; s < ND; ++s) {
            const double v = A[(size_t)s * L.n + i];
            const int J = agg_nb<DIM>(L, a, cx, s);
            if (J == I) acc[DIM] += v;
            else acc[s] += v;
        }
    });
    const int cn = L.cn;
    // a single coarse cell takes every coupling inside itself: its operator
    // is exactly 0 (zero row sums), while the summed terms above cancel
    // only to rounding, and 1 / rounding would inject a huge constant
    if (cn == 1) {
#pragma unroll
        for (int s = 0; s < ND; ++s) acc[s] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < ND; ++s) Ac[(size_t)s * cn + I] = acc[s];
    const double mi = acc[DIM] > 0.0 ? 1.0 / acc[DIM] : 0.0;
    mic[I] = mi;
    if (Ac32) {
#pragma unroll
        for (int s = 0; s < ND; ++s) Ac32[(size_t)s * cn + I] = (float)acc[s];
        mic32[I] = (float)mi;
    }
}

void launch_mg_coarsen(int dim, const MLevel *lev, int l, int cn, double *Ac, double *mic, float *Ac32, float *mic32,
                       hipStream_t s)
{
    if (cn <= 0) return;
    const dim3 g(ceil_div(cn, TILE)), b(TILE);
    if (dim == 2) hipLaunchKernelGGL(k_mg_coarsen<2>, g, b, 0, s, lev, l, Ac, mic, Ac32, mic32);
    else hipLaunchKernelGGL(k_mg_coarsen<3>, g, b, 0, s, lev, l, Ac, mic, Ac32, mic32);
}

// ------------------------------------------------------------- start

// start at iteration index k (mode 0: every solve, x = x0 or 0; mode 1:
// solves in K_RESTART, keep x): r_k = b - A x, p_(k-1) = 0; partial (b, b)
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_init(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k,
                                                  int mode)
{
    constexpr int ND = 2 * DIM + 1;
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RESTART) return;
    if (outer_idle(J)) return;
    const int pk = k & 1;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = J.n, sx = J.sx, sxy = J.sxy;
    auto A = G<T>(J.A);
    auto b = G<T>(J.b);
    auto x = G<T>(J.x), x0 = G<T>(J.x0);
    auto r = G<T>(pk ? J.rh : J.r), pz = G<T>(pk ? J.p0 : J.p1);
    const bool from_x0 = mode == 0 && J.x0;
    const bool keep_x = mode == 1;
    double bb = 0.0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *) {
            const T bi = b[i];
            T ri = bi;
            if (from_x0 || keep_x) {
                auto src = from_x0 ? x0 : x;
                T ax = T(0);
#pragma unroll
                for (int s = 0; s < ND; ++s) ax += A[(size_t)s * n + i] * src[nb_index<ND>(i, s, n, sx, sxy)];
                ri = bi - ax;
            }
            if (from_x0) x[i] = x0[i];
            else if (!keep_x) x[i] = T(0);
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

// ------------------------------------------------------------- iteration

template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_pq(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                const int *kbase, int koff)
{
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (!active(J, k) || outer_idle(J)) return;
    KState *st = J.st;
    const int pk = k & 1, pm = (k + 1) & 1;
    const bool first = k == st->k0;
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
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = J.n, sx = J.sx, sxy = J.sxy;
    auto A = G<T>(J.A);
    auto z = G<T>(J.v0);
    auto q = G<T>(J.v1);
    auto po = G<T>(pm ? J.p1 : J.p0), pn = G<T>(pk ? J.p1 : J.p0);
    double v = 0.0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *) {
            T qi = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                const int j = nb_index<ND>(i, s, n, sx, sxy);
                qi += A[(size_t)s * n + i] * ((z[j] - tz) + tb * po[j]);
            }
            const T pi = (z[i] - tz) + tb * po[i];
            pn[i] = pi;
            q[i] = qi;
            v += (double)pi * qi;
        });
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
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J)) return;
    KState *st = J.st;
    if (INIT ? !mg_live(J, k) : st->status != K_RUNNING) return;
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
    const T ta = (T)alpha, w = (T)MG_W;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = J.n, sx = J.sx, sxy = J.sxy;
    auto A = G<T>(J.A);
    auto mi = G<T>(J.minv);
    auto x = G<T>(J.x);
    auto p = G<T>(pk ? J.p1 : J.p0);
    auto q = G<T>(J.v1);
    auto rc = G<T>(pk ? J.rh : J.r), rn = G<T>(pn1 ? J.rh : J.r);
    auto bc = G<T>(J.lev[1].b);
    double rr = 0.0;
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        T bsum = T(0);
        for_children<DIM>(L, a, [&](int i, const int *) {
            T ax = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                const int j = nb_index<ND>(i, s, n, sx, sxy);
                const T rj = INIT ? rn[j] : rc[j] - ta * q[j];
                ax += A[(size_t)s * n + i] * (w * mi[j] * rj);
            }
            T ri;
            if (INIT) {
                ri = rn[i];
            } else {
                ri = rc[i] - ta * q[i];
                rn[i] = ri;
                x[i] = x[i] + ta * p[i];
            }
            rr += (double)ri * ri;
            bsum += ri - ax;
        });
        bc[I] = bsum;
    }
    double vv[1] = {rr};
    const int off[1] = {poff(J, pn1, PS_RR)};
    put_partials<1>(vv, J.part, off, tl.t);
}

// level l >= 1 (launch level): pre-smooth from zero and restrict
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_down(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                  const int *kbase, int koff)
{
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    const MLevel &L = J.lev[tl.lv];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = L.n, sx = L.nx, sxy = L.nx * L.ny;
    const T w = (T)MG_W;
    auto A = G<T>(L.A);
    auto mi = G<T>(L.minv);
    auto b = G<T>(L.b);
    auto bc = G<T>(J.lev[tl.lv + 1].b);
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        T bsum = T(0);
        for_children<DIM>(L, a, [&](int i, const int *) {
            T ax = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                const int j = nb_index<ND>(i, s, n, sx, sxy);
                ax += A[(size_t)s * n + i] * (w * mi[j] * b[j]);
            }
            bsum += b[i] - ax;
        });
        bc[I] = bsum;
    }
}

// level l >= 1 (launch level): prolong the coarse correction (scaled by
// MG_OG) onto the pre-smoothed value and post-smooth
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_up(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                const int *kbase, int koff)
{
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    const MLevel &L = J.lev[tl.lv];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = L.n, sx = L.nx, sxy = L.nx * L.ny;
    const T w = (T)MG_W, og = (T)MG_OG;
    auto A = G<T>(L.A);
    auto mi = G<T>(L.minv);
    auto b = G<T>(L.b);
    auto e = G<T>(L.e);
    auto ec = G<T>(J.lev[tl.lv + 1].e);
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *cx) {
            T ax = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                const int j = nb_index<ND>(i, s, n, sx, sxy);
                ax += A[(size_t)s * n + i] * (w * mi[j] * b[j] + og * ec[agg_nb<DIM>(L, a, cx, s)]);
            }
            const T xi = w * mi[i] * b[i] + og * ec[I];
            e[i] = xi + w * mi[i] * (b[i] - ax);
        });
    }
}

// level 0: prolong, post-smooth -> z_(k+1); partials (r_(k+1), z_(k+1)),
// sum(z_(k+1)), sum(r_(k+1))
template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_up0(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                 const int *kbase, int koff)
{
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (outer_idle(J) || !mg_live(J, k)) return;
    const int pn1 = (k + 1) & 1;
    const MLevel &L = J.lev[0];
    const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
    const int n = J.n, sx = J.sx, sxy = J.sxy;
    const T w = (T)MG_W, og = (T)MG_OG;
    auto A = G<T>(J.A);
    auto mi = G<T>(J.minv);
    auto r = G<T>(pn1 ? J.rh : J.r);
    auto z = G<T>(J.v0);
    auto ec = G<T>(J.lev[1].e);
    double vv[3] = {0.0, 0.0, 0.0};     // (r, z), sum z, sum r
    const int I0 = tl.t * L.cpt, I1 = min(L.cn, I0 + L.cpt);
    for (int I = I0 + threadIdx.x; I < I1; I += TILE) {
        const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
        for_children<DIM>(L, a, [&](int i, const int *cx) {
            T ax = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) {
                const int j = nb_index<ND>(i, s, n, sx, sxy);
                ax += A[(size_t)s * n + i] * (w * mi[j] * r[j] + og * ec[agg_nb<DIM>(L, a, cx, s)]);
            }
            const T ri = r[i];
            const T xi = w * mi[i] * ri + og * ec[I];
            const T zi = xi + w * mi[i] * (ri - ax);
            z[i] = zi;
            vv[0] += (double)ri * zi;
            vv[1] += (double)zi;
            vv[2] += (double)ri;
        });
    }
    const int off[3] = {poff(J, pn1, PS_RHO), poff(J, pn1, PS_Q), poff(J, pn1, PS_TT)};
    put_partials<3>(vv, J.part, off, tl.t);
}

// ------------------------------------------------------------- LDS levels
// Levels nglob .. coarsest of one solve in one workgroup: b and x of every
// level in local memory (level l at an offset, b then x), operators read
// from global memory.  V(2,2) with damped Jacobi, correction scaled by MG_OL.

template <int DIM, class T>
__device__ __forceinline__ int lds_parent(const MLevel &L, int i, double inx, double inxy)
{
    int fz = 0, rem = i;
    if (DIM == 3) {
        fz = fdiv(i, L.nx * L.ny, inxy);
        rem = i - fz * L.nx * L.ny;
    }
    const int fy = fdiv(rem, L.nx, inx);
    const int fx = rem - fy * L.nx;
    return (fx >> 1) + L.cnx * ((fy >> 1) + L.cny * (fz >> 1));
}

// x = x + w M (b - A x) on one level in local memory (two barriers)
template <int ND, class T>
__device__ __forceinline__ void lds_sweep(const MLevel &L, const T *b, T *x)
{
    const int n = L.n, sx = L.nx, sxy = L.nx * L.ny;
    auto A = G<T>(L.A);
    auto mi = G<T>(L.minv);
    const T w = (T)MG_W;
    T nv[MG_LPT];
#pragma unroll
    for (int c = 0; c < MG_LPT; ++c) {
        const int i = threadIdx.x + c * TILE;
        if (i < n) {
            T ax = T(0);
#pragma unroll
            for (int s = 0; s < ND; ++s) ax += A[(size_t)s * n + i] * x[nb_index<ND>(i, s, n, sx, sxy)];
            nv[c] = x[i] + w * mi[i] * (b[i] - ax);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MG_LPT; ++c) {
        const int i = threadIdx.x + c * TILE;
        if (i < n) x[i] = nv[c];
    }
    __syncthreads();
}

template <int DIM, class T>
__global__ __launch_bounds__(TILE) void k_mg_lds(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles,
                                                 const int *kbase, int koff)
{
    constexpr int ND = 2 * DIM + 1;
    const int k = kidx(kbase, koff);
    const JTile tl = tiles[blockIdx.x];
    const KJob &J = jobs[tl.j];
    if (outer_idle(J) || !mg_live(J, k)) return;
    extern __shared__ __align__(16) unsigned char mg_smem[];
    T *sh = reinterpret_cast<T *>(mg_smem);
    const MLevel *Lv = J.lev;
    const int L0 = J.nglob, M = J.nlev - 1;
    const T w = (T)MG_W, ol = (T)MG_OL;
    {
        auto bg = G<T>(Lv[L0].b);
        for (int i = threadIdx.x; i < Lv[L0].n; i += TILE) sh[i] = bg[i];
    }
    __syncthreads();
    // down: levels L0 .. M-1
    int o = 0;
    for (int l = L0; l < M; ++l) {
        const MLevel &L = Lv[l];
        const int n = L.n, sx = L.nx, sxy = L.nx * L.ny;
        T *b = sh + o, *x = sh + o + n, *bc = sh + o + 2 * n;
        auto A = G<T>(L.A);
        auto mi = G<T>(L.minv);
        for (int i = threadIdx.x; i < n; i += TILE) x[i] = w * mi[i] * b[i];
        __syncthreads();
        lds_sweep<ND, T>(L, b, x);
        const double icx = 1.0 / L.cnx, icxy = 1.0 / ((double)L.cnx * L.cny);
        for (int I = threadIdx.x; I < L.cn; I += TILE) {
            const Agg<DIM> a = agg_of<DIM>(L, I, icx, icxy);
            T bsum = T(0);
            for_children<DIM>(L, a, [&](int i, const int *) {
                T ax = T(0);
#pragma unroll
                for (int s = 0; s < ND; ++s) ax += A[(size_t)s * n + i] * x[nb_index<ND>(i, s, n, sx, sxy)];
                bsum += b[i] - ax;
            });
            bc[I] = bsum;
        }
        __syncthreads();
        o += 2 * n;
    }
    // coarsest level: one damped-Jacobi application (the single cell has a
    // zero operator and a zero inverse diagonal: x = 0)
    {
        const MLevel &L = Lv[M];
        auto mi = G<T>(L.minv);
        T *b = sh + o, *x = sh + o + L.n;
        for (int i = threadIdx.x; i < L.n; i += TILE) x[i] = w * mi[i] * b[i];
        __syncthreads();
    }
    // up: levels M-1 .. L0
    for (int l = M - 1; l >= L0; --l) {
        const MLevel &L = Lv[l];
        const int n = L.n;
        o -= 2 * n;
        T *b = sh + o, *x = sh + o + n;
        const T *xc = sh + o + 2 * n + L.cn;
        const double inx = 1.0 / L.nx, inxy = 1.0 / ((double)L.nx * L.ny);
        for (int i = threadIdx.x; i < n; i += TILE) x[i] += ol * xc[lds_parent<DIM, T>(L, i, inx, inxy)];
        __syncthreads();
        lds_sweep<ND, T>(L, b, x);
        lds_sweep<ND, T>(L, b, x);
    }
    {
        auto eg = G<T>(Lv[L0].e);
        const T *x = sh + Lv[L0].n;
        for (int i = threadIdx.x; i < Lv[L0].n; i += TILE) eg[i] = x[i];
    }
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
    case KI_MG_LDS: return (const void *)&k_mg_lds<DIM, T>;
    case KI_MG_UP: return (const void *)&k_mg_up<DIM, T>;
    case KI_MG_UP0: return (const void *)&k_mg_up0<DIM, T>;
    }
    return nullptr;
}

const void *mg_fn(int which, int nd, int fp32)
{
    if (nd == 5) return fp32 ? mg_fn_t<2, float>(which) : mg_fn_t<2, double>(which);
    return fp32 ? mg_fn_t<3, float>(which) : mg_fn_t<3, double>(which);
}

void launch_mg_init(int nd, int fp32, const KJob *j, const JTile *t, int nt, int k, int mode, hipStream_t s)
{
    if (nt <= 0) return;
    const dim3 g(nt), b(TILE);
    if (nd == 5) {
        if (fp32) hipLaunchKernelGGL((k_mg_init<2, float>), g, b, 0, s, j, t, k, mode);
        else hipLaunchKernelGGL((k_mg_init<2, double>), g, b, 0, s, j, t, k, mode);
    } else {
        if (fp32) hipLaunchKernelGGL((k_mg_init<3, float>), g, b, 0, s, j, t, k, mode);
        else hipLaunchKernelGGL((k_mg_init<3, double>), g, b, 0, s, j, t, k, mode);
    }
}

}  // namespace sol
