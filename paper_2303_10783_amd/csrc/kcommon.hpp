// Device helpers shared by the step kernels and the multigrid kernels:
// XCD-aware tile order, workgroup sums, the fence-free partial-sum
// protocol, DIA stencils and the Krylov status bookkeeping.
#pragma once
#include "sol_dev.hpp"

namespace sol {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + min(x, r) + k;
}

// v from the lane selected by DPP control CTRL (rows in ROWMASK; lanes
// without a source and rows outside the mask get 0)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_get(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum over the 64 lanes, returned in every lane.  Within each row of 16
// lanes, shifts by 1, 2, 4, 8 with zero fill leave the row total in lane 15;
// row broadcasts then add row 0 into row 1, row 2 into row 3, and lane 31
// into row 3: lane 63 holds the total.  A fixed tree, so every wave that sums
// the same values gets the same bits; all on the VALU (DPP), no LDS traffic.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_get<0x111, 0xf>(v);   // row_shr:1
    v += dpp_get<0x112, 0xf>(v);   // row_shr:2
    v += dpp_get<0x114, 0xf>(v);   // row_shr:4
    v += dpp_get<0x118, 0xf>(v);   // row_shr:8
    v += dpp_get<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_get<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum of K values over the 256 threads; result valid in thread 0
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (sh[k] + sh[K + k]) + (sh[2 * K + k] + sh[3 * K + k]);
    }
    __syncthreads();
}

// Reductions.  A kernel writes one partial sum per workgroup (plain stores);
// the next kernel on the stream (kernel boundaries make them visible) sums
// the partials of the tiles it needs in tile order, every workgroup in the
// same order, so all workgroups obtain bit-identical totals and no
// device-scope fence or atomic is needed.

// block totals of K values -> part[off[k] + t] (written by thread 0)
template <int K>
__device__ __forceinline__ void put_partials(double (&v)[K], double *part, const int (&off)[K], int t)
{
    __shared__ double sh[4 * K];
    block_sum<K>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) part[off[k] + t] = v[k];
    }
}

// out[k] = sum_{q < ntile} part[off[k] + q], identical in every thread and
// every workgroup: thread t adds q = t, t + 256, ... in that order, each
// wave adds its lanes in the fixed DPP tree, and after one barrier every
// thread adds the four wave totals in wave order.  (Broadcasting a total
// from thread 0 took two more barriers, each of which also waits for every
// load the waves have in flight.)  U > 1: the values of U consecutive q of
// a thread are loaded together, then added in the same order (one round trip
// per U of them), for the long per-case totals of one-workgroup kernels; the
// Krylov kernels total a few hundred tiles and keep U = 1 (its registers).
template <int K, int U = 1>
__device__ __forceinline__ void sum_partials(const double *part, const int (&off)[K], int ntile, double (&out)[K])
{
    __shared__ double sh[4 * K];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    int q = threadIdx.x;
    if constexpr (U > 1)
    for (; q + (U - 1) * TILE < ntile; q += U * TILE) {
        double v[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = part[off[k] + q + u * TILE];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    for (; q < ntile; q += TILE) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += part[off[k] + q];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[w * K + k] = acc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = (sh[k] + sh[K + k]) + (sh[2 * K + k] + sh[3 * K + k]);
}

// two consecutive elements of a vector (T = double or float) in one load;
// i must be even and the vector 2 sizeof(T)-aligned
template <class T>
struct Pair { T x, y; };
template <class T>
__device__ __forceinline__ Pair<T> load_pair(const void *base, int i)
{
    typedef T V __attribute__((ext_vector_type(2)));
    const V v = *(const __attribute__((address_space(1))) V *)((const __attribute__((address_space(1))) char *)base +
                                                                (unsigned)i * (unsigned)sizeof(T));
    return Pair<T>{v.x, v.y};
}

// neighbour offset of DIA slot s (slot order -sxy, -sx, -1, 0, +1, +sx, +sxy)
template <int ND>
__device__ __forceinline__ int slot_off(int s, int sx, int sxy)
{
    if (ND == 7) {
        switch (s) { case 0: return -sxy; case 1: return -sx; case 2: return -1; case 3: return 0;
                     case 4: return 1; case 5: return sx; default: return sxy; }
    }
    switch (s) { case 0: return -sx; case 1: return -1; case 2: return 0; case 3: return 1; default: return sx; }
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

template <class T>
using gptr = __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ gptr<T> G(const void *p) { return (gptr<T>)(p); }

// Read-only view of a global vector indexed by a 32-bit element index: the
// address is a uniform base plus a 32-bit byte offset, which the compiler
// emits as the scalar-base form of the global loads (one VGPR per address
// instead of two); kernels that gather many neighbour values hold fewer
// registers and more waves.  For vectors only: a vector of the largest
// grid sol_create accepts (2.9e8 rows) stays below 4 GiB, a 7-diagonal
// matrix would not.
template <class T>
struct RO {
    const __attribute__((address_space(1))) char *b;
    __device__ __forceinline__ T operator[](int i) const
    {
        return *(const __attribute__((address_space(1))) T *)(b + (unsigned)i * (unsigned)sizeof(T));
    }
};

template <class T>
__device__ __forceinline__ RO<T> R(const void *p) { return RO<T>{(const __attribute__((address_space(1))) char *)p}; }

// y_i = sum_s A[s][i] * f(i + off_s) in type T.  Slots whose neighbour lies
// outside the domain hold an exact 0 coefficient; their index is clamped
// into [0, n) so that no access leaves the arrays.
template <int ND, class T, class F>
__device__ __forceinline__ T kstencil(gptr<T> A, int n, int i, int sx, int sxy, F f)
{
    T acc = T(0);
#pragma unroll
    for (int s = 0; s < ND; ++s) {
        int j = i + slot_off<ND>(s, sx, sxy);
        j = j < 0 ? 0 : (j >= n ? n - 1 : j);
        acc += A[(size_t)s * n + i] * f(j);
    }
    return acc;
}

__device__ __forceinline__ const KJob &job_of(const KJob *jobs, const JTile *tiles, JTile &tl)
{
    tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    return jobs[tl.j];
}

__device__ __forceinline__ int poff(const KJob &J, int par, int slot) { return (par * NSLOT + slot) * J.ntile; }

// The status of a solve, read once for the whole workgroup.  Workgroup 0 of
// a launch may change it (convergence, breakdown) while the waves of a
// workgroup that starts later read it one by one.  Had they disagreed, the
// waves that returned at once would have left their slots of the block-wide
// sums stale, and the waves that went on would have derived their scalars,
// and then their row updates, from those slots.  Every kernel whose entry
// check reads a status that its own workgroup 0 may change takes it from
// here, once, before any other use of LDS.
__device__ __forceinline__ int wg_status(const KState *st)
{
    __shared__ int s;
    if (threadIdx.x == 0) s = st->status;
    __syncthreads();
    return s;
}

// an inner solve whose refinement no longer needs it
__device__ __forceinline__ bool outer_idle(const KJob &J)
{
    return J.role == ROLE_INNER && J.partner->status != K_RUNNING;
}

// status of a solve as seen by iteration k: RUNNING, or a (re)start whose
// first iteration is k
__device__ __forceinline__ bool active(const KJob &J, int k)
{
    const int s = wg_status(J.st);
    return s == K_RUNNING || (s == K_RESTART && k == J.st->k0);
}

// record a status change: workgroup 0 of the solve only
__device__ __forceinline__ void set_status(const JTile &tl, KState *st, int status, int it, double rr)
{
    if (tl.t == 0 && threadIdx.x == 0) {
        st->status = status;
        st->it = it;
        st->rr = rr;
    }
}

// record the start of a solve at iteration index k (workgroup 0)
__device__ __forceinline__ void mark_start(const JTile &tl, KState *st, int k, int mode)
{
    if (tl.t == 0 && threadIdx.x == 0) {
        st->k0 = k;
        st->half = 0;
        if (mode == 0) { st->it_base = 0; st->restarts = 0; st->status = K_RUNNING; }
        else { st->it_base = st->it; st->restarts += 1; }
    }
}

// convergence test at the start of iteration k; rr = ||r_k||^2 and bbp =
// total of the (b,b) partials left by the start kernels (used at k = k0)
__device__ __forceinline__ bool keep_going(const KJob &J, const JTile &tl, int k, double rr, double bbp)
{
    KState *st = J.st;
    const int it = st->it_base + (k - st->k0);
    double bb;
    if (k == st->k0) {
        bb = bbp;
        if (tl.t == 0 && threadIdx.x == 0) st->bb = bb;
    } else {
        bb = st->bb;
    }
    if (!finite(rr) || !finite(bb)) { set_status(tl, st, K_NONFINITE, it, rr); return false; }
    if (bb == 0.0) { set_status(tl, st, K_ZERO, it, rr); return false; }
    if (rr <= st->tol2 * bb) { set_status(tl, st, K_CONVERGED, it, rr); return false; }
    if (it >= st->max_iter) { set_status(tl, st, K_FAILED, it, rr); return false; }
    if (k == st->k0 && tl.t == 0 && threadIdx.x == 0) st->status = K_RUNNING;
    return true;
}


}  // namespace sol
