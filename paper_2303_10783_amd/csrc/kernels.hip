// HIP kernels (gfx950) of one time step of the decoupled solidification
// scheme: term-wise assembly, Jacobi-PCG / Jacobi-BiCGSTAB iterations with
// fused reductions, divergence / projection, phase update and commit.
//
// Launch model: every per-row kernel walks a table of tiles (256 rows each)
// covering one or many cases; workgroup b takes tile xcd_tile(b) so that the
// tiles one XCD executes are contiguous in memory (its L2 then holds the
// y/z neighbour rows of its own tiles).  Reductions: per-workgroup partial
// sums, totalled in a fixed order by the next kernel (deterministic; no
// device-scope fences, which on gfx950 would write back the whole L2).
#include "sol_dev.hpp"
#include "kernels.hpp"

namespace sol {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
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
// every workgroup
template <int K>
__device__ __forceinline__ void sum_partials(const double *part, const int (&off)[K], int ntile, double (&out)[K])
{
    __shared__ double sh[4 * K];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int q = threadIdx.x; q < ntile; q += TILE) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += part[off[k] + q];
    }
    block_sum<K>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k] = acc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = sh[k];
    __syncthreads();
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

// y_i = sum_s A[s][i] * f(i + off_s).  Slots whose neighbour lies outside the
// domain hold an exact 0 coefficient; their index is clamped into [0, n) so
// that no access leaves the arrays.
template <int ND, class TA, class F>
__device__ __forceinline__ double stencil(const TA *__restrict__ A, int n, int i, int sx, int sxy, F f)
{
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < ND; ++s) {
        int j = i + slot_off<ND>(s, sx, sxy);
        j = j < 0 ? 0 : (j >= n ? n - 1 : j);
        acc += (double)A[(size_t)s * n + i] * f(j);
    }
    return acc;
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// ----------------------------------------------------------- grid helpers

__device__ __forceinline__ int cell_index(const Phys &P, int i, int j, int k)
{
    return i + P.nx * (j + P.ny * k);
}

// velocity component a on the a-face with face number F (0..n_a) at the
// transverse cell coordinates q (q[a] ignored); wall faces carry 0
__device__ __forceinline__ double face_vel(const Phys &P, double *const *vel, int a, const int *q, int F)
{
    const int na = a == 0 ? P.nx : (a == 1 ? P.ny : P.nz);
    if (F <= 0 || F >= na) return 0.0;
    if (a == 0) return vel[0][(F - 1) + (P.nx - 1) * (q[1] + P.ny * q[2])];
    if (a == 1) return vel[1][q[0] + P.nx * ((F - 1) + (P.ny - 1) * q[2])];
    return vel[2][q[0] + P.nx * (q[1] + P.ny * (F - 1))];
}

__device__ __forceinline__ void decode(int row, int sx, int sy, int *q)
{
    q[0] = row % sx;
    const int rem = row / sx;
    q[1] = rem % sy;
    q[2] = rem / sy;
}

// conductance of a cooled wall seen from the adjacent cell centre: film h in
// series with the half cell h_a/(2k); a prescribed temperature is h -> inf
__device__ __forceinline__ double wall_cond(const Phys &P, int face, double ha)
{
    const int th = P.thermal[face];
    if (th == 1) return 1.0 / (1.0 / P.hc[face] + ha / (2.0 * P.kcond));
    if (th == 2) return 2.0 * P.kcond / ha;
    return 0.0;
}

__device__ __forceinline__ double wall_temp(const Phys &P, int face, double t)
{
    return P.thermal[face] == 2 ? P.Tw0[face] - P.Tramp[face] * t : P.Text[face];
}

// ---------------------------------------------------- offline assembly
// Constant-coefficient terms, assembled once (the term-wise split of
// Section 4): transient 1/dt, central diffusion (eq. 3.26) with no-slip
// half-cell ghosts for tangential velocity, free-slip (no shear), Dirichlet
// zero for wall-normal velocity neighbours; energy wall conductances; the
// Neumann pressure Laplacian -L = -D G (eq. 3.4) with its Jacobi inverse.
template <int DIM>
__global__ __launch_bounds__(TILE) void k_asm_const(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    constexpr int ND = 2 * DIM + 1;
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int s = tl.s;
    const int n = P.nsys[s];
    const int row = tl.t * TILE + threadIdx.x;
    if (row >= n) return;
    int q[3];
    decode(row, P.sdim[s][0], P.sdim[s][1], q);
    double a[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) a[k] = 0.0;
    if (s <= SW) {
        a[DIM] = P.idt;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const double dif = P.nu * P.ih2[ax];
            const bool em = q[ax] >= 1, ep = q[ax] <= P.sdim[s][ax] - 2;
            if (ax == s) {
                // neighbours along the normal: faces (or impermeable walls) at distance h
                a[DIM] += 2.0 * dif;
                a[DIM - 1 - ax] = em ? -dif : 0.0;
                a[DIM + 1 + ax] = ep ? -dif : 0.0;
            } else {
                if (em) { a[DIM] += dif; a[DIM - 1 - ax] = -dif; }
                else if (P.slip[2 * ax] == 0) a[DIM] += 2.0 * dif;
                if (ep) { a[DIM] += dif; a[DIM + 1 + ax] = -dif; }
                else if (P.slip[2 * ax + 1] == 0) a[DIM] += 2.0 * dif;
            }
        }
        double *Ac = c.Ac[s];
#pragma unroll
        for (int k = 0; k < ND; ++k) Ac[(size_t)k * n + row] = a[k];
    } else if (s == ST) {
        a[DIM] = P.idt;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const double dif = P.alpha * P.ih2[ax];
            for (int sd = 0; sd < 2; ++sd) {
                const bool ex = sd == 0 ? q[ax] >= 1 : q[ax] <= P.sdim[s][ax] - 2;
                const int slot = sd == 0 ? DIM - 1 - ax : DIM + 1 + ax;
                if (ex) { a[DIM] += dif; a[slot] = -dif; }
                else {
                    const double U = wall_cond(P, 2 * ax + sd, P.h[ax]);
                    a[DIM] += U / (P.rcp * P.h[ax]);
                }
            }
        }
        double *Ac = c.Ac[ST];
#pragma unroll
        for (int k = 0; k < ND; ++k) Ac[(size_t)k * n + row] = a[k];
    } else if (s == SP) {
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const bool em = q[ax] >= 1, ep = q[ax] <= P.sdim[s][ax] - 2;
            if (em) { a[DIM] += P.ih2[ax]; a[DIM - 1 - ax] = -P.ih2[ax]; }
            if (ep) { a[DIM] += P.ih2[ax]; a[DIM + 1 + ax] = -P.ih2[ax]; }
        }
        double *A = c.A[SP];
#pragma unroll
        for (int k = 0; k < ND; ++k) A[(size_t)k * n + row] = a[k];
        const double mi = a[DIM] > 0.0 ? 1.0 / a[DIM] : 1.0;
        c.minv[SP][row] = mi;
        if (c.A32[SP]) {
#pragma unroll
            for (int k = 0; k < ND; ++k) c.A32[SP][(size_t)k * n + row] = (float)a[k];
            c.minv32[SP][row] = (float)mi;
        }
    }
}

// ---------------------------------------------------- momentum assembly
// Predictor of eq. (3.3): A = const + upwind convection (eq. 4.4 rows, flux
// form, advecting velocity = mean of the two nearest level-n velocities of
// that component) + Carman-Kozeny drag (eq. 2.8) on the face;
// b = u^n/dt - (1/rho) dp^n/dx + Boussinesq force (eq. 2.9, vertical only).
template <int DIM>
__global__ __launch_bounds__(TILE) void k_asm_momentum(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    constexpr int ND = 2 * DIM + 1;
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int d = tl.s;
    const int n = P.nsys[d];
    const int row = tl.t * TILE + threadIdx.x;
    if (row >= n) return;
    int q[3];
    decode(row, P.sdim[d][0], P.sdim[d][1], q);
    int lo[3] = {q[0], q[1], q[2]}, hi[3] = {q[0], q[1], q[2]};
    hi[d] += 1;
    const int clo = cell_index(P, lo[0], lo[1], lo[2]);
    const int chi = cell_index(P, hi[0], hi[1], hi[2]);
    double *const vel[3] = {c.u, c.v, c.w};
    const double *Ac = c.Ac[d];
    double a[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) a[k] = Ac[(size_t)k * n + row];
    double dconv = 0.0;
    const int F = q[d] + 1;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        double vm, vp;
        if (ax == d) {
            const double uc = face_vel(P, vel, d, lo, F);
            vm = 0.5 * (face_vel(P, vel, d, lo, F - 1) + uc);
            vp = 0.5 * (uc + face_vel(P, vel, d, lo, F + 1));
        } else {
            vm = 0.5 * (face_vel(P, vel, ax, lo, q[ax]) + face_vel(P, vel, ax, hi, q[ax]));
            vp = 0.5 * (face_vel(P, vel, ax, lo, q[ax] + 1) + face_vel(P, vel, ax, hi, q[ax] + 1));
        }
        const double cw = -fmax(vm, 0.0) * P.ih[ax];
        const double cp = (fmax(vp, 0.0) - fmin(vm, 0.0)) * P.ih[ax];
        const double ce = fmin(vp, 0.0) * P.ih[ax];
        dconv += cp;
        const bool em = q[ax] >= 1, ep = q[ax] <= P.sdim[d][ax] - 2;
        a[DIM - 1 - ax] = em ? a[DIM - 1 - ax] + cw : 0.0;
        a[DIM + 1 + ax] = ep ? a[DIM + 1 + ax] + ce : 0.0;
    }
    const double gf = 0.5 * (c.gl[clo] + c.gl[chi]);
    const double sol = 1.0 - gf;
    const double drag = P.nu * 180.0 * sol * sol / (P.lambda2 * P.lambda2 * (gf * gf * gf + P.eps));
    a[DIM] += dconv + drag;
    double *A = c.A[d];
#pragma unroll
    for (int k = 0; k < ND; ++k) A[(size_t)k * n + row] = a[k];
    const double mi = 1.0 / a[DIM];
    c.minv[d][row] = mi;
    double rhs = vel[d][row] * P.idt - (c.p[chi] - c.p[clo]) / (P.rho * P.h[d]);
    if (d == DIM - 1) {
        const double Tf = 0.5 * (c.T[clo] + c.T[chi]);
        const double Cf = 0.5 * (c.Cl[clo] + c.Cl[chi]);
        rhs += P.grav * (P.betaT * (Tf - P.Tref) + P.betaC * (Cf - P.Cref));
    }
    c.b[d][row] = rhs;
    if (c.A32[d]) {
#pragma unroll
        for (int k = 0; k < ND; ++k) c.A32[d][(size_t)k * n + row] = (float)a[k];
        c.minv32[d][row] = (float)mi;
    }
}

// ---------------------------------------------- solute + energy assembly
// Solute (eqs. 3.8-3.10): I/dt + A_con(u^{n+1}) A_g, A_g = diag(1/(1 - (1-k_p)
// (1-g_l^n))) applied to the columns (C_l = A_g C substituted into the
// convection term); b = C^n/dt.  Energy (eq. 3.11): const (1/dt, alpha
// diffusion, wall conductances) + A_con(u^{n+1}); b = T^n/dt + wall terms at
// t_{n+1}.  vel_src 1: advecting field = projected u^{n+1} (the step);
// 0: the level-n field (stand-alone assembly).
template <int DIM>
__global__ __launch_bounds__(TILE) void k_asm_transport(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles, int vel_src)
{
    constexpr int ND = 2 * DIM + 1;
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int n = P.ncell;
    const int ci = tl.t * TILE + threadIdx.x;
    if (ci >= n) return;
    int q[3];
    decode(ci, P.nx, P.ny, q);
    double *const vel[3] = {vel_src ? c.un[0] : c.u, vel_src ? c.un[1] : c.v, vel_src ? c.un[2] : c.w};
    const double t_new = (double)(*c.step + 1) * P.dt;
    const double omk = 1.0 - P.kp;
    const double agP = 1.0 / (1.0 - omk * (1.0 - c.gl[ci]));
    const double *AcT = c.Ac[ST];
    double aC[ND], aT[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) { aC[k] = 0.0; aT[k] = AcT[(size_t)k * n + ci]; }
    double dconv = 0.0;
    double bT = c.T[ci] * P.idt;
    const int stride[3] = {1, P.nx, P.nx * P.ny};
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const double vm = face_vel(P, vel, ax, q, q[ax]);
        const double vp = face_vel(P, vel, ax, q, q[ax] + 1);
        const double cw = -fmax(vm, 0.0) * P.ih[ax];
        const double cp = (fmax(vp, 0.0) - fmin(vm, 0.0)) * P.ih[ax];
        const double ce = fmin(vp, 0.0) * P.ih[ax];
        dconv += cp;
        const int nax = P.sdim[SC][ax];
        const bool em = q[ax] >= 1, ep = q[ax] <= nax - 2;
        const int sm = DIM - 1 - ax, sp = DIM + 1 + ax;
        if (em) {
            const double agm = 1.0 / (1.0 - omk * (1.0 - c.gl[ci - stride[ax]]));
            aC[sm] = cw * agm;
            aT[sm] += cw;
        } else {
            aT[sm] = 0.0;
            const double U = wall_cond(P, 2 * ax, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax, t_new) / (P.rcp * P.h[ax]);
        }
        if (ep) {
            const double agp = 1.0 / (1.0 - omk * (1.0 - c.gl[ci + stride[ax]]));
            aC[sp] = ce * agp;
            aT[sp] += ce;
        } else {
            aT[sp] = 0.0;
            const double U = wall_cond(P, 2 * ax + 1, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax + 1, t_new) / (P.rcp * P.h[ax]);
        }
    }
    aC[DIM] = P.idt + dconv * agP;
    aT[DIM] += dconv;
    double *AC = c.A[SC], *AT = c.A[ST];
#pragma unroll
    for (int k = 0; k < ND; ++k) { AC[(size_t)k * n + ci] = aC[k]; AT[(size_t)k * n + ci] = aT[k]; }
    c.b[SC][ci] = c.C[ci] * P.idt;
    c.b[ST][ci] = bT;
    const double miC = 1.0 / aC[DIM], miT = 1.0 / aT[DIM];
    c.minv[SC][ci] = miC;
    c.minv[ST][ci] = miT;
    if (c.A32[SC]) {
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            c.A32[SC][(size_t)k * n + ci] = (float)aC[k];
            c.A32[ST][(size_t)k * n + ci] = (float)aT[k];
        }
        c.minv32[SC][ci] = (float)miC;
        c.minv32[ST][ci] = (float)miT;
    }
}

// ---------------------------------------------- pressure-correction rhs
// b = -(rho/dt) D u* (eq. 3.4); partial sums of b and (D u*)^2 per tile.
template <int DIM>
__global__ __launch_bounds__(TILE) void k_div_rhs(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles, int vel_src)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int ci = tl.t * TILE + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (ci < P.ncell) {
        int q[3];
        decode(ci, P.nx, P.ny, q);
        double *const vel[3] = {vel_src ? c.us[0] : c.u, vel_src ? c.us[1] : c.v, vel_src ? c.us[2] : c.w};
        double dv = 0.0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax)
            dv += (face_vel(P, vel, ax, q, q[ax] + 1) - face_vel(P, vel, ax, q, q[ax])) * P.ih[ax];
        const double b = -(P.rho * P.idt) * dv;
        c.b[SP][ci] = b;
        v[0] = b;
        v[1] = dv * dv;
    }
    const int nt = c.ntile_cell;
    const int off[2] = {0, nt};
    put_partials<2>(v, c.red_part, off, tl.t);
}

// remove the mean of the pressure rhs (consistency of the Neumann problem);
// workgroup 0 of each case records the mean and ||D u*||
__global__ __launch_bounds__(TILE) void k_sub_mean(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const int nt = c.ntile_cell;
    const int off[2] = {0, nt};
    double tot[2];
    sum_partials<2>(c.red_part, off, nt, tot);
    const double mean = tot[0] / (double)c.ph.ncell;
    const int ci = tl.t * TILE + threadIdx.x;
    if (ci < c.ph.ncell) c.b[SP][ci] -= mean;
    if (tl.t == 0 && threadIdx.x == 0) {
        c.red[R_SUMB] = tot[0];
        c.red[R_DIVSTAR] = sqrt(tot[1]);
        c.ks[SP].bmean = mean;
    }
}

// ------------------------------------------------------------ projection
// u^{n+1} = u* - (dt/rho) G phi on the interior faces (eq. 3.5), into un
__global__ __launch_bounds__(TILE) void k_project(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int d = tl.s;
    const int row = tl.t * TILE + threadIdx.x;
    if (row >= P.nsys[d]) return;
    int q[3];
    decode(row, P.sdim[d][0], P.sdim[d][1], q);
    const int clo = cell_index(P, q[0], q[1], q[2]);
    const int stride = d == 0 ? 1 : (d == 1 ? P.nx : P.nx * P.ny);
    const double g = (c.phi[clo + stride] - c.phi[clo]) * P.ih[d];
    c.un[d][row] = c.us[d][row] - (P.dt / P.rho) * g;
}

// ------------------------------------------------------ phase + commit
// Second split step (eq. 3.12) with liquidus (eq. 3.13) and lever rule
// (eq. 3.14): with H = T* + (L/c_p) g^n the liquid fraction is
//   solid    H < T_e                         g = 0
//   plateau  H < T_e + (L/c_p) g_eut         g = (H - T_e)/(L/c_p)  (isothermal)
//   mush     H < T_l + L/c_p                 larger root of a g^2 + b g + c
//                                            (eqs. 3.15-3.16), clipped to [0,1]
//   liquid   otherwise                       g = 1
// T^{n+1} = T* - (L/c_p)(g - g^n); C_l = C/(1 + (1-g)(k_p-1)), C_s = k_p C_l
// (eqs. 3.17-3.18).  Then the new state replaces level n: T, g_l, C, C_l,
// C_s, p += phi - mean(phi), and u, v, w take the projected velocities.
__device__ __forceinline__ void phase_point(const Phys &P, double Ts, double gn, double Cn,
                                            double &T, double &g)
{
    const double lam = P.lam, kp = P.kp, omk = 1.0 - P.kp;
    const double H = Ts + lam * gn;
    const double Tl = P.Tm + P.msp * Cn;
    const double Te = P.Tm + P.msp * P.Ce;
    double geut = 1.0 - (Te - Tl) / (omk * (Te - P.Tm));
    geut = fmin(fmax(geut, 0.0), 1.0);
    if (H < Te) {
        g = 0.0;
    } else if (H < Te + lam * geut) {
        g = (H - Te) / lam;
    } else if (H < Tl + lam) {
        const double a = omk;
        const double b = kp - gn * omk + omk * (P.Tm - Ts) / lam;
        const double cc = -(gn + Ts / lam) * kp + (Tl - omk * P.Tm) / lam;
        const double disc = fmax(b * b - 4.0 * a * cc, 0.0);
        const double sq = sqrt(disc);
        const double qq = -0.5 * (b + (b >= 0.0 ? sq : -sq));
        const double r1 = qq / a;
        const double r2 = qq != 0.0 ? cc / qq : r1;
        g = fmin(fmax(fmax(r1, r2), 0.0), 1.0);
    } else {
        g = 1.0;
    }
    T = Ts - lam * (g - gn);
}

template <int DIM>
__global__ __launch_bounds__(TILE) void k_phase_commit(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const Phys &P = c.ph;
    const int ci = tl.t * TILE + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (ci < P.ncell) {
        int q[3];
        decode(ci, P.nx, P.ny, q);
        const double Ts = c.Tstar[ci], gn = c.gl[ci], Cn = c.Cnew[ci];
        double T, g;
        phase_point(P, Ts, gn, Cn, T, g);
        const double Cl = Cn / (1.0 + (1.0 - g) * (P.kp - 1.0));
        c.T[ci] = T;
        c.gl[ci] = g;
        c.C[ci] = Cn;
        c.Cl[ci] = Cl;
        c.Cs[ci] = P.kp * Cl;
        const double mphi = c.ks[SP].xsum / (double)P.ncell;
        const double ph = c.phi[ci] - mphi;
        c.phi[ci] = ph;
        c.p[ci] += ph;
        // velocities: each cell commits the interior face on its + side
        double *const velv[3] = {c.u, c.v, c.w};
        double dv = 0.0;
        const double t_new = (double)(*c.step + 1) * P.dt;
        double wall = 0.0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const int na = ax == 0 ? P.nx : (ax == 1 ? P.ny : P.nz);
            if (q[ax] < na - 1) {
                int f;
                if (ax == 0) f = q[0] + (P.nx - 1) * (q[1] + P.ny * q[2]);
                else if (ax == 1) f = q[0] + P.nx * (q[1] + (P.ny - 1) * q[2]);
                else f = q[0] + P.nx * (q[1] + P.ny * q[2]);
                velv[ax][f] = c.un[ax][f];
            }
            double *const vs[3] = {c.un[0], c.un[1], c.un[2]};
            dv += (face_vel(P, vs, ax, q, q[ax] + 1) - face_vel(P, vs, ax, q, q[ax])) * P.ih[ax];
            if (q[ax] == 0) {
                const double U = wall_cond(P, 2 * ax, P.h[ax]);
                if (U > 0.0) wall += U / (P.rcp * P.h[ax]) * (Ts - wall_temp(P, 2 * ax, t_new));
            }
            if (q[ax] == na - 1) {
                const double U = wall_cond(P, 2 * ax + 1, P.h[ax]);
                if (U > 0.0) wall += U / (P.rcp * P.h[ax]) * (Ts - wall_temp(P, 2 * ax + 1, t_new));
            }
        }
        v[0] = Cn;
        v[1] = T + P.lam * g;
        v[2] = wall;
        v[3] = dv * dv;
    }
    const int nt = c.ntile_cell;
    const int off[4] = {0, nt, 2 * nt, 3 * nt};
    put_partials<4>(v, c.red_part, off, tl.t);
}

// per-case totals of the committed step (one workgroup per case); advances
// the step counter after every workgroup of k_phase_commit has read it
__global__ __launch_bounds__(TILE) void k_case_stats(const CaseDev *__restrict__ cases, const int32_t *__restrict__ cidx)
{
    const CaseDev &c = cases[cidx[blockIdx.x]];
    const int nt = c.ntile_cell;
    const int off[4] = {0, nt, 2 * nt, 3 * nt};
    double tot[4];
    sum_partials<4>(c.red_part, off, nt, tot);
    if (threadIdx.x == 0) {
        c.red[R_SUMC] = tot[0];
        c.red[R_SUMH] = tot[1];
        c.red[R_WALL] = tot[2];
        c.red[R_DIVNEW] = sqrt(tot[3]);
        *c.step += 1;
    }
}

// ------------------------------------------------------------- Krylov
// Jacobi-preconditioned CG (pressure) and BiCGSTAB (transport).  Each
// iteration is split at its global reductions.  A kernel of iteration k
// first totals the partial sums the previous kernels left (iteration k-1 in
// the buffers of parity (k-1)&1, iteration k in parity k&1), derives the
// scalars (alpha, beta, omega) and the convergence decision, identically in
// every workgroup, then works on its rows and writes its own partials.
// The preconditioned vector the matrix product needs at neighbour rows is
// recomputed there from vectors the previous kernel left unchanged, so no
// extra pass writes it; vectors overwritten while neighbours still read them
// are ping-ponged by iteration parity.  Workgroup 0 of a solve records a
// status change (converged, failed, restart); every other workgroup reaches
// the same decision from the same totals and stops with it.

typedef __attribute__((address_space(1))) double gdbl;

template <class T>
__device__ __forceinline__ gdbl *G(T *p) { return (gdbl *)p; }
template <class T>
__device__ __forceinline__ const gdbl *GC(const T *p) { return (const gdbl *)p; }

__device__ __forceinline__ const KJob &job_of(const KJob *jobs, const JTile *tiles, JTile &tl)
{
    tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    return jobs[tl.j];
}

__device__ __forceinline__ int poff(const KJob &J, int par, int slot) { return (par * NSLOT + slot) * J.ntile; }

// status of a solve as seen by iteration k: RUNNING, or a (re)start whose
// first iteration is k
__device__ __forceinline__ bool active(const KState *st, int k)
{
    const int s = st->status;
    return s == K_RUNNING || (s == K_RESTART && k == st->k0);
}

// record a terminal (or restart) status: workgroup 0 of the solve only
__device__ __forceinline__ void set_status(const JTile &tl, KState *st, int status, int it, double rr)
{
    if (tl.t == 0 && threadIdx.x == 0) {
        st->status = status;
        st->it = it;
        st->rr = rr;
    }
}

// Start of a solve at host iteration index k (mode 0: every solve, x = x0 or
// 0; mode 1: solves in K_RESTART, keep x).  r = b - A x, rh = r, p = v = 0;
// partials (r,Mr) or (rh,r), (r,r), (b,b) for iteration k.
template <int ND>
__global__ __launch_bounds__(TILE) void k_kinit(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k, int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (mode == 1 && st->status != K_RESTART) return;
    const int n = J.n;
    const int flip = k & 1;
    const gdbl *A = GC(J.A), *b = GC(J.b), *mi = GC(J.minv);
    gdbl *x = G(J.x), *r = G(J.r), *rh = G(J.rh);
    gdbl *po = G(flip ? J.p1 : J.p0), *vo = G(flip ? J.v1 : J.v0);
    const gdbl *x0 = GC(J.x0);
    double v[3] = {0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt;
    const int i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        double ri;
        if (mode == 0) {
            if (x0) {
                ri = b[i] - stencil<ND>(A, n, i, J.sx, J.sxy, [&](int j) { return x0[j]; });
                x[i] = x0[i];
            } else {
                ri = b[i];
                x[i] = 0.0;
            }
        } else {
            ri = b[i] - stencil<ND>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
        }
        r[i] = ri;
        rh[i] = ri;
        po[i] = 0.0;
        vo[i] = 0.0;
        v[0] += J.kind == K_CG ? ri * mi[i] * ri : ri * ri;
        v[1] += ri * ri;
        v[2] += b[i] * b[i];
    }
    const int par = (k + 1) & 1;               // = parity of iteration k-1
    const int off[3] = {poff(J, par, PS_RHO), poff(J, par, PS_RR), poff(J, par, PS_BB)};
    put_partials<3>(v, J.part, off, tl.t);
    if (tl.t == 0 && threadIdx.x == 0) {
        st->k0 = k;
        if (mode == 0) { st->it_base = 0; st->restarts = 0; st->status = K_RUNNING; }
        else { st->it_base = st->it; st->restarts += 1; }
    }
}

// convergence test at the start of iteration k (shared by CG and BiCGSTAB);
// returns false when the solve stops here
__device__ __forceinline__ bool test_convergence(const KJob &J, const JTile &tl, KState *st, int k,
                                                 double rr, double &bb)
{
    const int it = st->it_base + (k - st->k0);
    if (k == st->k0) {
        const int off[1] = {poff(J, (k + 1) & 1, PS_BB)};
        double t[1];
        sum_partials<1>(J.part, off, J.ntile, t);
        bb = t[0];
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

// CG, first half of iteration k: beta = rho_k / rho_{k-1}; p = M r + beta p;
// q = A p; partial (p, q)
template <int ND>
__global__ __launch_bounds__(TILE) void k_cg_a(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (!active(st, k)) return;
    const int pk = k & 1, pm = (k + 1) & 1;
    double s2[2];
    {
        const int off[2] = {poff(J, pm, PS_RHO), poff(J, pm, PS_RR)};
        sum_partials<2>(J.part, off, J.ntile, s2);
    }
    double bb;
    if (!test_convergence(J, tl, st, k, s2[1], bb)) return;
    double beta = 0.0;
    if (k != st->k0) {
        const int off[1] = {poff(J, pk, PS_RHO)};
        double t[1];
        sum_partials<1>(J.part, off, J.ntile, t);
        beta = s2[0] / t[0];
    }
    const int n = J.n;
    const gdbl *A = GC(J.A), *r = GC(J.r), *mi = GC(J.minv);
    const gdbl *po = GC(pk ? J.p1 : J.p0);
    gdbl *pn = G(pk ? J.p0 : J.p1), *q = G(J.t);
    double v[1] = {0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const double pi = mi[i] * r[i] + beta * po[i];
        const double qi = stencil<ND>(A, n, i, J.sx, J.sxy, [&](int j) { return mi[j] * r[j] + beta * po[j]; });
        pn[i] = pi;
        q[i] = qi;
        v[0] += pi * qi;
    }
    const int off[1] = {poff(J, pk, PS_Q)};
    put_partials<1>(v, J.part, off, tl.t);
}

// CG, second half: alpha = rho_k / (p, q); x += alpha p; r -= alpha q;
// partials (r, M r), (r, r) for iteration k+1
template <int ND>
__global__ __launch_bounds__(TILE) void k_cg_b(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (st->status != K_RUNNING) return;
    const int pk = k & 1, pm = (k + 1) & 1;
    double s2[2];
    {
        const int off[2] = {poff(J, pm, PS_RHO), poff(J, pk, PS_Q)};
        sum_partials<2>(J.part, off, J.ntile, s2);
    }
    if (!(s2[1] > 0.0) || !finite(s2[1])) {
        set_status(tl, st, finite(s2[1]) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0), 0.0);
        return;
    }
    const double alpha = s2[0] / s2[1];
    const gdbl *pn = GC(pk ? J.p0 : J.p1), *q = GC(J.t), *mi = GC(J.minv);
    gdbl *x = G(J.x), *r = G(J.r);
    double v[2] = {0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(J.n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        x[i] = x[i] + alpha * pn[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        v[0] += ri * mi[i] * ri;
        v[1] += ri * ri;
    }
    const int off[2] = {poff(J, pk, PS_RHO), poff(J, pk, PS_RR)};
    put_partials<2>(v, J.part, off, tl.t);
}

// BiCGSTAB (van der Vorst), right Jacobi preconditioning.
// a: beta = (rho_k/rho_{k-1})(alpha_{k-1}/omega_{k-1});
//    p = r + beta (p - omega v); v = A M p; partial (rh, v)
template <int ND>
__global__ __launch_bounds__(TILE) void k_bicg_a(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (!active(st, k)) return;
    const int pk = k & 1, pm = (k + 1) & 1;
    double s2[2];
    {
        const int off[2] = {poff(J, pm, PS_RHO), poff(J, pm, PS_RR)};
        sum_partials<2>(J.part, off, J.ntile, s2);
    }
    double bb;
    if (!test_convergence(J, tl, st, k, s2[1], bb)) return;
    const double rho = s2[0];
    double beta = 0.0, omega = 0.0;
    if (k != st->k0) {
        double s4[4];
        const int off[4] = {poff(J, pk, PS_RHO), poff(J, pm, PS_Q), poff(J, pm, PS_TS), poff(J, pm, PS_TT)};
        sum_partials<4>(J.part, off, J.ntile, s4);
        const double rho_prev = s4[0];
        const double alpha_prev = rho_prev / s4[1];
        omega = s4[3] > 0.0 ? s4[2] / s4[3] : 0.0;
        if (omega == 0.0 || rho == 0.0 || rho_prev == 0.0) {
            set_status(tl, st, K_RESTART, st->it_base + (k - st->k0), s2[1]);
            return;
        }
        beta = (rho / rho_prev) * (alpha_prev / omega);
    }
    const int n = J.n;
    const gdbl *A = GC(J.A), *r = GC(J.r), *mi = GC(J.minv), *rh = GC(J.rh);
    const gdbl *po = GC(pk ? J.p1 : J.p0), *vo = GC(pk ? J.v1 : J.v0);
    gdbl *pn = G(pk ? J.p0 : J.p1), *vn = G(pk ? J.v0 : J.v1);
    double v[1] = {0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const double pi = r[i] + beta * (po[i] - omega * vo[i]);
        const double vi = stencil<ND>(A, n, i, J.sx, J.sxy,
                                      [&](int j) { return mi[j] * (r[j] + beta * (po[j] - omega * vo[j])); });
        pn[i] = pi;
        vn[i] = vi;
        v[0] += rh[i] * vi;
    }
    const int off[1] = {poff(J, pk, PS_Q)};
    put_partials<1>(v, J.part, off, tl.t);
}

// b: alpha = rho_k / (rh, v); s = r - alpha v; t = A M s; partials (t,s), (t,t)
template <int ND>
__global__ __launch_bounds__(TILE) void k_bicg_b(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (st->status != K_RUNNING) return;
    const int pk = k & 1, pm = (k + 1) & 1;
    double s2[2];
    {
        const int off[2] = {poff(J, pm, PS_RHO), poff(J, pk, PS_Q)};
        sum_partials<2>(J.part, off, J.ntile, s2);
    }
    if (s2[1] == 0.0 || !finite(s2[1])) {
        set_status(tl, st, finite(s2[1]) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0), 0.0);
        return;
    }
    const double alpha = s2[0] / s2[1];
    const int n = J.n;
    const gdbl *A = GC(J.A), *r = GC(J.r), *mi = GC(J.minv);
    const gdbl *vn = GC(pk ? J.v0 : J.v1);
    gdbl *t = G(J.t);
    double v[2] = {0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const double si = r[i] - alpha * vn[i];
        const double ti = stencil<ND>(A, n, i, J.sx, J.sxy, [&](int j) { return mi[j] * (r[j] - alpha * vn[j]); });
        t[i] = ti;
        v[0] += ti * si;
        v[1] += ti * ti;
    }
    const int off[2] = {poff(J, pk, PS_TS), poff(J, pk, PS_TT)};
    put_partials<2>(v, J.part, off, tl.t);
}

// c: omega = (t,s)/(t,t); x += M (alpha p + omega s); r = s - omega t;
// partials (rh, r), (r, r) for iteration k+1
template <int ND>
__global__ __launch_bounds__(TILE) void k_bicg_c(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    KState *st = J.st;
    if (st->status != K_RUNNING) return;
    const int pk = k & 1, pm = (k + 1) & 1;
    double s4[4];
    {
        const int off[4] = {poff(J, pm, PS_RHO), poff(J, pk, PS_Q), poff(J, pk, PS_TS), poff(J, pk, PS_TT)};
        sum_partials<4>(J.part, off, J.ntile, s4);
    }
    const double alpha = s4[0] / s4[1];
    const double omega = s4[3] > 0.0 ? s4[2] / s4[3] : 0.0;
    const gdbl *pn = GC(pk ? J.p0 : J.p1), *vn = GC(pk ? J.v0 : J.v1), *t = GC(J.t);
    const gdbl *mi = GC(J.minv), *rh = GC(J.rh);
    gdbl *x = G(J.x), *r = G(J.r);
    double v[2] = {0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(J.n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const double si = r[i] - alpha * vn[i];
        x[i] = x[i] + mi[i] * (alpha * pn[i] + omega * si);
        const double ri = si - omega * t[i];
        r[i] = ri;
        v[0] += rh[i] * ri;
        v[1] += ri * ri;
    }
    const int off[2] = {poff(J, pk, PS_RHO), poff(J, pk, PS_RR)};
    put_partials<2>(v, J.part, off, tl.t);
}

// True residual b - A x of a solve that stopped as converged (or x = 0 when
// ||b|| = 0); partials of ||b - A x||^2, sum(b - A x), sum(x) into parity 0.
template <int ND>
__global__ __launch_bounds__(TILE) void k_kfinish(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    const int status = J.st->status;
    if (status != K_CONVERGED && status != K_ZERO) return;
    const int n = J.n;
    const gdbl *A = GC(J.A), *b = GC(J.b);
    gdbl *x = G(J.x);
    double v[3] = {0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        if (status == K_ZERO) {
            x[i] = 0.0;
        } else {
            const double rt = b[i] - stencil<ND>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
            v[0] += rt * rt;
            v[1] += rt;
            v[2] += x[i];
        }
    }
    const int off[3] = {poff(J, 0, PS_Q), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    put_partials<3>(v, J.part, off, tl.t);
}

// one workgroup per solve: totals of k_kfinish, verdict on the true residual
__global__ __launch_bounds__(TILE) void k_kdecide(const KJob *__restrict__ jobs, int njobs)
{
    const KJob &J = jobs[blockIdx.x];
    KState *st = J.st;
    const int status = st->status;
    if (status != K_CONVERGED && status != K_ZERO) return;
    const int off[3] = {poff(J, 0, PS_Q), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    double tot[3];
    sum_partials<3>(J.part, off, J.ntile, tot);
    if (threadIdx.x == 0) {
        st->tr2 = tot[0];
        st->tsum = tot[1];
        st->xsum = tot[2];
        if (status == K_ZERO || tot[0] <= st->tol2 * st->bb) st->status = K_DONE;
        else st->status = st->restarts >= 20 ? K_FAILED : K_RESTART;
    }
}

// ------------------------------------------------------------ CSR export
// Structural pattern of a system (in-domain neighbours, ascending columns)
// and its values from the DIA storage.
template <int DIM>
__global__ __launch_bounds__(TILE) void k_csr_count(const CaseDev *__restrict__ cd, int s, int32_t *cnt)
{
    const Phys &P = cd->ph;
    const int row = blockIdx.x * TILE + threadIdx.x;
    if (row >= P.nsys[s]) return;
    int q[3];
    decode(row, P.sdim[s][0], P.sdim[s][1], q);
    int k = 1;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) k += (q[ax] >= 1) + (q[ax] <= P.sdim[s][ax] - 2);
    cnt[row] = k;
}

// exclusive scan of cnt[0..n) into row_ptr[0..n] by one workgroup
__global__ __launch_bounds__(1024) void k_scan(const int32_t *cnt, int32_t *row_ptr, int n)
{
    __shared__ int32_t sh[1024];
    const int T = 1024;
    const int chunk = (n + T - 1) / T;
    const int b0 = threadIdx.x * chunk, b1 = min(n, b0 + chunk);
    int32_t s = 0;
    for (int i = b0; i < b1; ++i) s += cnt[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {
        int32_t add = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = sh[threadIdx.x] - s;
    for (int i = b0; i < b1; ++i) { row_ptr[i] = run; run += cnt[i]; }
    if (threadIdx.x == T - 1) row_ptr[n] = sh[T - 1];
}

template <int DIM>
__global__ __launch_bounds__(TILE) void k_csr_fill(const CaseDev *__restrict__ cd, int s, const int32_t *row_ptr,
                                                   int32_t *col, double *val)
{
    constexpr int ND = 2 * DIM + 1;
    const Phys &P = cd->ph;
    const int n = P.nsys[s];
    const int row = blockIdx.x * TILE + threadIdx.x;
    if (row >= n) return;
    int q[3];
    decode(row, P.sdim[s][0], P.sdim[s][1], q);
    const int sx = P.sdim[s][0], sxy = P.sdim[s][0] * P.sdim[s][1];
    const double *A = cd->A[s];
    int p = row_ptr[row];
#pragma unroll
    for (int slot = 0; slot < ND; ++slot) {
        bool ex;
        if (slot == DIM) ex = true;
        else if (slot < DIM) { const int ax = DIM - 1 - slot; ex = q[ax] >= 1; }
        else { const int ax = slot - DIM - 1; ex = q[ax] <= P.sdim[s][ax] - 2; }
        if (ex) {
            col[p] = row + slot_off<ND>(slot, sx, sxy);
            val[p] = A[(size_t)slot * n + row];
            ++p;
        }
    }
}

// ------------------------------------------------------------- utilities
__global__ void k_fill(double *x, double v, int n)
{
    const int i = blockIdx.x * TILE + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_set_status(KState *st, int n, int status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st[i].status = status;
}

// ============================================================ launchers

#define GRID(n) dim3((unsigned)(n)), dim3(TILE)

void launch_asm_const(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_asm_const<2>, GRID(nt), 0, s, c, t);
    else hipLaunchKernelGGL(k_asm_const<3>, GRID(nt), 0, s, c, t);
}
void launch_asm_momentum(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_asm_momentum<2>, GRID(nt), 0, s, c, t);
    else hipLaunchKernelGGL(k_asm_momentum<3>, GRID(nt), 0, s, c, t);
}
void launch_asm_transport(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_asm_transport<2>, GRID(nt), 0, s, c, t, vel_src);
    else hipLaunchKernelGGL(k_asm_transport<3>, GRID(nt), 0, s, c, t, vel_src);
}
void launch_div_rhs(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_div_rhs<2>, GRID(nt), 0, s, c, t, vel_src);
    else hipLaunchKernelGGL(k_div_rhs<3>, GRID(nt), 0, s, c, t, vel_src);
}
void launch_sub_mean(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_sub_mean, GRID(nt), 0, s, c, t);
}
void launch_project(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_project, GRID(nt), 0, s, c, t);
}
void launch_phase_commit(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) hipLaunchKernelGGL(k_phase_commit<2>, GRID(nt), 0, s, c, t);
    else hipLaunchKernelGGL(k_phase_commit<3>, GRID(nt), 0, s, c, t);
}

void launch_kinit(int nd, const KJob *j, const JTile *t, int nt, int k, int mode, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) hipLaunchKernelGGL(k_kinit<5>, GRID(nt), 0, s, j, t, k, mode);
    else hipLaunchKernelGGL(k_kinit<7>, GRID(nt), 0, s, j, t, k, mode);
}
void launch_kdecide(const KJob *j, int njobs, hipStream_t s)
{
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_kdecide, dim3(njobs), dim3(TILE), 0, s, j, njobs);
}
void launch_case_stats(const CaseDev *c, const int32_t *cidx, int ncase, hipStream_t s)
{
    if (ncase <= 0) return;
    hipLaunchKernelGGL(k_case_stats, dim3(ncase), dim3(TILE), 0, s, c, cidx);
}
void launch_kfinish(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) hipLaunchKernelGGL(k_kfinish<5>, GRID(nt), 0, s, j, t);
    else hipLaunchKernelGGL(k_kfinish<7>, GRID(nt), 0, s, j, t);
}
void launch_kiter(int which, int nd, const KJob *j, const JTile *t, int nt, int k, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) {
        switch (which) {
        case KI_CG_A: hipLaunchKernelGGL(k_cg_a<5>, GRID(nt), 0, s, j, t, k); break;
        case KI_CG_B: hipLaunchKernelGGL(k_cg_b<5>, GRID(nt), 0, s, j, t, k); break;
        case KI_BICG_A: hipLaunchKernelGGL(k_bicg_a<5>, GRID(nt), 0, s, j, t, k); break;
        case KI_BICG_B: hipLaunchKernelGGL(k_bicg_b<5>, GRID(nt), 0, s, j, t, k); break;
        default: hipLaunchKernelGGL(k_bicg_c<5>, GRID(nt), 0, s, j, t, k); break;
        }
    } else {
        switch (which) {
        case KI_CG_A: hipLaunchKernelGGL(k_cg_a<7>, GRID(nt), 0, s, j, t, k); break;
        case KI_CG_B: hipLaunchKernelGGL(k_cg_b<7>, GRID(nt), 0, s, j, t, k); break;
        case KI_BICG_A: hipLaunchKernelGGL(k_bicg_a<7>, GRID(nt), 0, s, j, t, k); break;
        case KI_BICG_B: hipLaunchKernelGGL(k_bicg_b<7>, GRID(nt), 0, s, j, t, k); break;
        default: hipLaunchKernelGGL(k_bicg_c<7>, GRID(nt), 0, s, j, t, k); break;
        }
    }
}
void launch_csr(int dim, const CaseDev *cd, int s, int n, int32_t *cnt, int32_t *row_ptr, int32_t *col,
                double *val, int build_pattern, hipStream_t st)
{
    if (n <= 0) return;
    const int nb = ceil_div(n, TILE);
    if (build_pattern) {
        if (dim == 2) hipLaunchKernelGGL(k_csr_count<2>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
        else hipLaunchKernelGGL(k_csr_count<3>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, row_ptr, n);
    }
    if (dim == 2) hipLaunchKernelGGL(k_csr_fill<2>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val);
    else hipLaunchKernelGGL(k_csr_fill<3>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val);
}
void launch_fill(double *x, double v, int n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(ceil_div(n, TILE)), dim3(TILE), 0, s, x, v, n);
}
void launch_set_status(KState *st, int n, int status, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_set_status, dim3(ceil_div(n, 64)), dim3(64), 0, s, st, n, status);
}

}  // namespace sol
