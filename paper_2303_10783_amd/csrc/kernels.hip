// HIP kernels (gfx950) of one time step of the decoupled solidification
// scheme: term-wise assembly, Jacobi-PCG and BiCGSTAB (one or two Jacobi
// sweeps as the preconditioner) iterations with fused reductions,
// divergence / projection, phase update and commit.
//
// Launch model: every per-row kernel walks a table of tiles (256 rows each)
// covering one or many cases; workgroup b takes tile xcd_tile(b) so that the
// tiles one XCD executes are contiguous in memory (its L2 then holds the
// y/z neighbour rows of its own tiles).  Reductions: per-workgroup partial
// sums, totalled in a fixed order by the next kernel (deterministic; no
// device-scope fences, which on gfx950 would write back the whole L2).
#include "sol_dev.hpp"
#include "kcommon.hpp"
#include "kernels.hpp"

#include <atomic>

namespace sol {

static std::atomic<long> g_dispatches{0};
void note_dispatch(long n) { g_dispatches.fetch_add(n, std::memory_order_relaxed); }
long dispatch_count() { return g_dispatches.load(std::memory_order_relaxed); }

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

// Constant (offline) coefficients of a momentum row (component s, face
// coordinates q): I/dt + viscous diffusion, no-slip walls at half a cell
// along the tangential axes; and of an energy row: I/dt + conduction, Robin
// wall conductances on the diagonal.  The offline assembly stores them; the
// per-step stencil-route kernels form them in registers with the same code
// (56 bytes per 7-point row less to read than the stored copy, the same
// doubles), the forward route reads the stored copy.
template <int DIM>
__device__ __forceinline__ void mom_const_row(const Phys &P, int s, const int *q, double (&a)[2 * DIM + 1])
{
#pragma unroll
    for (int k = 0; k < 2 * DIM + 1; ++k) a[k] = 0.0;
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
}

template <int DIM>
__device__ __forceinline__ void energy_const_row(const Phys &P, const int *q, double (&a)[2 * DIM + 1])
{
#pragma unroll
    for (int k = 0; k < 2 * DIM + 1; ++k) a[k] = 0.0;
    a[DIM] = P.idt;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const double dif = P.alpha * P.ih2[ax];
        for (int sd = 0; sd < 2; ++sd) {
            const bool ex = sd == 0 ? q[ax] >= 1 : q[ax] <= P.sdim[ST][ax] - 2;
            const int slot = sd == 0 ? DIM - 1 - ax : DIM + 1 + ax;
            if (ex) { a[DIM] += dif; a[slot] = -dif; }
            else {
                const double U = wall_cond(P, 2 * ax + sd, P.h[ax]);
                a[DIM] += U / (P.rcp * P.h[ax]);
            }
        }
    }
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
        mom_const_row<DIM>(P, s, q, a);
        double *Ac = c.Ac[s];
#pragma unroll
        for (int k = 0; k < ND; ++k) Ac[(size_t)k * n + row] = a[k];
    } else if (s == ST) {
        energy_const_row<DIM>(P, q, a);
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
// In the form of eq. (2.6) (P.mom1) the advecting velocity is u/g~ and the
// drag g~ (mu/rho) K^-1, the pressure gradient and the force carry g, with g
// = g_l^n on the face (mean of its two cells) and g~ = max(g, darcy_eps^(1/3)):
// below that liquid fraction the regularisation of g^3 in eq. (2.8)
// dominates, and g~ keeps 1/g finite and the drag large in solid cells.
// Form (2.7) multiplies by 1 and divides by 1, bit for bit the plain rows.
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
    double a[ND];
    mom_const_row<DIM>(P, d, q, a);
    const double gf = 0.5 * (c.gl[clo] + c.gl[chi]);
    const double gt = P.mom1 ? fmax(gf, P.gfloor) : 1.0;
    const double gw = P.mom1 ? gf : 1.0;
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
        vm = vm / gt;
        vp = vp / gt;
        const double cw = -fmax(vm, 0.0) * P.ih[ax];
        const double cp = (fmax(vp, 0.0) - fmin(vm, 0.0)) * P.ih[ax];
        const double ce = fmin(vp, 0.0) * P.ih[ax];
        dconv += cp;
        const bool em = q[ax] >= 1, ep = q[ax] <= P.sdim[d][ax] - 2;
        a[DIM - 1 - ax] = em ? a[DIM - 1 - ax] + cw : 0.0;
        a[DIM + 1 + ax] = ep ? a[DIM + 1 + ax] + ce : 0.0;
    }
    const double sol = 1.0 - gf;
    const double drag = gt * (P.nu * 180.0 * sol * sol / (P.lambda2 * P.lambda2 * (gf * gf * gf + P.eps)));
    a[DIM] += dconv + drag;
    double *A = c.A[d];
#pragma unroll
    for (int k = 0; k < ND; ++k) A[(size_t)k * n + row] = a[k];
    const double mi = 1.0 / a[DIM];
    c.minv[d][row] = mi;
    double rhs = vel[d][row] * P.idt - gw * ((c.p[chi] - c.p[clo]) / (P.rho * P.h[d]));
    if (d == DIM - 1) {
        const double Tf = 0.5 * (c.T[clo] + c.T[chi]);
        const double Cf = 0.5 * (c.Cl[clo] + c.Cl[chi]);
        rhs += gw * (P.grav * (P.betaT * (Tf - P.Tref) + P.betaC * (Cf - P.Cref)));
    }
    c.b[d][row] = rhs;
    if (c.A32[d]) {
#pragma unroll
        for (int k = 0; k < ND; ++k) c.A32[d][(size_t)k * n + row] = (float)a[k];
        c.minv32[d][row] = (float)mi;
    }
}

// ---------------------------------------------- solute + energy assembly
// Solute (eqs. 3.8-3.10): I/dt + (A_con(u^{n+1}) - A_dif) A_g, A_g =
// diag(1/(1 - (1-k_p)(1-g_l^n))) applied to the columns (C_l = A_g C
// substituted into the convection and diffusion terms); A_dif is the
// liquid diffusion div(g_l^n D_l grad .) of eq. 3.7 with g_l on a face the
// mean of its two cells and no flux through walls (absent when D_l = 0);
// b = C^n/dt.  Energy (eq. 3.11): const (1/dt, alpha
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
    double aC[ND], aT[ND];
    energy_const_row<DIM>(P, q, aT);
#pragma unroll
    for (int k = 0; k < ND; ++k) aC[k] = 0.0;
    double dconv = 0.0, ddif = 0.0;
    const double gP = c.gl[ci];
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
            const double gm = c.gl[ci - stride[ax]];
            const double agm = 1.0 / (1.0 - omk * (1.0 - gm));
            const double dm = P.Dl * (0.5 * (gP + gm)) * P.ih2[ax];
            ddif += dm;
            aC[sm] = (cw - dm) * agm;
            aT[sm] += cw;
        } else {
            aT[sm] = 0.0;
            const double U = wall_cond(P, 2 * ax, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax, t_new) / (P.rcp * P.h[ax]);
        }
        if (ep) {
            const double gp = c.gl[ci + stride[ax]];
            const double agp = 1.0 / (1.0 - omk * (1.0 - gp));
            const double dp = P.Dl * (0.5 * (gP + gp)) * P.ih2[ax];
            ddif += dp;
            aC[sp] = (ce - dp) * agp;
            aT[sp] += ce;
        } else {
            aT[sp] = 0.0;
            const double U = wall_cond(P, 2 * ax + 1, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax + 1, t_new) / (P.rcp * P.h[ax]);
        }
    }
    aC[DIM] = P.idt + (dconv + ddif) * agP;
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

// totals of k_div_rhs's partials, one workgroup per case: the mean of the
// pressure rhs (removed for the consistency of the Neumann problem by k_guess
// or k_sub_mean) and ||D u*||.  Totalled once per case: a total reads all of
// the case's partials (4096 x 2 at 128x128x64), which every workgroup of a
// per-tile kernel would otherwise repeat.
__global__ __launch_bounds__(TILE) void k_case_mean(const CaseDev *__restrict__ cases, const int32_t *__restrict__ cidx)
{
    const CaseDev &c = cases[cidx[blockIdx.x]];
    const int nt = c.ntile_cell;
    const int off[2] = {0, nt};
    double tot[2];
    sum_partials<2, 8>(c.red_part, off, nt, tot);
    if (threadIdx.x == 0) {
        c.red[R_SUMB] = tot[0];
        c.red[R_DIVSTAR] = sqrt(tot[1]);
        c.ks[SP].bmean = tot[0] / (double)c.ph.ncell;
    }
}

// remove the mean k_case_mean recorded from the pressure rhs
__global__ __launch_bounds__(TILE) void k_sub_mean(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const int ci = tl.t * TILE + threadIdx.x;
    if (ci < c.ph.ncell) c.b[SP][ci] -= c.ks[SP].bmean;
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

// Initial guesses of the pressure-correction and energy solves (the paper
// fixes none; the converged solution does not depend on it): extrapolation
// in time from the previous solutions of the same case, counted from the
// last reset of the history (creation, written fields, a failed step).
// With h solved steps in the history: h >= QUAD_GUESS_STEPS quadratic,
// 3 x^n - 3 x^(n-1) + x^(n-2); h >= 2 linear, 2 x^n - x^(n-1); before that
// phi = 0 and T* = T^n.  Started from rest, the quadratic guess is worse
// for the first steps of the transient and better afterwards (500x300
// cavity, energy BiCGSTAB iterations: step 3 linear 31 / quadratic 41,
// step 5 27 / 27, step 6 26 / 25, step 12 22 / 19, step 18 21 / 16).  The
// guess is written into the solution buffer, which the solve then takes as
// its initial guess; the history shifts by one.  The same pass removes the
// mean k_case_mean recorded from the pressure rhs (as k_sub_mean would).
constexpr int QUAD_GUESS_STEPS = 6;
__global__ __launch_bounds__(TILE) void k_guess(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const int i = tl.t * TILE + threadIdx.x;
    if (i >= c.ph.ncell) return;
    const int64_t h = *c.step - *c.hist;
    const double t0 = c.Tstar[i], t1 = c.Tprev[i], t2 = c.Tprev2[i];
    const double p0 = c.phi[i], p1 = c.phiprev[i], p2 = c.phiprev2[i];
    double tg, pg;
    if (h >= QUAD_GUESS_STEPS) {
        tg = 3.0 * (t0 - t1) + t2;
        pg = 3.0 * (p0 - p1) + p2;
    } else if (h >= 2) {
        tg = 2.0 * t0 - t1;
        pg = 2.0 * p0 - p1;
    } else {
        tg = c.T[i];
        pg = 0.0;
    }
    c.b[SP][i] -= c.ks[SP].bmean;
    c.Tstar[i] = tg;
    c.phi[i] = pg;
    c.Tprev2[i] = t1;
    c.phiprev2[i] = p1;
    c.Tprev[i] = t0;
    c.phiprev[i] = p0;
}

// Initial guesses of the momentum solves, by the same rule from the previous
// u* (before the history holds two steps: u^n); written into u*, the history
// shifts by one.
constexpr int QUAD_GUESS_MOM = QUAD_GUESS_STEPS;
__global__ __launch_bounds__(TILE) void k_guess_mom(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const CaseDev &c = cases[tl.c];
    const int d = tl.s;
    const int row = tl.t * TILE + threadIdx.x;
    if (row >= c.ph.nsys[d]) return;
    const int64_t h = *c.step - *c.hist;
    const double s0 = c.us[d][row], s1 = c.usprev[d][row], s2 = c.usprev2[d][row];
    double g;
    if (h >= QUAD_GUESS_MOM) g = 3.0 * (s0 - s1) + s2;
    else if (h >= 2) g = 2.0 * s0 - s1;
    else g = (d == 0 ? c.u : (d == 1 ? c.v : c.w))[row];
    c.us[d][row] = g;
    c.usprev2[d][row] = s1;
    c.usprev[d][row] = s0;
}

// history reset of every case of a group (hist = step)
__global__ void k_hist_reset(const CaseDev *__restrict__ cases, int ncase)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncase) *cases[c].hist = *cases[c].step;
}

// per-case totals of the committed step (one workgroup per case); advances
// the step counter after every workgroup of k_phase_commit has read it
__global__ __launch_bounds__(TILE) void k_case_stats(const CaseDev *__restrict__ cases, const int32_t *__restrict__ cidx)
{
    const CaseDev &c = cases[cidx[blockIdx.x]];
    const int nt = c.ntile_cell;
    const int off[4] = {0, nt, 2 * nt, 3 * nt};
    double tot[4];
    sum_partials<4, 4>(c.red_part, off, nt, tot);
    if (threadIdx.x == 0) {
        c.red[R_SUMC] = tot[0];
        c.red[R_SUMH] = tot[1];
        c.red[R_WALL] = tot[2];
        c.red[R_DIVNEW] = sqrt(tot[3]);
        *c.step += 1;
    }
}

// ------------------------------------------------------------- Krylov
// Jacobi-preconditioned CG (pressure) and BiCGSTAB (transport), templated on
// the vector / matrix type T (double; float for the inner solves of the
// mixed-precision refinement).  Every kernel of iteration k first totals the
// partial sums the previous kernels left (iteration k-1 in the buffers of
// parity (k+1)&1, iteration k in parity k&1), derives the scalars and the
// convergence decision identically in every workgroup, then works on its
// rows and writes its own partials.  Vectors a matrix product needs at
// neighbour rows are recomputed there from vectors the previous kernel left
// unchanged; vectors overwritten while neighbours still read them are
// ping-ponged by iteration parity.  Workgroup 0 of a solve records status
// changes; the other workgroups reach the same decision and stop with it.
//
// CG runs one kernel per iteration (the Chronopoulos-Gear arrangement of
// the same recurrences: both inner products of an iteration are taken
// together, so one global reduction separates consecutive iterations):
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M r,
//   w = A u, gamma = (r, u), delta = (w, u),
//   beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old).

// ---- BiCGSTAB (van der Vorst's recurrences) with two reductions per
// iteration.  r_k, p_k, v_k of iteration k live in the buffers of parity
// k & 1 (r / r1, p0 / p1, v0 / v1); rho_k = (rh, r_k) is kept per parity in
// st->gamma by workgroup 0.  Iteration k is two launches:
//   B(k): convergence test on ||r_k||^2 (from A(k-1); the start kernels
//         test r_k0); alpha_k = rho_k / (rh, v_k); s = r_k - alpha_k v_k;
//         t = A M s; partials (t,s), (t,t), (rh,s), (rh,t), (s,s)
//   A(k): if ||s|| already meets half the tolerance, x += alpha_k M p_k and
//         r_(k+1) = s, tested by B(k+1) (bicg_half_exit); otherwise
//         omega_k = (t,s) / (t,t); x += M (alpha_k p_k + omega_k s);
//         r_(k+1) = s - omega_k t; rho_(k+1) = (rh, r_(k+1)) expanded as
//         (rh,s) - omega_k (rh,t), so beta = (rho_(k+1)/rho_k)(alpha_k/omega_k)
//         needs no reduction of its own; p_(k+1) = r_(k+1) + beta (p_k -
//         omega_k v_k), v_(k+1) = A M p_(k+1); partials (rh, v_(k+1)) and
//         ||r_(k+1)||^2 from the rows themselves.
// s and p_(k+1) are recomputed at the neighbour rows a stencil needs.  The
// textbook arrangement takes a third reduction for (rh, r_(k+1)) and
// ||r_(k+1)||.  Here the norm is summed from r_(k+1) and tested one kernel
// later (x_(k+1) is written by then); expanding it in (s,s), (t,s), (t,t)
// instead cancels catastrophically when one step shrinks the residual by
// orders of magnitude, as the diagonally dominant momentum systems do.  rho
// has no such cancellation: (rh,s) vanishes in exact arithmetic.
//
// ---- Transport preconditioner M (template argument PD).  PD 1: the inverse
// diagonal.  PD 2: two Jacobi sweeps from zero, z1 = D^-1 f, z2 = z1 + D^-1
// (f - A z1), i.e. M f = D^-1 (f - N D^-1 f) with N = A - D the off-diagonal
// part; about half the iterations of PD 1 on the momentum and energy
// systems.  A product A M f at row i then reaches every cell within two
// stencil steps of i (13 in 2D, 25 in 3D); each is gathered once, with the
// vectors that define f there recomputed as for PD 1, and combined from
// registers.  A cell outside the domain is only reached through an exact 0
// coefficient (of row i, or of the neighbour row in between); its index is
// clamped into [0, n) like kstencil's.

template <int ND>
struct Ring2 {
    static constexpr int NC = ND == 5 ? 13 : 25;
    int d[NC][3];                 // (dx, dy, dz) of each cell
    int nb[ND][ND];               // cell reached by DIA slot s, then slot s2
};

// unit step along axis a of DIA slot s (slot order -z, -y, -x, 0, +x, +y, +z)
template <int ND>
constexpr int slot_step(int s, int a)
{
    const int u = s - ND / 2;
    const int m = u < 0 ? -u : u;
    return (m != 0 && m - 1 == a) ? (u < 0 ? -1 : 1) : 0;
}

template <int ND>
constexpr Ring2<ND> make_ring2()
{
    Ring2<ND> R{};
    int c = 0;
    const int zr = ND == 7 ? 2 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx)
                if ((dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz) <= 2) {
                    R.d[c][0] = dx;
                    R.d[c][1] = dy;
                    R.d[c][2] = dz;
                    ++c;
                }
    for (int s = 0; s < ND; ++s)
        for (int s2 = 0; s2 < ND; ++s2)
            for (int q = 0; q < Ring2<ND>::NC; ++q) {
                bool same = true;
                for (int a = 0; a < 3; ++a) same = same && R.d[q][a] == slot_step<ND>(s, a) + slot_step<ND>(s2, a);
                if (same) R.nb[s][s2] = q;
            }
    return R;
}

template <int ND>
struct Ring2Tab {
    static constexpr Ring2<ND> R = make_ring2<ND>();
};

// row of ring cell c of row i, clamped into [0, n)
template <int ND>
__device__ __forceinline__ int ring_row(int i, int c, int sx, int sxy, int n)
{
    constexpr Ring2<ND> R = Ring2Tab<ND>::R;
    const int j = i + R.d[c][0] + R.d[c][1] * sx + R.d[c][2] * sxy;
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// PD 2: (A M f)_i from y[c] = (D^-1 f) at the ring cells idx[c] of row i.
// Ad[s] views diagonal s, mi the inverse diagonal: every load is a uniform
// base plus the 32-bit offset of its cell, one register per ring cell for
// all vectors and diagonals.
template <int ND, class T>
__device__ __forceinline__ T ring_amf(const RO<T> (&Ad)[ND], RO<T> mi, const int (&idx)[Ring2<ND>::NC],
                                      const T (&y)[Ring2<ND>::NC])
{
    constexpr Ring2<ND> RG = Ring2Tab<ND>::R;
    constexpr int C = ND / 2;
    const int i = idx[RG.nb[C][C]];
    T acc = T(0);
#pragma unroll
    for (int s = 0; s < ND; ++s) {
        const int cj = RG.nb[s][C];
        const int j = idx[cj];
        T ns = T(0);
#pragma unroll
        for (int s2 = 0; s2 < ND; ++s2)
            if (s2 != C) ns += Ad[s2][j] * y[RG.nb[s][s2]];
        acc += Ad[s][i] * (y[cj] - mi[j] * ns);
    }
    return acc;
}

template <int ND, class T>
__device__ __forceinline__ void diag_views(const void *A, int n, RO<T> (&Ad)[ND])
{
#pragma unroll
    for (int s = 0; s < ND; ++s) Ad[s] = R<T>((const T *)A + (size_t)s * n);
}

// Jacobi inverse diagonal of row j in the staged B and first-iteration
// kernels.  FP64: the reciprocal of the stored diagonal, which those kernels
// read anyway (one correctly rounded division: the double the assembly
// stores in minv, so the staged and the gathering kernels still agree bit
// for bit), instead of streaming minv as an array of its own.  The staged A
// kernel keeps the array: at its five waves per SIMD the divisions' latency
// cost more than the 8 bytes per row they saved (30.7 -> 31.7 us at
// 128x128x64), where B, at eight, gained (25.2 -> 24.0 us).  FP32 reads
// minv32: the float reciprocal of the float diagonal is not the float of
// that double.
template <class T>
struct MinvOf {
    RO<T> dg, mi;
    __device__ __forceinline__ T operator()(int j) const
    {
        if constexpr (sizeof(T) == 8) return T(1) / dg[j];
        else return mi[j];
    }
};

// a * b + c rounded once, spelled out where two kernels must round alike
// and the compiler's own choice of products to fuse could differ between them
template <class T>
__device__ __forceinline__ T fmat(T a, T b, T c)
{
    if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

// PD 2 on a 5-point FP64 system, the tile [i0, i1) staged through LDS (KJob::
// staged; the FP32 inner solves were faster gathering per row).  The rows within two stencil steps of the tile are [i0 - 2 sx - 2,
// i1 + 2 sx + 2).  Pass 1 writes y = D^-1 f for each of them (0 outside
// [0, n): only exact-0 coefficients reach those), pass 2 z = M f = y -
// D^-1 N y for the rows within one step, pass 3 hands (A z)_i of each own
// row to out(i, .).  Each value is loaded once per workgroup instead of once
// per row that reaches it; the arithmetic and its order are those of
// ring_amf.  The dynamic LDS holds stage2_values(rpt, sx) values.
template <class T, class MI, class FY, class FO>
__device__ __forceinline__ void stage2_amf(const KJob &J, int i0, int i1, const RO<T> (&Ad)[5], MI Mi, FY fy,
                                           FO out)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *Y = reinterpret_cast<T *>(lds_raw);
    const int n = J.n, sx = J.sx;
    const int ylo = i0 - 2 * sx - 2, yn = (i1 - i0) + 4 * sx + 4;
    const int zlo = i0 - sx - 1, zn = (i1 - i0) + 2 * sx + 2;
    T *Z = Y + yn;
    for (int q = threadIdx.x; q < yn; q += TILE) {
        const int j = ylo + q;
        Y[q] = (j >= 0 && j < n) ? Mi(j) * fy(j) : T(0);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < zn; q += TILE) {
        const int j = zlo + q;
        T z = T(0);
        if (j >= 0 && j < n) {
            const int c = j - ylo;
            T ns = T(0);
            ns += Ad[0][j] * Y[c - sx];
            ns += Ad[1][j] * Y[c - 1];
            ns += Ad[3][j] * Y[c + 1];
            ns += Ad[4][j] * Y[c + sx];
            z = Y[c] - Mi(j) * ns;
        }
        Z[q] = z;
    }
    __syncthreads();
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const int c = i - zlo;
        T acc = T(0);
        acc += Ad[0][i] * Z[c - sx];
        acc += Ad[1][i] * Z[c - 1];
        acc += Ad[2][i] * Z[c];
        acc += Ad[3][i] * Z[c + 1];
        acc += Ad[4][i] * Z[c + sx];
        out(i, acc);
    }
}

// PD 1 on a 7-point system, the tile [i0, i1) staged through LDS (KJob::
// staged): pass 1 writes y = fy(j) (= M f at row j) for the rows within one
// grid row of the tile, [i0 - sx, i1 + sx) (0 outside [0, n): only exact-0
// coefficients reach those), pass 2 hands (A y)_i of each own row to out(i, .),
// its x and y neighbours read from LDS and its two z neighbours (a plane
// away, in other tiles) recomputed by fy from memory.  A row's M f is loaded
// once per workgroup instead of once per row whose stencil reaches it; the
// products and their order are kstencil's.  The dynamic LDS holds
// stage1_values(rpt, sx) values.
template <class T, class FY, class FO>
__device__ __forceinline__ void stage1_amf7(const KJob &J, int i0, int i1, const RO<T> (&Ad)[7], FY fy, FO out)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *Y = reinterpret_cast<T *>(lds_raw);
    const int n = J.n, sx = J.sx, sxy = J.sxy;
    const int ylo = i0 - sx, yn = (i1 - i0) + 2 * sx;
    for (int q = threadIdx.x; q < yn; q += TILE) {
        const int j = ylo + q;
        Y[q] = (j >= 0 && j < n) ? fy(j) : T(0);
    }
    __syncthreads();
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const int c = i - ylo;
        const int jm = i - sxy < 0 ? 0 : i - sxy, jp = i + sxy >= n ? n - 1 : i + sxy;
        T acc = T(0);
        acc += Ad[0][i] * fy(jm);
        acc += Ad[1][i] * Y[c - sx];
        acc += Ad[2][i] * Y[c - 1];
        acc += Ad[3][i] * Y[c];
        acc += Ad[4][i] * Y[c + 1];
        acc += Ad[5][i] * Y[c + sx];
        acc += Ad[6][i] * fy(jp);
        out(i, acc);
    }
}

// Start at iteration index k (mode 0: every solve, x = x0 or 0; mode 1:
// solves in K_RESTART, keep x): r_k = b - A x, rh = r_k; partials (rh, r_k),
// (r_k, r_k), (b, b).
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_bicg_init(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k, int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RESTART) return;
    if (outer_idle(J)) return;
    const int n = J.n;
    auto A = G<T>(J.A);
    auto b = G<T>(J.b);
    auto x = G<T>(J.x), r = G<T>((k & 1) ? J.r1 : J.r), rh = G<T>(J.rh);
    auto x0 = G<T>(J.x0);
    double v[3] = {0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        T ri;
        if (mode == 0) {
            if (J.x0) {
                ri = b[i] - kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return x0[j]; });
                if (J.x0 != J.x) x[i] = x0[i];     // a guess written into x stays
            } else {
                ri = b[i];
                x[i] = T(0);
            }
        } else {
            ri = b[i] - kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
        }
        r[i] = ri;
        rh[i] = ri;
        v[0] += (double)ri * ri;
        v[1] += (double)ri * ri;
        v[2] += (double)b[i] * b[i];
    }
    const int pk = k & 1;
    const int off[3] = {poff(J, pk, PS_RHO), poff(J, pk, PS_RR), poff(J, pk, PS_BB)};
    put_partials<3>(v, J.part, off, tl.t);
    mark_start(tl, J.st, k, mode);
}

// first iteration of a (re)start at k = k0: convergence test on r_k; p_k =
// r_k, v_k = A M p_k; partial (rh, v_k).  Two sweeps on a staged 5-point FP64
// solve: the tile's neighbourhood goes through LDS, as in the iteration
// kernels.
template <int ND, int PD, class T, bool S1 = false>
__global__ __launch_bounds__(TILE) void k_bicg_first(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (!active(J, k) || outer_idle(J)) return;
    const int pk = k & 1;
    double s3[3];
    {
        const int off[3] = {poff(J, pk, PS_RHO), poff(J, pk, PS_RR), poff(J, pk, PS_BB)};
        sum_partials<3>(J.part, off, J.ntile, s3);
    }
    if (!keep_going(J, tl, k, s3[1], s3[2])) return;
    if (tl.t == 0 && threadIdx.x == 0) J.st->gamma[pk] = s3[0];
    const int n = J.n;
    auto A = G<T>(J.A);
    auto r = G<T>(pk ? J.r1 : J.r), mi = G<T>(J.minv), rh = G<T>(J.rh);
    auto p = G<T>(pk ? J.p1 : J.p0), vv = G<T>(pk ? J.v1 : J.v0);
    double q = 0.0;
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    bool done = false;
    if constexpr (PD == 2 && ND == 5 && sizeof(T) == 8) {
        if (J.staged) {
            RO<T> Ad[ND];
            diag_views<ND, T>(J.A, n, Ad);
            const MinvOf<T> Mi{Ad[2], R<T>(J.minv)};
            const auto Rr = R<T>(pk ? J.r1 : J.r);
            stage2_amf<T>(J, i0, i1, Ad, Mi, [&](int j) { return Rr[j]; }, [&](int i, T vi) {
                p[i] = r[i];
                vv[i] = vi;
                q += (double)rh[i] * vi;
            });
            done = true;
        }
    }
    if constexpr (S1) {
        static_assert(ND == 7 && PD == 1, "one-sweep 7-point staging");
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        const MinvOf<T> Mi{Ad[3], R<T>(J.minv)};
        const auto Rr = R<T>(pk ? J.r1 : J.r);
        stage1_amf7<T>(J, i0, i1, Ad, [&](int j) { return Mi(j) * Rr[j]; }, [&](int i, T vi) {
            p[i] = r[i];
            vv[i] = vi;
            q += (double)rh[i] * vi;
        });
        done = true;
    }
    if (!done)
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        T vi;
        if constexpr (PD == 1) {
            vi = kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return mi[j] * r[j]; });
        } else {
            constexpr int NC = Ring2<ND>::NC;
            RO<T> Ad[ND];
            diag_views<ND, T>(J.A, n, Ad);
            const auto Mi = R<T>(J.minv), Rr = R<T>(pk ? J.r1 : J.r);
            int idx[NC];
            T y[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                idx[c] = ring_row<ND>(i, c, J.sx, J.sxy, n);
                y[c] = Mi[idx[c]] * Rr[idx[c]];
            }
            vi = ring_amf<ND, T>(Ad, Mi, idx, y);
        }
        p[i] = r[i];
        vv[i] = vi;
        q += (double)rh[i] * vi;
    }
    double v1[1] = {q};
    const int off[1] = {poff(J, pk, PS_Q)};
    put_partials<1>(v1, J.part, off, tl.t);
}

// B(k); kernels below
template <int ND, int PD, class T, bool S1 = false>
__device__ __forceinline__ void bicg_b_body(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff)
{
    const int k = (kbase ? *kbase : 0) + koff;
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (wg_status(J.st) != K_RUNNING || outer_idle(J)) return;
    const int pk = k & 1;
    double s2[2];
    {
        const int off[2] = {poff(J, pk, PS_Q), poff(J, pk, PS_RR)};
        sum_partials<2>(J.part, off, J.ntile, s2);
    }
    if (k > J.st->k0 && !keep_going(J, tl, k, s2[1], 0.0)) return;
    double s1[1] = {s2[0]};
    if (s1[0] == 0.0 || !finite(s1[0])) {
        set_status(tl, J.st, finite(s1[0]) ? K_RESTART : K_NONFINITE, J.st->it_base + (k - J.st->k0), 0.0);
        return;
    }
    const T alpha = (T)(J.st->gamma[pk] / s1[0]);
    const int n = J.n;
    auto A = G<T>(J.A);
    auto r = G<T>(pk ? J.r1 : J.r), mi = G<T>(J.minv), rh = G<T>(J.rh);
    auto vk = G<T>(pk ? J.v1 : J.v0);
    auto t = G<T>(J.t);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};     // (t,s) (t,t) (rh,s) (rh,t) (s,s)
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    if constexpr (S1) {
        static_assert(ND == 7 && PD == 1, "one-sweep 7-point staging");
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        const MinvOf<T> Mi{Ad[3], R<T>(J.minv)};
        const auto Rr = R<T>(pk ? J.r1 : J.r), Vk = R<T>(pk ? J.v1 : J.v0), Rh = R<T>(J.rh);
        stage1_amf7<T>(J, i0, i1, Ad, [&](int j) { return Mi(j) * (Rr[j] - alpha * Vk[j]); }, [&](int i, T ti) {
            const T si = Rr[i] - alpha * Vk[i];
            const T hi = Rh[i];
            t[i] = ti;
            const double sd = si, td = ti, hd = hi;
            v[0] += td * sd;
            v[1] += td * td;
            v[2] += hd * sd;
            v[3] += hd * td;
            v[4] += sd * sd;
        });
    } else if constexpr (PD == 2) {
        constexpr int NC = Ring2<ND>::NC;
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        const auto Mi = R<T>(J.minv), Rr = R<T>(pk ? J.r1 : J.r), Vk = R<T>(pk ? J.v1 : J.v0), Rh = R<T>(J.rh);
        bool done = false;
        if constexpr (ND == 5 && sizeof(T) == 8) {
            if (J.staged) {
                const MinvOf<T> Mf{Ad[2], Mi};
                stage2_amf<T>(J, i0, i1, Ad, Mf, [&](int j) { return Rr[j] - alpha * Vk[j]; }, [&](int i, T ti) {
                    const T si = Rr[i] - alpha * Vk[i];
                    const T hi = Rh[i];
                    t[i] = ti;
                    const double sd = si, td = ti, hd = hi;
                    v[0] += td * sd;
                    v[1] += td * td;
                    v[2] += hd * sd;
                    v[3] += hd * td;
                    v[4] += sd * sd;
                });
                done = true;
            }
        }
        if (!done)
        for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
            int idx[NC];
            T y[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                idx[c] = ring_row<ND>(i, c, J.sx, J.sxy, n);
                y[c] = Mi[idx[c]] * (Rr[idx[c]] - alpha * Vk[idx[c]]);
            }
            const T ti = ring_amf<ND, T>(Ad, Mi, idx, y);
            const T si = Rr[i] - alpha * Vk[i];
            const T hi = Rh[i];
            t[i] = ti;
            const double sd = si, td = ti, hd = hi;
            v[0] += td * sd;
            v[1] += td * td;
            v[2] += hd * sd;
            v[3] += hd * td;
            v[4] += sd * sd;
        }
    } else
    for (int i = i0 + threadIdx.x; i < i1; i += 2 * TILE) {
        const bool two = i + TILE < i1;
        const int i2 = two ? i + TILE : i;
        T sv[2], tv[2], hv[2];
        const int iv[2] = {i, i2};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int ii = iv[u];
            sv[u] = r[ii] - alpha * vk[ii];
            tv[u] = kstencil<ND, T>(A, n, ii, J.sx, J.sxy, [&](int j) { return mi[j] * (r[j] - alpha * vk[j]); });
            hv[u] = rh[ii];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !two) break;
            t[iv[u]] = tv[u];
            const double sd = sv[u], td = tv[u], hd = hv[u];
            v[0] += td * sd;
            v[1] += td * td;
            v[2] += hd * sd;
            v[3] += hd * td;
            v[4] += sd * sd;
        }
    }
    const int off[5] = {poff(J, pk, PS_TS), poff(J, pk, PS_TT), poff(J, pk, PS_RHS), poff(J, pk, PS_RHT),
                        poff(J, pk, PS_SS)};
    put_partials<5>(v, J.part, off, tl.t);
}

// A(k) when s_k = r_k - alpha_k v_k already meets half the tolerance (its
// norm from B(k)): x_(k+1) = x_k + alpha_k M p_k, the update without the
// stabilising half; r_(k+1) = s_k, whose norm B(k+1) takes for its test
// from the tile's partial copied here, and nothing else is formed (r, p, v
// of k+1 serve no converged solve, and a restart forms them from x).  The
// same code for the gathering and the staged kernels.  The true residual of
// x + alpha M p is s plus the drift of the recurrences, so half the
// tolerance leaves room for a drift up to the other half (near the FP64
// floor a solve that exited at the tolerance itself failed its check and
// broke down at every restart); and only before a solve's first restart,
// after which it takes whole iterations.
template <int ND, int PD, class T>
__device__ __forceinline__ void bicg_half_exit(const KJob &J, const JTile &tl, int pk, int pn, T ta)
{
    const int n = J.n;
    auto x = G<T>(J.x);
    const auto Mi = R<T>(J.minv), Pk = R<T>(pk ? J.p1 : J.p0);
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    if constexpr (PD == 1) {
        for (int i = i0 + threadIdx.x; i < i1; i += TILE) x[i] = x[i] + Mi[i] * (ta * Pk[i]);
    } else {
        // M f = D^-1 (f - N D^-1 f) at row i
        constexpr int C = ND / 2;
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
            T gs = T(0);
#pragma unroll
            for (int s2 = 0; s2 < ND; ++s2) {
                if (s2 == C) continue;
                const int j = min(max(i + slot_off<ND>(s2, J.sx, J.sxy), 0), n - 1);
                gs += Ad[s2][i] * (Mi[j] * (ta * Pk[j]));
            }
            x[i] = x[i] + Mi[i] * (ta * Pk[i] - gs);
        }
    }
    if (threadIdx.x == 0) J.part[poff(J, pn, PS_RR) + tl.t] = J.part[poff(J, pk, PS_SS) + tl.t];
    if (tl.t == 0 && threadIdx.x == 0) J.st->half = 1;      // read by the host only
}

// A(k); kernels below
template <int ND, int PD, class T, bool S1 = false>
__device__ __forceinline__ void bicg_a_body(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff)
{
    const int k = (kbase ? *kbase : 0) + koff;
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (wg_status(J.st) != K_RUNNING || outer_idle(J)) return;
    KState *st = J.st;
    const int pk = k & 1, pn = (k + 1) & 1;
    double s5[6];
    {
        const int off[6] = {poff(J, pk, PS_TS), poff(J, pk, PS_TT), poff(J, pk, PS_RHS), poff(J, pk, PS_RHT),
                            poff(J, pk, PS_Q), poff(J, pk, PS_SS)};
        sum_partials<6>(J.part, off, J.ntile, s5);
    }
    const double rho = st->gamma[pk];
    const double alpha = rho / s5[4];
    if (st->restarts == 0 && finite(alpha) && s5[5] <= 0.25 * st->tol2 * st->bb) {
        bicg_half_exit<ND, PD, T>(J, tl, pk, pn, (T)alpha);
        return;
    }
    const double omega = s5[1] > 0.0 ? s5[0] / s5[1] : 0.0;
    const double rho_n = s5[2] - omega * s5[3];
    // On a breakdown nothing is written: workgroup 0 records the restart,
    // and a workgroup of this launch that starts after it reads the new
    // status and returns at once, so a partial update by the others would
    // leave x half-advanced.  The restart starts from x_k.
    if (omega == 0.0 || rho_n == 0.0 || rho == 0.0 || !finite(rho_n) || !finite(alpha)) {
        set_status(tl, st, finite(rho_n) && finite(alpha) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0),
                   st->rr);
        return;
    }
    const double beta = (rho_n / rho) * (alpha / omega);
    if (tl.t == 0 && threadIdx.x == 0) st->gamma[pn] = rho_n;
    const T ta = (T)alpha, tw = (T)omega, tb = (T)beta;
    const int n = J.n;
    auto A = G<T>(J.A);
    auto rk = G<T>(pk ? J.r1 : J.r), rn = G<T>(pn ? J.r1 : J.r);
    auto pkv = G<T>(pk ? J.p1 : J.p0), pnv = G<T>(pn ? J.p1 : J.p0);
    auto vk = G<T>(pk ? J.v1 : J.v0), vn = G<T>(pn ? J.v1 : J.v0);
    auto t = G<T>(J.t), mi = G<T>(J.minv), rh = G<T>(J.rh), x = G<T>(J.x);
    double q[2] = {0.0, 0.0};       // (rh, v_(k+1)), ||r_(k+1)||^2
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    // p_(k+1) at row j from vectors no workgroup of this launch writes
    auto pnext = [&](int j) {
        const T rj = (rk[j] - ta * vk[j]) - tw * t[j];
        return rj + tb * (pkv[j] - tw * vk[j]);
    };
    if constexpr (S1) {
        static_assert(ND == 7 && PD == 1, "one-sweep 7-point staging");
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        const auto Mi = R<T>(J.minv);
        stage1_amf7<T>(J, i0, i1, Ad, [&](int j) { return Mi[j] * pnext(j); }, [&](int i, T vi) {
            const T si = rk[i] - ta * vk[i];
            const T xi = fmat(Mi[i], fmat(ta, pkv[i], tw * si), x[i]);     // x + M (alpha p + omega s)
            const T ri = si - tw * t[i];
            const T pi = pnext(i);
            const T hi = rh[i];
            x[i] = xi;
            rn[i] = ri;
            pnv[i] = pi;
            vn[i] = vi;
            q[0] += (double)hi * vi;
            q[1] += (double)ri * ri;
        });
    } else if constexpr (PD == 2) {
        constexpr int NC = Ring2<ND>::NC, C = ND / 2;
        constexpr Ring2<ND> RG = Ring2Tab<ND>::R;
        RO<T> Ad[ND];
        diag_views<ND, T>(J.A, n, Ad);
        const auto Mi = R<T>(J.minv), Rk = R<T>(pk ? J.r1 : J.r), Vk = R<T>(pk ? J.v1 : J.v0),
                   Pk = R<T>(pk ? J.p1 : J.p0), Tt = R<T>(J.t), Rh = R<T>(J.rh), X = R<T>(J.x);
        bool done = false;
        if constexpr (ND == 5 && sizeof(T) == 8) {
            if (J.staged) {
                auto pn = [&](int j) { return ((Rk[j] - ta * Vk[j]) - tw * Tt[j]) + tb * (Pk[j] - tw * Vk[j]); };
                stage2_amf<T>(J, i0, i1, Ad, [&](int j) { return Mi[j]; }, pn, [&](int i, T vi) {
                    T gs = T(0);
#pragma unroll
                    for (int s2 = 0; s2 < ND; ++s2) {
                        if (s2 == C) continue;
                        const int j = min(max(i + slot_off<ND>(s2, J.sx, J.sxy), 0), n - 1);
                        gs += Ad[s2][i] * (Mi[j] * (ta * Pk[j] + tw * (Rk[j] - ta * Vk[j])));
                    }
                    const T si = Rk[i] - ta * Vk[i];
                    const T xi = X[i] + Mi[i] * ((ta * Pk[i] + tw * si) - gs);
                    const T ri = si - tw * Tt[i];
                    const T pi = pn(i);
                    const T hi = Rh[i];
                    x[i] = xi;
                    rn[i] = ri;
                    pnv[i] = pi;
                    vn[i] = vi;
                    q[0] += (double)hi * vi;
                    q[1] += (double)ri * ri;
                });
                done = true;
            }
        }
        if (!done)
        for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
            int idx[NC];
            T y[NC], g[ND];
            T pi = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int j = ring_row<ND>(i, c, J.sx, J.sxy, n);
                idx[c] = j;
                const T sj = Rk[j] - ta * Vk[j];
                const T pc = (sj - tw * Tt[j]) + tb * (Pk[j] - tw * Vk[j]);
                if (c == RG.nb[C][C]) pi = pc;
                y[c] = Mi[j] * pc;
#pragma unroll
                for (int s2 = 0; s2 < ND; ++s2)
                    if (c == RG.nb[s2][C]) g[s2] = ta * Pk[j] + tw * sj;
            }
            const T vi = ring_amf<ND, T>(Ad, Mi, idx, y);
            // x += M (alpha p_k + omega s), the product at row i only
            T gs = T(0);
#pragma unroll
            for (int s2 = 0; s2 < ND; ++s2)
                if (s2 != C) gs += Ad[s2][i] * (Mi[idx[RG.nb[s2][C]]] * g[s2]);
            const T si = Rk[i] - ta * Vk[i];
            const T xi = X[i] + Mi[i] * (g[C] - gs);
            const T ri = si - tw * Tt[i];
            const T hi = Rh[i];
            x[i] = xi;
            rn[i] = ri;
            pnv[i] = pi;
            vn[i] = vi;
            q[0] += (double)hi * vi;
            q[1] += (double)ri * ri;
        }
    } else
    for (int i = i0 + threadIdx.x; i < i1; i += 2 * TILE) {
        const bool two = i + TILE < i1;
        const int i2 = two ? i + TILE : i;
        T xv[2], rv[2], pv[2], vv[2], hv[2];
        const int iv[2] = {i, i2};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int ii = iv[u];
            const T si = rk[ii] - ta * vk[ii];
            xv[u] = fmat(mi[ii], fmat(ta, pkv[ii], tw * si), x[ii]);     // x + M (alpha p + omega s)
            rv[u] = si - tw * t[ii];
            pv[u] = pnext(ii);
            vv[u] = kstencil<ND, T>(A, n, ii, J.sx, J.sxy, [&](int j) { return mi[j] * pnext(j); });
            hv[u] = rh[ii];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !two) break;
            const int ii = iv[u];
            x[ii] = xv[u];
            rn[ii] = rv[u];
            pnv[ii] = pv[u];
            vn[ii] = vv[u];
            q[0] += (double)hv[u] * vv[u];
            q[1] += (double)rv[u] * rv[u];
        }
    }
    const int off[2] = {poff(J, pn, PS_Q), poff(J, pn, PS_RR)};
    put_partials<2>(q, J.part, off, tl.t);
}

// B(k) and A(k) kernels.  One sweep: k_bicg_b / k_bicg_a.  Two sweeps,
// FP64: k_bicg2_b64 / k_bicg2_a64.  On 7-point systems (gathers only) they
// may use up to two waves' worth of registers per lane, so that a row's
// 60-180 gathers are issued together rather than in a chain of round trips;
// on 5-point systems (staged through LDS) the registers of four waves per
// SIMD (127 and 96 VGPRs instead of 215 and 145): four workgroups per CU,
// every workgroup of a 500x300 launch resident at once (the two-wave form
// left 10 of 74 per XCD for a second round), measured faster at 500x300
// (+4 %) and in the 64-cavity batch (+21 %); the 7-point pair lost 3 % with
// four.  k_bicg2_b32 / k_bicg2_a32 (FP32 inner solves) take the default.
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_bicg_b(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_b_body<ND, 1, T>(jobs, tiles, kbase, koff); }
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_bicg_a(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_a_body<ND, 1, T>(jobs, tiles, kbase, koff); }
// one sweep on 7-point systems whose tiles all go through LDS (stage1_amf7):
// kernels of their own, so that the gathering kernels keep their register
// budget and these theirs (72 VGPRs in the A kernel against 166)
template <class T>
__global__ __launch_bounds__(TILE) void k_bicg_b1s(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_b_body<7, 1, T, true>(jobs, tiles, kbase, koff); }
template <class T>
__global__ __launch_bounds__(TILE) void k_bicg_a1s(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_a_body<7, 1, T, true>(jobs, tiles, kbase, koff); }
template <int ND>
__global__ void k_bicg2_b64(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff);
template <int ND>
__global__ void k_bicg2_a64(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff);
template <>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(1, 4)))
void k_bicg2_b64<5>(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_b_body<5, 2, double>(jobs, tiles, kbase, koff); }
template <>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(1, 4)))
void k_bicg2_a64<5>(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_a_body<5, 2, double>(jobs, tiles, kbase, koff); }
template <>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_bicg2_b64<7>(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_b_body<7, 2, double>(jobs, tiles, kbase, koff); }
template <>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_bicg2_a64<7>(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_a_body<7, 2, double>(jobs, tiles, kbase, koff); }
template <int ND>
__global__ __launch_bounds__(TILE) void k_bicg2_b32(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_b_body<ND, 2, float>(jobs, tiles, kbase, koff); }
template <int ND>
__global__ __launch_bounds__(TILE) void k_bicg2_a32(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff) { bicg_a_body<ND, 2, float>(jobs, tiles, kbase, koff); }

// ---- CG start, first kernel (mode as for BiCGSTAB): r = b - A x into r_(k&1),
// s_(k&1) = 0, p = 0; partials (r, r), (b, b)
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_cg_init_a(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k, int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RESTART) return;
    if (outer_idle(J)) return;
    const int n = J.n;
    const int pk = k & 1;
    auto A = G<T>(J.A);
    auto b = G<T>(J.b);
    auto x = G<T>(J.x), x0 = G<T>(J.x0);
    auto r = G<T>(pk ? J.rh : J.r), so = G<T>(pk ? J.p1 : J.p0), p = G<T>(J.t);
    double v[2] = {0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        T ri;
        if (mode == 0) {
            if (J.x0) {
                ri = b[i] - kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return x0[j]; });
                if (J.x0 != J.x) x[i] = x0[i];     // a guess written into x stays
            } else {
                ri = b[i];
                x[i] = T(0);
            }
        } else {
            ri = b[i] - kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
        }
        r[i] = ri;
        so[i] = T(0);
        p[i] = T(0);
        v[0] += (double)ri * ri;
        v[1] += (double)b[i] * b[i];
    }
    const int pm = (k + 1) & 1;
    const int off[2] = {poff(J, pm, PS_RR), poff(J, pm, PS_BB)};
    put_partials<2>(v, J.part, off, tl.t);
    mark_start(tl, J.st, k, mode);
}

// CG start, second kernel: w = A M r into w_(k&1); partials (r, M r), (w, M r)
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_cg_init_b(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int k, int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && !(J.st->status == K_RESTART && J.st->k0 == k)) return;
    if (outer_idle(J)) return;
    const int n = J.n;
    const int pk = k & 1;
    auto A = G<T>(J.A);
    auto mi = G<T>(J.minv);
    auto r = G<T>(pk ? J.rh : J.r), w = G<T>(pk ? J.v1 : J.v0);
    double v[2] = {0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const T wi = kstencil<ND, T>(A, n, i, J.sx, J.sxy, [&](int j) { return mi[j] * r[j]; });
        w[i] = wi;
        const T ui = mi[i] * r[i];
        v[0] += (double)r[i] * ui;
        v[1] += (double)wi * ui;
    }
    const int pm = (k + 1) & 1;
    const int off[2] = {poff(J, pm, PS_RHO), poff(J, pm, PS_TS)};
    put_partials<2>(v, J.part, off, tl.t);
}

// CG iteration k (one kernel)
template <int ND, class T>
__global__ __launch_bounds__(TILE) void k_cg(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, const int *kbase, int koff)
{
    const int k = (kbase ? *kbase : 0) + koff;
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (!active(J, k) || outer_idle(J)) return;
    KState *st = J.st;
    const int pk = k & 1, pm = (k + 1) & 1;
    const bool first = k == st->k0;
    // this kernel writes its partials into the parity-k slots while other
    // workgroups may still be reading; so it reads only parity k-1 slots and
    // takes gamma_{k-1}, alpha_{k-1} from the scalars workgroup 0 recorded
    double s4[4];
    {
        const int off[4] = {poff(J, pm, PS_RHO), poff(J, pm, PS_TS), poff(J, pm, PS_RR), poff(J, pm, PS_BB)};
        sum_partials<4>(J.part, off, J.ntile, s4);
    }
    if (!keep_going(J, tl, k, s4[2], s4[3])) return;
    const double gam = s4[0], del = s4[1];
    double alpha, beta = 0.0;
    if (first) {
        alpha = gam / del;
    } else {
        beta = gam / st->gamma[pm];
        alpha = gam / (del - beta * gam / st->alpha[pm]);
    }
    if (!(alpha > 0.0) || !finite(alpha) || !finite(beta)) {
        set_status(tl, st, finite(alpha) ? K_RESTART : K_NONFINITE, st->it_base + (k - st->k0), s4[2]);
        return;
    }
    if (tl.t == 0 && threadIdx.x == 0) {
        st->alpha[pk] = alpha;
        st->gamma[pk] = gam;
    }
    const T ta = (T)alpha, tb = (T)beta;
    const int n = J.n;
    auto A = G<T>(J.A);
    auto mi = G<T>(J.minv);
    auto rc = G<T>(pk ? J.rh : J.r), rn = G<T>(pk ? J.r : J.rh);
    auto wc = G<T>(pk ? J.v1 : J.v0), wn = G<T>(pk ? J.v0 : J.v1);
    auto so = G<T>(pk ? J.p1 : J.p0), sn = G<T>(pk ? J.p0 : J.p1);
    auto p = G<T>(J.t), x = G<T>(J.x);
    double v[3] = {0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        const T mii = mi[i], ri = rc[i];
        const T pi = mii * ri + tb * p[i];
        p[i] = pi;
        const T si = wc[i] + tb * so[i];
        sn[i] = si;
        x[i] = x[i] + ta * pi;
        const T rni = ri - ta * si;
        rn[i] = rni;
        const T wi = kstencil<ND, T>(A, n, i, J.sx, J.sxy,
                                     [&](int j) { return mi[j] * (rc[j] - ta * (wc[j] + tb * so[j])); });
        wn[i] = wi;
        const T un = mii * rni;
        v[0] += (double)rni * un;
        v[1] += (double)wi * un;
        v[2] += (double)rni * rni;
    }
    const int off[3] = {poff(J, pk, PS_RHO), poff(J, pk, PS_TS), poff(J, pk, PS_RR)};
    put_partials<3>(v, J.part, off, tl.t);
}

// ---- verification of a plain FP64 solve on the true residual b - A x (or
// x = 0 when ||b|| = 0); partials of ||b - A x||^2, sum(b - A x), sum(x)
template <int ND>
__global__ __launch_bounds__(TILE) void k_kfinish(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    const int status = J.st->status;
    if (status != K_CONVERGED && status != K_ZERO) return;
    const int n = J.n;
    auto A = G<double>(J.A);
    auto b = G<double>(J.b);
    auto x = G<double>(J.x);
    double v[3] = {0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        if (status == K_ZERO) {
            x[i] = 0.0;
        } else {
            const double rt = b[i] - kstencil<ND, double>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
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

// ---- mixed precision: FP64 iterative refinement around an FP32 solve.
// Residual sweep (mode 0: fresh start, x = x0 or 0; mode 1: keep x):
// r = b - A x in FP64, its FP32 copy into aux (the inner rhs); partials
// ||r||^2, ||b||^2, sum(r), sum(x).
template <int ND>
__global__ __launch_bounds__(TILE) void k_ir_resid(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles, int mode)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    if (mode == 1 && J.st->status != K_RUNNING) return;
    const int n = J.n;
    auto A = G<double>(J.A);
    auto b = G<double>(J.b);
    auto x = G<double>(J.x), x0 = G<double>(J.x0);
    auto r32 = G<float>(J.aux);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int i0 = tl.t * J.rpt, i1 = min(n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) {
        double ri, xi;
        if (mode == 0 && !J.x0) {
            ri = b[i];
            xi = 0.0;
            x[i] = 0.0;
        } else if (mode == 0) {
            ri = b[i] - kstencil<ND, double>(A, n, i, J.sx, J.sxy, [&](int j) { return x0[j]; });
            xi = x0[i];
            if (J.x0 != J.x) x[i] = xi;
        } else {
            ri = b[i] - kstencil<ND, double>(A, n, i, J.sx, J.sxy, [&](int j) { return x[j]; });
            xi = x[i];
        }
        r32[i] = (float)ri;
        v[0] += ri * ri;
        v[1] += b[i] * b[i];
        v[2] += ri;
        v[3] += xi;
    }
    const int off[4] = {poff(J, 0, PS_RR), poff(J, 0, PS_BB), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    put_partials<4>(v, J.part, off, tl.t);
}

// one workgroup per refinement: verdict on the FP64 residual of the sweep;
// the inner solve's iterations are added to the count
__global__ __launch_bounds__(TILE) void k_ir_decide(const KJob *__restrict__ jobs, int njobs, int mode, int max_outer)
{
    const KJob &J = jobs[blockIdx.x];
    KState *st = J.st;
    if (mode == 1 && st->status != K_RUNNING) return;
    const int off[4] = {poff(J, 0, PS_RR), poff(J, 0, PS_BB), poff(J, 0, PS_TS), poff(J, 0, PS_TT)};
    double tot[4];
    sum_partials<4>(J.part, off, J.ntile, tot);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            st->bb = tot[1];
            st->outer = 0;
            st->inner_total = 0;
            st->restarts = 0;
        } else {
            st->outer += 1;
            st->inner_total += J.partner->it;
        }
        st->rr = tot[0];
        st->tr2 = tot[0];
        st->tsum = tot[2];
        st->xsum = tot[3];
        st->it = st->inner_total;
        if (!finite(tot[0]) || !finite(st->bb)) st->status = K_NONFINITE;
        else if (st->bb == 0.0) st->status = K_ZERO;
        else if (tot[0] <= st->tol2 * st->bb) st->status = K_DONE;
        else if (st->outer >= max_outer || st->inner_total >= st->max_iter) st->status = K_FAILED;
        else {
            st->status = K_RUNNING;
            // the next inner solve reduces its right-hand side r only as far
            // as the FP64 target still needs, (0.3 tol ||b|| / ||r||)^2,
            // bounded by what FP32 reaches (1e-5, or tol when looser) and by
            // at least halving r
            const double need = 0.09 * st->tol2 * st->bb / tot[0];
            J.partner->tol2 = fmin(0.25, fmax(fmax(st->tol2, 1e-10), need));
        }
    }
}

// x += d (FP64 += FP32 correction) for refinements still running; x = 0 for
// a zero right-hand side
template <int ND>
__global__ __launch_bounds__(TILE) void k_ir_update(const KJob *__restrict__ jobs, const JTile *__restrict__ tiles)
{
    JTile tl;
    const KJob &J = job_of(jobs, tiles, tl);
    const int status = J.st->status;
    if (status != K_RUNNING && status != K_ZERO) return;
    auto x = G<double>(J.x);
    auto d = G<float>(J.t);
    const int i0 = tl.t * J.rpt, i1 = min(J.n, i0 + J.rpt);
    for (int i = i0 + threadIdx.x; i < i1; i += TILE) x[i] = status == K_ZERO ? 0.0 : x[i] + (double)d[i];
}

// the zero-rhs verdict of a refinement becomes final after k_ir_update
__global__ void k_ir_close(const KJob *__restrict__ jobs, int njobs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs && jobs[j].st->status == K_ZERO) jobs[j].st->status = K_DONE;
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

// rows [r0, r1) of the system; entry p of the CSR arrays goes to
// col[p - base], val[p - base] (base = row_ptr[r0] when the arrays hold only
// that block of rows, 0 when they hold the whole system)
template <int DIM>
__global__ __launch_bounds__(TILE) void k_csr_fill(const CaseDev *__restrict__ cd, int s, const int32_t *row_ptr,
                                                   int32_t *col, double *val, int r0, int r1, int base)
{
    constexpr int ND = 2 * DIM + 1;
    const Phys &P = cd->ph;
    const int n = P.nsys[s];
    const int row = r0 + blockIdx.x * TILE + threadIdx.x;
    if (row >= r1 || row >= n) return;
    int q[3];
    decode(row, P.sdim[s][0], P.sdim[s][1], q);
    const int sx = P.sdim[s][0], sxy = P.sdim[s][0] * P.sdim[s][1];
    const double *A = cd->A[s];
    int p = row_ptr[row] - base;
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

// ------------------------------------------ forward (probing) assembly
// The paper's second route to the same systems (Section 4, the forward
// method, eqs. 4.5-4.7): the discrete equation of every unknown is written
// as a residual Eq(phi) = A phi - b, so that b = -Eq(0) and the entry of
// column j in row i is Eq(e)_i - Eq(0)_i for a probe vector e that is 1 on
// every cell of j's colour (i mod 3, j mod 3[, k mod 3]) and 0 elsewhere: no
// two cells of one colour meet in a 5/7-point stencil, so 9 (2D) or 27 (3D)
// probes recover every entry.  Only the terms that change every step are
// probed; the constant part (transient, diffusion, wall conductances of the
// term-wise split) comes from the offline assembly.  No probe vector is
// stored: a row sees a probe only on its own stencil, where a colour is 1 on
// at most one slot, so each row evaluates its residual once at phi = 0 and
// once per in-domain slot with phi = 1 on that slot's cell -- the probes of
// the colours that meet its stencil; the others give Eq(0) again.  The
// residuals are written with face fluxes (upwind value times the advecting
// velocity), not with the coefficient rows of the stencil kernels above.

// upwind face flux: advecting velocity times the upstream value (eq. 3.28)
__device__ __forceinline__ double upw(double v, double left, double right)
{
    return v >= 0.0 ? v * left : v * right;
}

// momentum predictor (eq. 3.3), varying part: convection + drag - b; the
// form of eq. (2.6) as in k_asm_momentum (advecting velocity u/g~; drag,
// pressure gradient and force scaled)
template <int DIM>
__global__ __launch_bounds__(TILE) void k_fwd_momentum(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles)
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
    // advecting velocities on the faces of the control volume
    double vm[3], vp[3];
    bool in[ND];
    const int F = q[d] + 1;
    const double gf = 0.5 * (c.gl[clo] + c.gl[chi]);
    const double gt = P.mom1 ? fmax(gf, P.gfloor) : 1.0;
    const double gw = P.mom1 ? gf : 1.0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        if (ax == d) {
            const double uc = face_vel(P, vel, d, lo, F);
            vm[ax] = 0.5 * (face_vel(P, vel, d, lo, F - 1) + uc);
            vp[ax] = 0.5 * (uc + face_vel(P, vel, d, lo, F + 1));
        } else {
            vm[ax] = 0.5 * (face_vel(P, vel, ax, lo, q[ax]) + face_vel(P, vel, ax, hi, q[ax]));
            vp[ax] = 0.5 * (face_vel(P, vel, ax, lo, q[ax] + 1) + face_vel(P, vel, ax, hi, q[ax] + 1));
        }
        vm[ax] = vm[ax] / gt;
        vp[ax] = vp[ax] / gt;
        in[DIM - 1 - ax] = q[ax] >= 1;
        in[DIM + 1 + ax] = q[ax] <= P.sdim[d][ax] - 2;
    }
    in[DIM] = true;
    const double sol = 1.0 - gf;
    const double drag = gt * (P.nu * 180.0 * sol * sol / (P.lambda2 * P.lambda2 * (gf * gf * gf + P.eps)));
    double b = vel[d][row] * P.idt - gw * ((c.p[chi] - c.p[clo]) / (P.rho * P.h[d]));
    if (d == DIM - 1) {
        const double Tf = 0.5 * (c.T[clo] + c.T[chi]);
        const double Cf = 0.5 * (c.Cl[clo] + c.Cl[chi]);
        b += gw * (P.grav * (P.betaT * (Tf - P.Tref) + P.betaC * (Cf - P.Cref)));
    }
    // Eq(phi) on the stencil: phi[k] is the probe's value on slot k
    auto eq = [&](const double *phi) {
        double r = 0.0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax)
            r += (upw(vp[ax], phi[DIM], phi[DIM + 1 + ax]) - upw(vm[ax], phi[DIM - 1 - ax], phi[DIM])) * P.ih[ax];
        return r + drag * phi[DIM] - b;
    };
    double phi[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) phi[k] = 0.0;
    const double r0 = eq(phi);
    const double *Ac = c.Ac[d];
    double a[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        a[k] = 0.0;
        if (in[k]) {
            phi[k] = 1.0;
            a[k] = Ac[(size_t)k * n + row] + (eq(phi) - r0);
            phi[k] = 0.0;
        }
    }
    double *A = c.A[d];
#pragma unroll
    for (int k = 0; k < ND; ++k) A[(size_t)k * n + row] = a[k];
    const double mi = 1.0 / a[DIM];
    c.minv[d][row] = mi;
    c.b[d][row] = -r0;
    if (c.A32[d]) {
#pragma unroll
        for (int k = 0; k < ND; ++k) c.A32[d][(size_t)k * n + row] = (float)a[k];
        c.minv32[d][row] = (float)mi;
    }
}

// solute (eqs. 3.7-3.10: transient, convection and liquid diffusion of
// C_l = A_g C) and energy (eq. 3.11, varying part: convection) residuals
template <int DIM>
__global__ __launch_bounds__(TILE) void k_fwd_transport(const CaseDev *__restrict__ cases, const Tile *__restrict__ tiles,
                                                        int vel_src)
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
    const int stride[3] = {1, P.nx, P.nx * P.ny};
    double vm[3], vp[3], dm[3], dp[3], ag[ND];
    bool in[ND];
    const double gP = c.gl[ci];
    ag[DIM] = 1.0 / (1.0 - omk * (1.0 - gP));
    in[DIM] = true;
    double bT = c.T[ci] * P.idt;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        vm[ax] = face_vel(P, vel, ax, q, q[ax]);
        vp[ax] = face_vel(P, vel, ax, q, q[ax] + 1);
        const int sm = DIM - 1 - ax, sp = DIM + 1 + ax;
        in[sm] = q[ax] >= 1;
        in[sp] = q[ax] <= P.sdim[SC][ax] - 2;
        dm[ax] = dp[ax] = 0.0;
        ag[sm] = ag[sp] = 0.0;
        if (in[sm]) {
            const double g = c.gl[ci - stride[ax]];
            ag[sm] = 1.0 / (1.0 - omk * (1.0 - g));
            dm[ax] = P.Dl * (0.5 * (gP + g)) * P.ih2[ax];
        } else {
            const double U = wall_cond(P, 2 * ax, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax, t_new) / (P.rcp * P.h[ax]);
        }
        if (in[sp]) {
            const double g = c.gl[ci + stride[ax]];
            ag[sp] = 1.0 / (1.0 - omk * (1.0 - g));
            dp[ax] = P.Dl * (0.5 * (gP + g)) * P.ih2[ax];
        } else {
            const double U = wall_cond(P, 2 * ax + 1, P.h[ax]);
            if (U > 0.0) bT += U * wall_temp(P, 2 * ax + 1, t_new) / (P.rcp * P.h[ax]);
        }
    }
    const double bC = c.C[ci] * P.idt;
    // solute: phi is C on the stencil, the fluxes act on C_l = A_g C; walls
    // carry no flux (zero face velocity, zero diffusive flux)
    auto eqC = [&](const double *phi) {
        double r = phi[DIM] * P.idt - bC;
        const double lP = ag[DIM] * phi[DIM];
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const double lW = ag[DIM - 1 - ax] * phi[DIM - 1 - ax], lE = ag[DIM + 1 + ax] * phi[DIM + 1 + ax];
            r += (upw(vp[ax], lP, lE) - upw(vm[ax], lW, lP)) * P.ih[ax];
            r -= dp[ax] * (lE - lP) - dm[ax] * (lP - lW);
        }
        return r;
    };
    // energy: convection of T* (the constant part, with the walls, is in Ac)
    auto eqT = [&](const double *phi) {
        double r = -bT;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax)
            r += (upw(vp[ax], phi[DIM], phi[DIM + 1 + ax]) - upw(vm[ax], phi[DIM - 1 - ax], phi[DIM])) * P.ih[ax];
        return r;
    };
    double phi[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) phi[k] = 0.0;
    const double r0C = eqC(phi), r0T = eqT(phi);
    const double *AcT = c.Ac[ST];
    double aC[ND], aT[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        aC[k] = aT[k] = 0.0;
        if (in[k]) {
            phi[k] = 1.0;
            aC[k] = eqC(phi) - r0C;
            aT[k] = AcT[(size_t)k * n + ci] + (eqT(phi) - r0T);
            phi[k] = 0.0;
        }
    }
    double *AC = c.A[SC], *AT = c.A[ST];
#pragma unroll
    for (int k = 0; k < ND; ++k) { AC[(size_t)k * n + ci] = aC[k]; AT[(size_t)k * n + ci] = aT[k]; }
    c.b[SC][ci] = -r0C;
    c.b[ST][ci] = -r0T;
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

// ============================================================ launchers

#define GRID(n) dim3((unsigned)(n)), dim3(TILE)

void launch_asm_const(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) SOL_LAUNCH(k_asm_const<2>, GRID(nt), 0, s, c, t);
    else SOL_LAUNCH(k_asm_const<3>, GRID(nt), 0, s, c, t);
}
void launch_asm_momentum(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s, int fwd)
{
    if (nt <= 0) return;
    if (fwd) {
        if (dim == 2) SOL_LAUNCH(k_fwd_momentum<2>, GRID(nt), 0, s, c, t);
        else SOL_LAUNCH(k_fwd_momentum<3>, GRID(nt), 0, s, c, t);
        return;
    }
    if (dim == 2) SOL_LAUNCH(k_asm_momentum<2>, GRID(nt), 0, s, c, t);
    else SOL_LAUNCH(k_asm_momentum<3>, GRID(nt), 0, s, c, t);
}
void launch_asm_transport(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s, int fwd)
{
    if (nt <= 0) return;
    if (fwd) {
        if (dim == 2) SOL_LAUNCH(k_fwd_transport<2>, GRID(nt), 0, s, c, t, vel_src);
        else SOL_LAUNCH(k_fwd_transport<3>, GRID(nt), 0, s, c, t, vel_src);
        return;
    }
    if (dim == 2) SOL_LAUNCH(k_asm_transport<2>, GRID(nt), 0, s, c, t, vel_src);
    else SOL_LAUNCH(k_asm_transport<3>, GRID(nt), 0, s, c, t, vel_src);
}
void launch_div_rhs(int dim, const CaseDev *c, const Tile *t, int nt, int vel_src, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) SOL_LAUNCH(k_div_rhs<2>, GRID(nt), 0, s, c, t, vel_src);
    else SOL_LAUNCH(k_div_rhs<3>, GRID(nt), 0, s, c, t, vel_src);
}
void launch_case_mean(const CaseDev *c, const int32_t *cidx, int ncase, hipStream_t s)
{
    if (ncase <= 0) return;
    SOL_LAUNCH(k_case_mean, GRID(ncase), 0, s, c, cidx);
}
void launch_sub_mean(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    SOL_LAUNCH(k_sub_mean, GRID(nt), 0, s, c, t);
}
void launch_project(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    SOL_LAUNCH(k_project, GRID(nt), 0, s, c, t);
}
void launch_phase_commit(int dim, const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (dim == 2) SOL_LAUNCH(k_phase_commit<2>, GRID(nt), 0, s, c, t);
    else SOL_LAUNCH(k_phase_commit<3>, GRID(nt), 0, s, c, t);
}

template <int ND, class T>
static const void *iter_fn_t(int which, bool two, bool s1)
{
    constexpr bool f64 = sizeof(T) == 8;
    switch (which) {
    case KI_CG: return (const void *)&k_cg<ND, T>;
    case KI_BICG_A:
        if (ND == 7 && !two && s1) return (const void *)&k_bicg_a1s<T>;
        if (!two) return (const void *)&k_bicg_a<ND, T>;
        return f64 ? (const void *)&k_bicg2_a64<ND> : (const void *)&k_bicg2_a32<ND>;
    case KI_BICG_B:
        if (ND == 7 && !two && s1) return (const void *)&k_bicg_b1s<T>;
        if (!two) return (const void *)&k_bicg_b<ND, T>;
        return f64 ? (const void *)&k_bicg2_b64<ND> : (const void *)&k_bicg2_b32<ND>;
    }
    return nullptr;
}

const void *kiter_fn(int which, int nd, int fp32, bool two, bool s1)
{
    if (which >= KI_MG_PQ) return mg_fn(which, nd, fp32);
    if (nd == 5) return fp32 ? iter_fn_t<5, float>(which, two, false) : iter_fn_t<5, double>(which, two, false);
    return fp32 ? iter_fn_t<7, float>(which, two, s1) : iter_fn_t<7, double>(which, two, s1);
}

// iteration index base of graph-replayed chunks
__global__ void k_kbase_add(int *kbase, int m) { if (threadIdx.x == 0 && blockIdx.x == 0) *kbase += m; }
__global__ void k_kbase_set(int *kbase, int v) { if (threadIdx.x == 0 && blockIdx.x == 0) *kbase = v; }

const void *kbase_add_fn() { return (const void *)&k_kbase_add; }

void launch_kbase_set(int *kbase, int v, hipStream_t s)
{
    SOL_LAUNCH(k_kbase_set, dim3(1), dim3(64), 0, s, kbase, v);
}

// deterministic right-hand side for the tile-size tuner: +1, -1, +1, ...
// (0 for the last entry of an odd count), so its sum is exactly 0 and the
// singular Neumann pressure system stays consistent
template <class T>
__global__ void k_tune_rhs(T *b, int n)
{
    const int i = blockIdx.x * TILE + threadIdx.x;
    if (i < n) b[i] = ((n & 1) && i == n - 1) ? T(0) : ((i & 1) ? T(-1) : T(1));
}
void launch_tune_rhs(void *b, int fp32, int n, hipStream_t s)
{
    if (n <= 0) return;
    if (fp32) SOL_LAUNCH(k_tune_rhs<float>, dim3(ceil_div(n, TILE)), dim3(TILE), 0, s, (float *)b, n);
    else SOL_LAUNCH(k_tune_rhs<double>, dim3(ceil_div(n, TILE)), dim3(TILE), 0, s, (double *)b, n);
}

template <int ND, class T>
static void launch_init_nd(int kind, bool two, bool s1, const KJob *j, const JTile *t, int nt, int k, int mode,
                           size_t smem, hipStream_t s)
{
    if (kind == K_CG) {
        SOL_LAUNCH((k_cg_init_a<ND, T>), GRID(nt), 0, s, j, t, k, mode);
        SOL_LAUNCH((k_cg_init_b<ND, T>), GRID(nt), 0, s, j, t, k, mode);
        return;
    }
    SOL_LAUNCH((k_bicg_init<ND, T>), GRID(nt), 0, s, j, t, k, mode);
    if (two) SOL_LAUNCH((k_bicg_first<ND, 2, T>), dim3(nt), dim3(TILE), smem, s, j, t, k);
    else if constexpr (ND == 7) {
        if (s1) SOL_LAUNCH((k_bicg_first<7, 1, T, true>), dim3(nt), dim3(TILE), smem, s, j, t, k);
        else SOL_LAUNCH((k_bicg_first<ND, 1, T>), GRID(nt), 0, s, j, t, k);
    } else SOL_LAUNCH((k_bicg_first<ND, 1, T>), GRID(nt), 0, s, j, t, k);
}

void launch_kinit(int kind, int nd, int fp32, bool two, bool s1, const KJob *j, const JTile *t, int nt, int k,
                  int mode, size_t smem, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) {
        if (fp32) launch_init_nd<5, float>(kind, two, false, j, t, nt, k, mode, smem, s);
        else launch_init_nd<5, double>(kind, two, false, j, t, nt, k, mode, smem, s);
    } else {
        if (fp32) launch_init_nd<7, float>(kind, two, s1, j, t, nt, k, mode, smem, s);
        else launch_init_nd<7, double>(kind, two, s1, j, t, nt, k, mode, smem, s);
    }
}

void launch_kfinish(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) SOL_LAUNCH(k_kfinish<5>, GRID(nt), 0, s, j, t);
    else SOL_LAUNCH(k_kfinish<7>, GRID(nt), 0, s, j, t);
}
void launch_kdecide(const KJob *j, int njobs, hipStream_t s)
{
    if (njobs <= 0) return;
    SOL_LAUNCH(k_kdecide, dim3(njobs), dim3(TILE), 0, s, j, njobs);
}
void launch_ir_resid(int nd, const KJob *j, const JTile *t, int nt, int mode, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) SOL_LAUNCH(k_ir_resid<5>, GRID(nt), 0, s, j, t, mode);
    else SOL_LAUNCH(k_ir_resid<7>, GRID(nt), 0, s, j, t, mode);
}
void launch_ir_decide(const KJob *j, int njobs, int mode, int max_outer, hipStream_t s)
{
    if (njobs <= 0) return;
    SOL_LAUNCH(k_ir_decide, dim3(njobs), dim3(TILE), 0, s, j, njobs, mode, max_outer);
}
void launch_ir_update(int nd, const KJob *j, const JTile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    if (nd == 5) SOL_LAUNCH(k_ir_update<5>, GRID(nt), 0, s, j, t);
    else SOL_LAUNCH(k_ir_update<7>, GRID(nt), 0, s, j, t);
}
void launch_ir_close(const KJob *j, int njobs, hipStream_t s)
{
    if (njobs <= 0) return;
    SOL_LAUNCH(k_ir_close, dim3(ceil_div(njobs, 64)), dim3(64), 0, s, j, njobs);
}
void launch_guess(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    SOL_LAUNCH(k_guess, GRID(nt), 0, s, c, t);
}
void launch_guess_mom(const CaseDev *c, const Tile *t, int nt, hipStream_t s)
{
    if (nt <= 0) return;
    SOL_LAUNCH(k_guess_mom, GRID(nt), 0, s, c, t);
}
void launch_hist_reset(const CaseDev *c, int ncase, hipStream_t s)
{
    if (ncase <= 0) return;
    SOL_LAUNCH(k_hist_reset, dim3(ceil_div(ncase, 64)), dim3(64), 0, s, c, ncase);
}
void launch_case_stats(const CaseDev *c, const int32_t *cidx, int ncase, hipStream_t s)
{
    if (ncase <= 0) return;
    SOL_LAUNCH(k_case_stats, dim3(ncase), dim3(TILE), 0, s, c, cidx);
}
void launch_csr(int dim, const CaseDev *cd, int s, int n, int32_t *cnt, int32_t *row_ptr, int32_t *col,
                double *val, int build_pattern, hipStream_t st)
{
    if (n <= 0) return;
    const int nb = ceil_div(n, TILE);
    if (build_pattern) {
        if (dim == 2) SOL_LAUNCH(k_csr_count<2>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
        else SOL_LAUNCH(k_csr_count<3>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
        SOL_LAUNCH(k_scan, dim3(1), dim3(1024), 0, st, cnt, row_ptr, n);
    }
    if (dim == 2) SOL_LAUNCH(k_csr_fill<2>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val, 0, n, 0);
    else SOL_LAUNCH(k_csr_fill<3>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val, 0, n, 0);
}
void launch_csr_pattern(int dim, const CaseDev *cd, int s, int n, int32_t *cnt, int32_t *row_ptr, hipStream_t st)
{
    if (n <= 0) return;
    const int nb = ceil_div(n, TILE);
    if (dim == 2) SOL_LAUNCH(k_csr_count<2>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
    else SOL_LAUNCH(k_csr_count<3>, dim3(nb), dim3(TILE), 0, st, cd, s, cnt);
    SOL_LAUNCH(k_scan, dim3(1), dim3(1024), 0, st, cnt, row_ptr, n);
}
void launch_csr_rows(int dim, const CaseDev *cd, int s, int r0, int r1, const int32_t *row_ptr, int base,
                     int32_t *col, double *val, hipStream_t st)
{
    if (r1 <= r0) return;
    const int nb = ceil_div(r1 - r0, TILE);
    if (dim == 2) SOL_LAUNCH(k_csr_fill<2>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val, r0, r1, base);
    else SOL_LAUNCH(k_csr_fill<3>, dim3(nb), dim3(TILE), 0, st, cd, s, row_ptr, col, val, r0, r1, base);
}
void launch_fill(double *x, double v, int n, hipStream_t s)
{
    if (n <= 0) return;
    SOL_LAUNCH(k_fill, dim3(ceil_div(n, TILE)), dim3(TILE), 0, s, x, v, n);
}
void launch_set_status(KState *st, int n, int status, hipStream_t s)
{
    if (n <= 0) return;
    SOL_LAUNCH(k_set_status, dim3(ceil_div(n, 64)), dim3(64), 0, s, st, n, status);
}

}  // namespace sol
