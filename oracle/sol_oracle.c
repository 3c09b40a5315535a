/*
 * sol_oracle.c -- plain, slow, FP64 CPU reference ("oracle") of one time step
 * of the fully decoupled operator-splitting solidification / macro-segregation
 * scheme (arXiv 2303.10783).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * What is computed (paper references are to sections / equations / Table 1 /
 * Algorithm 1 of the paper):
 *   - staggered uniform grid, Section 3 "Spatial discretization": u on the
 *     west-east faces, v on the south-north faces (w on bottom-top faces in
 *     3D), scalars at cell centres;  unknowns ordered x fastest (Section 4,
 *     eq. 4.2);  only interior faces carry velocity unknowns, wall faces are
 *     impermeable (velocity 0).
 *   - central fully implicit diffusion, eq. (3.26); implicit first-order upwind
 *     convection in flux form, eqs. (3.27)-(3.28) and the coefficient rows of
 *     eq. (4.4);
 *   - momentum predictor eq. (3.3) (momentum form 2.7, or the minimal
 *     model's form 2.6 on request) with Carman-Kozeny drag eq. (2.8) and
 *     Boussinesq force eq. (2.9);
 *   - pressure-correction Poisson eq. (3.4) and projection eq. (3.5);
 *   - matrix-based solute transport eqs. (3.6), (3.8)-(3.10), with the
 *     liquid diffusion of eq. (3.7) when D_l > 0;
 *   - split energy equation eqs. (3.11)-(3.12), liquidus eq. (3.13), lever
 *     rule eq. (3.14), quadratic eqs. (3.15)-(3.16), eutectic rule (text after
 *     eq. 3.16), concentration update eqs. (3.17)-(3.18);
 *   - the time loop of Algorithm 1, steps 1-8.
 * The paper names no linear solver: Jacobi-preconditioned CG is used for the
 * (symmetric) pressure system and Jacobi-preconditioned BiCGSTAB for the
 * transport systems, both stopped on the true residual.
 *
 * Readings of points the paper leaves open are listed where they are used
 * (tag "reading:").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { SYS_U = 0, SYS_V = 1, SYS_W = 2, SYS_P = 3, SYS_C = 4, SYS_T = 5, NSYS = 6 };
enum { TH_ADIABATIC = 0, TH_ROBIN = 1, TH_DIRICHLET = 2 };
enum { VEL_NOSLIP = 0, VEL_FREESLIP = 1 };
enum { MOM_PLAIN = 0, MOM_MINIMAL = 1 };   /* momentum form: eq. (2.7) / eq. (2.6) */

typedef struct {
    int32_t dim, nx, ny, nz;
    double lx, ly, lz;
    /* alloy */
    double rho, mu, cp, kcond, latent, beta_T, beta_C, lambda2;
    double T_m, m_sp, k_p, C_e, T_ref, C_ref, grav, darcy_eps;
    /* walls, order W E S N B T */
    int32_t thermal[6];
    double hc[6], T_ext[6], T_wall0[6], T_ramp[6];
    int32_t velocity[6];
    /* numerics */
    double dt, tol_p, tol_t;
    int32_t max_iter;
    /* 1 = use the printed order A_g*A_con (row scaling) for the solute
       matrix instead of A_con*A_g; only for a test that shows its solute
       conservation defect */
    int32_t literal_ag_order;
    /* liquid solute diffusivity D_l of eq. (3.7); 0 = the minimal model */
    double D_l;
    /* momentum form of the predictor: MOM_PLAIN, eq. (2.7) (the form the
       scheme's eq. 3.3 discretises), or MOM_MINIMAL, eq. (2.6) */
    int32_t mom_form;
} oc_case;

typedef struct {
    double *u, *v, *w, *p, *T, *C, *gl, *Cl, *Cs;
    int64_t step; /* completed steps; time = step * dt */
} oc_fields;

typedef struct {
    int32_t iters[NSYS];
    double rel_resid[NSYS];   /* final true ||b-Ax|| / ||b|| per system */
    double sum_resid[NSYS];   /* sum of the final true residual vector   */
    double sum_C;             /* sum of C^{n+1}                           */
    double sum_H;             /* sum of T^{n+1} + (L/c_p) g^{n+1}         */
    double wall_flux;         /* sum over cooled wall cells of
                                 U/(rho c_p h) (T*_P - T_ext)             */
    double div_star;          /* ||D u*||_2                               */
    double div_new;           /* ||D u^{n+1}||_2                          */
    double poisson_resid;     /* ||r_p||_2 of the pressure solve          */
} oc_stats;

/* simple CSR container owned by the oracle */
typedef struct {
    int n, nnz;
    int *row_ptr, *col;
    double *val, *rhs;
} oc_csr;

static int g_threads = 1;
void oc_set_threads(int n) { g_threads = n > 0 ? n : 1; }

/* ------------------------------------------------------------------ grid */

static double h_of(const oc_case *c, int a)
{
    if (a == 0) return c->lx / c->nx;
    if (a == 1) return c->ly / c->ny;
    return c->lz / c->nz;
}

static void cell_dims(const oc_case *c, int n[3])
{
    n[0] = c->nx; n[1] = c->ny; n[2] = (c->dim == 3) ? c->nz : 1;
}

/* grid of the unknowns of a system: velocity component d lives on the
   interior d-faces, so its extent along d is one less than the cell count */
void oc_sys_dims(const oc_case *c, int sys, int d[3])
{
    cell_dims(c, d);
    if (sys == SYS_U) d[0] -= 1;
    if (sys == SYS_V) d[1] -= 1;
    if (sys == SYS_W) d[2] -= 1;
    if (sys == SYS_W && c->dim != 3) { d[0] = d[1] = d[2] = 0; }
    if (d[0] < 0) d[0] = 0;
    if (d[1] < 0) d[1] = 0;
    if (d[2] < 0) d[2] = 0;
}

int oc_sys_rows(const oc_case *c, int sys)
{
    int d[3];
    oc_sys_dims(c, sys, d);
    return d[0] * d[1] * d[2];
}

static int lin(const int n[3], int i, int j, int k) { return i + n[0] * (j + n[1] * k); }

/* velocity component a on the a-face with face number F along a (0..n_a),
   other coordinates = cell coordinates q[]; wall faces carry 0 */
static double face_vel(const oc_case *c, double *const vel[3], int a, const int q[3], int F)
{
    int n[3], d[3], r[3];
    cell_dims(c, n);
    if (F <= 0 || F >= n[a]) return 0.0;
    d[0] = n[0]; d[1] = n[1]; d[2] = n[2];
    d[a] -= 1;
    r[0] = q[0]; r[1] = q[1]; r[2] = q[2];
    r[a] = F - 1;
    return vel[a][lin(d, r[0], r[1], r[2])];
}

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* One assembled row: diagonal, neighbour coefficients along each axis and
   side (side 0 = minus/back, side 1 = plus/front), presence flags, rhs. */
typedef struct {
    double diag, nb[3][2], rhs;
    int has[3][2];
} row_t;

static void row_clear(row_t *r)
{
    memset(r, 0, sizeof(*r));
}

/* Write rows into CSR with ascending columns:
   [-d0*d1, -d0, -1, 0, +1, +d0, +d0*d1]; in-domain neighbours only; an entry
   whose value happens to be zero is kept (structural). */
static void csr_put(oc_csr *m, const int d[3], int row, const row_t *r, int *pos)
{
    int p = *pos;
    const int off[3] = {1, d[0], d[0] * d[1]};
    for (int a = 2; a >= 0; --a)
        if (r->has[a][0]) { m->col[p] = row - off[a]; m->val[p] = r->nb[a][0]; ++p; }
    m->col[p] = row; m->val[p] = r->diag; ++p;
    for (int a = 0; a < 3; ++a)
        if (r->has[a][1]) { m->col[p] = row + off[a]; m->val[p] = r->nb[a][1]; ++p; }
    m->rhs[row] = r->rhs;
    m->row_ptr[row + 1] = p;
    *pos = p;
}

/* --------------------------------------------------- upwind convection row
   Flux-form first-order upwind across one axis of a control volume whose
   minus/plus faces carry the advecting velocities vm / vp (eq. 3.28 and the
   coefficient triple of eq. 4.4):
       [ -max(vm,0) ; max(vp,0) - min(vm,0) ; min(vp,0) ] / h              */
static void upwind(double vm, double vp, double h, double *cw, double *cp, double *ce)
{
    *cw = -dmax(vm, 0.0) / h;
    *cp = (dmax(vp, 0.0) - dmin(vm, 0.0)) / h;
    *ce = dmin(vp, 0.0) / h;
}

/* Carman-Kozeny drag coefficient (mu/rho) K^{-1}, eq. (2.8);
   reading: g^3 regularised by darcy_eps so that K^{-1} stays finite in solid */
static double darcy(const oc_case *c, double g)
{
    double nu = c->mu / c->rho;
    return nu * 180.0 * (1.0 - g) * (1.0 - g) / (c->lambda2 * c->lambda2 * (g * g * g + c->darcy_eps));
}

/* ------------------------------------------------ momentum predictor, eq. (3.3)
   System for velocity component d on the interior d-faces.
     A = I/dt + Conv(u^n) - nu Lap + (mu/rho) K^{-1}
     b = u^n/dt - (1/rho) d p^n / dx_d + f_d
   reading: flux-form upwind with the advecting velocity on each face of the
   face-centred control volume taken as the arithmetic mean of the two
   nearest level-n velocities of that component;  no-slip walls tangential to
   the unknown act through a half-cell ghost (2 nu / h^2 on the diagonal);
   free-slip walls carry no shear; a wall-normal neighbour is a Dirichlet 0;
   Boussinesq force on the vertical component only, hydrostatic part dropped,
   T and C_l at level n averaged onto the face.
   Momentum form (2.6) (mom_form = MOM_MINIMAL): the same predictor with the
   advecting velocity u/g_l, the pressure gradient, the drag and the force
   multiplied by g_l:
     A = I/dt + Conv(u^n / g~) - nu Lap + (mu/rho) g~ K^{-1}(g)
     b = u^n/dt - (g/rho) d p^n / dx_d + g f_d
   readings: g is g_l^n on the face, the mean of its two cells (as for the
   drag of eq. 2.8);  g~ = max(g, darcy_eps^(1/3)), the liquid fraction below
   which the regularisation of g^3 in eq. (2.8) dominates, so that 1/g~
   stays finite and the drag g~ K^{-1} stays large in solid cells (with g
   itself it would vanish there);  the pressure correction and the
   projection, eqs. (3.4)-(3.5), are unchanged, so a steady state (phi = 0)
   satisfies the discrete (2.6). */
static void assemble_momentum(const oc_case *c, const oc_fields *f, int d, oc_csr *m)
{
    int n[3], sd[3];
    cell_dims(c, n);
    oc_sys_dims(c, d, sd);
    double *const vel[3] = {f->u, f->v, f->w};
    const double nu = c->mu / c->rho;
    const int vert = c->dim - 1;
    const int minimal = c->mom_form == MOM_MINIMAL;
    const double gfloor = cbrt(c->darcy_eps);
    int pos = 0;
    m->row_ptr[0] = 0;
    for (int k = 0; k < sd[2]; ++k)
    for (int j = 0; j < sd[1]; ++j)
    for (int i = 0; i < sd[0]; ++i) {
        int q[3] = {i, j, k};
        int row = lin(sd, i, j, k);
        int F = q[d] + 1;                 /* face number along d */
        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
        lo[d] = F - 1; hi[d] = F;         /* the two cells sharing the face */
        int clo = lin(n, lo[0], lo[1], lo[2]);
        int chi = lin(n, hi[0], hi[1], hi[2]);
        double gf = 0.5 * (f->gl[clo] + f->gl[chi]);
        double gt = minimal ? dmax(gf, gfloor) : 1.0;   /* g~ of form (2.6) */
        double gw = minimal ? gf : 1.0;                 /* g on p and f   */
        row_t r;
        row_clear(&r);
        for (int a = 0; a < c->dim; ++a) {
            double h = h_of(c, a);
            double cw, cp, ce;
            if (a == d) {
                /* neighbours: faces F-1 and F+1 along d */
                double vm = 0.5 * (face_vel(c, vel, d, lo, F - 1) + face_vel(c, vel, d, lo, F));
                double vp = 0.5 * (face_vel(c, vel, d, lo, F) + face_vel(c, vel, d, lo, F + 1));
                upwind(vm / gt, vp / gt, h, &cw, &cp, &ce);
                r.has[a][0] = (q[a] >= 1);
                r.has[a][1] = (q[a] <= sd[a] - 2);
                r.diag += 2.0 * nu / (h * h) + cp;
                if (r.has[a][0]) r.nb[a][0] = -nu / (h * h) + cw;
                if (r.has[a][1]) r.nb[a][1] = -nu / (h * h) + ce;
            } else {
                /* tangential neighbours; advecting a-velocity on the
                   control-volume faces = mean over the two cells lo/hi */
                double vm = 0.5 * (face_vel(c, vel, a, lo, q[a]) + face_vel(c, vel, a, hi, q[a]));
                double vp = 0.5 * (face_vel(c, vel, a, lo, q[a] + 1) + face_vel(c, vel, a, hi, q[a] + 1));
                upwind(vm / gt, vp / gt, h, &cw, &cp, &ce);
                r.diag += cp;
                for (int s = 0; s < 2; ++s) {
                    int exists = s == 0 ? (q[a] >= 1) : (q[a] <= sd[a] - 2);
                    r.has[a][s] = exists;
                    if (exists) {
                        r.diag += nu / (h * h);
                        r.nb[a][s] = -nu / (h * h) + (s == 0 ? cw : ce);
                    } else if (c->velocity[2 * a + s] == VEL_NOSLIP) {
                        r.diag += 2.0 * nu / (h * h);
                    }
                }
            }
        }
        r.diag += 1.0 / c->dt + gt * darcy(c, gf);
        r.rhs = vel[d][row] / c->dt - gw * ((f->p[chi] - f->p[clo]) / (c->rho * h_of(c, d)));
        if (d == vert) {
            double Tf = 0.5 * (f->T[clo] + f->T[chi]);
            double Cf = 0.5 * (f->Cl[clo] + f->Cl[chi]);
            /* f = g(1 - beta_T (T - T_ref) - beta_C (C_l - C_ref)) along -z:
               vertical component without the hydrostatic part */
            r.rhs += gw * (c->grav * (c->beta_T * (Tf - c->T_ref) + c->beta_C * (Cf - c->C_ref)));
        }
        csr_put(m, sd, row, &r, &pos);
    }
    m->nnz = pos;
}

/* divergence of a face field at cell q: sum_a (v_{a,+} - v_{a,-}) / h_a */
static double cell_div(const oc_case *c, double *const vel[3], const int q[3])
{
    double s = 0.0;
    for (int a = 0; a < c->dim; ++a)
        s += (face_vel(c, vel, a, q, q[a] + 1) - face_vel(c, vel, a, q, q[a])) / h_of(c, a);
    return s;
}

/* ------------------------------------------- pressure correction, eq. (3.4)
   (-L) phi = -(rho/dt) D u*,  L = D G: the 5/7-point Laplacian with
   homogeneous Neumann walls.  reading: the rhs is made consistent by removing
   its mean (the operator is singular). */
static void assemble_poisson(const oc_case *c, double *const ustar[3], oc_csr *m)
{
    int n[3];
    cell_dims(c, n);
    int pos = 0;
    m->row_ptr[0] = 0;
    for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
    for (int i = 0; i < n[0]; ++i) {
        int q[3] = {i, j, k};
        row_t r;
        row_clear(&r);
        for (int a = 0; a < c->dim; ++a) {
            double h = h_of(c, a);
            for (int s = 0; s < 2; ++s) {
                int exists = s == 0 ? (q[a] >= 1) : (q[a] <= n[a] - 2);
                r.has[a][s] = exists;
                if (exists) { r.diag += 1.0 / (h * h); r.nb[a][s] = -1.0 / (h * h); }
            }
        }
        r.rhs = -(c->rho / c->dt) * cell_div(c, ustar, q);
        csr_put(m, n, lin(n, i, j, k), &r, &pos);
    }
    m->nnz = pos;
    double mean = 0.0;
    for (int i = 0; i < m->n; ++i) mean += m->rhs[i];
    mean /= (double)m->n;
    for (int i = 0; i < m->n; ++i) m->rhs[i] -= mean;
}

/* ------------------------------- solute transport, eqs. (3.6), (3.8)-(3.10)
   (I/dt + A_con(u^{n+1}) A_g) C^{n+1} = C^n / dt,
   (A_g)_jj = 1 / (1 - (1 - k_p)(1 - g_l,j^n)).
   reading: C_l^{n+1} = A_g C^{n+1} substituted into the convection term gives
   A_con A_g (column scaling); the printed A_g*A_con (row scaling) is kept
   behind literal_ag_order for a test.  Flux-form upwind with the face
   velocities u^{n+1}; walls carry no flux.
   Liquid diffusion (eq. 3.7, the A_lap term of eq. 3.9): the diffusive flux
   g_l^n D_l grad C_l^{n+1} across a face, with g_l on the face the mean of
   its two cells (reading, as for the drag), C_l = A_g C substituted as for
   convection (columns scaled); zero flux through walls; D_l = 0 is the
   minimal model. */
static void assemble_solute(const oc_case *c, const oc_fields *f, double *const unew[3], oc_csr *m)
{
    int n[3];
    cell_dims(c, n);
    int pos = 0;
    m->row_ptr[0] = 0;
    const int off[3] = {1, n[0], n[0] * n[1]};
    for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
    for (int i = 0; i < n[0]; ++i) {
        int q[3] = {i, j, k};
        int row = lin(n, i, j, k);
        row_t r;
        row_clear(&r);
        double agP = 1.0 / (1.0 - (1.0 - c->k_p) * (1.0 - f->gl[row]));
        double conv_diag = 0.0, dif_diag = 0.0;
        for (int a = 0; a < c->dim; ++a) {
            double h = h_of(c, a);
            double vm = face_vel(c, unew, a, q, q[a]);
            double vp = face_vel(c, unew, a, q, q[a] + 1);
            double cw, cp, ce;
            upwind(vm, vp, h, &cw, &cp, &ce);
            conv_diag += cp;
            r.has[a][0] = (q[a] >= 1);
            r.has[a][1] = (q[a] <= n[a] - 2);
            for (int s = 0; s < 2; ++s) {
                if (!r.has[a][s]) continue;
                int nb = row + (s == 0 ? -off[a] : off[a]);
                double agN = 1.0 / (1.0 - (1.0 - c->k_p) * (1.0 - f->gl[nb]));
                double gface = 0.5 * (f->gl[row] + f->gl[nb]);
                double dcoef = c->D_l * gface / (h * h);
                double cf = ((s == 0) ? cw : ce) - dcoef;
                dif_diag += dcoef;
                r.nb[a][s] = c->literal_ag_order ? agP * cf : cf * agN;
            }
        }
        r.diag = 1.0 / c->dt + (conv_diag + dif_diag) * agP;
        r.rhs = f->C[row] / c->dt;
        csr_put(m, n, row, &r, &pos);
    }
    m->nnz = pos;
}

/* series conductance of a cooled wall seen from the cell centre:
   convective film (h) in series with the half cell (h_a / (2 k));
   a prescribed wall temperature is the limit h -> infinity */
static double wall_U(const oc_case *c, int face, double h)
{
    if (c->thermal[face] == TH_ROBIN) return 1.0 / (1.0 / c->hc[face] + h / (2.0 * c->kcond));
    if (c->thermal[face] == TH_DIRICHLET) return 2.0 * c->kcond / h;
    return 0.0;
}

static double wall_T(const oc_case *c, int face, double t)
{
    if (c->thermal[face] == TH_DIRICHLET) return c->T_wall0[face] - c->T_ramp[face] * t;
    return c->T_ext[face];
}

/* ------------------------------------ energy, first split step, eq. (3.11)
   (I/dt + A_con(u^{n+1}) - alpha Lap) T* = T^n/dt + wall terms,
   alpha = k/(rho c_p).  Cooled walls: q = U (T_P - T_ext), i.e.
   U/(rho c_p h) on the diagonal and U T_ext/(rho c_p h) in the rhs;
   adiabatic walls: nothing.  t_new = time level n+1 (for T(t) walls). */
static void assemble_energy(const oc_case *c, const oc_fields *f, double *const unew[3], double t_new, oc_csr *m)
{
    int n[3];
    cell_dims(c, n);
    const double alpha = c->kcond / (c->rho * c->cp);
    int pos = 0;
    m->row_ptr[0] = 0;
    for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
    for (int i = 0; i < n[0]; ++i) {
        int q[3] = {i, j, k};
        int row = lin(n, i, j, k);
        row_t r;
        row_clear(&r);
        r.rhs = f->T[row] / c->dt;
        r.diag = 1.0 / c->dt;
        for (int a = 0; a < c->dim; ++a) {
            double h = h_of(c, a);
            double vm = face_vel(c, unew, a, q, q[a]);
            double vp = face_vel(c, unew, a, q, q[a] + 1);
            double cw, cp, ce;
            upwind(vm, vp, h, &cw, &cp, &ce);
            r.diag += cp;
            for (int s = 0; s < 2; ++s) {
                int exists = s == 0 ? (q[a] >= 1) : (q[a] <= n[a] - 2);
                r.has[a][s] = exists;
                if (exists) {
                    r.diag += alpha / (h * h);
                    r.nb[a][s] = -alpha / (h * h) + (s == 0 ? cw : ce);
                } else {
                    int face = 2 * a + s;
                    double U = wall_U(c, face, h);
                    if (U > 0.0) {
                        r.diag += U / (c->rho * c->cp * h);
                        r.rhs += U * wall_T(c, face, t_new) / (c->rho * c->cp * h);
                    }
                }
            }
        }
        csr_put(m, n, row, &r, &pos);
    }
    m->nnz = pos;
}

/* ------------------------------------------------------------ linear algebra */

static void spmv(const oc_csr *m, const double *x, double *y)
{
    int i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (i = 0; i < m->n; ++i) {
        double s = 0.0;
        for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p) s += m->val[p] * x[m->col[p]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    int i;
#pragma omp parallel for num_threads(g_threads) schedule(static) reduction(+ : s)
    for (i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void true_residual(const oc_csr *m, const double *x, double *r)
{
    spmv(m, x, r);
    for (int i = 0; i < m->n; ++i) r[i] = m->rhs[i] - r[i];
}

static double diag_of(const oc_csr *m, int i)
{
    for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p)
        if (m->col[p] == i) return m->val[p];
    return 0.0;
}

/* Jacobi-preconditioned conjugate gradients for the symmetric pressure
   system; stops when the true residual satisfies ||b - A x|| <= tol ||b||.
   b = 0 gives x = 0.  Returns iterations, or -1 when max_iter is reached.
   On return rres = the true residual vector. */
int oc_pcg(const oc_csr *m, double *x, double tol, int max_iter, double *rres, double *relres)
{
    int n = m->n;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *minv = malloc(sizeof(double) * n);
    int it = 0, ret = 0;
    double bn = sqrt(dot(n, m->rhs, m->rhs));
    if (bn == 0.0) {
        for (int i = 0; i < n; ++i) { x[i] = 0.0; rres[i] = 0.0; }
        *relres = 0.0;
        goto done;
    }
    for (int i = 0; i < n; ++i) minv[i] = 1.0 / diag_of(m, i);
    true_residual(m, x, r);
    for (;;) {
        if (sqrt(dot(n, r, r)) <= tol * bn) break;
        for (int i = 0; i < n; ++i) { z[i] = minv[i] * r[i]; p[i] = z[i]; }
        double rz = dot(n, r, z);
        int conv = 0;
        while (it < max_iter) {
            spmv(m, p, q);
            double alpha = rz / dot(n, p, q);
            for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bn) { conv = 1; break; }
            for (int i = 0; i < n; ++i) z[i] = minv[i] * r[i];
            double rz_new = dot(n, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        /* confirm on the true residual; restart from it if the recursion drifted */
        true_residual(m, x, r);
        if (!conv) { ret = -1; break; }
    }
    true_residual(m, x, rres);
    *relres = sqrt(dot(n, rres, rres)) / bn;
done:
    free(r); free(z); free(p); free(q); free(minv);
    return ret < 0 ? -1 : it;
}

/* Jacobi right-preconditioned BiCGSTAB (van der Vorst, 1992) for the
   nonsymmetric transport systems; same stopping rule as oc_pcg.  A breakdown
   (rho = 0 or omega = 0) restarts from the current iterate. */
int oc_bicgstab(const oc_csr *m, double *x, double tol, int max_iter, double *rres, double *relres)
{
    int n = m->n;
    double *r = malloc(sizeof(double) * n), *rh = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double *ph = malloc(sizeof(double) * n), *s = malloc(sizeof(double) * n);
    double *sh = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
    double *minv = malloc(sizeof(double) * n);
    int it = 0, ret = 0;
    double bn = sqrt(dot(n, m->rhs, m->rhs));
    if (bn == 0.0) {
        for (int i = 0; i < n; ++i) { x[i] = 0.0; rres[i] = 0.0; }
        *relres = 0.0;
        goto done;
    }
    for (int i = 0; i < n; ++i) minv[i] = 1.0 / diag_of(m, i);
    true_residual(m, x, r);
    for (;;) {
        if (sqrt(dot(n, r, r)) <= tol * bn) break;
        if (it >= max_iter) { ret = -1; break; }
        /* (re)start */
        for (int i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
        double rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int conv = 0;
        while (it < max_iter) {
            double rho = dot(n, rh, r);
            if (rho == 0.0) break;
            double beta = (rho / rho_old) * (alpha / omega);
            for (int i = 0; i < n; ++i) { p[i] = r[i] + beta * (p[i] - omega * v[i]); ph[i] = minv[i] * p[i]; }
            spmv(m, ph, v);
            alpha = rho / dot(n, rh, v);
            for (int i = 0; i < n; ++i) { s[i] = r[i] - alpha * v[i]; sh[i] = minv[i] * s[i]; }
            spmv(m, sh, t);
            double tt = dot(n, t, t);
            omega = tt > 0.0 ? dot(n, t, s) / tt : 0.0;
            for (int i = 0; i < n; ++i) { x[i] += alpha * ph[i] + omega * sh[i]; r[i] = s[i] - omega * t[i]; }
            rho_old = rho;
            ++it;
            if (sqrt(dot(n, r, r)) <= tol * bn) { conv = 1; break; }
            if (omega == 0.0) break;
        }
        true_residual(m, x, r);
        (void)conv;
    }
    true_residual(m, x, rres);
    *relres = sqrt(dot(n, rres, rres)) / bn;
done:
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(minv);
    return ret < 0 ? -1 : it;
}

/* ------------------------------------------------------------ phase update
   Second split step of the energy equation, eq. (3.12), with the liquidus
   eq. (3.13) and lever rule eq. (3.14): the liquid fraction g = g_l^{n+1}
   solves a g^2 + b g + c = 0, eqs. (3.15)-(3.16),
     a = 1 - k_p,
     b = k_p - g^n (1 - k_p) + (c_p/L)(1 - k_p)(T_m - T*),
     c = -(g^n + (c_p/L) T*) k_p + (c_p/L)(T_l - (1 - k_p) T_m),
   keeping the larger root, limited to [0, 1]; then T^{n+1} = T* - (L/c_p)
   (g - g^n).  reading of the eutectic rule (its flowchart is not in the
   text): at T_e = T_m + m_sp C_e the change is isothermal and T may fall
   below T_e only once the cell is fully solid.  With H = T* + (L/c_p) g^n
   (conserved by the split step) and g_eut the lever fraction at T_e:
     H <  T_e                    -> g = 0            (solid)
     H <  T_e + (L/c_p) g_eut    -> g = (H - T_e)/(L/c_p)   (plateau, T = T_e)
     H <  T_l + L/c_p            -> larger root of the quadratic (mushy)
     otherwise                   -> g = 1            (liquid)
   Then C_l = C / (1 + (1 - g)(k_p - 1)), C_s = k_p C_l, eqs. (3.17)-(3.18). */
void oc_phase_cell(const oc_case *c, double Tstar, double gn, double Cnew,
                   double *T_out, double *g_out, double *Cl_out, double *Cs_out, int *branch)
{
    const double lam = c->latent / c->cp;
    const double kp = c->k_p;
    const double H = Tstar + lam * gn;
    const double Tl = c->T_m + c->m_sp * Cnew;
    const double Te = c->T_m + c->m_sp * c->C_e;
    double geut = 1.0 - (Te - Tl) / ((1.0 - kp) * (Te - c->T_m));
    if (geut < 0.0) geut = 0.0;
    if (geut > 1.0) geut = 1.0;
    double g;
    int br;
    if (H < Te) { g = 0.0; br = 0; }
    else if (H < Te + lam * geut) { g = (H - Te) / lam; br = 1; }
    else if (H < Tl + lam) {
        double a = 1.0 - kp;
        double b = kp - gn * (1.0 - kp) + (1.0 - kp) * (c->T_m - Tstar) / lam;
        double cc = -(gn + Tstar / lam) * kp + (Tl - (1.0 - kp) * c->T_m) / lam;
        double disc = b * b - 4.0 * a * cc;
        if (disc < 0.0) disc = 0.0;
        /* both roots, evaluated without cancellation (Numerical Recipes
           form q = -(b + sign(b) sqrt(disc))/2, roots q/a and c/q) */
        double sq = sqrt(disc);
        double qq = -0.5 * (b + (b >= 0.0 ? sq : -sq));
        double r1 = qq / a;
        double r2 = (qq != 0.0) ? cc / qq : r1;
        g = r1 > r2 ? r1 : r2;
        if (g < 0.0) g = 0.0;
        if (g > 1.0) g = 1.0;
        br = 2;
    } else { g = 1.0; br = 3; }
    double T = Tstar - lam * (g - gn);
    double Cl = Cnew / (1.0 + (1.0 - g) * (kp - 1.0));
    *T_out = T; *g_out = g; *Cl_out = Cl; *Cs_out = kp * Cl;
    if (branch) *branch = br;
}

void oc_phase(const oc_case *c, int n, const double *Tstar, const double *gn, const double *Cnew,
              double *T, double *g, double *Cl, double *Cs, int *branch)
{
    for (int i = 0; i < n; ++i)
        oc_phase_cell(c, Tstar[i], gn[i], Cnew[i], &T[i], &g[i], &Cl[i], &Cs[i], branch ? &branch[i] : NULL);
}

/* ------------------------------------------------------------ public assembly */

static int nnz_bound(const oc_case *c, int sys) { return (2 * c->dim + 1) * oc_sys_rows(c, sys); }

static oc_csr csr_new(int n, int nnzmax)
{
    oc_csr m;
    m.n = n; m.nnz = 0;
    m.row_ptr = calloc((size_t)n + 1, sizeof(int));
    m.col = malloc(sizeof(int) * (size_t)(nnzmax > 0 ? nnzmax : 1));
    m.val = malloc(sizeof(double) * (size_t)(nnzmax > 0 ? nnzmax : 1));
    m.rhs = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    return m;
}

static void csr_free(oc_csr *m) { free(m->row_ptr); free(m->col); free(m->val); free(m->rhs); }

/* Assemble system `sys` from the fields f.  For the momentum systems the
   level-n fields are used; for SYS_P the face field `vel` is u*; for SYS_C and
   SYS_T the face field `vel` is the advecting u^{n+1}; t_new is the new time
   level (prescribed wall temperatures).  Output arrays are caller-owned and
   sized rows+1 / (2*dim+1)*rows / (2*dim+1)*rows / rows.  Returns nnz. */
int oc_assemble(const oc_case *c, const oc_fields *f, double *vu, double *vv, double *vw,
                double t_new, int sys, int *row_ptr, int *col, double *val, double *rhs)
{
    int n = oc_sys_rows(c, sys);
    oc_csr m;
    m.n = n; m.row_ptr = row_ptr; m.col = col; m.val = val; m.rhs = rhs; m.nnz = 0;
    double *const vel[3] = {vu, vv, vw};
    row_ptr[0] = 0;
    if (n == 0) return 0;
    switch (sys) {
    case SYS_U: case SYS_V: case SYS_W: assemble_momentum(c, f, sys, &m); break;
    case SYS_P: assemble_poisson(c, vel, &m); break;
    case SYS_C: assemble_solute(c, f, vel, &m); break;
    case SYS_T: assemble_energy(c, f, vel, t_new, &m); break;
    default: return -1;
    }
    return m.nnz;
}

/* ------------------------------------------------------------- time step */

static void face_counts(const oc_case *c, int nf[3])
{
    for (int a = 0; a < 3; ++a) nf[a] = oc_sys_rows(c, a);
}

/* One time step of Algorithm 1.  f holds level n on entry and level n+1 on a
   successful return (0).  On a solver failure (-1) f is left at level n.
   `inter` (nullable) receives u*, v*, w*, phi, T* (sizes of u, v, w, cells,
   cells). */
int oc_step(const oc_case *c, oc_fields *f, oc_stats *st, double *iu, double *iv, double *iw,
            double *iphi, double *iTstar)
{
    int n3[3], nf[3];
    cell_dims(c, n3);
    face_counts(c, nf);
    const int N = n3[0] * n3[1] * n3[2];
    const double t_new = (double)(f->step + 1) * c->dt;
    double *vel_n[3] = {f->u, f->v, f->w};
    double *ustar[3], *unew[3];
    int ret = 0;
    oc_stats s;
    memset(&s, 0, sizeof(s));
    for (int a = 0; a < 3; ++a) {
        ustar[a] = calloc((size_t)(nf[a] > 0 ? nf[a] : 1), sizeof(double));
        unew[a] = calloc((size_t)(nf[a] > 0 ? nf[a] : 1), sizeof(double));
    }
    double *phi = calloc(N, sizeof(double)), *rres = calloc(N + 1, sizeof(double));
    double *rv = calloc((size_t)(nf[0] + nf[1] + nf[2] + 1), sizeof(double));
    double *Cnew = malloc(sizeof(double) * N), *Tstar = malloc(sizeof(double) * N);
    double *Tn = malloc(sizeof(double) * N), *gn = malloc(sizeof(double) * N);
    double *Cl = malloc(sizeof(double) * N), *Cs = malloc(sizeof(double) * N);
    double *pn = malloc(sizeof(double) * N);

    /* step 1: momentum predictor u* (eq. 3.3), initial guess u^n */
    for (int d = 0; d < c->dim; ++d) {
        int nr = nf[d];
        if (nr == 0) continue;
        oc_csr m = csr_new(nr, nnz_bound(c, d));
        oc_assemble(c, f, f->u, f->v, f->w, t_new, d, m.row_ptr, m.col, m.val, m.rhs);
        memcpy(ustar[d], vel_n[d], sizeof(double) * nr);
        double rel;
        int it = oc_bicgstab(&m, ustar[d], c->tol_t, c->max_iter, rv, &rel);
        s.iters[d] = it; s.rel_resid[d] = rel;
        for (int i = 0; i < nr; ++i) s.sum_resid[d] += rv[i];
        csr_free(&m);
        if (it < 0) { ret = -1; goto out; }
    }
    /* step 2: pressure correction (eq. 3.4), phi_0 = 0, zero-mean phi */
    {
        int nr = N;
        oc_csr m = csr_new(nr, nnz_bound(c, SYS_P));
        oc_assemble(c, f, ustar[0], ustar[1], ustar[2], t_new, SYS_P, m.row_ptr, m.col, m.val, m.rhs);
        for (int i = 0; i < N; ++i) {
            int q[3] = {i % n3[0], (i / n3[0]) % n3[1], i / (n3[0] * n3[1])};
            double dv = cell_div(c, ustar, q);
            s.div_star += dv * dv;
        }
        s.div_star = sqrt(s.div_star);
        double rel;
        int it = oc_pcg(&m, phi, c->tol_p, c->max_iter, rres, &rel);
        s.iters[SYS_P] = it; s.rel_resid[SYS_P] = rel;
        double pr = 0.0;
        for (int i = 0; i < N; ++i) { s.sum_resid[SYS_P] += rres[i]; pr += rres[i] * rres[i]; }
        s.poisson_resid = sqrt(pr);
        csr_free(&m);
        if (it < 0) { ret = -1; goto out; }
        double mean = 0.0;
        for (int i = 0; i < N; ++i) mean += phi[i];
        mean /= (double)N;
        for (int i = 0; i < N; ++i) phi[i] -= mean;
    }
    /* step 3: projection (eq. 3.5) u^{n+1} = u* - dt/rho G phi, p^{n+1} = p^n + phi */
    for (int d = 0; d < c->dim; ++d) {
        int sd[3];
        oc_sys_dims(c, d, sd);
        double h = h_of(c, d);
        for (int k = 0; k < sd[2]; ++k)
        for (int j = 0; j < sd[1]; ++j)
        for (int i = 0; i < sd[0]; ++i) {
            int q[3] = {i, j, k};
            int row = lin(sd, i, j, k);
            int lo[3] = {i, j, k}, hi[3] = {i, j, k};
            lo[d] = q[d]; hi[d] = q[d] + 1;
            double g = (phi[lin(n3, hi[0], hi[1], hi[2])] - phi[lin(n3, lo[0], lo[1], lo[2])]) / h;
            unew[d][row] = ustar[d][row] - c->dt / c->rho * g;
        }
    }
    for (int i = 0; i < N; ++i) pn[i] = f->p[i] + phi[i];
    for (int i = 0; i < N; ++i) {
        int q[3] = {i % n3[0], (i / n3[0]) % n3[1], i / (n3[0] * n3[1])};
        double dv = cell_div(c, unew, q);
        s.div_new += dv * dv;
    }
    s.div_new = sqrt(s.div_new);
    /* step 4: solute (eq. 3.10), initial guess C^n */
    {
        oc_csr m = csr_new(N, nnz_bound(c, SYS_C));
        oc_assemble(c, f, unew[0], unew[1], unew[2], t_new, SYS_C, m.row_ptr, m.col, m.val, m.rhs);
        memcpy(Cnew, f->C, sizeof(double) * N);
        double rel;
        int it = oc_bicgstab(&m, Cnew, c->tol_t, c->max_iter, rres, &rel);
        s.iters[SYS_C] = it; s.rel_resid[SYS_C] = rel;
        for (int i = 0; i < N; ++i) s.sum_resid[SYS_C] += rres[i];
        csr_free(&m);
        if (it < 0) { ret = -1; goto out; }
    }
    /* steps 5-6: T* (eq. 3.11), initial guess T^n (T_l enters in step 7) */
    {
        oc_csr m = csr_new(N, nnz_bound(c, SYS_T));
        oc_assemble(c, f, unew[0], unew[1], unew[2], t_new, SYS_T, m.row_ptr, m.col, m.val, m.rhs);
        memcpy(Tstar, f->T, sizeof(double) * N);
        double rel;
        int it = oc_bicgstab(&m, Tstar, c->tol_t, c->max_iter, rres, &rel);
        s.iters[SYS_T] = it; s.rel_resid[SYS_T] = rel;
        for (int i = 0; i < N; ++i) s.sum_resid[SYS_T] += rres[i];
        csr_free(&m);
        if (it < 0) { ret = -1; goto out; }
        /* heat leaving through cooled walls, per unit cell volume, at T* */
        for (int i = 0; i < N; ++i) {
            int q[3] = {i % n3[0], (i / n3[0]) % n3[1], i / (n3[0] * n3[1])};
            for (int a = 0; a < c->dim; ++a)
                for (int sd = 0; sd < 2; ++sd) {
                    int wall = sd == 0 ? (q[a] == 0) : (q[a] == n3[a] - 1);
                    if (!wall) continue;
                    double h = h_of(c, a);
                    double U = wall_U(c, 2 * a + sd, h);
                    if (U > 0.0) s.wall_flux += U / (c->rho * c->cp * h) * (Tstar[i] - wall_T(c, 2 * a + sd, t_new));
                }
        }
    }
    /* steps 7-8: phase update and C_l, C_s (eqs. 3.12-3.18) */
    memcpy(gn, f->gl, sizeof(double) * N);
    oc_phase(c, N, Tstar, gn, Cnew, Tn, f->gl, Cl, Cs, NULL);
    {
        const double lam = c->latent / c->cp;
        for (int i = 0; i < N; ++i) { s.sum_C += Cnew[i]; s.sum_H += Tn[i] + lam * f->gl[i]; }
    }
    /* commit level n+1 */
    for (int d = 0; d < c->dim; ++d) memcpy(vel_n[d], unew[d], sizeof(double) * nf[d]);
    memcpy(f->p, pn, sizeof(double) * N);
    memcpy(f->T, Tn, sizeof(double) * N);
    memcpy(f->C, Cnew, sizeof(double) * N);
    memcpy(f->Cl, Cl, sizeof(double) * N);
    memcpy(f->Cs, Cs, sizeof(double) * N);
    f->step += 1;
    if (iu) memcpy(iu, ustar[0], sizeof(double) * nf[0]);
    if (iv) memcpy(iv, ustar[1], sizeof(double) * nf[1]);
    if (iw && c->dim == 3) memcpy(iw, ustar[2], sizeof(double) * nf[2]);
    if (iphi) memcpy(iphi, phi, sizeof(double) * N);
    if (iTstar) memcpy(iTstar, Tstar, sizeof(double) * N);
out:
    if (st) *st = s;
    for (int a = 0; a < 3; ++a) { free(ustar[a]); free(unew[a]); }
    free(phi); free(rres); free(rv); free(Cnew); free(Tstar); free(Tn); free(gn); free(Cl); free(Cs); free(pn);
    return ret;
}

/* Solve a caller-given CSR system with the oracle's Krylov methods
   (kind 0 = Jacobi-PCG, 1 = Jacobi-BiCGSTAB); x holds the initial guess on
   entry.  Returns iterations or -1. */
int oc_solve(int kind, int n, int *row_ptr, int *col, double *val, double *rhs,
             double *x, double tol, int max_iter, double *relres)
{
    oc_csr m;
    m.n = n; m.nnz = row_ptr[n]; m.row_ptr = row_ptr; m.col = col; m.val = val; m.rhs = rhs;
    double *r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int it = kind == 0 ? oc_pcg(&m, x, tol, max_iter, r, relres)
                       : oc_bicgstab(&m, x, tol, max_iter, r, relres);
    free(r);
    return it;
}
