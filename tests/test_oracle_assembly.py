"""Pins of the oracle's assembled systems against facts that do not come from
the oracle itself: closed-form sparsity counts, an independent forward-probe
assembly (the paper's second assembly route, Section 4), exactness of the
stencils on polynomials, conservation identities, M-matrix signs, the
closed-form spectrum of the Neumann Laplacian, and steady 1D solutions
(plane Couette/Poiseuille-type, Darcy's law, a conducting slab)."""
import numpy as np
import pytest

import oracle
from oracle import forward
import workloads as W

SYS = oracle


def _perturbed(case, seed=1, gl_range=(0.0, 1.0), vel_amp=1e-3):
    o = oracle.Oracle(case)
    f = o.fields()
    rng = np.random.default_rng(seed)
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-vel_amp, vel_amp, f[k].size)
    f["gl"] = rng.uniform(*gl_range, f["gl"].size)
    f["p"] = rng.uniform(-1.0, 1.0, f["p"].size)
    f["T"] = f["T"] + rng.uniform(-3, 3, f["T"].size)
    f["Cl"] = f["Cl"] + rng.uniform(-1, 1, f["Cl"].size)
    return f


def _cases():
    c2 = W.cavity_2d(7, 5)
    c2fs = W.cavity_2d(6, 4)
    for b in c2fs["bcs"]:
        b["velocity"] = W.VELOCITY_FREESLIP
    c2fs["bcs"][3] = W.face_bc(W.THERMAL_DIRICHLET, T0=480.0, b=0.5)
    c3 = W.box_3d(5, 4, 3, lx=0.05, ly=0.04, lz=0.03)
    c3["bcs"][5] = W.face_bc(W.THERMAL_ROBIN, h=50.0, T_ext=400.0, velocity=W.VELOCITY_FREESLIP)
    # liquid solute diffusion (eq. 3.7), large enough to dominate the solute rows
    c2d = W.cavity_2d(7, 5, alloy=W.sn10pb_alloy(D_l=2e-4))
    c3d = W.box_3d(5, 4, 3, lx=0.05, ly=0.04, lz=0.03, alloy=W.sn10pb_alloy(D_l=2e-4))
    # momentum form (2.6); the perturbed g_l spans solid cells and the floor
    c2m = W.with_momentum(c2fs, W.MOMENTUM_MINIMAL)
    c3m = W.with_momentum(c3, W.MOMENTUM_MINIMAL)
    return [c2, c2fs, c3, c2d, c3d, c2m, c3m]


@pytest.mark.parametrize("case", _cases(), ids=["2d", "2d-freeslip-dirichlet", "3d", "2d-Dl", "3d-Dl",
                                                "2d-mom26", "3d-mom26"])
def test_forward_probe_equals_stencil_assembly(case):
    """Forward method (colour probes of a residual function) reproduces the
    directly assembled matrices and right-hand sides up to rounding."""
    f = _perturbed(case)
    o = oracle.Oracle(case, fields=f)
    rng = np.random.default_rng(7)
    vel = tuple(rng.uniform(-1e-3, 1e-3, max(1, f[k].size)) for k in ("u", "v", "w"))
    dim = case["grid"]["dim"]
    for sys in range(6):
        if dim == 2 and sys == SYS.SYS_W:
            continue
        v = vel if sys in (SYS.SYS_P, SYS.SYS_C, SYS.SYS_T) else None
        A, b, rp, ci = o.assemble(sys, vel=v, t_new=0.37)
        Af, bf = forward.forward_assemble(case, o.fields(), sys, vel=v, t_new=0.37)
        assert np.array_equal(A.indptr, Af.indptr)
        assert np.array_equal(A.indices, Af.indices)
        scale = abs(A).sum(axis=1).A1 + abs(b)
        assert (abs(A - Af).sum(axis=1).A1 / scale).max() < 64 * np.finfo(float).eps
        assert (abs(b - bf) / scale).max() < 64 * np.finfo(float).eps


def _nnz_closed_form(d):
    nx, ny, nz = d
    n = nx * ny * nz
    return n + 2 * ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1))


@pytest.mark.parametrize("dims", [(2, 50, 30, 1), (2, 7, 1, 1), (3, 5, 4, 3), (3, 2, 2, 2)])
def test_sparsity_closed_form(dims):
    dim, nx, ny, nz = dims
    if dim == 2:
        case = W.cavity_2d(nx, ny)
    else:
        case = W.box_3d(nx, ny, nz)
    o = oracle.Oracle(case)
    cell = (nx, ny, nz if dim == 3 else 1)
    for sys in range(6):
        if dim == 2 and sys == SYS.SYS_W:
            continue
        d = list(cell)
        if sys < 3:
            d[sys] -= 1
        if min(d) <= 0:
            assert o.rows(sys) == 0
            continue
        A, b, rp, ci = o.assemble(sys, vel=(o.f["u"], o.f["v"], o.f["w"]))
        assert A.shape[0] == d[0] * d[1] * d[2]
        assert A.nnz == _nnz_closed_form(d)
        if dim == 2 and sys >= 3:
            assert A.nnz == 5 * nx * ny - 2 * nx - 2 * ny
        for i in range(A.shape[0]):   # columns strictly ascending per row
            cols = ci[rp[i]:rp[i + 1]]
            assert np.all(np.diff(cols) > 0)


def _grid_xy(case, sys=SYS.SYS_T):
    g = case["grid"]
    nx, ny = g["nx"], g["ny"]
    hx, hy = g["lx"] / nx, g["ly"] / ny
    if sys == SYS.SYS_U:
        x = np.arange(1, nx) * hx
        y = (np.arange(ny) + 0.5) * hy
    elif sys == SYS.SYS_V:
        x = (np.arange(nx) + 0.5) * hx
        y = np.arange(1, ny) * hy
    else:
        x = (np.arange(nx) + 0.5) * hx
        y = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(x, y, indexing="xy")
    return X.ravel(), Y.ravel(), hx, hy


def test_diffusion_exact_on_quadratics_and_symmetric():
    """Central diffusion: -alpha * Lap_h of x^2 + 3y^2 is -8 alpha exactly at
    interior rows; the operator is symmetric and annihilates constants with
    adiabatic walls (row sums 0)."""
    case = W.make_case(2, 9, 7, 1, 0.09, 0.07, 1.0)      # all walls adiabatic
    o = oracle.Oracle(case)
    zero = tuple(np.zeros(max(1, o.f[k].size)) for k in ("u", "v", "w"))
    A, b, _, _ = o.assemble(SYS.SYS_T, vel=zero)
    dt = case["numerics"]["dt"]
    al = case["alloy"]
    alpha = al["k"] / (al["rho"] * al["cp"])
    D = A.toarray() - np.eye(A.shape[0]) / dt
    X, Y, hx, hy = _grid_xy(case)
    phi = X ** 2 + 3 * Y ** 2
    val = D @ phi
    inner = (X > hx) & (X < 0.09 - hx) & (Y > hy) & (Y < 0.07 - hy)
    np.testing.assert_allclose(val[inner], -alpha * 8.0, rtol=1e-9)
    np.testing.assert_allclose(D, D.T, atol=1e-12 * abs(D).max())
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-10 * abs(D).max())


@pytest.mark.parametrize("shape", [(4, 3), (5, 2), (3, 3, 2)])
def test_neumann_laplacian_spectrum_closed_form(shape):
    """Eigenvalues of -L (Neumann, uniform grid) are sums over axes of
    (4/h^2) sin^2(k pi / (2n)), k = 0..n-1 (DCT-II modes)."""
    if len(shape) == 2:
        case = W.make_case(2, shape[0], shape[1], 1, 0.04, 0.03, 1.0)
        hs = [0.04 / shape[0], 0.03 / shape[1]]
    else:
        case = W.make_case(3, *shape, 0.03, 0.02, 0.01)
        hs = [0.03 / shape[0], 0.02 / shape[1], 0.01 / shape[2]]
    o = oracle.Oracle(case)
    zero = tuple(np.zeros(max(1, o.f[k].size)) for k in ("u", "v", "w"))
    A, b, _, _ = o.assemble(SYS.SYS_P, vel=zero)
    ev = np.sort(np.linalg.eigvalsh(A.toarray()))
    lam1d = [(4.0 / h ** 2) * np.sin(np.arange(n) * np.pi / (2 * n)) ** 2 for n, h in zip(shape, hs)]
    grid = lam1d[0]
    for l in lam1d[1:]:
        grid = np.add.outer(grid, l).ravel()
    np.testing.assert_allclose(ev, np.sort(grid), rtol=1e-12, atol=1e-9 * ev.max())


def test_upwind_exact_for_linear_and_conservative():
    """Upwind convection with a uniform velocity is exact for linear profiles
    away from walls; its columns sum to zero for any face velocity (flux
    form) and its off-diagonals are non-positive (M-matrix)."""
    case = W.make_case(2, 10, 8, 1, 0.10, 0.08, 1.0)
    o = oracle.Oracle(case)
    nx, ny = 10, 8
    U0 = 2e-3
    u = np.full((nx - 1) * ny, U0)
    v = np.zeros(nx * (ny - 1))
    A, b, _, _ = o.assemble(SYS.SYS_C, vel=(u, v, np.zeros(1)))   # g_l = 1: A_g = I
    dt = case["numerics"]["dt"]
    Cm = A.toarray() - np.eye(A.shape[0]) / dt
    X, Y, hx, hy = _grid_xy(case)
    phi = 3.0 * X - 5.0 * Y + 1.0
    val = Cm @ phi
    inner = (X > hx) & (X < 0.10 - hx)
    np.testing.assert_allclose(val[inner], U0 * 3.0, rtol=1e-10)
    # arbitrary (not divergence free) velocities, both signs
    rng = np.random.default_rng(3)
    u = rng.uniform(-1e-3, 1e-3, u.size)
    v = rng.uniform(-1e-3, 1e-3, v.size)
    A, b, _, _ = o.assemble(SYS.SYS_T, vel=(u, v, np.zeros(1)))
    off = A - np.diag(A.diagonal())
    assert off.max() <= 0.0
    zero = tuple(np.zeros(max(1, o.f[k].size)) for k in ("u", "v", "w"))
    A0, _, _, _ = o.assemble(SYS.SYS_T, vel=zero)
    conv = (A - A0).toarray()
    np.testing.assert_allclose(conv.sum(axis=0), 0.0, atol=1e-12 * abs(conv).max())


def test_solute_matrix_Ag_limits_and_column_sums():
    """A_g = diag(1/(k_p + (1-k_p) g_l)): g_l = 1 gives plain upwind, g_l = 0
    gives upwind / k_p, and for any g_l the columns of
    I/dt + A_con A_g sum to 1/dt (solute conservation, eq. 3.10).  The
    printed order A_g A_con breaks the column identity."""
    case = W.make_case(2, 6, 5, 1, 0.06, 0.05, 1.0)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1e-3, 1e-3, 5 * 5)
    v = rng.uniform(-1e-3, 1e-3, 6 * 4)
    vel = (u, v, np.zeros(1))
    kp = case["alloy"]["k_p"]
    dt = case["numerics"]["dt"]
    I = np.eye(30) / dt
    f = oracle.Oracle(case).fields()
    A1 = oracle.Oracle(case, fields=f).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    f0 = dict(f, gl=np.zeros(30))
    A0 = oracle.Oracle(case, fields=f0).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    np.testing.assert_allclose(A0 - I, (A1 - I) / kp, rtol=1e-12, atol=1e-14)
    fr = dict(f, gl=rng.uniform(0, 1, 30))
    Ar = oracle.Oracle(case, fields=fr).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    np.testing.assert_allclose(Ar.sum(axis=0), 1.0 / dt, rtol=1e-13)
    Al = oracle.Oracle(case, fields=fr, literal_ag_order=True).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    assert abs(Al.sum(axis=0) - 1.0 / dt).max() > 1e-3


def _steady(case):
    case["numerics"]["dt"] = 1e12
    return case


def test_freeslip_channel_parabola_exact():
    """Steady u-momentum driven by a uniform pressure drop between impermeable
    walls at x = 0, l_x, free-slip at y walls: u(x) = G x (l_x - x) / (2 mu),
    reproduced exactly at the face nodes (a parabola is exact for central
    differences with Dirichlet end nodes).  Also pins the sign of the
    pressure-gradient force (flow runs down the pressure drop)."""
    nx, ny, lx, ly = 12, 3, 0.012, 0.003
    case = _steady(W.make_case(2, nx, ny, 1, lx, ly, 1.0, dT_amp=0.0))
    for b in case["bcs"]:
        b["velocity"] = W.VELOCITY_FREESLIP
    G = 3.0
    f = oracle.Oracle(case).fields()
    xc = (np.arange(nx) + 0.5) * lx / nx
    f["p"] = np.tile(-G * xc, ny)
    o = oracle.Oracle(case, fields=f)
    A, b, _, _ = o.assemble(SYS.SYS_U)
    u, it, rel = oracle.solve(A, b, kind="bicgstab", tol=1e-14)
    x = np.tile(np.arange(1, nx) * lx / nx, ny)
    mu = case["alloy"]["mu"]
    exact = G * x * (lx - x) / (2 * mu)
    np.testing.assert_allclose(u, exact, rtol=1e-9)


def test_noslip_channel_second_order():
    """Plane Poiseuille flow between no-slip walls (half-cell ghost): the
    mid-channel profile converges to G y (l_y - y)/(2 mu) at second order."""
    errs = []
    for ny in (8, 16, 32):
        lx, ly = 0.4, 0.01
        nx = 40
        case = _steady(W.make_case(2, nx, ny, 1, lx, ly, 1.0, dT_amp=0.0))
        G = 1e-3
        f = oracle.Oracle(case).fields()
        xc = (np.arange(nx) + 0.5) * lx / nx
        f["p"] = np.tile(-G * xc, ny)
        o = oracle.Oracle(case, fields=f)
        A, b, _, _ = o.assemble(SYS.SYS_U)
        u, it, rel = oracle.solve(A, b, kind="bicgstab", tol=1e-13, max_iter=20000)
        u = u.reshape(ny, nx - 1)[:, (nx - 1) // 2]
        y = (np.arange(ny) + 0.5) * ly / ny
        exact = G * y * (ly - y) / (2 * case["alloy"]["mu"])
        errs.append(abs(u - exact).max() / exact.max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 5e-3
    assert np.all(rates > 1.8), (errs, rates)


def test_darcy_law_and_buoyancy_direction():
    """In a uniform mush with a uniform thermal buoyancy force the steady
    vertical predictor velocity away from walls obeys Darcy's law
    v = K f / nu with the Carman-Kozeny permeability (eq. 2.8), and warm
    liquid rises (v > 0 for T > T_ref with beta_T > 0)."""
    nx, ny = 8, 8
    case = _steady(W.make_case(2, nx, ny, 1, 0.008, 0.008, 1.0, dT_amp=0.0))
    al = case["alloy"]
    al["darcy_eps"] = 0.0
    g0, dT = 0.5, 2.0
    f = oracle.Oracle(case).fields()
    f["gl"] = np.full(nx * ny, g0)
    f["T"] = f["T"] + dT
    o = oracle.Oracle(case, fields=f)
    A, b, _, _ = o.assemble(SYS.SYS_V)
    v, it, rel = oracle.solve(A, b, kind="bicgstab", tol=1e-14)
    v = v.reshape(ny - 1, nx)[2:-2, 2:-2]
    K = al["lambda2"] ** 2 * g0 ** 3 / (180.0 * (1 - g0) ** 2)
    force = al["g"] * al["beta_T"] * dT
    nu = al["mu"] / al["rho"]
    np.testing.assert_allclose(v, K * force / nu, rtol=1e-6)
    assert np.all(v > 0)


def test_conducting_slab_linear_profile():
    """Steady conduction through a slab cooled by a film (h, T_ext) on the
    west side and held at T_E on the east side: the exact temperature is
    linear, T = T_ext + q (1/h + x/k), q = (T_E - T_ext)/(1/h + l_x/k); the
    half-cell series resistance makes the grid solution exact."""
    nx, lx = 10, 0.05
    case = _steady(W.make_case(2, nx, 1, 1, lx, 0.01, 1.0, dT_amp=0.0))
    hc, Text, TE = 150.0, 300.0, 520.0
    case["bcs"][0] = W.face_bc(W.THERMAL_ROBIN, h=hc, T_ext=Text)
    case["bcs"][1] = W.face_bc(W.THERMAL_DIRICHLET, T0=TE, b=0.0)
    o = oracle.Oracle(case)
    zero = tuple(np.zeros(max(1, o.f[k].size)) for k in ("u", "v", "w"))
    A, b, _, _ = o.assemble(SYS.SYS_T, vel=zero)
    T, it, rel = oracle.solve(A, b, kind="bicgstab", tol=1e-15)
    k = case["alloy"]["k"]
    x = (np.arange(nx) + 0.5) * lx / nx
    q = (TE - Text) / (1.0 / hc + lx / k)
    np.testing.assert_allclose(T, Text + q * (1.0 / hc + x / k), rtol=1e-11)


def test_momentum_advecting_velocity_exact_for_linear():
    """Momentum convection (flux form, face-averaged advecting velocity): with
    uniform u^n = U0 at the interior x-faces, the x-convection of a linear
    u* is U0 du*/dx at rows two faces away from the walls; with uniform
    v^n = V0 the y-convection of a linear u* is V0 du*/dy away from walls."""
    nx, ny, lx, ly = 10, 9, 0.10, 0.09
    case = W.make_case(2, nx, ny, 1, lx, ly, 1.0, dT_amp=0.0)
    base = oracle.Oracle(case).fields()
    X, Y, hx, hy = _grid_xy(case, SYS.SYS_U)
    A0, _, _, _ = oracle.Oracle(case, fields=base).assemble(SYS.SYS_U)
    for U0, V0 in ((1.5e-3, 0.0), (0.0, -2.0e-3)):
        f = dict(base)
        f["u"] = np.full((nx - 1) * ny, U0)
        f["v"] = np.full(nx * (ny - 1), V0)
        A, _, _, _ = oracle.Oracle(case, fields=f).assemble(SYS.SYS_U)
        conv = (A - A0).toarray()
        phi = 2.0 * X + 7.0 * Y
        val = conv @ phi
        inner = (X > 1.5 * hx) & (X < lx - 1.5 * hx) & (Y > hy) & (Y < ly - hy)
        np.testing.assert_allclose(val[inner], U0 * 2.0 + V0 * 7.0, rtol=1e-10)



# ----------------------------------------------------- liquid diffusion

def _dl_case(D=1e-4, nx=9, ny=7, nz=1):
    al = W.sn10pb_alloy(D_l=D)
    if nz == 1:
        return W.make_case(2, nx, ny, 1, nx * 1e-3, ny * 1e-3, 1.0, alloy=al)
    return W.make_case(3, nx, ny, nz, nx * 1e-3, ny * 1e-3, nz * 1e-3, alloy=al)


@pytest.mark.parametrize("nz", [1, 5])
def test_liquid_diffusion_exact_for_quadratic_Cl_and_linear_gl(nz):
    """The diffusion rows of the solute matrix (eq. 3.7) acting on C = C_l /
    A_g give -div(g_l D_l grad C_l) exactly on rows away from the walls when
    g_l is linear and C_l quadratic in every axis (face means of a linear g_l
    are exact, differences of a quadratic C_l are exact face gradients, and
    the central difference of the quadratic flux is exact)."""
    case = _dl_case(nz=nz)
    al = case["alloy"]
    D, kp = al["D_l"], al["k_p"]
    g = case["grid"]
    n = (g["nx"], g["ny"], g["nz"])
    h = (g["lx"] / n[0], g["ly"] / n[1], g["lz"] / n[2])
    dim = g["dim"]
    k, j, i = np.meshgrid(*(np.arange(n[a]) for a in (2, 1, 0)), indexing="ij")
    x = [((i + 0.5) * h[0]).ravel(), ((j + 0.5) * h[1]).ravel(), ((k + 0.5) * h[2]).ravel()]
    a_g, b_g = (0.3, 40.0, 25.0, 30.0), None
    gl = a_g[0] + sum(a_g[1 + a] * x[a] for a in range(dim))
    cq = (2.0, 500.0, -300.0, 400.0)
    Cl = 10.0 + sum(cq[a] * x[a] + 1e4 * (a + 1) * x[a] ** 2 for a in range(dim))
    f = oracle.Oracle(case).fields()
    f["gl"] = gl
    o = oracle.Oracle(case, fields=f)
    zero = tuple(np.zeros(max(1, f[kk].size)) for kk in ("u", "v", "w"))
    A, _, _, _ = o.assemble(SYS.SYS_C, vel=zero)
    C = Cl * (kp + (1.0 - kp) * gl)
    lhs = A @ C - C / case["numerics"]["dt"]
    # -sum_a d/dx_a (g D dCl/dx_a) = -D sum_a (g_a' Cl_a' + g Cl_a'')
    exact = -D * sum(a_g[1 + a] * (cq[a] + 2e4 * (a + 1) * x[a]) + gl * 2e4 * (a + 1) for a in range(dim))
    inner = np.ones(C.size, bool)
    for a, idx in enumerate((i.ravel(), j.ravel(), k.ravel())[:dim]):
        inner &= (idx >= 1) & (idx <= n[a] - 2)
    np.testing.assert_allclose(lhs[inner], exact[inner], rtol=1e-9, atol=1e-9 * abs(exact).max())


def test_liquid_diffusion_conserves_solute():
    """With diffusion the solute matrix still has column sums 1/dt (zero-flux
    walls, symmetric face coefficients), so sum C is conserved for any g_l
    and flow; the printed row order breaks it."""
    case = _dl_case(D=3e-4)
    rng = np.random.default_rng(12)
    f = oracle.Oracle(case).fields()
    f["gl"] = rng.uniform(0.0, 1.0, f["gl"].size)
    vel = tuple(rng.uniform(-1e-3, 1e-3, max(1, f[kk].size)) for kk in ("u", "v", "w"))
    dt = case["numerics"]["dt"]
    A = oracle.Oracle(case, fields=f).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    np.testing.assert_allclose(A.sum(axis=0), 1.0 / dt, rtol=1e-13)
    f0 = dict(f, gl=np.ones(f["gl"].size))
    zero = tuple(np.zeros(max(1, f[kk].size)) for kk in ("u", "v", "w"))
    A1 = oracle.Oracle(case, fields=f0).assemble(SYS.SYS_C, vel=zero)[0].toarray()
    L = A1 - np.eye(A1.shape[0]) / dt                   # g_l = 1: D_l times the Neumann Laplacian
    np.testing.assert_allclose(L, L.T, rtol=0, atol=1e-12 * abs(L).max())
    np.testing.assert_allclose(L.sum(axis=1), 0.0, atol=1e-12 * abs(L).max())
    assert np.all(np.diag(L) > 0)
    Al = oracle.Oracle(case, fields=f, literal_ag_order=True).assemble(SYS.SYS_C, vel=vel)[0].toarray()
    assert abs(Al.sum(axis=0) - 1.0 / dt).max() > 1e-3
