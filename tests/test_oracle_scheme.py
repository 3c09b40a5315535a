"""Pins of the oracle's solves and whole time step: dense direct solves on
tiny grids, divergence after projection, residual-corrected solute and
energy conservation (with the printed A_g order as a planted defect), and
the Neumann closed-form solution of the one-dimensional Stefan problem."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import erf, erfc

import oracle
import workloads as W


def _perturbed_fields(case, seed=2):
    rng = np.random.default_rng(seed)
    o = oracle.Oracle(case)
    f = o.fields()
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-1e-3, 1e-3, f[k].size)
    f["gl"] = rng.uniform(0.0, 1.0, f["gl"].size)
    f["p"] = rng.uniform(-1.0, 1.0, f["p"].size)
    return f


@pytest.mark.parametrize("dim", [2, 3])
def test_krylov_matches_dense_direct(dim):
    case = W.cavity_2d(6, 5) if dim == 2 else W.box_3d(4, 3, 3, lx=0.04, ly=0.03, lz=0.03)
    f = _perturbed_fields(case)
    o = oracle.Oracle(case, fields=f)
    rng = np.random.default_rng(4)
    vel = tuple(rng.uniform(-1e-3, 1e-3, max(1, f[k].size)) for k in ("u", "v", "w"))
    for sys in range(6):
        if dim == 2 and sys == oracle.SYS_W:
            continue
        v = vel if sys in (oracle.SYS_P, oracle.SYS_C, oracle.SYS_T) else None
        A, b, _, _ = o.assemble(sys, vel=v)
        Ad = A.toarray()
        if sys == oracle.SYS_P:
            x, it, rel = oracle.solve(A, b, kind="cg", tol=1e-14)
            x = x - x.mean()
            ref = np.linalg.lstsq(Ad, b, rcond=None)[0]
            ref = ref - ref.mean()
        else:
            x, it, rel = oracle.solve(A, b, kind="bicgstab", tol=1e-14)
            ref = np.linalg.solve(Ad, b)
        assert it >= 0
        assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_projection_divergence_bound_and_tight_tolerance():
    """D u^{n+1} = -(dt/rho) r_p (up to the mean of D u*, which is zero), so
    ||D u^{n+1}|| equals (dt/rho) ||r_p||; at tight tolerance the projected
    field is divergence free to 1e-12 relative to D u*."""
    case = W.cavity_2d(12, 8, tol=1e-10)
    o = oracle.Oracle(case)
    st = o.step(3)
    rho, dt = case["alloy"]["rho"], case["numerics"]["dt"]
    for s in st:
        assert abs(s["div_new"] - dt / rho * s["poisson_resid"]) <= 1e-6 * s["div_new"] + 1e-12 * s["div_star"]
    case2 = W.cavity_2d(12, 8, tol=1e-14)
    st2 = oracle.Oracle(case2).step(3)
    for s in st2:
        assert s["div_new"] <= 1e-12 * s["div_star"]


def _sums(f, case):
    lam = case["alloy"]["latent"] / case["alloy"]["cp"]
    return f["C"].sum(), (f["T"] + lam * f["gl"]).sum()


@pytest.mark.parametrize("tol", [1e-10, 1e-14])
def test_conservation_residual_corrected(tol):
    """Solute: sum C^{n+1} - sum C^n + dt sum r_C = 0; energy:
    sum(T + L/c_p g)^{n+1} - sum(...)^n + dt sum_walls U/(rho c_p h)(T* - T_ext)
    + dt sum r_T = 0, both to 1e-12 relative, at any solver tolerance."""
    case = W.cavity_2d(20, 12, tol=tol)
    o = oracle.Oracle(case)
    dt = case["numerics"]["dt"]
    for _ in range(6):
        C0, H0 = _sums(o.fields(), case)
        s = o.step(1)[0]
        C1, H1 = _sums(o.fields(), case)
        assert abs(C1 - C0 + dt * s["sum_resid"][oracle.SYS_C]) <= 1e-12 * abs(C0)
        assert abs(H1 - H0 + dt * s["wall_flux"] + dt * s["sum_resid"][oracle.SYS_T]) <= 1e-12 * abs(H0)
        assert abs(s["sum_C"] - C1) <= 1e-13 * abs(C1)


def test_printed_Ag_order_breaks_solute_conservation():
    """Planted defect: the row-scaled A_g*A_con does not conserve solute once
    a non-uniform composition is carried through mushy cells (it does while
    g_l = 1 everywhere)."""
    case = W.cavity_2d(16, 10, tol=1e-13)
    f = oracle.Oracle(case).fields()
    rng = np.random.default_rng(9)
    f["gl"] = rng.uniform(0.2, 1.0, f["gl"].size)
    f["u"] = rng.uniform(-1e-3, 1e-3, f["u"].size)
    f["v"] = rng.uniform(-1e-3, 1e-3, f["v"].size)
    f["C"] = rng.uniform(8.0, 12.0, f["C"].size)
    good = oracle.Oracle(case, fields=f)
    bad = oracle.Oracle(case, fields=f, literal_ag_order=True)
    dt = case["numerics"]["dt"]
    C0 = f["C"].sum()
    sg = good.step(1)[0]
    sb = bad.step(1)[0]
    eg = abs(good.fields()["C"].sum() - C0 + dt * sg["sum_resid"][oracle.SYS_C]) / C0
    eb = abs(bad.fields()["C"].sum() - C0 + dt * sb["sum_resid"][oracle.SYS_C]) / C0
    assert eg < 1e-12
    assert eb > 1e-9


def _neumann_lambda(St_s, St_l):
    """Root of St_s/(e^{l^2} erf l) - St_l/(e^{l^2} erfc l) = l sqrt(pi)
    (two-phase Stefan problem, equal diffusivities; Carslaw & Jaeger)."""
    f = lambda l: St_s / (math.exp(l * l) * erf(l)) - St_l / (math.exp(l * l) * erfc(l)) - l * math.sqrt(math.pi)
    return brentq(f, 1e-6, 3.0)


def _stefan_case(nx, dt, Tw, dTl, lx=0.1):
    al = W.sn10pb_alloy(beta_T=0.0, beta_C=0.0)
    Te = al["T_m"] + al["m_sp"] * al["C_e"]
    case = W.make_case(2, nx, 1, 1, lx, 0.01, 1.0, C0=al["C_e"], alloy=al,
                       T0=Te + dTl, dT_amp=0.0, dt=dt, tol_p=1e-13, tol_t=1e-13)
    case["bcs"][0] = W.face_bc(W.THERMAL_DIRICHLET, T0=Tw, b=0.0)
    return case, Te


def test_neumann_stefan_first_order():
    """Isothermal (eutectic-composition) solidification from a cold wall in a
    still melt: front s(t) = 2 lam_N sqrt(alpha t) and the erf/erfc
    temperature profiles.  The latent-heat split lags the front by O(dt), so
    h and dt are refined together with dt = 3 h^2/alpha; the front error then
    falls first order in h."""
    Tw, dTl, t_end = 400.0, 5.0, 20.0
    errs, terrs = [], []
    for nx, dt in ((100, 0.1), (200, 0.025), (400, 0.00625)):
        case, Te = _stefan_case(nx, dt, Tw, dTl)
        al = case["alloy"]
        alpha = al["k"] / (al["rho"] * al["cp"])
        St_s = al["cp"] * (Te - Tw) / al["latent"]
        St_l = al["cp"] * dTl / al["latent"]
        lamN = _neumann_lambda(St_s, St_l)
        o = oracle.Oracle(case)
        nsteps = int(round(t_end / dt))
        o.step(nsteps)
        f = o.fields()
        h = 0.1 / nx
        s_num = h * np.sum(1.0 - f["gl"])
        s_ex = 2 * lamN * math.sqrt(alpha * t_end)
        errs.append(abs(s_num - s_ex) / s_ex)
        x = (np.arange(nx) + 0.5) * h
        eta = x / (2 * math.sqrt(alpha * t_end))
        Tex = np.where(x < s_ex, Tw + (Te - Tw) * erf(eta) / erf(lamN),
                       Te + dTl - dTl * erfc(eta) / erfc(lamN))
        terrs.append(np.abs(f["T"] - Tex).max())
    assert abs(lamN - 0.1769) < 2e-3
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[-1] < 0.012, errs
    assert errs[0] / errs[-1] > 3.5, errs           # first order over 4x refinement of h
    assert terrs[-1] < 0.3 * terrs[0] and terrs[-1] < 1.0, terrs    # max |T - T_exact| in K


def test_still_melt_without_buoyancy_stays_at_rest():
    """beta_T = beta_C = 0 (hydrostatic part dropped): the velocity stays
    exactly zero and C stays uniform while the cavity loses heat."""
    al = W.sn10pb_alloy(beta_T=0.0, beta_C=0.0)
    case = W.make_case(2, 10, 6, 1, 0.1, 0.06, 1.0, alloy=al,
                       bcs=W.west_cooled_bcs())
    o = oracle.Oracle(case)
    o.step(5)
    f = o.fields()
    assert not f["u"].any() and not f["v"].any()
    assert np.all(f["C"] == 10.0)
    lam = case["alloy"]["latent"] / case["alloy"]["cp"]
    H0 = (case["init"]["T"] + lam * case["init"]["gl"]).sum()
    assert (f["T"] + lam * f["gl"]).sum() < H0 and (f["gl"] < 1.0).any()


# ---------------------------------------------------------------------------
# Wiring of the time step (Algorithm 1): which face velocity advects C and T*
# (u^{n+1} after the projection, eqs. 3.10-3.11), which C sets the liquidus of
# the phase update (C^{n+1}, eq. 3.13), which g_l scales the solute columns
# (g_l^n, the A_g of eq. 3.9).  Flux-form upwind conserves for any face field
# and the rest-state pins have u = 0, so these need pins of their own.
# ---------------------------------------------------------------------------

def _liquid_melt(dT_amp, seed=3, nx=24, ny=16):
    al = W.sn10pb_alloy()
    Tl = al["T_m"] + al["m_sp"] * 10.0
    return W.make_case(2, nx, ny, 1, nx * 1e-3, ny * 1e-3, 1.0, T0=Tl + 5.0, dT_amp=dT_amp,
                       bcs=W.west_cooled_bcs(), seed=seed, tol_p=1e-12, tol_t=1e-12)


def _solve_with(case, fields, sys, vel):
    """Solve one transport system of a step, assembled from `fields` (level n)
    with the face field `vel` as the advecting velocity, by a dense solve."""
    o = oracle.Oracle(case, fields=fields)
    A, b, _, _ = o.assemble(sys, vel=vel)
    return np.linalg.solve(A.toarray(), b)


def test_solute_advected_by_projected_velocity_stays_uniform():
    """All-liquid melt (T0 = T_l + 5 K, +-2 K perturbation) with uniform C:
    thermal buoyancy drives a flow, and C must stay exactly uniform, because
    the divergence-free u^{n+1} carries the uniform field without sources.
    Planted mistake: the same step's solute system advected by u* (not yet
    projected) makes C drift by far more than rounding."""
    case = _liquid_melt(2.0)
    o = oracle.Oracle(case)
    o.step(2)
    drift_planted = 0.0
    for _ in range(5):
        fn = o.fields()
        o.step(1, keep_intermediate=True)
        f = o.fields()
        assert np.ptp(f["C"]) == 0.0 and np.all(f["gl"] == 1.0)
        assert np.abs(f["u"]).max() > 1e-6          # the melt does move
        ustar = (o.intermediate["u"], o.intermediate["v"], np.zeros(1))
        drift_planted = max(drift_planted, np.ptp(_solve_with(case, fn, oracle.SYS_C, ustar)))
    assert drift_planted > 1e-9 * 10.0, drift_planted


def test_temperature_advected_by_projected_velocity_stays_uniform():
    """Uniform T, adiabatic walls, composition perturbed by +-0.5 wt%:
    solutal buoyancy drives the flow, and T* (hence T, all liquid) must stay
    exactly uniform under the divergence-free u^{n+1}.  Planted mistake: the
    energy system advected by u* drifts."""
    case = _liquid_melt(0.0)
    case["bcs"] = [W.face_bc() for _ in range(6)]
    rng = np.random.default_rng(5)
    case["init"]["C"] = 10.0 + rng.uniform(-0.5, 0.5, case["init"]["C"].size)
    case["init"]["Cl"] = case["init"]["C"].copy()
    o = oracle.Oracle(case)
    drift_planted = 0.0
    for _ in range(5):
        fn = o.fields()
        o.step(1, keep_intermediate=True)
        f = o.fields()
        assert np.ptp(f["T"]) == 0.0 and np.ptp(o.intermediate["Tstar"]) == 0.0
        assert np.abs(f["u"]).max() > 1e-5
        ustar = (o.intermediate["u"], o.intermediate["v"], np.zeros(1))
        drift_planted = max(drift_planted, np.ptp(_solve_with(case, fn, oracle.SYS_T, ustar)))
    assert drift_planted > 1e-9 * case["T0"], drift_planted


def _mushy_state(case, seed=7):
    """A flowing, partly solid state: random face velocities, g_l in
    [0.3, 0.95], C around C0, and T on the liquidus of the liquid
    concentration (eqs. 2.19-2.20), so every cell is mushy."""
    rng = np.random.default_rng(seed)
    al = case["alloy"]
    f = {k: np.array(v, copy=True) for k, v in case["init"].items()}
    for k in ("u", "v"):
        f[k] = rng.uniform(-2e-3, 2e-3, f[k].size)
    n = f["T"].size
    f["gl"] = rng.uniform(0.3, 0.95, n)
    f["C"] = 10.0 + rng.uniform(-1.0, 1.0, n)
    f["Cl"] = f["C"] / (al["k_p"] + (1.0 - al["k_p"]) * f["gl"])
    f["Cs"] = al["k_p"] * f["Cl"]
    f["T"] = al["T_m"] + al["m_sp"] * f["Cl"] - rng.uniform(0.0, 0.5, n)
    return f


def test_mushy_cells_sit_on_liquidus_of_new_composition():
    """After a step through a flowing mush, every cell left mushy satisfies
    T^{n+1} = T_m + m_sp C_l^{n+1} (eq. 2.20) with C_l^{n+1} from C^{n+1} and
    g_l^{n+1} (eq. 3.17): the liquidus of the phase update is T_l(C^{n+1})
    (eq. 3.13).  Planted mistake: the update with T_l(C^n) leaves the cells
    off that line by the composition change of the step."""
    case = W.cavity_2d(20, 12, lx=0.02, ly=0.012, tol=1e-13)
    al = case["alloy"]
    fn = _mushy_state(case)
    o = oracle.Oracle(case, fields=fn)
    o.step(1, keep_intermediate=True)
    f = o.fields()
    mush = (f["gl"] > 0.0) & (f["gl"] < 1.0)
    assert mush.sum() > 0.9 * mush.size
    off = np.abs(f["T"] - (al["T_m"] + al["m_sp"] * f["Cl"]))[mush]
    assert off.max() <= 1e-11 * al["T_m"], off.max()
    assert np.abs(f["C"] - fn["C"]).max() > 1e-3           # composition did move
    T, g, _, _, _ = o.phase(o.intermediate["Tstar"], fn["gl"], fn["C"])
    Cl = f["C"] / (1.0 + (1.0 - g) * (al["k_p"] - 1.0))
    m2 = (g > 0.0) & (g < 1.0)
    assert np.abs(T - (al["T_m"] + al["m_sp"] * Cl))[m2].max() > 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_step_rebuilt_from_forward_matrices(dim):
    """One whole step of the oracle against the same step rebuilt from the
    independent forward-method matrices (residual probing, Section 4) and
    dense direct solves, in the order of Algorithm 1: u* from the level-n
    fields; phi from u* (eq. 3.4, least squares, mean-free); u^{n+1} by the
    projection (eq. 3.5); C^{n+1} with u^{n+1} and g_l^n (eq. 3.10); T* with
    u^{n+1} (eq. 3.11); phase update with T*, g_l^n and C^{n+1}
    (eqs. 3.12-3.18)."""
    from oracle import forward
    if dim == 2:
        case = W.cavity_2d(9, 7, lx=0.009, ly=0.007, tol=1e-14)
    else:
        case = W.box_3d(6, 5, 4, lx=0.006, ly=0.005, lz=0.004, tol=1e-14)
    case["numerics"]["tol_p"] = 1e-14
    fn = _mushy_state(case) if dim == 2 else dict(case["init"])
    if dim == 3:
        rng = np.random.default_rng(8)
        fn = {k: np.array(v, copy=True) for k, v in fn.items()}
        for k in ("u", "v", "w"):
            fn[k] = rng.uniform(-2e-3, 2e-3, fn[k].size)
        fn["gl"] = rng.uniform(0.3, 1.0, fn["gl"].size)
        fn["T"] = fn["T"] - rng.uniform(0.0, 3.0, fn["T"].size)
    al, nm = case["alloy"], case["numerics"]
    g = case["grid"]
    n = (g["nx"], g["ny"], g["nz"] if dim == 3 else 1)
    h = (g["lx"] / n[0], g["ly"] / n[1], (g["lz"] / n[2]) if dim == 3 else 1.0)
    fw = dict(fn)
    if dim == 2:
        fw["w"] = np.zeros(0)
    ustar = []
    for d in range(dim):
        A, b = forward.forward_assemble(case, fw, d)
        ustar.append(np.linalg.solve(A.toarray(), b))
    A, b = forward.forward_assemble(case, fw, oracle.SYS_P, vel=tuple(ustar) + ((np.zeros(0),) if dim == 2 else ()))
    phi = np.linalg.lstsq(A.toarray(), b, rcond=None)[0]
    phi = phi - phi.mean()
    P = phi.reshape(n[2], n[1], n[0])
    unew = []
    for d in range(dim):
        ax = 2 - d
        grad = np.diff(P, axis=ax) / h[d]
        unew.append(ustar[d] - nm["dt"] / al["rho"] * grad.ravel())
    vel = tuple(unew) + ((np.zeros(0),) if dim == 2 else ())
    A, b = forward.forward_assemble(case, fw, oracle.SYS_C, vel=vel)
    Cnew = np.linalg.solve(A.toarray(), b)
    A, b = forward.forward_assemble(case, fw, oracle.SYS_T, vel=vel, t_new=nm["dt"])
    Tstar = np.linalg.solve(A.toarray(), b)
    o = oracle.Oracle(case, fields=fn)
    T, gl, Cl, Cs, _ = o.phase(Tstar, fn["gl"], Cnew)
    o.step(1, keep_intermediate=True)
    f = o.fields()
    def r(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    for d, k in enumerate("uvw"[:dim]):
        assert r(o.intermediate[k], ustar[d]) < 1e-10, k
        assert r(f[k], unew[d]) < 1e-10, k
    assert r(o.intermediate["phi"], phi) < 1e-10
    assert r(f["p"], fn["p"] + phi) < 1e-10 or np.linalg.norm(f["p"] - fn["p"] - phi) < 1e-10
    assert r(f["C"], Cnew) < 1e-12
    assert r(o.intermediate["Tstar"], Tstar) < 1e-12
    assert r(f["T"], T) < 1e-12 and np.abs(f["gl"] - gl).max() < 1e-10
    assert r(f["Cl"], Cl) < 1e-12 and r(f["Cs"], Cs) < 1e-12


# ---------------------------------------------- liquid solute diffusion

def test_liquid_diffusion_cosine_mode_decays_at_the_discrete_rate():
    """Eq. (3.7) in a still, fully liquid 1D bar (no buoyancy, adiabatic
    walls): C - C0 = A cos(pi x / L) is an eigenvector of the discrete
    Neumann Laplacian (DCT-II mode 1) with eigenvalue
    (4 D_l / h^2) sin^2(pi h / (2 L)), so each implicit step divides its
    amplitude by 1 + dt lambda_h exactly; the mean stays C0."""
    nx, L, D, dt, A0, nsteps = 40, 0.04, 1e-5, 0.5, 0.5, 20
    al = W.sn10pb_alloy(beta_T=0.0, beta_C=0.0, D_l=D)
    Tl = al["T_m"] + al["m_sp"] * 10.0
    case = W.make_case(2, nx, 1, 1, L, 1e-3, 1.0, alloy=al, T0=Tl + 20.0, dT_amp=0.0, dt=dt,
                       tol_p=1e-14, tol_t=1e-14)
    h = L / nx
    x = (np.arange(nx) + 0.5) * h
    mode = np.cos(np.pi * x / L)
    case["init"]["C"] = 10.0 + A0 * mode
    case["init"]["Cl"] = case["init"]["C"].copy()
    o = oracle.Oracle(case)
    o.step(nsteps)
    f = o.fields()
    assert np.all(f["gl"] == 1.0) and not f["u"].any()
    lam = 4.0 * D / h ** 2 * math.sin(math.pi * h / (2.0 * L)) ** 2
    expect = 10.0 + A0 * mode * (1.0 + dt * lam) ** (-nsteps)
    np.testing.assert_allclose(f["C"], expect, rtol=1e-12)
    assert abs(f["C"].mean() - 10.0) < 1e-13 * 10.0
    assert (1.0 + dt * lam) ** (-nsteps) < 0.6         # the mode did decay


def test_liquid_diffusion_acts_on_the_liquid_concentration():
    """A mushy, still state (no buoyancy, u = 0) whose liquid concentration
    C_l = C / (k_p + (1 - k_p) g_l) is uniform while g_l and hence C vary:
    eq. (3.7) diffuses C_l, so C^{n+1} = C^n.  Planted mistake: diffusing the
    mixture C itself (A_g = I, the same face coefficients) moves C."""
    al = W.sn10pb_alloy(beta_T=0.0, beta_C=0.0, D_l=1e-4)
    case = W.make_case(2, 12, 9, 1, 0.012, 0.009, 1.0, alloy=al, dT_amp=0.0, tol_p=1e-14, tol_t=1e-14)
    rng = np.random.default_rng(21)
    n = case["init"]["T"].size
    kp = al["k_p"]
    gl = rng.uniform(0.3, 0.9, n)
    Cl0 = 12.0
    f = {k: np.array(v, copy=True) for k, v in case["init"].items()}
    f["gl"] = gl
    f["Cl"] = np.full(n, Cl0)
    f["C"] = Cl0 * (kp + (1.0 - kp) * gl)
    f["Cs"] = kp * f["Cl"]
    f["T"] = al["T_m"] + al["m_sp"] * Cl0 + 0.0 * gl
    o = oracle.Oracle(case, fields=f)
    o.step(1)
    assert np.array_equal(o.fields()["C"], f["C"])
    # planted: the mixture diffused instead (A_g = I), same face g_l
    o2 = oracle.Oracle(case, fields=f)
    A, b, _, _ = o2.assemble(oracle.SYS_C, vel=tuple(np.zeros(max(1, f[k].size)) for k in ("u", "v", "w")))
    Id = np.eye(n) / case["numerics"]["dt"]
    ag = 1.0 / (kp + (1.0 - kp) * gl)
    M = (A.toarray() - Id) / ag[None, :]               # the diffusion rows without the A_g columns
    planted = np.linalg.solve(Id + M, b)
    assert np.abs(planted - f["C"]).max() > 1e-6


# ------------------------------------------- freckle cavity (Example 2)

@pytest.mark.parametrize("dim", [2, 3])
def test_freckle_recipe_perturbation_and_symmetry(dim):
    """Example 2's set-up: Pb-48%Sn at 216 degC, bottom wall T0 - b t, top
    wall T0, C = 1.0001 C0 on the vertical centre line.  The perturbation
    sits on the middle columns only; the Sn-rich (lighter, beta_C > 0)
    centre column rises; the cavity and its perturbation are mirror
    symmetric about the centre plane(s), so the velocity is too (to the
    solver tolerance)."""
    c = W.freckle_case(dim, tol=1e-13, mesh=(30, 90, 1) if dim == 2 else (12, 12, 36),
                       slip_sides=(dim == 3))
    c["numerics"]["tol_t"] = 1e-14
    g = c["grid"]
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    C = c["init"]["C"].reshape(nz, ny, nx)
    C0 = c["C0"]
    mid = [nx // 2 - 1, nx // 2]
    hot = np.zeros_like(C, bool)
    if dim == 2:
        hot[:, :, mid] = True
    else:
        hot[:, ny // 2 - 1:ny // 2 + 1, nx // 2 - 1:nx // 2 + 1] = True
    assert np.all(C[hot] == 1.0001 * C0) and np.all(C[~hot] == C0)
    bot, top = (2, 3) if dim == 2 else (4, 5)
    assert c["bcs"][bot]["thermal"] == W.THERMAL_DIRICHLET and c["bcs"][bot]["b"] == 0.05
    assert c["bcs"][top]["thermal"] == W.THERMAL_DIRICHLET and c["bcs"][top]["b"] == 0.0
    assert abs(c["bcs"][top]["T0"] - (216.0 + 273.15)) < 1e-12
    o = oracle.Oracle(c)
    o.step(10)
    f = o.fields()
    if dim == 2:
        v = f["v"].reshape(ny - 1, nx)
        assert np.all(v[ny // 3:2 * ny // 3, mid] > 0)
        assert np.abs(v - v[:, ::-1]).max() <= 1e-10 * np.abs(v).max()
    else:
        w = f["w"].reshape(nz - 1, ny, nx)
        assert np.all(w[nz // 3:2 * nz // 3, ny // 2 - 1:ny // 2 + 1, nx // 2 - 1:nx // 2 + 1] > 0)
        for ax in (1, 2):
            assert np.abs(w - np.flip(w, axis=ax)).max() <= 1e-10 * np.abs(w).max()
