"""Pins of the oracle's momentum predictor in the minimal model's form,
eq. (2.6): u_t + (u/g_l).grad u = div(nu grad u) - (g_l/rho) grad p
- (mu g_l/rho) K^-1 u + g_l f, against facts that do not come from the
oracle's own arithmetic:

* in fully liquid melt the two forms coincide (the paper's remark after
  eq. 2.7), so with g_l = 1 the systems and whole time steps must equal
  those of eq. (2.7) bit for bit;
* first-order upwinding is positively homogeneous in the advecting
  velocity, so in a uniform mush g0 the convection of (2.6) is that of
  eq. (2.7) with the velocity field u/g0, and the two matrices differ only
  on the diagonal, by (g0 - 1) times the drag of (2.7);
* the right-hand side is linear in the pressure gradient and the force, so
  with u^n = 0 and a uniform g0 the (2.6) right-hand side is g0 times that
  of (2.7);
* in solid cells (g_l = 0) the pressure gradient and the force vanish and
  the drag is the floor darcy_eps^(1/3) times the drag of (2.7) there (the
  reading that keeps the flow stopped);
* the forward-probe route assembles the same (2.6) systems (tests of the
  assembly module).

The drag of (2.7) is read off the oracle's own (2.7) systems as a
difference of diagonals (K^-1 = 0 at g_l = 1), not retyped."""
import numpy as np
import pytest

import oracle
import workloads as W

EPS = np.finfo(float).eps


def _cases():
    c2 = W.cavity_2d(9, 6, seed=3)
    c3 = W.box_3d(6, 5, 4, lx=0.06, ly=0.05, lz=0.04, seed=4)
    c3["bcs"][2] = W.face_bc(velocity=W.VELOCITY_FREESLIP)
    return [c2, c3]


IDS = ["2d", "3d"]


def _fields(case, seed, gl=None, vel_amp=1e-3):
    f = oracle.Oracle(case).fields()
    rng = np.random.default_rng(seed)
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-vel_amp, vel_amp, f[k].size) if vel_amp else np.zeros(f[k].size)
    f["p"] = rng.uniform(-2.0, 2.0, f["p"].size)
    f["T"] = f["T"] + rng.uniform(-3.0, 3.0, f["T"].size)
    f["Cl"] = f["Cl"] + rng.uniform(-1.0, 1.0, f["Cl"].size)
    f["gl"] = rng.uniform(0.0, 1.0, f["gl"].size) if gl is None else np.full(f["gl"].size, float(gl))
    return f


def _momentum_systems(case):
    return [0, 1] if case["grid"]["dim"] == 2 else [0, 1, 2]


def _asm(case, form, f, s):
    A, b, _, _ = oracle.Oracle(W.with_momentum(case, form), fields=f).assemble(s)
    return A.tocsr(), b


@pytest.mark.parametrize("case", _cases(), ids=IDS)
def test_liquid_systems_equal_plain_form(case):
    f = _fields(case, 1, gl=1.0)
    for s in _momentum_systems(case):
        A1, b1 = _asm(case, W.MOMENTUM_MINIMAL, f, s)
        A2, b2 = _asm(case, W.MOMENTUM_PLAIN, f, s)
        assert np.array_equal(A1.indptr, A2.indptr) and np.array_equal(A1.indices, A2.indices)
        assert np.array_equal(A1.data, A2.data), s
        assert np.array_equal(b1, b2), s


@pytest.mark.parametrize("case", _cases(), ids=IDS)
def test_liquid_steps_equal_plain_form(case):
    """Five whole steps of a melt that stays liquid (started 5 K above the
    liquidus, so the buoyancy drives a flow): identical fields."""
    al = case["alloy"]
    T0 = al["T_m"] + al["m_sp"] * case["C0"] + 5.0
    c = W.make_case(case["grid"]["dim"], case["grid"]["nx"], case["grid"]["ny"], case["grid"]["nz"],
                    case["grid"]["lx"], case["grid"]["ly"], case["grid"]["lz"], T0=T0, dT_amp=2.0,
                    bcs=case["bcs"], tol_p=1e-12, tol_t=1e-12, seed=5)
    out = {}
    for form in (W.MOMENTUM_PLAIN, W.MOMENTUM_MINIMAL):
        o = oracle.Oracle(W.with_momentum(c, form))
        o.step(5)
        out[form] = o.fields()
    assert out[W.MOMENTUM_PLAIN]["gl"].min() == 1.0
    assert np.abs(out[W.MOMENTUM_PLAIN]["v"]).max() > 0.0
    for k in ("u", "v", "w", "p", "T", "C"):
        assert np.array_equal(out[W.MOMENTUM_PLAIN][k], out[W.MOMENTUM_MINIMAL][k]), k


@pytest.mark.parametrize("g0", [0.8, 0.35, 0.05])
@pytest.mark.parametrize("case", _cases(), ids=IDS)
def test_uniform_mush_convection_of_u_over_g(case, g0):
    """A_(2.6)(u; g0) - A_(2.7)(u/gt; g0) = diag((gt - 1) drag_(2.7)(g0)),
    gt = max(g0, darcy_eps^(1/3)) (g0 = 0.05 lies below that floor), entry
    by entry to a few ulp of each entry's scale; the convective parts
    dominate the off-diagonal entries (a missing 1/gt would move them by
    ~25-1900 %)."""
    gt = max(g0, float(np.cbrt(case["alloy"]["darcy_eps"])))
    f = _fields(case, 2, gl=g0)
    fs = dict(f)
    for k in ("u", "v", "w"):
        fs[k] = f[k] / gt
    f0, f1 = dict(f), dict(f)
    for k in ("u", "v", "w"):
        f0[k] = np.zeros(f[k].size)
        f1[k] = np.zeros(f[k].size)
    f1["gl"] = np.ones(f["gl"].size)
    for s in _momentum_systems(case):
        A1, _ = _asm(case, W.MOMENTUM_MINIMAL, f, s)
        A2, _ = _asm(case, W.MOMENTUM_PLAIN, fs, s)
        Ad, _ = _asm(case, W.MOMENTUM_PLAIN, f0, s)
        Al, _ = _asm(case, W.MOMENTUM_PLAIN, f1, s)
        drag = Ad.diagonal() - Al.diagonal()
        assert drag.min() > 0.0
        D = (A1 - A2).tocsr()
        off = D.copy()
        off.setdiag(0.0)
        # scale of an entry: its diffusion and convection parts, and the
        # velocities whose face mean (which may cancel) was divided by gt
        g = case["grid"]
        hmin = min(g["lx"] / g["nx"], g["ly"] / g["ny"], g["lz"] / g["nz"] if g["dim"] == 3 else 1.0)
        vmax = max(np.abs(f[k]).max() for k in ("u", "v", "w") if f[k].size)
        scale = np.abs(A1).toarray() + np.abs(A2).toarray() + np.abs(Al).toarray() + vmax / (gt * hmin)
        assert (np.abs(off.toarray()) <= 8 * EPS * scale).all(), s
        want = (gt - 1.0) * drag
        dscale = np.abs(A1.diagonal()) + np.abs(A2.diagonal()) + np.abs(Ad.diagonal())
        assert (np.abs(D.diagonal() - want) <= 16 * EPS * dscale).all(), s
        # the convective part of the off-diagonals is what was checked
        conv = np.abs((A2 - Al).toarray())
        np.fill_diagonal(conv, 0.0)
        assert conv.max() > 10 * np.abs(Al.toarray() - np.diag(Al.diagonal())).max()


@pytest.mark.parametrize("g0", [0.8, 0.35, 0.02])
@pytest.mark.parametrize("case", _cases(), ids=IDS)
def test_uniform_mush_rhs_scales_with_g(case, g0):
    """u^n = 0: b_(2.6) = g0 b_(2.7), for the pressure gradient alone
    (T = T_ref, C_l = C_ref) and for the buoyancy alone (p = 0), each to an
    ulp or two (also below the floor: only 1/g and the drag use it)."""
    al = case["alloy"]
    f = _fields(case, 3, gl=g0, vel_amp=0.0)
    fp, ff = dict(f), dict(f)
    fp["T"] = np.full(f["T"].size, al["T_ref"])
    fp["Cl"] = np.full(f["Cl"].size, al["C_ref"])
    ff["p"] = np.zeros(f["p"].size)
    for fx in (fp, ff):
        for s in _momentum_systems(case):
            _, b1 = _asm(case, W.MOMENTUM_MINIMAL, fx, s)
            _, b2 = _asm(case, W.MOMENTUM_PLAIN, fx, s)
            if fx is ff and s != case["grid"]["dim"] - 1:
                assert not np.any(b1) and not np.any(b2)
                continue
            assert np.abs(b2).max() > 0.0
            assert (np.abs(b1 - g0 * b2) <= 2 * EPS * np.abs(b1)).all(), s


@pytest.mark.parametrize("case", _cases(), ids=IDS)
def test_solid_cells_drag_floor_and_no_forcing(case):
    """g_l = 0: no pressure gradient or force in b, and the drag is the
    floor g~ = darcy_eps^(1/3) times the drag of (2.7) at g_l = 0."""
    f = _fields(case, 4, gl=0.0, vel_amp=0.0)
    f1 = dict(f)
    f1["gl"] = np.ones(f["gl"].size)
    gfloor = np.cbrt(case["alloy"]["darcy_eps"])
    for s in _momentum_systems(case):
        A1, b1 = _asm(case, W.MOMENTUM_MINIMAL, f, s)
        A2, _ = _asm(case, W.MOMENTUM_PLAIN, f, s)
        Al, _ = _asm(case, W.MOMENTUM_PLAIN, f1, s)
        assert not np.any(b1)
        drag2 = A2.diagonal() - Al.diagonal()
        drag1 = A1.diagonal() - Al.diagonal()
        assert (np.abs(drag1 - gfloor * drag2) <= 16 * EPS * A2.diagonal()).all(), s
        # still far above the transient term: the flow is held
        assert drag1.min() > 1e3 / case["numerics"]["dt"]
