"""GPU parity, through the C ABI, of the momentum predictor in the minimal
model's form, eq. (2.6) (SOL_OPT_MOMENTUM = SOL_MOMENTUM_MINIMAL): advecting
velocity u/g_l; pressure gradient, Carman-Kozeny drag (eq. 2.8) and force
scaled by g_l.  The systems of both assembly routes against both oracle
routes, on states whose g_l spans solid cells, the floor of the
regularisation, mush and liquid; time steps against the oracle (FP64 and
mixed precision); equality with eq. (2.7) in liquid melt; a batch that mixes
the two forms against its cases run alone."""
import numpy as np
import pytest

import oracle
from oracle import forward
import workloads as W

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
FIELDS = ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")


@pytest.fixture(scope="module")
def sol():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2303_10783_amd as sol
    sol.load()
    return sol


@pytest.fixture(scope="module")
def dev(sol):
    return sol.TorchDevice(0)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.size == 0:
        return 0.0
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def field_errors(got, ref):
    out = {}
    for k in FIELDS:
        a, b = got[k], ref[k]
        if len(b) == 0 or (k == "w" and len(a) == 0):
            continue
        if k == "p":
            a, b = a - a.mean(), b - b.mean()
        out[k] = rel(a, b)
    return out


def _minimal(case):
    return W.with_momentum(case, W.MOMENTUM_MINIMAL)


def _perturbed(case, seed=17):
    """g_l uniform on [0, 1] with exact 0 (solid) and 1 (liquid) cells, so
    the rows meet every regime of the form: solid, below and above the
    floor darcy_eps^(1/3), liquid."""
    rng = np.random.default_rng(seed)
    f = {k: np.array(v, dtype=np.float64, copy=True) for k, v in case["init"].items()}
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-2e-3, 2e-3, f[k].size)
    n = f["T"].size
    f["gl"] = rng.uniform(0.0, 1.0, n)
    f["gl"][::7] = 0.0
    f["gl"][3::11] = 1.0
    f["p"] = rng.uniform(-2.0, 2.0, n)
    f["T"] = f["T"] + rng.uniform(-20.0, 5.0, n)
    f["C"] = f["C"] + rng.uniform(-1.0, 1.0, n)
    f["Cl"] = f["C"] / (f["gl"] + case["alloy"]["k_p"] * (1 - f["gl"]))
    return f


def _asm_cases():
    c2 = W.cavity_2d(37, 23, seed=5)
    c2fs = W.cavity_2d(19, 11, seed=6)
    for bc in c2fs["bcs"]:
        bc["velocity"] = W.VELOCITY_FREESLIP
    c3 = W.box_3d(13, 9, 6, lx=0.013, ly=0.009, lz=0.006, seed=7)
    c3["bcs"][1] = W.face_bc(velocity=W.VELOCITY_FREESLIP)
    return [_minimal(c) for c in (c2, c2fs, c3)]


def _row_ulps(va, vb, rp, rhs_a, rhs_b, scale_rows):
    dv = np.add.reduceat(np.abs(va - vb), rp[:-1])
    return max((dv / scale_rows).max(), (np.abs(rhs_a - rhs_b) / scale_rows).max()) / EPS


@pytest.mark.parametrize("case", _asm_cases(), ids=["2d", "2d-freeslip", "3d"])
def test_systems_match_oracle_both_routes(sol, dev, case):
    """Momentum systems of the form (2.6): stencil route within 4 ulp of the
    row scale of the oracle's rows, forward route within 8 ulp of the
    oracle's stencil rows and its forward probing; patterns bit-exact.  The
    same state's (2.7) systems differ by far more (the test sees the form)."""
    print(f"[gpu] momentum form (2.6) systems, {case['name']}", flush=True)
    f = _perturbed(case)
    g = sol.Case(case, device=dev, write_init=False)
    g.write_fields(f)
    orc = oracle.Oracle(case, fields=f)
    plain = oracle.Oracle(W.with_momentum(case, W.MOMENTUM_PLAIN), fields=f)
    fo = orc.fields()
    systems = [0, 1] if case["grid"]["dim"] == 2 else [0, 1, 2]
    mask = sum(1 << s for s in systems)
    g.assemble(mask)
    stencil = {s: g.read_matrix(s) for s in systems}
    g.set_assembly("forward")
    g.assemble(mask)
    worst = {}
    for s in systems:
        A, b, orp, oci = orc.assemble(s)
        Af, bf = forward.forward_assemble(case, fo, s)
        scale = np.add.reduceat(np.abs(A.data), A.indptr[:-1]) + np.abs(b)
        rp, ci, va, rhs = stencil[s]
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci), s
        e_st = _row_ulps(va, A.data, rp, rhs, b, scale)
        assert e_st <= 4.0, (s, e_st)
        rp2, ci2, va2, rhs2 = g.read_matrix(s)
        assert np.array_equal(rp2, orp) and np.array_equal(ci2, oci), s
        e_fo = _row_ulps(va2, A.data, rp, rhs2, b, scale)
        e_ff = _row_ulps(va2, Af.tocsr().data, rp, rhs2, bf, scale)
        assert max(e_fo, e_ff) <= 8.0, (s, e_fo, e_ff)
        A2, b2, _, _ = plain.assemble(s)
        assert _row_ulps(va, A2.data, rp, rhs, b2, scale) > 1e6, s
        worst[s] = (round(e_st, 2), round(e_fo, 2), round(e_ff, 2))
    print("form (2.6), ulp of the row scale (stencil vs oracle, forward vs oracle stencil, vs oracle forward):",
          worst, flush=True)
    g.close()


def _liquid_melt(dim, seed):
    if dim == 2:
        c = W.cavity_2d(24, 16, seed=seed, tol=1e-12)
    else:
        c = W.box_3d(10, 8, 6, lx=0.010, ly=0.008, lz=0.006, seed=seed, tol=1e-12)
    al = c["alloy"]
    T0 = al["T_m"] + al["m_sp"] * c["C0"] + 5.0
    g = c["grid"]
    return W.make_case(dim, g["nx"], g["ny"], g["nz"], g["lx"], g["ly"], g["lz"], T0=T0, dT_amp=2.0,
                       bcs=c["bcs"], tol_p=1e-12, tol_t=1e-12, seed=seed)


@pytest.mark.parametrize("dim", [2, 3])
def test_liquid_melt_equals_plain_form_bitwise(sol, dev, dim):
    """Fully liquid melt (g_l = 1 throughout): the two forms coincide, so
    the GPU fields of five steps are bit-identical."""
    case = _liquid_melt(dim, 30 + dim)
    out = {}
    for form in (W.MOMENTUM_PLAIN, W.MOMENTUM_MINIMAL):
        g = sol.Case(W.with_momentum(case, form), device=dev)
        g.step(5)
        out[form] = g.read_fields()
        g.close()
    assert out[W.MOMENTUM_PLAIN]["gl"].min() == 1.0
    assert np.abs(out[W.MOMENTUM_PLAIN]["v"]).max() > 0.0
    for k in FIELDS:
        assert np.array_equal(out[W.MOMENTUM_PLAIN][k], out[W.MOMENTUM_MINIMAL][k]), k


def _step_case(name):
    if name == "2d-mush":
        return _minimal(W.cavity_2d(37, 23, tol=1e-13, seed=21, T_ext=250.0, h=2000.0)), 6
    if name == "3d-mush":
        return _minimal(W.box_3d(9, 7, 5, lx=0.009, ly=0.007, lz=0.005, tol=1e-13, seed=22,
                                 T_ext=250.0, h=2000.0)), 4
    raise KeyError(name)


@pytest.mark.parametrize("precision", [W.PRECISION_FP64, W.PRECISION_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name", ["2d-mush", "3d-mush"])
def test_steps_match_oracle(sol, dev, name, precision):
    """A cooled cavity developing a mush, stepped in the form (2.6): every
    field within 1e-9 (FP64) / 1e-8 (mixed) of the oracle at pressure
    tolerance 1e-13 and transport 1e-14; the (2.7) fields of the same steps
    are ~1e-2 away in u, v, p."""
    case, nsteps = _step_case(name)
    case["numerics"]["tol_t"] = 1e-14
    print(f"[gpu] momentum form (2.6) steps, {name}, precision {precision}", flush=True)
    o = oracle.Oracle(case)
    o.step(nsteps)
    ref = o.fields()
    c = dict(case)
    c["numerics"] = dict(case["numerics"], precision=precision)
    g = sol.Case(c, device=dev)
    st = g.step(nsteps)
    got = g.read_fields()
    g.close()
    errs = field_errors(got, ref)
    gate = 1e-9 if precision == W.PRECISION_FP64 else 1e-8
    assert max(errs.values()) < gate, errs
    for s in range(6):
        assert st["rel_resid"][s] <= (1e-13 if s == 3 else 1e-14) * (1 + 1e-6)
    if precision == W.PRECISION_FP64:
        p = oracle.Oracle(W.with_momentum(case, W.MOMENTUM_PLAIN))
        p.step(nsteps)
        far = field_errors(p.fields(), ref)
        assert min(far["u"], far["v"], far["p"]) > 1e-4, far


def test_steps_from_solid_and_mush_match_oracle(sol, dev):
    """Two steps from a state with solid cells (g_l = 0), cells below the
    floor of the regularisation, mush and liquid, all moving: FP64 fields
    within 1e-9 of the oracle."""
    case = _minimal(W.cavity_2d(21, 13, tol=1e-13, seed=23))
    case["numerics"]["tol_t"] = 1e-14
    f = _perturbed(case, seed=29)
    o = oracle.Oracle(case, fields=f)
    o.step(2)
    g = sol.Case(case, device=dev, write_init=False)
    g.write_fields(f)
    g.step(2)
    errs = field_errors(g.read_fields(), o.fields())
    g.close()
    assert max(errs.values()) < 1e-9, errs


def test_batch_mixing_forms_equals_alone(sol, dev):
    """One batch launch serves a (2.6) case and a (2.7) case: each equals
    the same case advanced alone, bit for bit."""
    ca = _minimal(W.cavity_2d(30, 18, seed=41, T_ext=250.0, h=2000.0))
    cb = W.cavity_2d(26, 20, seed=42, T_ext=250.0, h=2000.0)
    alone = []
    for c in (ca, cb):
        g = sol.Case(c, device=dev)
        g.step(4)
        alone.append(g.read_fields())
        g.close()
    a = sol.Case(ca, device=dev)
    b = sol.Case(cb, device=dev)
    bt = sol.Batch([a, b])
    bt.step([4, 4])
    bt.close()
    for g, ref in zip((a, b), alone):
        got = g.read_fields()
        for k in FIELDS:
            assert np.array_equal(got[k], ref[k]), k
        g.close()


def test_option_validation(sol, dev):
    import paper_2303_10783_amd.binding as B
    a = sol.Case(W.cavity_2d(12, 8, seed=51), device=dev)
    with pytest.raises(B.SolError) as e:
        a.set_momentum(7)
    assert e.value.code == B.SOL_EINVAL
    b = sol.Case(W.cavity_2d(12, 8, seed=52), device=dev)
    bt = sol.Batch([a, b])
    with pytest.raises(B.SolError) as e:
        a.set_momentum(W.MOMENTUM_MINIMAL)
    assert e.value.code == B.SOL_EBUSY
    bt.close()
    a.set_momentum(W.MOMENTUM_MINIMAL)
    a.step(1)
    a.close()
    b.close()
