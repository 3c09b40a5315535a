"""GPU parity of the forward (residual-probing) assembly route, through the
C ABI (SOL_OPT_ASSEMBLY = SOL_ASSEMBLY_FORWARD; Section 4, eqs. 4.5-4.7):
the systems it writes equal the stencil route's and the oracle's (both of
its routes: row-by-row stencils and its own forward probing) up to a few
ulp of each row's scale, with the pattern bit-exact, and time steps
assembled this way match the oracle."""
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


def _perturbed(case, seed=11):
    rng = np.random.default_rng(seed)
    f = {k: np.array(v, dtype=np.float64, copy=True) for k, v in case["init"].items()}
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-2e-3, 2e-3, f[k].size)
    n = f["T"].size
    f["gl"] = rng.uniform(0.0, 1.0, n)
    f["p"] = rng.uniform(-2.0, 2.0, n)
    f["T"] = f["T"] + rng.uniform(-20.0, 5.0, n)
    f["C"] = f["C"] + rng.uniform(-1.0, 1.0, n)
    f["Cl"] = f["C"] / (f["gl"] + case["alloy"]["k_p"] * (1 - f["gl"]))
    return f


def _cases():
    c2 = W.cavity_2d(37, 23, seed=5)
    c2fs = W.cavity_2d(19, 11, seed=6)
    for bc in c2fs["bcs"]:
        bc["velocity"] = W.VELOCITY_FREESLIP
    c2fs["bcs"][3] = W.face_bc(W.THERMAL_DIRICHLET, T0=470.0, b=0.3, velocity=W.VELOCITY_FREESLIP)
    c3 = W.box_3d(13, 9, 6, lx=0.013, ly=0.009, lz=0.006, seed=7)
    c3["bcs"][5] = W.face_bc(W.THERMAL_ROBIN, h=150.0, T_ext=350.0)
    c2d = W.cavity_2d(37, 23, seed=5, alloy=W.sn10pb_alloy(D_l=5e-5))
    c3d = W.box_3d(13, 9, 6, lx=0.013, ly=0.009, lz=0.006, seed=7, alloy=W.sn10pb_alloy(D_l=5e-5))
    return [c2, c2fs, c3, c2d, c3d]


def _ulps(va, vb, rp, rhs_a, rhs_b, scale_rows):
    """Largest row-summed difference of the values and the largest rhs
    difference, in units of eps times the row scale."""
    dv = np.add.reduceat(np.abs(va - vb), rp[:-1])
    return max((dv / scale_rows).max(), (np.abs(rhs_a - rhs_b) / scale_rows).max()) / EPS


@pytest.mark.parametrize("case", _cases(), ids=["2d", "2d-freeslip-dirichlet", "3d", "2d-Dl", "3d-Dl"])
def test_forward_assembly_equals_stencil_and_oracle(sol, dev, case):
    """Same handle, same state: the momentum, solute and energy systems of
    the forward route against the stencil route, the oracle's stencil
    assembly and the oracle's forward probing (numpy face fluxes): pattern
    bit-exact; values and right-hand sides within 8 ulp of the row scale
    (the forward residual subtracts Eq(0) = -b, so each entry carries the
    rounding of b)."""
    f = _perturbed(case)
    g = sol.Case(case, device=dev, write_init=False)
    g.write_fields(f)
    vel = (f["u"], f["v"], f["w"] if f["w"].size else np.zeros(1))
    orc = oracle.Oracle(case, fields=f)
    fo = orc.fields()
    dim = case["grid"]["dim"]
    systems = [s for s in (0, 1, 2, 4, 5) if not (dim == 2 and s == 2)]
    g.assemble(0x3F)
    stencil = {s: g.read_matrix(s) for s in systems}
    g.set_assembly("forward")
    g.assemble(0x3F)
    worst = {}
    for s in systems:
        rp, ci, va, rhs = g.read_matrix(s)
        rps, cis, vas, rhss = stencil[s]
        assert np.array_equal(rp, rps) and np.array_equal(ci, cis), s
        v = vel if s >= 3 else None
        A, b, orp, oci = orc.assemble(s, vel=v)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci), s
        Af, bf = forward.forward_assemble(case, fo, s, vel=v, t_new=case["numerics"]["dt"])
        scale = np.add.reduceat(np.abs(A.data), A.indptr[:-1]) + np.abs(b)
        e_st = _ulps(va, vas, rp, rhs, rhss, scale)
        e_or = _ulps(va, A.data, rp, rhs, b, scale)
        e_fw = _ulps(va, Af.tocsr().data, rp, rhs, bf, scale)
        worst[s] = (round(e_st, 2), round(e_or, 2), round(e_fw, 2))
        assert max(e_st, e_or, e_fw) <= 8.0, (s, e_st, e_or, e_fw)
    print("forward route, ulp of the row scale vs (stencil route, oracle stencil, oracle forward):", worst)
    g.close()


@pytest.mark.parametrize("precision", [W.PRECISION_FP64, W.PRECISION_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name", ["2d-37x23", "3d-9x7x5", "2d-Dl"])
def test_forward_assembly_steps_match_oracle(sol, dev, name, precision):
    """Time steps whose momentum, solute and energy systems come from the
    forward route match the oracle per field (1e-9 FP64, 1e-8 mixed) at
    pressure tolerance 1e-13 and transport 1e-14."""
    if name == "2d-37x23":
        case = W.cavity_2d(37, 23, tol=1e-13, seed=1)
    elif name == "3d-9x7x5":
        case = W.box_3d(9, 7, 5, lx=0.009, ly=0.007, lz=0.005, tol=1e-13, seed=3)
    else:
        case = W.cavity_2d(37, 23, tol=1e-13, seed=11, alloy=W.sn10pb_alloy(D_l=5e-5), T_ext=250.0, h=2000.0)
    case["numerics"]["tol_t"] = 1e-14
    o = oracle.Oracle(case)
    o.step(5)
    ref = o.fields()
    case["numerics"]["precision"] = precision
    g = sol.Case(case, device=dev)
    g.set_assembly("forward")
    st = g.step(5)
    got = g.read_fields()
    g.close()
    gate = 1e-9 if precision == W.PRECISION_FP64 else 1e-8
    for k in FIELDS:
        a, b = got[k], ref[k]
        if len(b) == 0 or (k == "w" and len(a) == 0):
            continue
        if k == "p":
            a, b = a - a.mean(), b - b.mean()
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert e < gate, (k, e)
    for s in range(6):
        assert st["rel_resid"][s] <= (1e-13 if s == 3 else 1e-14) * (1 + 1e-6)


def test_batch_rejects_mixed_assembly_routes(sol, dev):
    import paper_2303_10783_amd.binding as B
    a = sol.Case(W.cavity_2d(20, 12, seed=81), device=dev)
    b = sol.Case(W.cavity_2d(24, 12, seed=82), device=dev)
    b.set_assembly("forward")
    with pytest.raises(B.SolError) as e:
        sol.Batch([a, b])
    assert e.value.code == B.SOL_EINVAL
    a.set_assembly("forward")
    bt = sol.Batch([a, b])
    bt.step([1, 1])
    bt.close()
    a.close()
    b.close()
