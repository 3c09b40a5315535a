"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects invalid arguments before any device work."""
import ctypes as C
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sol.h")


@pytest.fixture(scope="module")
def sol():
    import paper_2303_10783_amd as sol
    from paper_2303_10783_amd import build as b
    if not os.path.exists(b.OUT):
        b.build()
    sol.load()
    return sol


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sol_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(sol):
    L = sol.load()
    names = _declared()
    assert "sol_create" in names and "sol_step" in names and "sol_batch_step" in names
    for n in names:
        assert hasattr(L, n), n
    from paper_2303_10783_amd import binding
    assert sorted(binding.exported_symbols()) == names


def _structs(sol, case):
    from paper_2303_10783_amd import binding
    return binding.make_structs(case)


@pytest.mark.parametrize("mutate,field", [
    (lambda c: c["grid"].update(nx=1), "nx"),
    (lambda c: c["grid"].update(dim=4), "dim"),
    (lambda c: c["numerics"].update(dt=0.0), "dt"),
    (lambda c: c["numerics"].update(dt=float("nan")), "dt"),
    (lambda c: c["numerics"].update(tol_p=0.0), "tolerance"),
    (lambda c: c["numerics"].update(max_iter=0), "max_iter"),
    (lambda c: c["alloy"].update(k_p=1.2), "k_p"),
    (lambda c: c["alloy"].update(m_sp=2.33), "m_sp"),
    (lambda c: c["alloy"].update(rho=-1.0), "rho"),
    (lambda c: c["alloy"].update(D_l=-1e-9), "D_l"),
    (lambda c: c["bcs"][0].update(h=-5.0), "Robin"),
    (lambda c: c["grid"].update(lx=0.0), "lengths"),
])
def test_invalid_arguments_rejected_before_device_work(sol, mutate, field):
    from paper_2303_10783_amd import binding
    case = W.cavity_2d(8, 6)
    mutate(case)
    grid, alloy, bcs, num = binding.make_structs(case)
    h = C.c_void_p()
    rc = sol.load().sol_create(C.byref(grid), C.byref(alloy), C.byref(bcs), C.byref(num), None, C.byref(h))
    assert rc == binding.SOL_EINVAL
    assert h.value is None
    assert sol.load().sol_last_error().decode()


def test_null_arguments(sol):
    from paper_2303_10783_amd import binding
    L = sol.load()
    h = C.c_void_p()
    assert L.sol_create(None, None, None, None, None, C.byref(h)) == binding.SOL_EINVAL
    assert L.sol_step(None, 1, None) == binding.SOL_EINVAL
    assert L.sol_read_fields(None, 1, None) == binding.SOL_EINVAL
    assert L.sol_batch_create(None, 0, C.byref(h)) == binding.SOL_EINVAL
    L.sol_destroy(None)
    L.sol_batch_destroy(None)
    assert L.sol_dispatch_count(None) == binding.SOL_EINVAL


def test_dispatch_count_without_device_work(sol):
    """The dispatch counter is readable without a device and does not move
    for calls rejected before any device work."""
    from paper_2303_10783_amd import binding
    n0 = binding.dispatch_count()
    L = sol.load()
    assert L.sol_step(None, 1, None) == binding.SOL_EINVAL
    assert binding.dispatch_count() == n0 >= 0


def test_footprint_scales_with_cells(sol):
    # both 2D grids end their multigrid hierarchy on the same 25 x 15 level,
    # whose dense inverse (375^2 doubles) is a per-case constant
    f1 = sol.sol_footprint_bytes(W.cavity_2d(100, 60))
    f2 = sol.sol_footprint_bytes(W.cavity_2d(200, 120))
    f3 = sol.sol_footprint_bytes(W.box_3d(32, 32, 32))
    per_cell = (f2 - f1) / (200 * 120 - 100 * 60)
    assert 300 < per_cell < 1500                   # bytes per cell, 2D
    assert 3.0 < f2 / f1 < 4.5
    assert f3 / 32 ** 3 > f2 / (200 * 120)         # 3D stores 7 diagonals


def _defines():
    out = {}
    for name, val in re.findall(r"#define\s+(SOL_[A-Z0-9_]+)\s+(-?\d+)\b", open(HEADER).read()):
        out[name] = int(val)
    return out


def test_binding_constants_match_header():
    """The marshalling layer's numeric constants are the header's."""
    from paper_2303_10783_amd import binding as B
    d = _defines()
    for name in ("SOL_OK", "SOL_EINVAL", "SOL_ENOMEM", "SOL_ENOCONV", "SOL_ENONFINITE", "SOL_EDEVICE", "SOL_EBUSY"):
        assert getattr(B, name) == d[name], name
    assert (B.OPT_GRAPH, B.OPT_PRECOND, B.OPT_TPRECOND) == (d["SOL_OPT_GRAPH"], d["SOL_OPT_PRECOND"], d["SOL_OPT_TPRECOND"])
    assert (B.OPT_ASSEMBLY, B.OPT_MOMENTUM, B.OPT_MG_FUSE) == (d["SOL_OPT_ASSEMBLY"], d["SOL_OPT_MOMENTUM"],
                                                               d["SOL_OPT_MG_FUSE"])
    assert B.ASSEMBLY == dict(stencil=d["SOL_ASSEMBLY_STENCIL"], forward=d["SOL_ASSEMBLY_FORWARD"])
    assert (B.MOMENTUM_PLAIN, B.MOMENTUM_MINIMAL) == (d["SOL_MOMENTUM_PLAIN"], d["SOL_MOMENTUM_MINIMAL"])
    import workloads as W
    assert (W.MOMENTUM_PLAIN, W.MOMENTUM_MINIMAL) == (d["SOL_MOMENTUM_PLAIN"], d["SOL_MOMENTUM_MINIMAL"])
    assert B.PRECOND == dict(jacobi=d["SOL_PRECOND_JACOBI"], mg=d["SOL_PRECOND_MG"])
    assert B.TPRECOND == dict(jacobi=d["SOL_TPRECOND_JACOBI"], jacobi2=d["SOL_TPRECOND_JACOBI2"],
                              auto=d["SOL_TPRECOND_AUTO"])
    kc = {k: v for k, v in d.items() if k.startswith("SOL_KCLASS_")}
    assert sorted(B.KCLASS.values()) == sorted(kc.values())
    assert len(B.KCLASS) == d["SOL_NKCLASS"]


def test_set_option_rejects_null_handle(sol):
    from paper_2303_10783_amd import binding as B
    L = sol.load()
    for opt, val in ((B.OPT_GRAPH, 1), (B.OPT_PRECOND, 0), (B.OPT_TPRECOND, 2), (B.OPT_ASSEMBLY, 1),
                     (B.OPT_MOMENTUM, 1), (B.OPT_MG_FUSE, 0)):
        assert L.sol_set_option(None, opt, val) == B.SOL_EINVAL


# the calls of the problem statement: each declaration's comment names the
# passage of the paper that defines the operation
PAPER_CALLS = ("sol_create", "sol_write_fields", "sol_read_fields", "sol_system_size", "sol_assemble",
               "sol_read_matrix", "sol_step", "sol_footprint_bytes", "sol_batch_create", "sol_batch_step")


def _comment_before(txt, name):
    """The comment block closest above the declaration of `name` (a comment
    may head a group of declarations, as for the two batch calls)."""
    i = re.search(r"\b(int|void|const char \*)\s+" + name + r"\s*\(", txt).start()
    j = txt.rfind("*/", 0, i)
    k = txt.rfind("/*", 0, j)
    assert 0 <= k < j, name
    return txt[k:j]


@pytest.mark.parametrize("name", PAPER_CALLS)
def test_header_cites_defining_passage(name):
    txt = open(HEADER).read()
    c = _comment_before(txt, name)
    assert re.search(r"(eqs?\.\s*\d\.\d+|Algorithm 1|Section \d|Table 1)", c), (name, c)
