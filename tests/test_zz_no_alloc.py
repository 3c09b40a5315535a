"""GPU test of the allocation-free CSR export (sol_read_matrix_noalloc)
through the C ABI: its output equals sol_read_matrix's bit for bit (pattern
and values come from the same kernels), on two calls in a row on one GPU,
the first exporting 128x128x64 systems (7.2 million entries: several row
blocks through the fixed device scratch), the second a smaller 2D case
(one block), and a system beyond the scratch's maximum is refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sol():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2303_10783_amd as sol
    sol.load()
    return sol


def _perturb(case, seed):
    rng = np.random.default_rng(seed)
    f = {k: np.array(v, dtype=np.float64, copy=True) for k, v in case["init"].items()}
    for k in ("u", "v", "w"):
        f[k] = rng.uniform(-2e-3, 2e-3, f[k].size)
    f["gl"] = rng.uniform(0.0, 1.0, f["gl"].size)
    f["p"] = rng.uniform(-1.0, 1.0, f["p"].size)
    return f


def _compare_all(g, dim):
    for s in range(6):
        if dim == 2 and s == 2:
            continue
        a = g.read_matrix(s)
        b = g.read_matrix(s, noalloc=True)
        for x, y, name in zip(a, b, ("row_ptr", "col_idx", "val", "rhs")):
            assert x.dtype == y.dtype and x.shape == y.shape, (s, name)
            assert np.array_equal(x, y), (s, name)


def test_noalloc_export_equals_export(sol):
    dev = sol.TorchDevice(0)
    big = W.box_3d(128, 128, 64)
    print("[gpu] noalloc export: 128x128x64, then 37x23", flush=True)
    g = sol.Case(big, device=dev, write_init=False)
    g.write_fields(_perturb(big, 1))
    g.assemble(0x3F)
    _compare_all(g, 3)
    g.step(1)                     # the systems of a step, exported again
    _compare_all(g, 3)
    g.close()
    small = W.cavity_2d(37, 23, seed=2)
    g = sol.Case(small, device=dev, write_init=False)
    g.write_fields(_perturb(small, 3))
    g.assemble(0x3F)
    _compare_all(g, 2)
    g.close()


def test_noalloc_export_refuses_oversize_system(sol):
    import paper_2303_10783_amd.binding as B
    dev = sol.TorchDevice(0)
    case = W.cavity_2d(2050, 2046, lx=0.205, ly=0.2046)      # 4 194 300 pressure rows
    g = sol.Case(case, device=dev)
    with pytest.raises(B.SolError) as e:
        g.read_matrix(3, noalloc=True)
    assert e.value.code == B.SOL_EINVAL and "scratch" in str(e.value)
    rp, ci, va, rhs = g.read_matrix(0, noalloc=True)           # u: 2049 x 2046 rows, fits
    assert rp[-1] == ci.size
    g.close()
