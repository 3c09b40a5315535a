"""GPU check of the fused coarse multigrid levels (SOL_OPT_MG_FUSE): two
consecutive smoothed coarse levels run in one launch each way, every
workgroup recomputing its halo in local memory.  The fused cycle must give
the per-level cycle's results bit for bit: the same fields, iteration counts
and residuals, on 2D and 3D grids with odd counts, with one fused pair, with
a pair and a level left alone, at FP64 and in the FP32 inner solves of
mixed precision, alone and in a batch whose cases have different numbers of
levels (pair and single launches side by side)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

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


def _case(shape, precision, seed):
    if len(shape) == 2:
        nx, ny = shape
        if ny < 8:
            return W.cavity_2d(nx, ny, lx=nx * 1e-4, ly=ny * 1e-4, seed=seed, precision=precision)
        return W.cavity_2d(*shape, seed=seed, precision=precision)
    nx, ny, nz = shape
    return W.box_3d(nx, ny, nz, lx=nx * 1e-3, ly=ny * 1e-3, lz=nz * 1e-3, seed=seed, precision=precision)


# coarse levels above the exact one: (301, 183) and the 3D grids have two
# (one fused pair); (600, 400) has three (a pair and a single level);
# (8000, 2) is one cell high from level 1 on and (256, 256, 2) one cell deep,
# so their bricks straddle single-cell axes
SHAPES = [(301, 183), (600, 400), (72, 40, 40), (97, 75, 53), (8000, 2), (256, 256, 2)]


@pytest.mark.parametrize("precision", [W.PRECISION_FP64, W.PRECISION_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES, ids=["x".join(map(str, s)) for s in SHAPES])
def test_fused_equals_per_level_bitwise(sol, dev, shape, precision):
    case = _case(shape, precision, seed=sum(shape))
    print(f"[gpu] fused coarse levels {shape} precision {precision}", flush=True)
    out = []
    for fuse in (False, True):
        g = sol.Case(case, device=dev)
        g.set_mg_fuse(fuse)
        st = g.step(3)
        out.append((g.read_fields(), st))
        g.close()
    (fa, sa), (fb, sb) = out
    assert sa["iters_total"] == sb["iters_total"], (sa["iters_total"], sb["iters_total"])
    assert sa["rel_resid"] == sb["rel_resid"]
    for k in FIELDS:
        assert np.array_equal(fa[k], fb[k]), k


def test_fused_batch_with_different_level_counts(sol, dev):
    cases = W.batch_cases(n_cases=10, seed=5, precision=W.PRECISION_FP64)
    res = []
    for fuse in (False, True):
        hs = [sol.Case(c, device=dev) for c in cases]
        for h in hs:
            h.set_mg_fuse(fuse)
        bt = sol.Batch(hs)
        bt.step([3] * len(hs))
        bt.close()
        res.append([h.read_fields() for h in hs])
        for h in hs:
            h.close()
    for a, b in zip(*res):
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), k


def test_fused_matches_oracle(sol, dev):
    """A fused 2D cycle against the oracle at tight tolerances, per field."""
    case = W.cavity_2d(301, 183, seed=61, tol=3e-13)
    case["numerics"]["tol_t"] = 1e-14
    g = sol.Case(case, device=dev)
    g.step(2)
    got = g.read_fields()
    g.close()
    o = oracle.Oracle(case, threads=8)
    o.step(2)
    ref = o.fields()
    for k in FIELDS:
        a, b = got[k], ref[k]
        if len(b) == 0:
            continue
        if k == "p":
            a, b = a - a.mean(), b - b.mean()
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert e < 1e-9, (k, e)
