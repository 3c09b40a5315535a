"""GPU parity, through the C ABI, of the parts the time-marching runs of the
other parity tests do not reach:

* the phase update in all four branches of the enthalpy classification
  (solid, eutectic plateau, mush, liquid; eqs. 3.12-3.18 and the eutectic
  rule stated after eq. 3.16), including cells that remelt;
* the advecting field of the solute and energy solves (u^{n+1}), through two
  invariants that hold exactly for the projected velocity;
* batched and served (continuous batching) runs against the oracle, per case
  and per field, not only against the same cases advanced alone.
"""
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


# ----------------------------------------------------------------- phase

def _branch_fields(case, seed):
    """Level-n fields whose enthalpy H = T + (L/c_p) g_l spans the four
    branches of the phase update for a cell-wise composition C in [5, 15]:
    solid (H < T_e), eutectic plateau (T_e <= H < T_e + (L/c_p) g_eut),
    mush (up to T_l(C) + L/c_p) and liquid; g_l^n is drawn independently of
    H, so heated cells (remelting: H above the present state's enthalpy)
    occur in every branch.  A few cells sit exactly on a branch boundary of
    H."""
    rng = np.random.default_rng(seed)
    al = case["alloy"]
    lam = al["latent"] / al["cp"]
    kp = al["k_p"]
    n = case["init"]["T"].size
    f = {k: np.array(v, copy=True) for k, v in case["init"].items()}
    C = rng.uniform(5.0, 15.0, n)
    gn = rng.uniform(0.0, 1.0, n)
    gn[::11] = 0.0
    gn[5::13] = 1.0
    Tl = al["T_m"] + al["m_sp"] * C
    Te = al["T_m"] + al["m_sp"] * al["C_e"]
    geut = np.clip(1.0 - (Te - Tl) / ((1.0 - kp) * (Te - al["T_m"])), 0.0, 1.0)
    target = rng.integers(0, 4, n)
    lo = np.select([target == 0, target == 1, target == 2, target == 3],
                   [Te - 40.0, Te, Te + lam * geut, Tl + lam])
    hi = np.select([target == 0, target == 1, target == 2, target == 3],
                   [Te, Te + lam * geut, Tl + lam, Tl + lam + 30.0])
    H = lo + rng.uniform(0.0, 1.0, n) * (hi - lo)
    edge = np.arange(n) % 17 == 3
    H[edge] = lo[edge]
    f["C"] = C
    f["gl"] = gn
    f["T"] = H - lam * gn
    f["Cl"] = C / (kp + (1.0 - kp) * gn)
    f["Cs"] = kp * f["Cl"]
    return f


@pytest.mark.parametrize("dim", [2, 3])
def test_phase_update_all_branches(sol, dev, dim):
    """One step of a still, buoyancy-free melt (u = p = 0, adiabatic walls,
    dt = 1e-6 s, so T* stays near T^n) from fields that put cells in every
    branch; the GPU's T^{n+1}, g_l^{n+1}, C_l^{n+1}, C_s^{n+1} against the
    oracle's phase update of the GPU's own T*, g_l^n and C^{n+1}, cell by
    cell.  The oracle's branch output must show all four branches, remelting
    cells among them."""
    al = W.sn10pb_alloy(beta_T=0.0, beta_C=0.0)
    if dim == 2:
        case = W.make_case(2, 61, 37, 1, 0.061, 0.037, 1.0, alloy=al, dt=1e-6, tol_p=1e-13, tol_t=1e-14)
    else:
        case = W.make_case(3, 17, 13, 11, 0.017, 0.013, 0.011, alloy=al, dt=1e-6, tol_p=1e-13, tol_t=1e-14)
    f = _branch_fields(case, seed=40 + dim)
    print(f"[gpu] phase branches {dim}D, {f['T'].size} cells", flush=True)
    g = sol.Case(case, device=dev, write_init=False)
    g.write_fields(f)
    g.step(1)
    got = g.read_fields()
    Tstar = g.read_fields(("Tstar",))["Tstar"]
    g.close()
    assert not got["u"].any() and not got["v"].any()
    np.testing.assert_allclose(got["C"], f["C"], rtol=1e-13, atol=0)
    orc = oracle.Oracle(case, fields=f)
    T, gl, Cl, Cs, br = orc.phase(Tstar, f["gl"], got["C"])
    counts = np.bincount(br, minlength=4)
    print("cells per branch (solid, plateau, mush, liquid):", counts.tolist(), flush=True)
    assert np.all(counts >= 50), counts
    remelt = gl > f["gl"] + 1e-3
    assert remelt.sum() >= 50 and (remelt & (br == 3)).any() and (remelt & (br == 2)).any()
    assert (gl < f["gl"] - 1e-3).sum() >= 50            # and cells that solidify
    assert np.all(np.abs(got["T"] - T) <= 1e-14 * np.abs(T)), np.abs(got["T"] - T).max()
    assert np.all(np.abs(got["gl"] - gl) <= 1e-12), np.abs(got["gl"] - gl).max()
    for b in range(4):                                   # branch values as such
        m = br == b
        if b == 0:
            assert np.all(got["gl"][m] == 0.0)
        if b == 1:
            Te = al["T_m"] + al["m_sp"] * al["C_e"]
            assert np.all(np.abs(got["T"][m] - Te) <= 1e-13 * Te)
        if b == 3:
            assert np.all(got["gl"][m] == 1.0)
    # C_l, C_s: eqs. (3.17)-(3.18) from the GPU's own g (the denominator
    # 1 + (1 - g)(k_p - 1) >= k_p may round differently by an ulp of 1 when
    # contracted to a fused multiply-add: <= 3.4e-15 relative), and against
    # the oracle within what the g tolerance allows
    kp = al["k_p"]
    own = got["C"] / (1.0 + (1.0 - got["gl"]) * (kp - 1.0))
    assert np.all(np.abs(got["Cl"] - own) <= 1e-14 * own)
    assert np.all(np.abs(got["Cs"] - kp * own) <= 1e-14 * kp * own)
    assert np.all(np.abs(got["Cl"] - Cl) <= (1e-14 + 1e-12 / kp) * Cl)
    assert rel(got["Cs"], Cs) < 1e-13


# ----------------------------------------------------------- invariants

def _liquid_melt(dim, dT_amp, precision):
    al = W.sn10pb_alloy()
    Tl = al["T_m"] + al["m_sp"] * 10.0
    if dim == 2:
        return W.make_case(2, 40, 24, 1, 0.040, 0.024, 1.0, T0=Tl + 5.0, dT_amp=dT_amp, seed=3,
                           bcs=W.west_cooled_bcs(), tol_p=1e-12, tol_t=1e-12, precision=precision)
    return W.make_case(3, 16, 12, 10, 0.016, 0.012, 0.010, T0=Tl + 5.0, dT_amp=dT_amp, seed=3,
                       bcs=W.west_cooled_bcs(), tol_p=1e-12, tol_t=1e-12, precision=precision)


@pytest.mark.parametrize("precision", [W.PRECISION_FP64, W.PRECISION_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_projected_velocity_keeps_uniform_fields(sol, dev, dim, precision):
    """The solute and energy systems are advected by the divergence-free
    u^{n+1} (eqs. 3.10-3.11), which carries a uniform field without sources:
    (a) an all-liquid melt (T0 = T_l + 5 K, +-2 K) with uniform C keeps C
    uniform while thermal buoyancy stirs it; (b) a uniform T with the
    composition perturbed by +-0.5 wt% (adiabatic walls) keeps T uniform
    while solutal buoyancy stirs it.  Advecting with u* instead drifts by
    ~1e-4 (the oracle's planted-mistake pins)."""
    case = _liquid_melt(dim, 2.0, precision)
    g = sol.Case(case, device=dev)
    g.step(6)
    f = g.read_fields()
    g.close()
    assert np.abs(f["u"]).max() > 1e-6
    assert np.ptp(f["C"]) <= 1e-14 * 10.0 and np.all(f["gl"] == 1.0), np.ptp(f["C"])
    case = _liquid_melt(dim, 0.0, precision)
    case["bcs"] = [W.face_bc() for _ in range(6)]
    rng = np.random.default_rng(5)
    case["init"]["C"] = 10.0 + rng.uniform(-0.5, 0.5, case["init"]["C"].size)
    case["init"]["Cl"] = case["init"]["C"].copy()
    g = sol.Case(case, device=dev)
    g.step(6)
    f = g.read_fields()
    Ts = g.read_fields(("Tstar",))["Tstar"]
    g.close()
    assert np.abs(f["u"]).max() > 1e-6
    assert np.ptp(f["T"]) <= 1e-14 * case["T0"] and np.ptp(Ts) <= 1e-14 * case["T0"], (np.ptp(f["T"]), np.ptp(Ts))


# ------------------------------------------------- batched and served

def _tight(case, tol_p=1e-13, tol_t=1e-14):
    case["numerics"]["tol_p"] = tol_p
    case["numerics"]["tol_t"] = tol_t
    return case


def test_batched_cavities_match_oracle(sol, dev):
    """Eight cavities of the batched recipe (uneven sizes 3e3-1e5 cells,
    aspect ratio, cooling coefficient and C0 drawn from the seed) advanced
    together, FP64 and mixed precision, against the oracle run on each case
    alone: every field of every case within 1e-9 (FP64) and 1e-8 (mixed)
    after 3 steps at pressure tolerance 3e-13 and transport 1e-14 (the
    pressure systems of the larger cavities round their true residual to
    ~1.2e-13 in FP64, so 1e-13 is below their floor)."""
    cases = [_tight(c, tol_p=3e-13) for c in W.batch_cases(8, seed=3, precision=W.PRECISION_FP64, tol=3e-13)]
    print("[gpu] batched vs oracle:", [(c["grid"]["nx"], c["grid"]["ny"]) for c in cases], flush=True)
    refs = []
    for c in cases:
        o = oracle.Oracle(c, threads=8)
        o.step(3)
        refs.append(o.fields())
    for precision, gate in ((W.PRECISION_FP64, 1e-9), (W.PRECISION_MIXED, 1e-8)):
        for c in cases:
            c["numerics"]["precision"] = precision
        gs = [sol.Case(c, device=dev) for c in cases]
        b = sol.Batch(gs)
        st = b.step([3] * len(gs))
        b.close()
        worst = 0.0
        for i, (g, ref) in enumerate(zip(gs, refs)):
            errs = field_errors(g.read_fields(), ref)
            worst = max(worst, max(errs.values()))
            for k, e in errs.items():
                assert e < gate, (precision, i, k, errs)
            assert st[i]["rel_resid"][3] <= 3e-13 * (1 + 1e-6)
            g.close()
        print(f"precision {precision}: worst field error vs oracle {worst:.1e}", flush=True)
    for c in cases:
        c["numerics"]["precision"] = W.PRECISION_FP64


def test_served_stream_matches_oracle_and_alone(sol, dev):
    """Continuous batching of a Poisson stream (mixed precision, tight
    tolerances) with one request of 400 x 330 = 132 000 cells among small
    ones.  Every served result matches the oracle per field within 1e-8.
    Against the same case advanced alone: bit-identical below 131 072
    cells; the large case solves a larger coarse multigrid level exactly when
    it runs alone than inside a batch, so alone and served agree to the
    solver tolerance band, not bit for bit."""
    from paper_2303_10783_amd.serve import Request, Server
    reqs = [_tight(c) for c in W.served_arrivals(6, seed=5, rate=200.0, scale=0.004, tol=1e-13)]
    big = _tight(W.cavity_2d(400, 330, lx=0.08, ly=0.066, seed=131, precision=W.PRECISION_MIXED), tol_p=2e-13)
    big["arrival_s"] = reqs[2]["arrival_s"]
    reqs.insert(3, big)
    requests = [Request(case=c, steps=3 + (i % 2), arrival=c["arrival_s"], rid=i) for i, c in enumerate(reqs)]
    print("[gpu] served vs oracle:", [r.case["grid"]["nx"] * r.case["grid"]["ny"] * r.case["grid"]["nz"]
                                      for r in requests], flush=True)
    srv = Server(device=dev, max_active=3)
    out = srv.run(requests)
    assert out["requests"] == len(requests)
    admits = [t for t, ev, _ in srv.log if ev == "admit"]
    finishes = [t for t, ev, _ in srv.log if ev == "finish"]
    assert min(finishes) < max(admits)               # admitted while others ran
    for r in out["done"]:
        c = r.case
        o = oracle.Oracle(c, threads=8)
        o.step(r.steps)
        errs = field_errors(r.result, o.fields())
        for k, e in errs.items():
            assert e < 1e-8, (r.rid, k, errs)
        g = sol.Case(c, device=dev)
        g.step(r.steps)
        alone = g.read_fields()
        g.close()
        n = c["grid"]["nx"] * c["grid"]["ny"] * c["grid"]["nz"]
        if n < 131072:
            for k in FIELDS:
                assert np.array_equal(r.result[k], alone[k]), (r.rid, k)
        else:
            e2 = field_errors(r.result, alone)
            print(f"request {r.rid} ({n} cells): served vs alone", {k: f"{v:.1e}" for k, v in e2.items()})
            assert max(e2[k] for k in ("T", "C", "gl", "Cl", "Cs")) < 1e-11, e2
            assert max(e2.values()) < 1e-8, e2
    print("served:", {k: v for k, v in out.items() if k != "done"})


def _box_case():
    case = W.workload_case("C3", tol=1e-12)
    case["numerics"]["tol_t"] = 1e-13
    return case


_BOX_REF = {}


def _box_oracle_fields():
    if not _BOX_REF:
        o = oracle.Oracle(_box_case(), threads=16)
        o.step(2)
        _BOX_REF.update(o.fields())
    return _BOX_REF


@pytest.mark.parametrize("precision", [W.PRECISION_FP64, W.PRECISION_MIXED], ids=["fp64", "mixed"])
def test_box_128x128x64_matches_oracle(sol, dev, precision):
    """The 3D workload at full size (128 x 128 x 64 cells) against the
    oracle, per field, after 2 steps with the pressure solved to 1e-12 and
    the transport systems to 1e-13 on both sides: within 1e-9 in FP64 and
    1e-8 in mixed precision (FP32 Krylov inside FP64 refinement)."""
    case = _box_case()
    print(f"[gpu] 128x128x64 vs oracle, precision {precision}", flush=True)
    ref = _box_oracle_fields()
    case["numerics"]["precision"] = precision
    g = sol.Case(case, device=dev)
    st = g.step(2)
    errs = field_errors(g.read_fields(), ref)
    g.close()
    print("per-field rel L2 vs oracle:", {k: f"{v:.1e}" for k, v in errs.items()}, "iters", st["iters"], flush=True)
    gate = 1e-9 if precision == W.PRECISION_FP64 else 1e-8
    for k, e in errs.items():
        assert e < gate, (k, errs)
    for s in range(6):
        assert st["rel_resid"][s] <= (1e-12 if s == 3 else 1e-13) * (1 + 1e-6)
