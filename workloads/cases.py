"""Seeded synthetic workloads shared by the oracle side and the HIP side.

This module holds case descriptions (grid, alloy constants, wall conditions,
solver settings) and seeded random draws only.  It performs none of the
scheme's arithmetic: every quantity of the method (stencils, Darcy drag,
buoyancy, phase relations, solves) is computed independently by the oracle
and by the HIP library from the plain parameters given here.

Physical constants follow the Sn-10%Pb column of the alloy property table
(Table 1 of the paper) where the workload definitions below do not fix them;
the workload definitions override Table 1 where both give a value
(melting point, liquidus slope, partition coefficient, dendrite arm spacing,
expansion coefficients, density, viscosity).

Face order everywhere: W, E, S, N, B, T  (x-min, x-max, y-min, y-max,
z-min, z-max).  In 2D only the first four faces exist and gravity acts along
-y; in 3D gravity acts along -z.
"""
from __future__ import annotations

import copy
import math

import numpy as np

FACES = ("W", "E", "S", "N", "B", "T")

THERMAL_ADIABATIC = 0
THERMAL_ROBIN = 1       # convective cooling q = h (T - T_ext)
THERMAL_DIRICHLET = 2   # prescribed wall temperature T(t) = T0 - b t

VELOCITY_NOSLIP = 0
VELOCITY_FREESLIP = 1

PRECISION_FP64 = 0
PRECISION_MIXED = 1     # FP32 Krylov inside FP64 iterative refinement

MOMENTUM_PLAIN = 0      # momentum form of eq. (2.7), the one the scheme's eq. (3.3) discretises
MOMENTUM_MINIMAL = 1    # the minimal model's form, eq. (2.6)

FIELD_NAMES = ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")


def sn10pb_alloy(**override) -> dict:
    """Alloy constants of the benchmark cavity workloads (SI units, K, wt%)."""
    a = dict(
        rho=7000.0,        # kg/m^3
        mu=1.0e-3,         # Pa s
        cp=260.0,          # J/(kg K)      Table 1, Sn-10%Pb
        k=55.0,            # W/(m K)       Table 1, Sn-10%Pb
        latent=6.1e4,      # J/kg          Table 1, Sn-10%Pb
        beta_T=6.0e-5,     # 1/K
        beta_C=-5.0e-3,    # 1/wt%
        lambda2=1.85e-5,   # m, secondary dendrite arm spacing
        T_m=505.0,         # K, melting point at C = 0
        m_sp=-2.33,        # K/wt%, liquidus slope
        k_p=0.0656,        # partition coefficient
        C_e=38.1,          # wt%, eutectic composition (Table 1, Sn-10%Pb)
        g=9.81,            # m/s^2, magnitude of gravity
        D_l=0.0,           # liquid solute diffusivity (minimal model: none)
        darcy_eps=1.0e-3,  # regularisation of g^3 in the Carman-Kozeny drag
        T_ref=None,        # filled by make_case: initial uniform temperature
        C_ref=None,        # filled by make_case: initial uniform concentration
    )
    a.update(override)
    return a


def pb48sn_alloy(**override) -> dict:
    """Pb-48%Sn column of the alloy property table (Table 1), temperatures
    converted to kelvin (melting point 327.5 degC)."""
    a = dict(
        rho=9000.0, mu=1.0e-3, cp=200.0, k=50.0, latent=5.35e4,
        beta_T=1.0e-4, beta_C=4.5e-3, lambda2=40.0e-6,
        T_m=327.5 + 273.15, m_sp=-2.334, k_p=0.307, C_e=61.9,
        g=9.81, D_l=0.0, darcy_eps=1.0e-3, T_ref=None, C_ref=None,
    )
    a.update(override)
    return a


def face_bc(thermal=THERMAL_ADIABATIC, h=0.0, T_ext=0.0, T0=0.0, b=0.0,
            velocity=VELOCITY_NOSLIP) -> dict:
    return dict(thermal=int(thermal), h=float(h), T_ext=float(T_ext),
                T0=float(T0), b=float(b), velocity=int(velocity))


def make_case(dim, nx, ny, nz, lx, ly, lz, *, C0=10.0, alloy=None, bcs=None,
              dt=0.01, tol_p=1e-10, tol_t=1e-10, max_iter=200000,
              precision=PRECISION_FP64, seed=0, T0=None, dT_amp=0.1,
              name="case", momentum=MOMENTUM_PLAIN) -> dict:
    """Return a case: parameters plus seeded initial fields.

    Initial state (a still, fully liquid melt): u = v = w = p = 0, C = C0,
    g_l = 1, C_l = C0, C_s = 0 (unused before the first step), and
    T = T0 + U(-dT_amp, dT_amp) drawn per cell in lexicographic order
    (x fastest) from numpy's default_rng(seed).  T0 defaults to the liquidus
    temperature at C0 (the examples start at T0 = T_l), computed from the
    straight liquidus line T_m + m_sp C0 of the alloy.  `momentum` selects
    the momentum form (MOMENTUM_PLAIN or MOMENTUM_MINIMAL).
    """
    if dim == 2:
        nz, lz = 1, 1.0
    alloy = sn10pb_alloy() if alloy is None else copy.deepcopy(alloy)
    if T0 is None:
        T0 = alloy["T_m"] + alloy["m_sp"] * C0
    if alloy.get("T_ref") is None:
        alloy["T_ref"] = float(T0)
    if alloy.get("C_ref") is None:
        alloy["C_ref"] = float(C0)
    if bcs is None:
        bcs = [face_bc() for _ in range(6)]
    bcs = [dict(b) for b in bcs]
    assert len(bcs) == 6
    grid = dict(dim=int(dim), nx=int(nx), ny=int(ny), nz=int(nz),
                lx=float(lx), ly=float(ly), lz=float(lz))
    numerics = dict(dt=float(dt), tol_p=float(tol_p), tol_t=float(tol_t),
                    max_iter=int(max_iter), precision=int(precision))
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    dT = rng.uniform(-dT_amp, dT_amp, n) if dT_amp > 0 else np.zeros(n)
    init = dict(
        u=np.zeros((nx - 1) * ny * nz),
        v=np.zeros(nx * (ny - 1) * nz),
        w=np.zeros(nx * ny * (nz - 1)) if dim == 3 else np.zeros(0),
        p=np.zeros(n),
        T=float(T0) + dT,
        C=np.full(n, float(C0)),
        gl=np.ones(n),
        Cl=np.full(n, float(C0)),
        Cs=np.zeros(n),
    )
    return dict(name=name, grid=grid, alloy=alloy, bcs=bcs,
                numerics=numerics, init=init, seed=int(seed), C0=float(C0),
                T0=float(T0), momentum=int(momentum))


def momentum_form(case) -> int:
    """Momentum form of a case (cases built before the key existed: PLAIN)."""
    return int(case.get("momentum", MOMENTUM_PLAIN))


def with_momentum(case, form) -> dict:
    """Copy of `case` with the momentum form set (fields shared by value)."""
    c = copy.deepcopy(case)
    c["momentum"] = int(form)
    return c


def field_sizes(grid) -> dict:
    nx, ny, nz, dim = grid["nx"], grid["ny"], grid["nz"], grid["dim"]
    n = nx * ny * nz
    return dict(u=(nx - 1) * ny * nz, v=nx * (ny - 1) * nz,
                w=nx * ny * (nz - 1) if dim == 3 else 0,
                p=n, T=n, C=n, gl=n, Cl=n, Cs=n)


# ---------------------------------------------------------------------------
# The benchmark cavities.  2D: 0.10 m x 0.06 m (the 5:3 cavity of the
# solidification benchmarks), cooled through the west wall by h = 400 W/m^2K
# to 298 K, other walls adiabatic, all walls rigid and no-slip.
# ---------------------------------------------------------------------------

def west_cooled_bcs(h=400.0, T_ext=298.0, velocity=VELOCITY_NOSLIP):
    bcs = [face_bc(velocity=velocity) for _ in range(6)]
    bcs[0] = face_bc(THERMAL_ROBIN, h=h, T_ext=T_ext, velocity=velocity)
    return bcs


def cavity_2d(nx=50, ny=30, *, lx=0.10, ly=0.06, C0=10.0, h=400.0,
              T_ext=298.0, dt=0.01, tol=1e-10, precision=PRECISION_FP64,
              seed=0, max_iter=200000, name=None, alloy=None,
              momentum=MOMENTUM_PLAIN) -> dict:
    return make_case(2, nx, ny, 1, lx, ly, 1.0, C0=C0, alloy=alloy,
                     bcs=west_cooled_bcs(h, T_ext), dt=dt, tol_p=tol,
                     tol_t=tol, max_iter=max_iter, precision=precision,
                     seed=seed, name=name or f"cavity2d_{nx}x{ny}",
                     momentum=momentum)


def box_3d(nx=128, ny=128, nz=64, *, lx=0.10, ly=0.10, lz=0.05, C0=10.0,
           h=400.0, T_ext=298.0, dt=0.01, tol=1e-10,
           precision=PRECISION_FP64, seed=0, max_iter=200000, name=None,
           alloy=None, momentum=MOMENTUM_PLAIN) -> dict:
    return make_case(3, nx, ny, nz, lx, ly, lz, C0=C0, alloy=alloy,
                     bcs=west_cooled_bcs(h, T_ext), dt=dt, tol_p=tol,
                     tol_t=tol, max_iter=max_iter, precision=precision,
                     seed=seed, name=name or f"box3d_{nx}x{ny}x{nz}",
                     momentum=momentum)


# Named workloads (grid, steps).  C1 is small enough for the oracle to run in
# full; C2 is the throughput workload; C3 is the 3D box.
WORKLOADS = {
    "C1": dict(kind="2d", nx=50, ny=30, steps=200),
    "C2": dict(kind="2d", nx=500, ny=300, steps=1000),
    "C3": dict(kind="3d", nx=128, ny=128, nz=64, steps=500),
}


def workload_case(key, **kw) -> dict:
    w = WORKLOADS[key]
    if w["kind"] == "2d":
        return cavity_2d(w["nx"], w["ny"], name=key, **kw)
    return box_3d(w["nx"], w["ny"], w["nz"], name=key, **kw)


def batch_cases(n_cases=64, seed=0, *, n_min=6000, n_max=96000,
                r_min=0.5, r_max=4.0, h_min=200.0, h_max=800.0,
                c_min=5.0, c_max=15.0, ly=0.06, precision=PRECISION_MIXED,
                tol=1e-10) -> list:
    """Uneven 2D cavities for the batched workload.

    Per case: aspect ratio R ~ U[r_min, r_max], cell count N ~ U[n_min, n_max],
    n_x = round(sqrt(N R)), n_y = round(N / n_x), l_y fixed, l_x = R l_y,
    cooling coefficient h ~ U[h_min, h_max], C0 ~ U[c_min, c_max].
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_cases):
        R = rng.uniform(r_min, r_max)
        N = rng.uniform(n_min, n_max)
        h = rng.uniform(h_min, h_max)
        C0 = rng.uniform(c_min, c_max)
        nx = max(2, int(round(math.sqrt(N * R))))
        ny = max(2, int(round(N / nx)))
        out.append(cavity_2d(nx, ny, lx=R * ly, ly=ly, C0=C0, h=h,
                             precision=precision, tol=tol,
                             seed=seed * 1000 + i, name=f"batch{i}"))
    return out


def served_arrivals(n_requests, seed=0, *, rate=20.0, p3d=0.5,
                    n2d=(6000, 384000), n3d=(32768, 3538944),
                    r_range=(0.5, 4.0), h_range=(200.0, 800.0),
                    c_range=(5.0, 15.0), precision=PRECISION_MIXED,
                    tol=1e-10, scale=1.0) -> list:
    """Poisson arrivals (exponential gaps at `rate` per second) of 2D and 3D
    cases with log-uniform cell counts, seeded aspect ratio, h and C0.

    `scale` shrinks the cell-count bounds (for short runs); the recipe is
    otherwise unchanged.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        is3d = rng.uniform() < p3d
        R = rng.uniform(*r_range)
        h = rng.uniform(*h_range)
        C0 = rng.uniform(*c_range)
        lo, hi = (n3d if is3d else n2d)
        lo, hi = max(8.0, lo * scale), max(16.0, hi * scale)
        N = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        if is3d:
            # x : y : z = R : 1 : 0.5 shaped box, z vertical
            ny = max(2, int(round((N / (0.5 * R)) ** (1.0 / 3.0))))
            nx = max(2, int(round(R * ny)))
            nz = max(2, int(round(0.5 * ny)))
            case = box_3d(nx, ny, nz, lx=0.05 * R, ly=0.05, lz=0.025, C0=C0,
                          h=h, precision=precision, tol=tol,
                          seed=seed * 100000 + i, name=f"req{i}")
        else:
            nx = max(2, int(round(math.sqrt(N * R))))
            ny = max(2, int(round(N / nx)))
            case = cavity_2d(nx, ny, lx=0.06 * R, ly=0.06, C0=C0, h=h,
                             precision=precision, tol=tol,
                             seed=seed * 100000 + i, name=f"req{i}")
        case["arrival_s"] = t
        out.append(case)
    return out


# ---------------------------------------------------------------------------
# Freckle cavities (Example 2 of the paper): Pb-48%Sn, C0 = 48 wt%, a still
# melt at T0 = 216 degC, the bottom wall held at T(t) = T0 - b t with
# b = 0.05 K/s, the top wall at T0, the side walls adiabatic; the solute
# perturbation C = 1.0001 C0 on the vertical centre line starts the density
# inversion.  Meshes 30 x 90 (R = 1:3) and 90 x 30 (R = 3:1) in 2D,
# 30 x 30 x 90 and 90 x 30 x 30 in 3D, dt = 0.01 s.  The cavity dimensions
# are not given in the text: square cells of `cell` metres (1 mm) are taken.
# The centre line is the middle column of cells (the two middle columns, or
# the 2 x 2 middle columns in 3D, when the count is even).
# ---------------------------------------------------------------------------

FRECKLE_MESHES = {
    (2, "1:3"): (30, 90, 1), (2, "3:1"): (90, 30, 1),
    (3, "1:1:3"): (30, 30, 90), (3, "3:1:1"): (90, 30, 30),
}


def _middle(n):
    return [n // 2] if n % 2 else [n // 2 - 1, n // 2]


def freckle_case(dim=2, R=None, *, cell=1e-3, T0_C=216.0, b=0.05, C0=48.0, slip_sides=False,
                 dt=0.01, tol=1e-10, precision=PRECISION_FP64, mesh=None, name=None) -> dict:
    """The freckle-formation cavity with its centre-line solute perturbation;
    `mesh` overrides the paper's mesh (same recipe on another grid)."""
    R = R or ("1:3" if dim == 2 else "1:1:3")
    nx, ny, nz = mesh or FRECKLE_MESHES[(dim, R)]
    T0 = T0_C + 273.15
    vert = VELOCITY_FREESLIP if slip_sides else VELOCITY_NOSLIP
    bcs = [face_bc(velocity=vert) for _ in range(6)]
    bot, top = (2, 3) if dim == 2 else (4, 5)
    bcs[bot] = face_bc(THERMAL_DIRICHLET, T0=T0, b=b)
    bcs[top] = face_bc(THERMAL_DIRICHLET, T0=T0, b=0.0)
    case = make_case(dim, nx, ny, nz, nx * cell, ny * cell, nz * cell, C0=C0, alloy=pb48sn_alloy(),
                     bcs=bcs, dt=dt, tol_p=tol, tol_t=tol, precision=precision, T0=T0, dT_amp=0.0,
                     name=name or f"freckle{dim}d_{R}")
    C = case["init"]["C"].reshape(nz if dim == 3 else 1, ny, nx)
    if dim == 2:
        for i in _middle(nx):
            C[:, :, i] = 1.0001 * C0
    else:
        for j in _middle(ny):
            for i in _middle(nx):
                C[:, j, i] = 1.0001 * C0
    case["init"]["C"] = C.ravel()
    case["init"]["Cl"] = case["init"]["C"].copy()      # fully liquid: C_l = C
    return case
