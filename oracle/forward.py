"""Forward (residual-probing) matrix assembly -- an independent second route
to the same linear systems, used to cross-check the oracle's stencil
assembly.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Section 4 of the paper ("Forward method", eqs. 4.5-4.7): the discrete
equation of every unknown is coded directly as a residual Eq(Phi) = A Phi - b;
then b = -Eq(0), and the matrix entries come from evaluating Eq on probe
vectors that are 1 on one colour of cells and 0 elsewhere.  With colours
(i mod 3, j mod 3[, k mod 3]) no two unknowns of one colour meet in any row's
stencil, so 9 probes (2D) or 27 probes (3D) recover every entry.  The paper
states the result equals the directly assembled matrix up to rounding.

Here Eq is written with numpy array operations on (z, y, x)-shaped arrays,
face fluxes first and then their differences, i.e. a different code path
from the row-by-row stencil assembly in sol_oracle.c.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SYS_U, SYS_V, SYS_W, SYS_P, SYS_C, SYS_T = range(6)


def _ax(a):            # physical axis (0=x,1=y,2=z) -> numpy axis of (z,y,x)
    return 2 - a


def _take(arr, a, sl):
    idx = [slice(None)] * 3
    idx[_ax(a)] = sl
    return arr[tuple(idx)]


def _pad(arr, a, before, after, value=0.0):
    w = [(0, 0)] * 3
    w[_ax(a)] = (before, after)
    return np.pad(arr, w, constant_values=value)


class Geometry:
    def __init__(self, case):
        g = case["grid"]
        self.dim = g["dim"]
        self.n = (g["nx"], g["ny"], g["nz"] if self.dim == 3 else 1)
        self.h = (g["lx"] / g["nx"], g["ly"] / g["ny"],
                  g["lz"] / g["nz"] if self.dim == 3 else 1.0)
        self.cell_shape = (self.n[2], self.n[1], self.n[0])

    def sys_shape(self, sys):
        n = list(self.n)
        if sys in (SYS_U, SYS_V, SYS_W):
            n[sys] -= 1
        return (n[2], n[1], n[0])

    def full_face(self, vec, a):
        """Velocity component a on all a-faces (walls = 0), shape with n_a+1."""
        shp = list(self.cell_shape)
        shp[_ax(a)] -= 1
        inner = np.asarray(vec, dtype=np.float64).reshape(shp) if np.prod(shp) else np.zeros(shp)
        return _pad(inner, a, 1, 1)


def _upwind_flux(vel, phi_minus, phi_plus):
    """Face flux vel * (upstream value), eq. (3.28)."""
    return np.where(vel >= 0.0, vel * phi_minus, vel * phi_plus)


def eq_momentum(case, fields, d, phi):
    """Residual of eq. (3.3) for velocity component d: A phi - b.  With the
    momentum form of eq. (2.6) (case["momentum"] == 1) the convection is
    that of the advecting velocity u/g~ and the pressure gradient, the drag
    and the force carry g (g: g_l on the face, the mean of its two cells;
    g~ = max(g, darcy_eps^(1/3)), the reading of the stencil oracle)."""
    G = Geometry(case)
    al, nm, bcs = case["alloy"], case["numerics"], case["bcs"]
    nu = al["mu"] / al["rho"]
    dt = nm["dt"]
    shp = G.sys_shape(d)
    phi = np.asarray(phi, dtype=np.float64).reshape(shp)
    un = np.asarray(fields["uvw"[d]], dtype=np.float64).reshape(shp)
    vel = [G.full_face(fields["uvw"[a]], a) if a < G.dim else None for a in range(3)]
    # the upwind choice depends on the sign of the advecting velocity only,
    # so the flux difference divided by g~ > 0 is the convection of u/g~
    gl = np.asarray(fields["gl"], dtype=np.float64).reshape(G.cell_shape)
    gf = 0.5 * (_take(gl, d, slice(0, -1)) + _take(gl, d, slice(1, None)))
    if int(case.get("momentum", 0)) == 1:
        gt = np.maximum(gf, np.cbrt(al["darcy_eps"]))
        gw = gf
    else:
        gt = np.ones_like(gf)
        gw = np.ones_like(gf)
    res = (phi - un) / dt
    phi_full = _pad(phi, d, 1, 1)          # face numbers 0..n_d, walls 0
    for a in range(G.dim):
        h = G.h[a]
        if a == d:
            # control-volume faces at cell centres 0..n_d-1
            vf = vel[d]
            vcv = 0.5 * (_take(vf, d, slice(0, -1)) + _take(vf, d, slice(1, None)))
            flux = _upwind_flux(vcv, _take(phi_full, d, slice(0, -1)),
                                _take(phi_full, d, slice(1, None)))
            res = res + ((_take(flux, d, slice(1, None)) - _take(flux, d, slice(0, -1))) / h) / gt
            grad = (_take(phi_full, d, slice(1, None)) - _take(phi_full, d, slice(0, -1))) / h
            lap = (_take(grad, d, slice(1, None)) - _take(grad, d, slice(0, -1))) / h
            res = res - nu * lap
        else:
            # control-volume faces at the a-faces 0..n_a; advecting velocity
            # = mean of the a-velocity of the two cells sharing the d-face
            va = vel[a]
            vcv = 0.5 * (_take(va, d, slice(0, -1)) + _take(va, d, slice(1, None)))
            php = _pad(phi, a, 1, 1)
            flux = _upwind_flux(vcv, _take(php, a, slice(0, -1)), _take(php, a, slice(1, None)))
            res = res + ((_take(flux, a, slice(1, None)) - _take(flux, a, slice(0, -1))) / h) / gt
            inner = (_take(phi, a, slice(1, None)) - _take(phi, a, slice(0, -1))) / h
            lo_wall = 2.0 * _take(phi, a, slice(0, 1)) / h        # (phi - 0)/(h/2)
            hi_wall = -2.0 * _take(phi, a, slice(-1, None)) / h    # (0 - phi)/(h/2)
            if bcs[2 * a]["velocity"] != 0:
                lo_wall = 0.0 * lo_wall
            if bcs[2 * a + 1]["velocity"] != 0:
                hi_wall = 0.0 * hi_wall
            grad = np.concatenate([lo_wall, inner, hi_wall], axis=_ax(a))
            lap = (_take(grad, a, slice(1, None)) - _take(grad, a, slice(0, -1))) / h
            res = res - nu * lap
    # Carman-Kozeny drag on the face, eq. (2.8)
    kinv = 180.0 * (1.0 - gf) ** 2 / (al["lambda2"] ** 2 * (gf ** 3 + al["darcy_eps"]))
    res = res + nu * gt * kinv * phi
    # pressure gradient at level n
    p = np.asarray(fields["p"], dtype=np.float64).reshape(G.cell_shape)
    res = res + gw * (_take(p, d, slice(1, None)) - _take(p, d, slice(0, -1))) / (al["rho"] * G.h[d])
    # Boussinesq force on the vertical component, eq. (2.9)
    if d == G.dim - 1:
        T = np.asarray(fields["T"], dtype=np.float64).reshape(G.cell_shape)
        Cl = np.asarray(fields["Cl"], dtype=np.float64).reshape(G.cell_shape)
        Tf = 0.5 * (_take(T, d, slice(0, -1)) + _take(T, d, slice(1, None)))
        Cf = 0.5 * (_take(Cl, d, slice(0, -1)) + _take(Cl, d, slice(1, None)))
        f = al["g"] * (al["beta_T"] * (Tf - al["T_ref"]) + al["beta_C"] * (Cf - al["C_ref"]))
        res = res - gw * f
    return res.ravel()


def _neumann_lap(G, phi, coef=1.0):
    out = np.zeros_like(phi)
    for a in range(G.dim):
        h = G.h[a]
        grad = (_take(phi, a, slice(1, None)) - _take(phi, a, slice(0, -1))) / h
        grad = _pad(grad, a, 1, 1)        # zero flux through walls
        out = out + coef * (_take(grad, a, slice(1, None)) - _take(grad, a, slice(0, -1))) / h
    return out


def _div(G, vel):
    out = np.zeros(G.cell_shape)
    for a in range(G.dim):
        out = out + (_take(vel[a], a, slice(1, None)) - _take(vel[a], a, slice(0, -1))) / G.h[a]
    return out


def eq_poisson(case, ustar, phi):
    """Residual of eq. (3.4) written as (-L) phi - rhs with a mean-free rhs."""
    G = Geometry(case)
    al, nm = case["alloy"], case["numerics"]
    phi = np.asarray(phi, dtype=np.float64).reshape(G.cell_shape)
    vel = [G.full_face(ustar[a], a) if a < G.dim else None for a in range(3)]
    rhs = -(al["rho"] / nm["dt"]) * _div(G, vel)
    rhs = rhs - rhs.mean()
    return (-_neumann_lap(G, phi) - rhs).ravel()


def eq_solute(case, fields, unew, C):
    """Residual of eq. (3.10): (C - C^n)/dt + div(u C_l) - div(g_l D_l grad C_l),
    C_l = A_g C (the diffusion term is eq. 3.7's; g_l on a face is the mean
    of its two cells, zero flux through walls)."""
    G = Geometry(case)
    al, nm = case["alloy"], case["numerics"]
    C = np.asarray(C, dtype=np.float64).reshape(G.cell_shape)
    Cn = np.asarray(fields["C"], dtype=np.float64).reshape(G.cell_shape)
    gl = np.asarray(fields["gl"], dtype=np.float64).reshape(G.cell_shape)
    Cl = C / (1.0 - (1.0 - al["k_p"]) * (1.0 - gl))           # eq. (3.8)
    vel = [G.full_face(unew[a], a) if a < G.dim else None for a in range(3)]
    res = (C - Cn) / nm["dt"]
    for a in range(G.dim):
        p = _pad(Cl, a, 1, 1)
        flux = _upwind_flux(vel[a], _take(p, a, slice(0, -1)), _take(p, a, slice(1, None)))
        res = res + (_take(flux, a, slice(1, None)) - _take(flux, a, slice(0, -1))) / G.h[a]
    D = al.get("D_l", 0.0) or 0.0
    if D > 0.0:
        for a in range(G.dim):
            h = G.h[a]
            gface = 0.5 * (_take(gl, a, slice(1, None)) + _take(gl, a, slice(0, -1)))
            dflux = _pad(D * gface * (_take(Cl, a, slice(1, None)) - _take(Cl, a, slice(0, -1))) / h, a, 1, 1)
            res = res - (_take(dflux, a, slice(1, None)) - _take(dflux, a, slice(0, -1))) / h
    return res.ravel()


def eq_energy(case, fields, unew, T, t_new):
    """Residual of eq. (3.11) with convective / prescribed-temperature walls."""
    G = Geometry(case)
    al, nm, bcs = case["alloy"], case["numerics"], case["bcs"]
    rcp = al["rho"] * al["cp"]
    alpha = al["k"] / rcp
    T = np.asarray(T, dtype=np.float64).reshape(G.cell_shape)
    Tn = np.asarray(fields["T"], dtype=np.float64).reshape(G.cell_shape)
    vel = [G.full_face(unew[a], a) if a < G.dim else None for a in range(3)]
    res = (T - Tn) / nm["dt"] - _neumann_lap(G, T, alpha)
    for a in range(G.dim):
        p = _pad(T, a, 1, 1)
        flux = _upwind_flux(vel[a], _take(p, a, slice(0, -1)), _take(p, a, slice(1, None)))
        res = res + (_take(flux, a, slice(1, None)) - _take(flux, a, slice(0, -1))) / G.h[a]
        for s, sl in ((0, slice(0, 1)), (1, slice(-1, None))):
            bc = bcs[2 * a + s]
            h = G.h[a]
            if bc["thermal"] == 1:
                U, Tw = 1.0 / (1.0 / bc["h"] + h / (2.0 * al["k"])), bc["T_ext"]
            elif bc["thermal"] == 2:
                U, Tw = 2.0 * al["k"] / h, bc["T0"] - bc["b"] * t_new
            else:
                continue
            wall = np.zeros(G.cell_shape)
            idx = [slice(None)] * 3
            idx[_ax(a)] = sl
            wall[tuple(idx)] = U * (T[tuple(idx)] - Tw) / (rcp * h)
            res = res + wall
    return res.ravel()


def probe_assemble(G: Geometry, sys: int, eq):
    """Recover (A, b) of a linear residual map eq(x) = A x - b by colour
    probing (9 probes in 2D, 27 in 3D); structural pattern = in-domain
    5/7-point neighbours, columns ascending."""
    shp = G.sys_shape(sys)
    nz, ny, nx = shp
    n = nx * ny * nz
    if n == 0:
        return sp.csr_matrix((0, 0)), np.zeros(0)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    colour = (i % 3) + 3 * (j % 3) + 9 * (k % 3)
    r0 = eq(np.zeros(n))
    b = -r0
    ncol = 27 if G.dim == 3 else 9
    resp = {}
    for c in range(ncol):
        x = (colour == c).astype(np.float64)
        if x.any():
            resp[c] = eq(x) - r0
    rows, cols, vals = [], [], []
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    # ascending column order: -z, -y, -x, 0, +x, +y, +z
    order = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    del offs
    row_index = np.arange(n)
    for (dx, dy, dz) in order:
        if G.dim == 2 and dz != 0:
            continue
        ii, jj, kk = i + dx, j + dy, k + dz
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
        col = ii + nx * (jj + ny * kk)
        ccol = (ii % 3) + 3 * (jj % 3) + 9 * (kk % 3)
        v = np.zeros(n)
        for c in np.unique(ccol[ok]):
            m = ok & (ccol == c)
            v[m] = resp[int(c)][row_index[m]]
        rows.append(row_index[ok]); cols.append(col[ok]); vals.append(v[ok])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sort_indices()
    return A, b


def forward_assemble(case, fields, sys, vel=None, t_new=None):
    """(A, b) of system `sys` by the forward method; vel = (u*, v*, w*) for the
    pressure system and the advecting u^{n+1} for solute / energy."""
    G = Geometry(case)
    f = dict(fields)
    f["uvw"] = (fields["u"], fields["v"], fields["w"])
    if vel is None:
        vel = f["uvw"]
    if t_new is None:
        t_new = case["numerics"]["dt"]
    if sys in (SYS_U, SYS_V, SYS_W):
        return probe_assemble(G, sys, lambda x: eq_momentum(case, f, sys, x))
    if sys == SYS_P:
        return probe_assemble(G, sys, lambda x: eq_poisson(case, vel, x))
    if sys == SYS_C:
        return probe_assemble(G, sys, lambda x: eq_solute(case, fields, vel, x))
    if sys == SYS_T:
        return probe_assemble(G, sys, lambda x: eq_energy(case, fields, vel, x, t_new))
    raise ValueError(sys)
