"""Python access to the plain FP64 CPU oracle (``sol_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark may import this package; the product library and
its binding never do.  The oracle shares no code with the HIP path.

The C file is compiled with gcc (plain ``-O2 -std=c99``, no fast-math, no
FMA contraction) into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sol_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

SYS_U, SYS_V, SYS_W, SYS_P, SYS_C, SYS_T = range(6)
SYSTEM_NAMES = ("u", "v", "w", "p", "C", "T")


def build(force: bool = False) -> str:
    """Compile the oracle (always when force, else only when stale)."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
           "-fopenmp", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Case(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("rho", C.c_double), ("mu", C.c_double), ("cp", C.c_double),
        ("kcond", C.c_double), ("latent", C.c_double), ("beta_T", C.c_double),
        ("beta_C", C.c_double), ("lambda2", C.c_double),
        ("T_m", C.c_double), ("m_sp", C.c_double), ("k_p", C.c_double),
        ("C_e", C.c_double), ("T_ref", C.c_double), ("C_ref", C.c_double),
        ("grav", C.c_double), ("darcy_eps", C.c_double),
        ("thermal", C.c_int32 * 6), ("hc", C.c_double * 6),
        ("T_ext", C.c_double * 6), ("T_wall0", C.c_double * 6),
        ("T_ramp", C.c_double * 6), ("velocity", C.c_int32 * 6),
        ("dt", C.c_double), ("tol_p", C.c_double), ("tol_t", C.c_double),
        ("max_iter", C.c_int32), ("literal_ag_order", C.c_int32),
        ("D_l", C.c_double),
        ("mom_form", C.c_int32),
    ]


class _Fields(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in
                ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")] + \
               [("step", C.c_int64)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 6), ("rel_resid", C.c_double * 6),
                ("sum_resid", C.c_double * 6), ("sum_C", C.c_double),
                ("sum_H", C.c_double), ("wall_flux", C.c_double),
                ("div_star", C.c_double), ("div_new", C.c_double),
                ("poisson_resid", C.c_double)]

    def as_dict(self):
        return dict(iters=list(self.iters), rel_resid=list(self.rel_resid),
                    sum_resid=list(self.sum_resid), sum_C=self.sum_C,
                    sum_H=self.sum_H, wall_flux=self.wall_flux,
                    div_star=self.div_star, div_new=self.div_new,
                    poisson_resid=self.poisson_resid)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.oc_sys_rows.argtypes = [C.POINTER(_Case), C.c_int]
        L.oc_sys_rows.restype = C.c_int
        L.oc_assemble.argtypes = [C.POINTER(_Case), C.POINTER(_Fields), dp, dp, dp,
                                  C.c_double, C.c_int, ip, ip, dp, dp]
        L.oc_assemble.restype = C.c_int
        L.oc_step.argtypes = [C.POINTER(_Case), C.POINTER(_Fields), C.POINTER(_Stats),
                              dp, dp, dp, dp, dp]
        L.oc_step.restype = C.c_int
        L.oc_phase.argtypes = [C.POINTER(_Case), C.c_int, dp, dp, dp, dp, dp, dp, dp, ip]
        L.oc_phase.restype = None
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_solve.argtypes = [C.c_int, C.c_int, ip, ip, dp, dp, dp, C.c_double, C.c_int, dp]
        L.oc_solve.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_case_struct(case: dict, literal_ag_order: bool = False) -> _Case:
    g, al, nm = case["grid"], case["alloy"], case["numerics"]
    s = _Case()
    s.dim, s.nx, s.ny = g["dim"], g["nx"], g["ny"]
    s.nz = g["nz"] if g["dim"] == 3 else 1
    s.lx, s.ly, s.lz = g["lx"], g["ly"], g["lz"]
    s.rho, s.mu, s.cp, s.kcond = al["rho"], al["mu"], al["cp"], al["k"]
    s.latent, s.beta_T, s.beta_C = al["latent"], al["beta_T"], al["beta_C"]
    s.lambda2, s.T_m, s.m_sp, s.k_p = al["lambda2"], al["T_m"], al["m_sp"], al["k_p"]
    s.C_e, s.T_ref, s.C_ref = al["C_e"], al["T_ref"], al["C_ref"]
    s.grav, s.darcy_eps = al["g"], al["darcy_eps"]
    for i, b in enumerate(case["bcs"]):
        s.thermal[i] = b["thermal"]
        s.hc[i] = b["h"]
        s.T_ext[i] = b["T_ext"]
        s.T_wall0[i] = b["T0"]
        s.T_ramp[i] = b["b"]
        s.velocity[i] = b["velocity"]
    s.dt, s.tol_p, s.tol_t = nm["dt"], nm["tol_p"], nm["tol_t"]
    s.max_iter = nm["max_iter"]
    s.literal_ag_order = 1 if literal_ag_order else 0
    s.D_l = float(al.get("D_l", 0.0) or 0.0)
    s.mom_form = int(case.get("momentum", 0))
    return s


FIELDS = ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")


class Oracle:
    """State of one case advanced by the oracle (all fields FP64, host)."""

    def __init__(self, case: dict, fields: dict | None = None,
                 literal_ag_order: bool = False, threads: int = 1):
        self.case = case
        self.cs = make_case_struct(case, literal_ag_order)
        self.L = lib()
        self.L.oc_set_threads(int(threads))
        src = case["init"] if fields is None else fields
        self.f = {k: np.array(src[k], dtype=np.float64, copy=True) for k in FIELDS}
        if self.f["w"].size == 0:
            self.f["w"] = np.zeros(1)  # never read in 2D
        self.step_index = int(src.get("step", 0)) if isinstance(src, dict) else 0
        self.last_stats = None
        self.intermediate = None

    # -- helpers
    def rows(self, sys: int) -> int:
        return self.L.oc_sys_rows(C.byref(self.cs), sys)

    def _fields_struct(self):
        fs = _Fields()
        for k in FIELDS:
            setattr(fs, k, _dp(self.f[k]))
        fs.step = self.step_index
        return fs

    def fields(self) -> dict:
        out = {k: self.f[k].copy() for k in FIELDS}
        if self.cs.dim == 2:
            out["w"] = np.zeros(0)
        return out

    # -- operations
    def step(self, nsteps: int = 1, keep_intermediate: bool = False):
        """Advance nsteps time steps (Algorithm 1).  Returns per-step stats."""
        stats = []
        N = self.rows(SYS_P)
        for _ in range(nsteps):
            fs = self._fields_struct()
            st = _Stats()
            inter = None
            if keep_intermediate:
                inter = dict(u=np.zeros(max(1, self.rows(SYS_U))),
                             v=np.zeros(max(1, self.rows(SYS_V))),
                             w=np.zeros(max(1, self.rows(SYS_W))),
                             phi=np.zeros(N), Tstar=np.zeros(N))
                args = [_dp(inter[k]) for k in ("u", "v", "w", "phi", "Tstar")]
            else:
                args = [None] * 5
            rc = self.L.oc_step(C.byref(self.cs), C.byref(fs), C.byref(st), *args)
            if rc != 0:
                raise RuntimeError(f"oracle step failed (no convergence) at step {self.step_index}")
            self.step_index = fs.step
            self.last_stats = st.as_dict()
            stats.append(self.last_stats)
            if keep_intermediate:
                inter["u"] = inter["u"][: self.rows(SYS_U)]
                inter["v"] = inter["v"][: self.rows(SYS_V)]
                inter["w"] = inter["w"][: self.rows(SYS_W)]
                self.intermediate = inter
        return stats

    def assemble(self, sys: int, vel=None, t_new=None):
        """CSR matrix (scipy) and rhs of system `sys` from the current fields.

        Momentum systems use the level-n fields.  For the pressure system
        `vel` = (u*, v*, w*); for the solute and energy systems `vel` is the
        advecting face velocity (defaults to the current velocity field).
        Also returns the raw (row_ptr, col_idx) int32 arrays.
        """
        n = self.rows(sys)
        nd = 2 * self.cs.dim + 1
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(max(1, nd * n), dtype=np.int32)
        va = np.zeros(max(1, nd * n))
        rhs = np.zeros(max(1, n))
        if vel is None:
            vel = (self.f["u"], self.f["v"], self.f["w"])
        vel = [np.ascontiguousarray(x, dtype=np.float64) if x is not None and len(x) else np.zeros(1)
               for x in vel]
        for a in range(self.cs.dim):
            if vel[a].size < self.rows(a):
                raise ValueError(f"velocity component {a}: {vel[a].size} values for {self.rows(a)} faces")
        if t_new is None:
            t_new = (self.step_index + 1) * self.cs.dt
        fs = self._fields_struct()
        nnz = self.L.oc_assemble(C.byref(self.cs), C.byref(fs), _dp(vel[0]), _dp(vel[1]),
                                 _dp(vel[2]), float(t_new), sys, _ip(rp), _ip(ci), _dp(va), _dp(rhs))
        ci, va, rhs = ci[:nnz], va[:nnz], rhs[:n]
        A = sp.csr_matrix((va, ci, rp), shape=(n, n))
        return A, rhs, rp, ci

    def phase(self, Tstar, gn, Cnew):
        """Phase update of eqs. (3.12)-(3.18) per cell; returns T, g, Cl, Cs, branch."""
        Tstar = np.ascontiguousarray(Tstar, dtype=np.float64)
        gn = np.ascontiguousarray(gn, dtype=np.float64)
        Cnew = np.ascontiguousarray(Cnew, dtype=np.float64)
        n = Tstar.size
        T, g, Cl, Cs = (np.zeros(n) for _ in range(4))
        br = np.zeros(n, dtype=np.int32)
        self.L.oc_phase(C.byref(self.cs), n, _dp(Tstar), _dp(gn), _dp(Cnew),
                        _dp(T), _dp(g), _dp(Cl), _dp(Cs), _ip(br))
        return T, g, Cl, Cs, br


def solve(A, b, x0=None, kind="cg", tol=1e-13, max_iter=100000):
    """Solve A x = b with the oracle's Jacobi-PCG (kind="cg") or Jacobi-
    BiCGSTAB (kind="bicgstab").  Returns (x, iterations, relative residual)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rp = np.ascontiguousarray(A.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    va = np.ascontiguousarray(A.data, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    rel = C.c_double(0.0)
    it = lib().oc_solve(0 if kind == "cg" else 1, n, _ip(rp), _ip(ci), _dp(va), _dp(b),
                        _dp(x), float(tol), int(max_iter), C.byref(rel))
    return x, it, rel.value


def run(case: dict, nsteps: int, threads: int = 1):
    """Run a case for nsteps from its initial fields; returns (fields, stats)."""
    o = Oracle(case, threads=threads)
    stats = o.step(nsteps)
    return o.fields(), stats
