"""ctypes binding of libsol.so (the C ABI in include/sol.h).

Argument marshalling only: every step of the time step runs in the HIP
kernels of the library.  When the library is missing the import fails
loudly; there is no fallback path.

PyTorch supplies device memory (its caching allocator, through the
sol_device_ctx alloc/free callbacks) and the stream the library queues on.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsol.so")

SOL_OK, SOL_EINVAL, SOL_ENOMEM, SOL_ENOCONV, SOL_ENONFINITE, SOL_EDEVICE, SOL_EBUSY = 0, -1, -2, -3, -4, -5, -6
SYS_U, SYS_V, SYS_W, SYS_P, SYS_C, SYS_T = range(6)
FIELD_BITS = dict(u=0, v=1, w=2, p=3, T=4, C=5, gl=6, Cl=7, Cs=8,
                  ustar=9, vstar=10, wstar=11, phi=12, Tstar=13)
STATE_FIELDS = ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")
NFIELDS = 14
KCLASS = dict(cg=0, bicg_a=1, bicg_b=2, bicg_c=3, asm_mom=4, asm_trn=5, phase=6,
              mg_pq=7, mg_down0=8, mg_up0=9, mg_coarse=10)
OPT_GRAPH, OPT_PRECOND, OPT_TPRECOND, OPT_ASSEMBLY, OPT_MOMENTUM, OPT_MG_FUSE = 1, 2, 3, 4, 5, 6
ASSEMBLY = dict(stencil=0, forward=1)
MOMENTUM_PLAIN, MOMENTUM_MINIMAL = 0, 1     # eq. (2.7) / eq. (2.6)
PRECOND = dict(jacobi=0, mg=1)
TPRECOND = dict(jacobi=0, jacobi2=1, auto=2)


class SolError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sol error {code}: {msg}")
        self.code = code


class sol_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double)]


class sol_alloy(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("rho", "mu", "cp", "k", "latent", "beta_T", "beta_C", "lambda2", "T_m", "m_sp",
                 "k_p", "C_e", "T_ref", "C_ref", "g", "D_l", "darcy_eps")]


class sol_face_bc(C.Structure):
    _fields_ = [("thermal", C.c_int32), ("h", C.c_double), ("T_ext", C.c_double),
                ("T0", C.c_double), ("b", C.c_double), ("velocity", C.c_int32)]


class sol_bcs(C.Structure):
    _fields_ = [("face", sol_face_bc * 6)]


class sol_numerics(C.Structure):
    _fields_ = [("dt", C.c_double), ("tol_p", C.c_double), ("tol_t", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class sol_device_ctx(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class sol_step_stats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 6), ("iters_total", C.c_int64 * 6),
                ("rel_resid", C.c_double * 6), ("sum_resid", C.c_double * 6),
                ("sum_C", C.c_double), ("sum_H", C.c_double), ("wall_flux", C.c_double),
                ("div_star", C.c_double), ("div_new", C.c_double), ("step", C.c_int64),
                ("redone", C.c_int64)]

    def as_dict(self):
        return dict(iters=list(self.iters), iters_total=list(self.iters_total),
                    rel_resid=list(self.rel_resid), sum_resid=list(self.sum_resid),
                    sum_C=self.sum_C, sum_H=self.sum_H, wall_flux=self.wall_flux,
                    div_star=self.div_star, div_new=self.div_new, step=self.step, redone=self.redone)


_lib = None


def load():
    """Load libsol.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} not found: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIBPATH)
    P, I32, U32 = C.c_void_p, C.c_int32, C.c_uint32
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    sig = {
        "sol_create": ([C.POINTER(sol_grid), C.POINTER(sol_alloy), C.POINTER(sol_bcs),
                        C.POINTER(sol_numerics), C.POINTER(sol_device_ctx), C.POINTER(P)], I32),
        "sol_destroy": ([P], None),
        "sol_write_fields": ([P, U32, C.POINTER(dp)], I32),
        "sol_read_fields": ([P, U32, C.POINTER(dp)], I32),
        "sol_system_size": ([P, I32, ip, ip], I32),
        "sol_assemble": ([P, U32], I32),
        "sol_read_matrix": ([P, I32, ip, ip, dp, dp], I32),
        "sol_read_matrix_noalloc": ([P, I32, ip, ip, dp, dp], I32),
        "sol_step": ([P, I32, C.POINTER(sol_step_stats)], I32),
        "sol_footprint_bytes": ([C.POINTER(sol_grid), C.POINTER(sol_numerics), C.POINTER(C.c_size_t)], I32),
        "sol_batch_create": ([C.POINTER(P), I32, C.POINTER(P)], I32),
        "sol_batch_step": ([P, C.POINTER(I32), C.POINTER(sol_step_stats)], I32),
        "sol_batch_destroy": ([P], None),
        "sol_set_timing": ([P, I32], I32),
        "sol_get_timing": ([P, I32, C.POINTER(C.c_int64), dp, dp], I32),
        "sol_set_option": ([P, I32, C.c_int64], I32),
        "sol_dispatch_count": ([C.POINTER(C.c_int64)], I32),
        "sol_autotune": ([P, ip], I32),
        "sol_last_error": ([], C.c_char_p),
        "sol_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def exported_symbols():
    return ["sol_create", "sol_destroy", "sol_write_fields", "sol_read_fields", "sol_system_size",
            "sol_assemble", "sol_read_matrix", "sol_read_matrix_noalloc", "sol_step", "sol_footprint_bytes",
            "sol_batch_create", "sol_batch_step", "sol_batch_destroy", "sol_set_timing",
            "sol_get_timing", "sol_set_option", "sol_autotune", "sol_last_error", "sol_version",
            "sol_dispatch_count"]


def dispatch_count() -> int:
    """Device work items (kernel dispatches, graph nodes, state copies) the
    library has queued in this process so far."""
    n = C.c_int64(0)
    check(load().sol_dispatch_count(C.byref(n)))
    return n.value


def check(rc):
    if rc != SOL_OK:
        raise SolError(rc, load().sol_last_error().decode())
    return rc


# ------------------------------------------------------------- marshalling

def make_structs(case: dict):
    g, a, nm = case["grid"], case["alloy"], case["numerics"]
    grid = sol_grid(g["dim"], g["nx"], g["ny"], g["nz"] if g["dim"] == 3 else 1,
                    g["lx"], g["ly"], g["lz"] if g["dim"] == 3 else 1.0)
    alloy = sol_alloy(a["rho"], a["mu"], a["cp"], a["k"], a["latent"], a["beta_T"], a["beta_C"],
                      a["lambda2"], a["T_m"], a["m_sp"], a["k_p"], a["C_e"], a["T_ref"], a["C_ref"],
                      a["g"], a.get("D_l", 0.0), a["darcy_eps"])
    bcs = sol_bcs()
    for i, b in enumerate(case["bcs"]):
        bcs.face[i] = sol_face_bc(b["thermal"], b["h"], b["T_ext"], b["T0"], b["b"], b["velocity"])
    num = sol_numerics(nm["dt"], nm["tol_p"], nm["tol_t"], nm["max_iter"], nm["precision"])
    return grid, alloy, bcs, num


def sol_footprint_bytes(case: dict) -> int:
    grid, _, _, num = make_structs(case)
    out = C.c_size_t(0)
    check(load().sol_footprint_bytes(C.byref(grid), C.byref(num), C.byref(out)))
    return out.value


class TorchDevice:
    """Device memory from torch's caching allocator and torch's current
    stream, handed to the library through sol_device_ctx."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dev_index = self.device.index or 0
        st = self.stream
        c_alloc = torch.cuda.caching_allocator_alloc
        c_delete = torch.cuda.caching_allocator_delete
        on_device = torch.cuda.device

        def _alloc(nbytes, user):
            with on_device(dev_index):
                return c_alloc(int(nbytes), dev_index, st)

        def _free(ptr, user):
            c_delete(ptr)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.ctx = sol_device_ctx(C.c_void_p(self.stream.cuda_stream), self._alloc, self._free, None)


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # release every handle while torch (its allocator) is still alive;
    # batches before the cases they reference
    objs = sorted(list(_live), key=lambda o: 0 if isinstance(o, Batch) else 1)
    for obj in objs:
        try:
            obj.close()
        except Exception:
            pass


class Case:
    """One case (handle) of the library; fields are numpy FP64 arrays on the host side."""

    def __init__(self, case: dict, device: TorchDevice | None = None, write_init: bool = True):
        L = load()
        self.case = case
        self.dev = device
        self.grid, self.alloy, self.bcs, self.num = make_structs(case)
        h = C.c_void_p()
        ctx = C.byref(device.ctx) if device is not None else None
        check(L.sol_create(C.byref(self.grid), C.byref(self.alloy), C.byref(self.bcs),
                           C.byref(self.num), ctx, C.byref(h)))
        self.h = h
        _live.add(self)
        self.sizes = {}
        g = case["grid"]
        nx, ny, nz = g["nx"], g["ny"], g["nz"] if g["dim"] == 3 else 1
        n = nx * ny * nz
        self.sizes = dict(u=(nx - 1) * ny * nz, v=nx * (ny - 1) * nz,
                          w=nx * ny * (nz - 1) if g["dim"] == 3 else 0,
                          p=n, T=n, C=n, gl=n, Cl=n, Cs=n)
        self.sizes.update(ustar=self.sizes["u"], vstar=self.sizes["v"], wstar=self.sizes["w"], phi=n, Tstar=n)
        form = int(case.get("momentum", MOMENTUM_PLAIN))
        if form != MOMENTUM_PLAIN:
            self.set_momentum(form)
        if write_init:
            self.write_fields(case["init"])

    def close(self):
        if self.h:
            load().sol_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def write_fields(self, fields: dict):
        arrs = (C.POINTER(C.c_double) * NFIELDS)()
        keep = []
        mask = 0
        for k, v in fields.items():
            if k not in STATE_FIELDS:
                continue
            a = np.ascontiguousarray(v, dtype=np.float64)
            if a.size != self.sizes[k]:
                raise ValueError(f"field {k}: {a.size} values, expected {self.sizes[k]}")
            keep.append(a)
            arrs[FIELD_BITS[k]] = a.ctypes.data_as(C.POINTER(C.c_double))
            mask |= 1 << FIELD_BITS[k]
        check(load().sol_write_fields(self.h, mask, arrs))

    def read_fields(self, names=STATE_FIELDS) -> dict:
        arrs = (C.POINTER(C.c_double) * NFIELDS)()
        out = {}
        mask = 0
        for k in names:
            a = np.zeros(max(1, self.sizes[k]))
            out[k] = a
            arrs[FIELD_BITS[k]] = a.ctypes.data_as(C.POINTER(C.c_double))
            mask |= 1 << FIELD_BITS[k]
        check(load().sol_read_fields(self.h, mask, arrs))
        return {k: v[: self.sizes[k]] for k, v in out.items()}

    def step(self, nsteps: int = 1) -> dict:
        st = sol_step_stats()
        check(load().sol_step(self.h, int(nsteps), C.byref(st)))
        return st.as_dict()

    def assemble(self, mask: int = 0x3F):
        check(load().sol_assemble(self.h, mask))

    def system_size(self, sys: int):
        r, z = C.c_int32(0), C.c_int32(0)
        check(load().sol_system_size(self.h, sys, C.byref(r), C.byref(z)))
        return r.value, z.value

    def read_matrix(self, sys: int, noalloc: bool = False):
        """CSR export of a system; noalloc selects sol_read_matrix_noalloc."""
        n, nnz = self.system_size(sys)
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(max(1, nnz), dtype=np.int32)
        va = np.zeros(max(1, nnz))
        rhs = np.zeros(max(1, n))
        fn = load().sol_read_matrix_noalloc if noalloc else load().sol_read_matrix
        check(fn(self.h, sys, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                     ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                     va.ctypes.data_as(C.POINTER(C.c_double)),
                                     rhs.ctypes.data_as(C.POINTER(C.c_double))))
        return rp, ci[:nnz], va[:nnz], rhs[:n]

    def set_graph(self, on: bool):
        check(load().sol_set_option(self.h, OPT_GRAPH, 1 if on else 0))

    def set_precond(self, name: str):
        """Pressure-CG preconditioner: 'mg' (default) or 'jacobi'."""
        check(load().sol_set_option(self.h, OPT_PRECOND, PRECOND[name]))

    def set_assembly(self, name: str):
        """'stencil' (closed-form rows) or 'forward' (residual probing)."""
        check(load().sol_set_option(self.h, OPT_ASSEMBLY, ASSEMBLY[name]))

    def set_mg_fuse(self, on: bool):
        """Coarse multigrid levels in fused pairs (default) or one launch each."""
        check(load().sol_set_option(self.h, OPT_MG_FUSE, 1 if on else 0))

    def set_momentum(self, form: int):
        """Momentum form of the predictor: MOMENTUM_PLAIN (eq. 2.7, default)
        or MOMENTUM_MINIMAL (eq. 2.6)."""
        check(load().sol_set_option(self.h, OPT_MOMENTUM, int(form)))

    def set_tprecond(self, name: str):
        """BiCGSTAB preconditioner of the momentum, solute and energy solves:
        'auto' (default: two Jacobi sweeps in 2D, one in 3D), 'jacobi2' (two)
        or 'jacobi' (one)."""
        check(load().sol_set_option(self.h, OPT_TPRECOND, TPRECOND[name]))

    def autotune(self) -> int:
        r = C.c_int32(0)
        check(load().sol_autotune(self.h, C.byref(r)))
        return r.value

    def set_timing(self, on: bool):
        check(load().sol_set_timing(self.h, 1 if on else 0))

    def timing(self, kclass: str):
        n, ms, by = C.c_int64(0), C.c_double(0), C.c_double(0)
        check(load().sol_get_timing(self.h, KCLASS[kclass], C.byref(n), C.byref(ms), C.byref(by)))
        return dict(launches=n.value, ms=ms.value, bytes=by.value)


class Batch:
    """Several cases advanced together (one launch per kernel for all)."""

    def __init__(self, cases):
        self.cases = list(cases)
        arr = (C.c_void_p * len(self.cases))(*[c.h.value for c in self.cases])
        b = C.c_void_p()
        check(load().sol_batch_create(arr, len(self.cases), C.byref(b)))
        self.b = b
        _live.add(self)

    def step(self, nsteps):
        if isinstance(nsteps, int):
            nsteps = [nsteps] * len(self.cases)
        ns = (C.c_int32 * len(self.cases))(*[int(x) for x in nsteps])
        st = (sol_step_stats * len(self.cases))()
        check(load().sol_batch_step(self.b, ns, st))
        return [s.as_dict() for s in st]

    def close(self):
        if self.b:
            load().sol_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
