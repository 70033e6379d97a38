"""ctypes binding of ``libdbs.so`` (the C ABI declared in ``include/dbs.h``).

Argument marshalling only: every step of the PISO path runs in the HIP
kernels of the library.  There is no CPU fallback; loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbs.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENAN, ECOURANT, EBOUNDS = 0, -1, -2, -3, -4, -5, -6, -7
_KIND = {"wall": 0, "inlet": 1, "outlet": 2, "empty": 3, "wave": 4}
_MODEL = {"brooks_corey": 0, "van_genuchten": 1}
_PREC = {"fp64": 0, "mixed": 1}

EXPORTS = (
    "dbs_create", "dbs_set_static", "dbs_set_state", "dbs_step", "dbs_get_state",
    "dbs_set_state_dev", "dbs_get_state_dev", "dbs_set_stream", "dbs_get_stats",
    "dbs_last_error", "dbs_destroy", "dbs_set_profiling", "dbs_kernel_time",
    "dbs_kernel_name", "dbs_kernel_classes", "dbs_reset_profiling",
    "dbs_debug_pressure_solve", "dbs_debug_step_trace",
    "dbs_batch_create", "dbs_batch_size", "dbs_batch_set_static", "dbs_batch_set_state",
    "dbs_batch_get_state", "dbs_batch_set_state_dev", "dbs_batch_get_state_dev",
    "dbs_batch_get_stats", "dbs_batch_step", "dbs_set_graph", "dbs_autotune", "dbs_set_tuning", "dbs_set_time",
    "dbs_pressure_solve_noalloc",
)


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Physics(C.Structure):
    _fields_ = [("rho_l", C.c_double), ("rho_g", C.c_double), ("mu_l", C.c_double),
                ("mu_g", C.c_double), ("g", C.c_double * 3), ("c_alpha", C.c_double),
                ("kr_model", C.c_int), ("kr_m", C.c_double), ("s_lirr", C.c_double),
                ("s_girr", C.c_double), ("pc_model", C.c_int), ("pc0", C.c_double),
                ("pc_exp", C.c_double), ("a_pcirr", C.c_double), ("a_pcmax", C.c_double),
                ("eps_pc", C.c_double), ("sigma", C.c_double),
                ("contact_angle", C.c_double)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int), ("U", C.c_double * 3), ("alpha", C.c_double),
                ("p", C.c_double), ("wave", C.c_double * 3)]


class Controls(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_corr", C.c_int), ("mom_maxit", C.c_int),
                ("transpose_visc", C.c_int), ("mules_iter", C.c_int), ("p_tol", C.c_double),
                ("p_maxit", C.c_int), ("precision", C.c_int), ("mg_pre", C.c_int),
                ("mg_post", C.c_int), ("max_courant", C.c_double), ("bounds_tol", C.c_double),
                ("target_courant", C.c_double), ("dt_max", C.c_double),
                ("mom_tol", C.c_double), ("n_alpha_sub", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_longlong), ("p_iters", C.c_int * 16),
                ("p_relres", C.c_double * 16), ("mg_levels", C.c_int),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("phase_volume", C.c_double), ("max_courant", C.c_double),
                ("time", C.c_double), ("dt", C.c_double), ("mom_sweeps", C.c_int),
                ("mom_relres", C.c_double), ("p_bnorm", C.c_double * 16),
                ("p_res0", C.c_double * 16), ("max_div", C.c_double),
                ("p_guess_order", C.c_int), ("p_guess_change", C.c_int * 16)]


_DP = C.POINTER(C.c_double)
_lib = None


class DBSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dbs error {code}: {msg}")
        self.code = code


def lib():
    """Load libdbs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2003_08374_amd.build` (no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        L.dbs_create.argtypes = [C.POINTER(Grid), C.POINTER(Physics), C.POINTER(BC),
                                 C.POINTER(Controls), C.POINTER(H)]
        L.dbs_set_static.argtypes = [H, _DP, _DP]
        L.dbs_set_state.argtypes = [H, _DP, _DP, _DP, _DP]
        L.dbs_step.argtypes = [H, C.c_int]
        L.dbs_batch_step.argtypes = [H, C.c_int]
        L.dbs_get_state.argtypes = [H, _DP, _DP, _DP, _DP, _DP]
        L.dbs_set_state_dev.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]
        L.dbs_get_state_dev.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        L.dbs_set_stream.argtypes = [H, C.c_void_p]
        L.dbs_get_stats.argtypes = [H, C.POINTER(Stats)]
        L.dbs_last_error.argtypes = [H]
        L.dbs_last_error.restype = C.c_char_p
        L.dbs_destroy.argtypes = [H]
        L.dbs_destroy.restype = None
        L.dbs_set_profiling.argtypes = [H, C.c_ulonglong]
        L.dbs_kernel_time.argtypes = [H, C.c_int, C.POINTER(C.c_longlong), _DP]
        L.dbs_kernel_name.argtypes = [C.c_int]
        L.dbs_kernel_name.restype = C.c_char_p
        L.dbs_kernel_classes.argtypes = []
        L.dbs_reset_profiling.argtypes = [H]
        L.dbs_reset_profiling.restype = None
        L.dbs_debug_pressure_solve.argtypes = [H, _DP, _DP, _DP, C.POINTER(C.c_int), _DP]
        L.dbs_debug_step_trace.argtypes = [H] + [_DP] * 10
        L.dbs_batch_create.argtypes = [C.c_int, C.POINTER(Grid), C.POINTER(Physics),
                                       C.POINTER(BC), C.POINTER(Controls), C.POINTER(H)]
        L.dbs_batch_size.argtypes = [H]
        L.dbs_batch_set_static.argtypes = [H, C.c_int, _DP, _DP]
        L.dbs_batch_set_state.argtypes = [H, C.c_int, _DP, _DP, _DP, _DP]
        L.dbs_batch_get_state.argtypes = [H, C.c_int, _DP, _DP, _DP, _DP, _DP]
        L.dbs_batch_set_state_dev.argtypes = [H, C.c_int] + [C.c_void_p] * 5
        L.dbs_batch_get_state_dev.argtypes = [H, C.c_int] + [C.c_void_p] * 6
        L.dbs_batch_get_stats.argtypes = [H, C.c_int, C.POINTER(Stats)]
        L.dbs_set_graph.argtypes = [H, C.c_int]
        L.dbs_autotune.argtypes = [H] + [C.POINTER(C.c_int)] * 6 + [_DP]
        L.dbs_set_tuning.argtypes = [H] + [C.c_int] * 7
        L.dbs_set_time.argtypes = [H, C.c_double]
        L.dbs_pressure_solve_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(C.c_int), C.c_int,
                                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                                 C.c_int, C.POINTER(C.c_int), _DP, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def nfaces(shape):
    nx, ny, nz = shape
    return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)


def make_structs(case, precision=None, p_tol=None, mg=None, max_courant=0.0, bounds_tol=0.0):
    g = Grid()
    g.nx, g.ny, g.nz = case.shape
    g.dx, g.dy, g.dz = case.h
    p = Physics()
    fl = case.fluids
    p.rho_l, p.rho_g, p.mu_l, p.mu_g = fl["rho_l"], fl["rho_g"], fl["mu_l"], fl["mu_g"]
    for a in range(3):
        p.g[a] = case.g[a]
    p.c_alpha = case.c_alpha
    p.kr_model = _MODEL[case.kr["model"]]
    p.kr_m = case.kr["m"]
    p.s_lirr = case.kr.get("s_lirr", 0.0)
    p.s_girr = case.kr.get("s_girr", 0.0)
    p.pc_model = _MODEL[case.pc["model"]]
    p.pc0 = case.pc["pc0"]
    p.pc_exp = case.pc["exp"]
    p.a_pcirr = case.pc.get("a_irr", 0.0)
    p.a_pcmax = case.pc.get("a_max", 1.0)
    p.eps_pc = case.pc.get("eps", 1e-3)
    p.sigma = float(getattr(case, "sigma", 0.0))
    p.contact_angle = float(getattr(case, "contact_angle", 0.0))
    bcs = (BC * 6)()
    for b in range(6):
        d = case.bc[b]
        bcs[b].kind = _KIND[d["kind"]]
        for a in range(3):
            bcs[b].U[a] = d.get("U", (0.0, 0.0, 0.0))[a]
        bcs[b].alpha = d.get("alpha", 0.0)
        bcs[b].p = d.get("p", 0.0)
        for q in range(3):
            bcs[b].wave[q] = d.get("wave", (0.0, 0.0, 0.0))[q]
    c = Controls()
    c.dt = case.dt
    c.n_corr = case.n_corr
    c.mom_maxit = int(case.mom_maxit)
    c.mom_tol = float(case.mom_tol)
    c.n_alpha_sub = int(getattr(case, "n_alpha_sub", 1))
    c.transpose_visc = int(case.transpose_visc)
    c.mules_iter = int(case.mules_iter)
    c.p_tol = case.p_tol if p_tol is None else p_tol
    c.p_maxit = case.p_maxit
    c.precision = _PREC[precision or case.precision]
    c.mg_pre, c.mg_post = mg if mg else (0, 0)
    c.max_courant = max_courant
    c.bounds_tol = bounds_tol
    c.target_courant = float(getattr(case, "target_courant", 0.0))
    c.dt_max = float(getattr(case, "dt_max", 0.0))
    return g, p, bcs, c


NOALLOC_BYTES = 64 << 20
NOALLOC_MAX_CELLS = 1 << 19


def pressure_solve_noalloc(case, rAU, b, x, tol, maxit=2000, precision="fp64", stream=None):
    """dbs_pressure_solve_noalloc on device buffers given as raw pointers
    (e.g. torch ``data_ptr()``) of nx*ny*nz doubles; the mesh and the kinds
    of the six domain faces come from ``case``.  Returns (iterations,
    relative residual); raises DBSError on failure."""
    g = Grid()
    g.nx, g.ny, g.nz = case.shape
    g.dx, g.dy, g.dz = case.h
    kinds = (C.c_int * 6)(*[_KIND[bc["kind"]] for bc in case.bc])
    it = C.c_int()
    rr = C.c_double()
    rc = lib().dbs_pressure_solve_noalloc(C.byref(g), kinds, _PREC[precision], rAU, b, x,
                                          float(tol), int(maxit), C.byref(it), C.byref(rr),
                                          stream)
    if rc != OK:
        raise DBSError(rc, lib().dbs_last_error(None).decode())
    return it.value, rr.value


class _Handle:
    """Methods shared by single-sample and batch handles."""

    h = None

    def _check(self, rc, h="self"):
        if rc != OK:
            msg = ""
            if h == "self" and getattr(self, "h", None):
                msg = lib().dbs_last_error(self.h).decode()
            raise DBSError(rc, msg)
        return rc

    _STEP = "dbs_step"

    def step(self, n=1, check=True):
        rc = getattr(lib(), self._STEP)(self.h, int(n))
        if check:
            self._check(rc)
        return rc

    def set_stream(self, stream):
        self._check(lib().dbs_set_stream(self.h, stream))

    def set_graph(self, on=True):
        """Replay steps from captured HIP graphs (see dbs_set_graph)."""
        self._check(lib().dbs_set_graph(self.h, int(bool(on))))

    def autotune(self):
        """Tune tile depth, sweeps, coarse sweeps, bottom depth and sweep
        fusion on the current state (which is left unchanged)."""
        v = [C.c_int() for _ in range(6)]
        ms = C.c_double()
        self._check(lib().dbs_autotune(self.h, *[C.byref(x) for x in v], C.byref(ms)))
        return {"kz": v[0].value, "sweeps": v[1].value, "coarse_sweeps": v[2].value,
                "bottom_shift": v[3].value, "fused": v[4].value, "coarse_block": v[5].value,
                "ms": ms.value}

    def set_time(self, t):
        self._check(lib().dbs_set_time(self.h, float(t)))

    def set_tuning(self, kz=0, sweeps=2, coarse_sweeps=2, bottom_shift=0, fused=1,
                   kz_coarse=0, coarse_block=0):
        self._check(lib().dbs_set_tuning(self.h, int(kz), int(kz_coarse), int(sweeps),
                                         int(coarse_sweeps), int(bottom_shift), int(fused),
                                         int(coarse_block)))

    @staticmethod
    def _stats_dict(s, n):
        return {"steps": s.steps, "p_iters": list(s.p_iters)[:n],
                "p_relres": list(s.p_relres)[:n], "mg_levels": s.mg_levels,
                "alpha_min": s.alpha_min, "alpha_max": s.alpha_max,
                "phase_volume": s.phase_volume, "max_courant": s.max_courant,
                "time": s.time, "dt": s.dt, "mom_sweeps": s.mom_sweeps,
                "mom_relres": s.mom_relres, "p_bnorm": list(s.p_bnorm)[:n],
                "p_res0": list(s.p_res0)[:n], "max_div": s.max_div,
                "p_guess_order": s.p_guess_order,
                "p_guess_change": list(s.p_guess_change)[:n]}

    # -------------------------------------------------------------- profiling
    def set_profiling(self, mask):
        self._check(lib().dbs_set_profiling(self.h, C.c_ulonglong(mask)))

    def reset_profiling(self):
        lib().dbs_reset_profiling(self.h)

    def kernel_times(self):
        L = lib()
        out = {}
        for c in range(L.dbs_kernel_classes()):
            n = C.c_longlong()
            ms = C.c_double()
            self._check(L.dbs_kernel_time(self.h, c, C.byref(n), C.byref(ms)))
            if n.value:
                out[L.dbs_kernel_name(c).decode()] = (n.value, ms.value)
        return out

    @staticmethod
    def kernel_class(name):
        L = lib()
        for c in range(L.dbs_kernel_classes()):
            if L.dbs_kernel_name(c).decode() == name:
                return c
        raise KeyError(name)

    def close(self):
        if getattr(self, "h", None):
            lib().dbs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _flat_faces(F):
    if isinstance(F, (tuple, list)):
        F = np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in F])
    return np.ascontiguousarray(F, dtype=np.float64)


def _split_faces(F, shape):
    nx, ny, nz = shape
    n1 = (nx + 1) * ny * nz
    n2 = n1 + nx * (ny + 1) * nz
    return (F[:n1], F[n1:n2], F[n2:])


class Solver(_Handle):
    """One single-domain problem resident on the current HIP device."""

    def __init__(self, case, precision=None, p_tol=None, mg=None, max_courant=0.0,
                 bounds_tol=0.0, state=None):
        self.case = case
        self.shape = tuple(case.shape)
        self.nc = int(np.prod(self.shape))
        self.nf = nfaces(self.shape)
        L = lib()
        g, p, bcs, c = make_structs(case, precision, p_tol, mg, max_courant, bounds_tol)
        h = C.c_void_p()
        self._check(L.dbs_create(C.byref(g), C.byref(p), bcs, C.byref(c), C.byref(h)), None)
        self.h = h
        phi = np.ascontiguousarray(case.phi, dtype=np.float64).reshape(self.nc)
        kinv = np.ascontiguousarray(case.kinv, dtype=np.float64).reshape(self.nc)
        self._check(L.dbs_set_static(h, _ptr(phi), _ptr(kinv)))
        if state is None:
            F = None
            if getattr(case, "F", None) is not None:
                F = np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in case.F])
            state = {"alpha": case.alpha, "U": case.U, "p_rgh": case.p_rgh, "F": F}
        self.set_state(state)

    def set_state(self, st):
        a = np.ascontiguousarray(st["alpha"], dtype=np.float64).reshape(self.nc)
        U = np.ascontiguousarray(st["U"], dtype=np.float64).reshape(3 * self.nc)
        pr = np.ascontiguousarray(st["p_rgh"], dtype=np.float64).reshape(self.nc)
        F = st.get("F")
        if F is not None:
            if isinstance(F, (tuple, list)):
                F = np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in F])
            F = np.ascontiguousarray(F, dtype=np.float64)
            assert F.size == self.nf
        self._check(lib().dbs_set_state(self.h, _ptr(a), _ptr(U), _ptr(pr), _ptr(F)))

    def state(self):
        a = np.zeros(self.nc)
        U = np.zeros(3 * self.nc)
        pr = np.zeros(self.nc)
        p = np.zeros(self.nc)
        F = np.zeros(self.nf)
        self._check(lib().dbs_get_state(self.h, _ptr(a), _ptr(U), _ptr(pr), _ptr(p), _ptr(F)))
        nx, ny, nz = self.shape
        n1 = (nx + 1) * ny * nz
        n2 = n1 + nx * (ny + 1) * nz
        return {"alpha": a, "U": U.reshape(3, self.nc), "p_rgh": pr, "p": p,
                "F": (F[:n1], F[n1:n2], F[n2:])}

    def set_state_dev(self, alpha, U, p_rgh, F=None, stream=None):
        """Device buffers given as raw pointers (e.g. torch ``data_ptr()``)."""
        self._check(lib().dbs_set_state_dev(self.h, alpha, U, p_rgh, F, stream))

    def get_state_dev(self, alpha=None, U=None, p_rgh=None, p=None, F=None, stream=None):
        self._check(lib().dbs_get_state_dev(self.h, alpha, U, p_rgh, p, F, stream))

    def stats(self):
        s = Stats()
        self._check(lib().dbs_get_stats(self.h, C.byref(s)))
        return self._stats_dict(s, self.case.n_corr)

    def pressure_solve(self, rAU, b, x0=None):
        rAU = np.ascontiguousarray(rAU, dtype=np.float64).ravel()
        b = np.ascontiguousarray(b, dtype=np.float64).ravel()
        x = np.zeros(self.nc) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).copy()
        it = C.c_int()
        rr = C.c_double()
        self._check(lib().dbs_debug_pressure_solve(self.h, _ptr(rAU), _ptr(b), _ptr(x),
                                                   C.byref(it), C.byref(rr)))
        return x, it.value, rr.value

    TRACE = ("A", "rAU", "Shat", "Ustar", "HbyA", "phiHbyA", "b", "Rp", "Rm", "alphaPhi")

    def trace_step(self):
        nc, nf = self.nc, self.nf
        size = {"A": nf, "rAU": nc, "Shat": 3 * nc, "Ustar": 3 * nc, "HbyA": 3 * nc,
                "phiHbyA": nf, "b": nc, "Rp": nc, "Rm": nc, "alphaPhi": nf}
        out = {k: np.zeros(size[k]) for k in self.TRACE}
        self._check(lib().dbs_debug_step_trace(self.h, *[_ptr(out[k]) for k in self.TRACE]))
        return out



class BatchSolver(_Handle):
    """Many independent samples advanced together (one launch per stage).

    The cases share fluids, closures, gravity, dt and solver controls; each
    has its own mesh, boundary values, porosity, permeability and state."""
    _STEP = "dbs_batch_step"

    def __init__(self, cases, precision=None, p_tol=None, mg=None, max_courant=0.0,
                 bounds_tol=0.0):
        cases = list(cases)
        assert cases, "empty batch"
        self.cases = cases
        n = len(cases)
        grids = (Grid * n)()
        bcs = (BC * (6 * n))()
        phys = ctl = None
        for i, cs in enumerate(cases):
            g, p, b6, c = make_structs(cs, precision, p_tol, mg, max_courant, bounds_tol)
            grids[i] = g
            for b in range(6):
                bcs[6 * i + b] = b6[b]
            if phys is None:
                phys, ctl = p, c
            elif bytes(p) != bytes(phys) or bytes(c) != bytes(ctl):
                # one physics and one set of controls serve the whole batch
                raise ValueError(f"sample {i} ({cs.name}) differs from sample 0 in its "
                                 "fluids, models, constants or controls")
        h = C.c_void_p()
        self._check(lib().dbs_batch_create(n, grids, C.byref(phys), bcs, C.byref(ctl),
                                           C.byref(h)), None)
        self.h = h
        self.n = n
        self.shapes = [tuple(cs.shape) for cs in cases]
        for i, cs in enumerate(cases):
            nc = int(np.prod(cs.shape))
            phi = np.ascontiguousarray(cs.phi, dtype=np.float64).reshape(nc)
            kinv = np.ascontiguousarray(cs.kinv, dtype=np.float64).reshape(nc)
            self._check(lib().dbs_batch_set_static(h, i, _ptr(phi), _ptr(kinv)))
            F = getattr(cs, "F", None)
            self.set_state(i, {"alpha": cs.alpha, "U": cs.U, "p_rgh": cs.p_rgh,
                               "F": None if F is None else _flat_faces(F)})

    def set_state(self, i, st):
        nc = int(np.prod(self.shapes[i]))
        a = np.ascontiguousarray(st["alpha"], dtype=np.float64).reshape(nc)
        U = np.ascontiguousarray(st["U"], dtype=np.float64).reshape(3 * nc)
        pr = np.ascontiguousarray(st["p_rgh"], dtype=np.float64).reshape(nc)
        F = st.get("F")
        if F is not None:
            F = _flat_faces(F)
            assert F.size == nfaces(self.shapes[i])
        self._check(lib().dbs_batch_set_state(self.h, int(i), _ptr(a), _ptr(U), _ptr(pr),
                                              _ptr(F)))

    def state(self, i):
        shape = self.shapes[i]
        nc = int(np.prod(shape))
        a, U, pr, p = np.zeros(nc), np.zeros(3 * nc), np.zeros(nc), np.zeros(nc)
        F = np.zeros(nfaces(shape))
        self._check(lib().dbs_batch_get_state(self.h, int(i), _ptr(a), _ptr(U), _ptr(pr),
                                              _ptr(p), _ptr(F)))
        return {"alpha": a, "U": U.reshape(3, nc), "p_rgh": pr, "p": p,
                "F": _split_faces(F, shape)}

    def stats(self, i):
        s = Stats()
        self._check(lib().dbs_batch_get_stats(self.h, int(i), C.byref(s)))
        return self._stats_dict(s, self.cases[0].n_corr)
