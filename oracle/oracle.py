"""ctypes binding of the plain FP64 CPU oracle (``libdbs_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  It never imports the HIP product
package, and the product package never imports it.

Cases are duck-typed objects with the attributes produced by the seeded input
generators (shape, h, fluids, g, c_alpha, kr, pc, bc, dt, n_corr, mom_maxit,
mom_tol, n_alpha_sub, transpose_visc, p_tol, p_maxit, phi, kinv).  State dicts
hold flat float64 arrays: alpha (nc), U (3, nc), p_rgh (nc), p (nc), F = (Fx, Fy, Fz).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbs_oracle.so")

_KIND = {"wall": 0, "inlet": 1, "outlet": 2, "empty": 3, "wave": 4}
_MODEL = {"brooks_corey": 0, "van_genuchten": 1}


class OracleCase(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
        ("rho_l", C.c_double), ("rho_g", C.c_double),
        ("mu_l", C.c_double), ("mu_g", C.c_double),
        ("g", C.c_double * 3),
        ("c_alpha", C.c_double),
        ("kr_model", C.c_int), ("kr_m", C.c_double),
        ("pc_model", C.c_int), ("pc0", C.c_double), ("pc_exp", C.c_double),
        ("s_lirr", C.c_double), ("s_girr", C.c_double),
        ("a_pcirr", C.c_double), ("a_pcmax", C.c_double), ("eps_pc", C.c_double),
        ("bc_kind", C.c_int * 6),
        ("bc_U", (C.c_double * 3) * 6),
        ("bc_alpha", C.c_double * 6),
        ("bc_p", C.c_double * 6),
        ("dt", C.c_double),
        ("n_corr", C.c_int), ("mom_maxit", C.c_int), ("transpose_visc", C.c_int),
        ("mules_iter", C.c_int),
        ("p_tol", C.c_double), ("p_maxit", C.c_int),
        ("bc_wave", (C.c_double * 3) * 6),
        ("t0", C.c_double),
        ("sigma", C.c_double),
        ("contact_angle", C.c_double),
        ("target_courant", C.c_double), ("dt_max", C.c_double),
        ("mom_tol", C.c_double), ("n_alpha_sub", C.c_int),
    ]


class OracleInfo(C.Structure):
    _fields_ = [
        ("p_iters", C.c_int * 16),
        ("p_relres", C.c_double * 16),
        ("alpha_min", C.c_double), ("alpha_max", C.c_double),
        ("phase_volume", C.c_double), ("max_div", C.c_double),
        ("dt_last", C.c_double), ("t_end", C.c_double),
        ("mom_sweeps", C.c_int), ("mom_relres", C.c_double),
        ("p_bnorm", C.c_double * 16),
    ]


_DP = C.POINTER(C.c_double)


class OracleTrace(C.Structure):
    _fields_ = [(n, _DP) for n in (
        "A", "Rp", "Rm", "alphaPhi", "alpha_new", "rAU", "Shat", "Ustar",
        "HbyA", "phiHbyA", "b", "aP", "aON", "aNO", "B")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no FMA contraction)."""
    src = os.path.join(_HERE, "dbs_oracle.c")
    hdr = os.path.join(_HERE, "dbs_oracle.h")
    stale = (not os.path.exists(LIB_PATH) or
             max(os.path.getmtime(src), os.path.getmtime(hdr)) > os.path.getmtime(LIB_PATH))
    if force or stale:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
            "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB_PATH)
        L.dbso_closures.argtypes = [C.POINTER(OracleCase), C.c_double, _DP, _DP, _DP, _DP]
        L.dbso_closures.restype = None
        L.dbso_init_flux.argtypes = [C.POINTER(OracleCase)] + [_DP] * 6
        L.dbso_init_flux.restype = C.c_int
        L.dbso_inlet_values.argtypes = [C.POINTER(OracleCase), C.c_int, C.c_double, _DP]
        L.dbso_inlet_values.restype = C.c_int
        L.dbso_step.argtypes = ([C.POINTER(OracleCase)] + [_DP] * 11 +
                                [C.c_int, C.POINTER(OracleInfo), C.POINTER(OracleTrace)])
        L.dbso_step.restype = C.c_int
        L.dbso_alpha_advance.argtypes = ([C.POINTER(OracleCase)] + [_DP] * 7 +
                                         [C.c_int, _DP])
        L.dbso_alpha_advance.restype = C.c_int
        L.dbso_curvature.argtypes = [C.POINTER(OracleCase)] + [_DP] * 6
        L.dbso_curvature.restype = C.c_int
        L.dbso_pressure_apply.argtypes = [C.POINTER(OracleCase), _DP, _DP, _DP]
        L.dbso_pressure_apply.restype = C.c_int
        L.dbso_pressure_solve.argtypes = [C.POINTER(OracleCase), _DP, _DP, _DP,
                                          C.c_double, C.c_int, C.POINTER(C.c_int), _DP]
        L.dbso_pressure_solve.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def make_case(cs) -> OracleCase:
    o = OracleCase()
    o.nx, o.ny, o.nz = cs.shape
    o.hx, o.hy, o.hz = cs.h
    fl = cs.fluids
    o.rho_l, o.rho_g, o.mu_l, o.mu_g = fl["rho_l"], fl["rho_g"], fl["mu_l"], fl["mu_g"]
    for a in range(3):
        o.g[a] = cs.g[a]
    o.c_alpha = cs.c_alpha
    o.kr_model = _MODEL[cs.kr["model"]]
    o.kr_m = cs.kr["m"]
    o.s_lirr = cs.kr.get("s_lirr", 0.0)
    o.s_girr = cs.kr.get("s_girr", 0.0)
    o.pc_model = _MODEL[cs.pc["model"]]
    o.pc0 = cs.pc["pc0"]
    o.pc_exp = cs.pc["exp"]
    o.a_pcirr = cs.pc.get("a_irr", 0.0)
    o.a_pcmax = cs.pc.get("a_max", 1.0)
    o.eps_pc = cs.pc.get("eps", 1e-3)
    for b in range(6):
        bc = cs.bc[b]
        o.bc_kind[b] = _KIND[bc["kind"]]
        for a in range(3):
            o.bc_U[b][a] = bc.get("U", (0.0, 0.0, 0.0))[a]
        o.bc_alpha[b] = bc.get("alpha", 0.0)
        o.bc_p[b] = bc.get("p", 0.0)
        wave = bc.get("wave", (0.0, 0.0, 0.0))
        for q in range(3):
            o.bc_wave[b][q] = wave[q]
    o.t0 = float(getattr(cs, "t0", 0.0))
    o.sigma = float(getattr(cs, "sigma", 0.0))
    o.contact_angle = float(getattr(cs, "contact_angle", 0.0))
    o.target_courant = float(getattr(cs, "target_courant", 0.0))
    o.dt_max = float(getattr(cs, "dt_max", 0.0))
    o.dt = cs.dt
    o.n_corr = cs.n_corr
    o.mom_maxit = int(cs.mom_maxit)
    o.mom_tol = float(cs.mom_tol)
    o.n_alpha_sub = int(getattr(cs, "n_alpha_sub", 1))
    o.transpose_visc = int(cs.transpose_visc)
    o.mules_iter = int(cs.mules_iter)
    o.p_tol = cs.p_tol
    o.p_maxit = cs.p_maxit
    return o


def nfaces(shape):
    nx, ny, nz = shape
    return ((nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1))


def closures(cs, alpha: float):
    o = make_case(cs)
    out = [C.c_double() for _ in range(4)]
    lib().dbso_closures(C.byref(o), float(alpha), *[C.byref(v) for v in out])
    return tuple(v.value for v in out)


def curvature(cs, alpha: np.ndarray, F=None) -> np.ndarray:
    """Interface curvature kappa = -div(grad(alpha)/|grad(alpha)|) per cell
    (CSF, Sec. 2.2), penalized at clear/porous faces when the case imposes a
    contact angle; F (face fluxes) only picks outlet backflow values."""
    o = make_case(cs)
    a = np.ascontiguousarray(alpha, dtype=np.float64).reshape(-1)
    if F is None:
        F = [np.zeros(n) for n in nfaces(cs.shape)]
    F = [np.ascontiguousarray(f, dtype=np.float64) for f in F]
    k = np.zeros(a.size)
    kv = np.ascontiguousarray(cs.kinv, dtype=np.float64).reshape(-1)
    rc = lib().dbso_curvature(C.byref(o), _ptr(a), _ptr(kv), *[_ptr(f) for f in F], _ptr(k))
    if rc:
        raise ValueError(f"dbso_curvature failed ({rc})")
    return k


def init_flux(cs, U: np.ndarray):
    o = make_case(cs)
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(3, -1)
    Us = [np.ascontiguousarray(U[a]) for a in range(3)]
    F = [np.zeros(n) for n in nfaces(cs.shape)]
    rc = lib().dbso_init_flux(C.byref(o), *[_ptr(u) for u in Us], *[_ptr(f) for f in F])
    if rc:
        raise ValueError(f"dbso_init_flux failed ({rc})")
    return tuple(F)


def inlet_values(cs, b: int, t: float) -> np.ndarray:
    """(n_faces, 4) array of the U and alpha that inlet side b prescribes at
    time t, faces in the order of that side's face array."""
    o = make_case(cs)
    nx, ny, nz = cs.shape
    side = (ny * nz, nx * nz, nx * ny)[b // 2]
    out = np.zeros((side, 4))
    n = lib().dbso_inlet_values(C.byref(o), int(b), float(t), _ptr(out))
    if n != side:
        raise ValueError(f"dbso_inlet_values failed ({n})")
    return out


def initial_state(cs) -> dict:
    """State dict from the case's initial fields (F from U when not given)."""
    nc = int(np.prod(cs.shape))
    st = {
        "alpha": np.ascontiguousarray(cs.alpha, dtype=np.float64).reshape(nc).copy(),
        "U": np.ascontiguousarray(cs.U, dtype=np.float64).reshape(3, nc).copy(),
        "p_rgh": np.ascontiguousarray(cs.p_rgh, dtype=np.float64).reshape(nc).copy(),
    }
    if getattr(cs, "F", None) is not None:
        st["F"] = tuple(np.ascontiguousarray(f, dtype=np.float64).copy() for f in cs.F)
    else:
        st["F"] = init_flux(cs, st["U"])
    st["p"] = np.zeros(nc)
    st["t"] = float(getattr(cs, "t0", 0.0))
    return st


def step(cs, state: dict, nsteps: int, trace: bool = False, check: bool = True):
    """Advance a copy of ``state`` by nsteps; returns (state, info[, trace]).
    The state's time ``t`` (default: the case's t0) is where the steps start."""
    o = make_case(cs)
    t0 = float(state.get("t", getattr(cs, "t0", 0.0)))
    o.t0 = t0
    nc = int(np.prod(cs.shape))
    nf = nfaces(cs.shape)
    phi = np.ascontiguousarray(cs.phi, dtype=np.float64).reshape(nc)
    kinv = np.ascontiguousarray(cs.kinv, dtype=np.float64).reshape(nc)
    a = state["alpha"].astype(np.float64).copy()
    U = [state["U"][d].astype(np.float64).copy() for d in range(3)]
    prgh = state["p_rgh"].astype(np.float64).copy()
    p = np.zeros(nc)
    F = [np.asarray(f, dtype=np.float64).copy() for f in state["F"]]
    info = OracleInfo()
    tr = None
    tarr = {}
    if trace:
        tr = OracleTrace()
        sizes = {"A": sum(nf), "Rp": nc, "Rm": nc, "alphaPhi": sum(nf), "alpha_new": nc,
                 "rAU": nc, "Shat": 3 * nc, "Ustar": 3 * nc, "HbyA": 3 * nc,
                 "phiHbyA": sum(nf), "b": nc, "aP": nc, "aON": sum(nf), "aNO": sum(nf),
                 "B": 3 * nc}
        for k, n in sizes.items():
            tarr[k] = np.zeros(n)
            setattr(tr, k, _ptr(tarr[k]))
    rc = lib().dbso_step(C.byref(o), _ptr(phi), _ptr(kinv), _ptr(a), _ptr(U[0]), _ptr(U[1]),
                         _ptr(U[2]), _ptr(prgh), _ptr(p), _ptr(F[0]), _ptr(F[1]), _ptr(F[2]),
                         int(nsteps), C.byref(info), C.byref(tr) if tr is not None else None)
    if check and rc:
        raise RuntimeError(f"dbso_step failed ({rc})")
    out = {"alpha": a, "U": np.stack(U), "p_rgh": prgh, "p": p, "F": tuple(F), "rc": rc,
           "t": info.t_end if nsteps > 0 else t0}
    inf = {
        "p_iters": list(info.p_iters)[: cs.n_corr],
        "p_relres": list(info.p_relres)[: cs.n_corr],
        "alpha_min": info.alpha_min, "alpha_max": info.alpha_max,
        "phase_volume": info.phase_volume, "max_div": info.max_div,
        "dt_last": info.dt_last,
        "mom_sweeps": info.mom_sweeps, "mom_relres": info.mom_relres,
        "p_bnorm": list(info.p_bnorm)[: cs.n_corr],
    }
    if trace:
        return out, inf, tarr
    return out, inf


def alpha_advance(cs, alpha, F, p_rgh=None, nsteps=1, t0=None):
    """Saturation transport alone: nsteps stages of cs.dt (each in
    cs.n_alpha_sub sub-cycles) with F and p_rgh fixed.  Returns (alpha, mean
    limited flux of the last stage as a concatenated x|y|z face array)."""
    o = make_case(cs)
    if t0 is not None:
        o.t0 = float(t0)
    nc = int(np.prod(cs.shape))
    phi = np.ascontiguousarray(cs.phi, dtype=np.float64).reshape(nc)
    kinv = np.ascontiguousarray(cs.kinv, dtype=np.float64).reshape(nc)
    a = np.ascontiguousarray(alpha, dtype=np.float64).reshape(nc).copy()
    F = [np.ascontiguousarray(f, dtype=np.float64) for f in F]
    pr = np.zeros(nc) if p_rgh is None else np.ascontiguousarray(p_rgh, dtype=np.float64).reshape(nc)
    aphi = np.zeros(sum(nfaces(cs.shape)))
    rc = lib().dbso_alpha_advance(C.byref(o), _ptr(phi), _ptr(kinv), _ptr(a), *[_ptr(f) for f in F],
                                  _ptr(pr), int(nsteps), _ptr(aphi))
    if rc:
        raise ValueError(f"dbso_alpha_advance failed ({rc})")
    return a, aphi


def pressure_apply(cs, rAU: np.ndarray, x: np.ndarray) -> np.ndarray:
    o = make_case(cs)
    rAU = np.ascontiguousarray(rAU, dtype=np.float64).ravel()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.zeros_like(x)
    if lib().dbso_pressure_apply(C.byref(o), _ptr(rAU), _ptr(x), _ptr(y)):
        raise ValueError("dbso_pressure_apply failed")
    return y


def pressure_solve(cs, rAU, b, x0=None, tol=1e-14, maxit=100000):
    o = make_case(cs)
    rAU = np.ascontiguousarray(rAU, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).ravel().copy()
    it = C.c_int()
    rr = C.c_double()
    rc = lib().dbso_pressure_solve(C.byref(o), _ptr(rAU), _ptr(b), _ptr(x), float(tol),
                                   int(maxit), C.byref(it), C.byref(rr))
    if rc:
        raise RuntimeError(f"dbso_pressure_solve failed ({rc})")
    return x, it.value, rr.value
