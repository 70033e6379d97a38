"""Small cases that pin the oracle (and later the HIP path) to closed forms
and invariants.  Built only from the seeded generators' vocabulary."""
from __future__ import annotations

import numpy as np

from paper_2003_08374_amd import workloads as W

# Table 1 air viscosity (the benchmark workloads override it to 1.8e-5)
AIR_T1 = {"rho": 1.0, "mu": 1.76e-5}


def column_1d(n, h, axis=0, phi=0.5, kinv=1e11, alpha0=1.0, U_in=1e-4, g=(0.0, 0.0, 0.0),
              fl=None, kr=None, pc=None, dt=1e-3, bc_lo=None, bc_hi=None, name="column"):
    """1D column of n cells along ``axis`` (the two other axes are empty)."""
    shape = [1, 1, 1]
    shape[axis] = n
    shape = tuple(shape)
    hh = [h, h, h]
    nx, ny, nz = shape
    U = np.zeros((3, nz, ny, nx))
    U[axis] = U_in
    bc = [W.empty() for _ in range(6)]
    vin = [0.0, 0.0, 0.0]
    vin[axis] = U_in
    bc[2 * axis] = bc_lo if bc_lo is not None else W.inlet(vin, alpha0)
    bc[2 * axis + 1] = bc_hi if bc_hi is not None else W.outlet(0.0, alpha0)
    c = W.Case(name=name, shape=shape, h=tuple(hh), fluids=fl or W.fluids(W.WATER, AIR_T1),
               g=tuple(g), bc=bc, phi=np.full((nz, ny, nx), phi),
               kinv=np.full((nz, ny, nx), kinv), alpha=np.full((nz, ny, nx), alpha0), U=U,
               p_rgh=np.zeros((nz, ny, nx)), dt=dt, p_tol=1e-14, p_maxit=100000)
    if kr is not None:
        c = c.replace(kr=kr)
    if pc is not None:
        c = c.replace(pc=pc)
    return c


def poiseuille(ny, H=1e-3, nx=4, G=1.0, dt=1e-2, L=None):
    """Solid-free channel between walls y = 0 and y = H, pressure drop G*L
    imposed by two fixed-pressure ends; water everywhere, no gravity."""
    h = H / ny
    L = L if L is not None else nx * h
    hx = L / nx
    shape = (nx, ny, 1)
    bc = [W.outlet(G * L, 1.0), W.outlet(0.0, 1.0), W.wall(), W.wall(), W.empty(), W.empty()]
    return W.Case(name=f"poiseuille_{ny}", shape=shape, h=(hx, h, hx),
                  fluids=W.fluids(W.WATER, W.AIR), g=(0.0, 0.0, 0.0), bc=bc,
                  phi=np.ones((1, ny, nx)), kinv=np.zeros((1, ny, nx)),
                  alpha=np.ones((1, ny, nx)), U=np.zeros((3, 1, ny, nx)),
                  p_rgh=np.zeros((1, ny, nx)), dt=dt, p_tol=1e-14, p_maxit=100000)


def closed_box_2d(nx, ny, h, fl, g=(0.0, -9.81, 0.0), phi=None, kinv=None, alpha=None,
                  dt=1e-4, name="closed_box"):
    bc = [W.wall(), W.wall(), W.wall(), W.wall(), W.empty(), W.empty()]
    shp = (1, ny, nx)
    return W.Case(name=name, shape=(nx, ny, 1), h=(h, h, h), fluids=fl, g=tuple(g), bc=bc,
                  phi=np.ones(shp) if phi is None else phi,
                  kinv=np.zeros(shp) if kinv is None else kinv,
                  alpha=np.zeros(shp) if alpha is None else alpha,
                  U=np.zeros((3,) + shp), p_rgh=np.zeros(shp), dt=dt, p_tol=1e-14,
                  p_maxit=100000)


def random_3d(shape=(6, 5, 4), seed=0, h=1e-4, dt=2e-5, g=(0.0, -9.81, 0.0), U_in=5e-3):
    """Small heterogeneous 3D case: random porous/clear cells, random alpha."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    shp = (nz, ny, nx)
    porous = rng.random(shp) < 0.6
    phi = np.where(porous, rng.uniform(0.2, 0.5, shp), 1.0)
    kinv = np.where(porous, 10.0 ** rng.uniform(9, 11, shp), 0.0)
    alpha = np.clip(rng.uniform(-0.3, 1.3, shp), 0.0, 1.0)
    U = rng.uniform(-1e-3, 1e-3, (3,) + shp)
    bc = [W.inlet((U_in, 0.0, 0.0), 1.0), W.outlet(0.0, 0.0), W.wall(), W.wall(), W.wall(),
          W.wall()]
    return W.Case(name=f"random3d_{seed}", shape=shape, h=(h, h, h),
                  fluids=W.fluids(W.WATER, W.OIL), g=tuple(g), bc=bc, phi=phi, kinv=kinv,
                  alpha=alpha, U=U, p_rgh=rng.uniform(-1, 1, shp), dt=dt, p_tol=1e-14,
                  p_maxit=100000,
                  kr={"model": "van_genuchten", "m": 0.5},
                  pc={"model": "brooks_corey", "pc0": 100.0, "exp": 0.5})
