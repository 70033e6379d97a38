"""Seeded synthetic workloads shaped after the paper's cases.

This module only builds inputs: meshes, fluid and model constants, boundary
conditions and seeded porosity / permeability / initial fields.  It holds
none of the method's arithmetic and imports neither the HIP binding nor the
oracle, so both sides can take their inputs from it.

Fluid properties follow the paper's Table 1 (water, air, oil) with the
viscosity overrides of the benchmark workloads (air 1.8e-5 Pa s, oil
5e-3 Pa s); model constants follow Table 2 unless a workload fixes others.
The paper's own case geometries exist only as figures, so the 3D fractured
media below are synthetic stand-ins for its fractured-matrix application
(Sec. 5.2): log-normal permeability with an 8-cell correlation length,
uniform porosity, and planar solid-free fractures.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

WATER = {"rho": 1000.0, "mu": 1e-3}
AIR = {"rho": 1.0, "mu": 1.8e-5}
OIL = {"rho": 800.0, "mu": 5e-3}
GRAVITY = 9.81


def fluids(l, g):
    return {"rho_l": l["rho"], "mu_l": l["mu"], "rho_g": g["rho"], "mu_g": g["mu"]}


def wall():
    return {"kind": "wall"}


def empty():
    return {"kind": "empty"}


def inlet(U, alpha):
    return {"kind": "inlet", "U": tuple(float(u) for u in U), "alpha": float(alpha)}


def outlet(p=0.0, backflow_alpha=0.0):
    return {"kind": "outlet", "p": float(p), "alpha": float(backflow_alpha)}


def wave(amplitude, period, depth):
    """Linear-wave inlet (x faces): surface depth + A sin(2 pi t / T)."""
    return {"kind": "wave", "wave": (float(amplitude), float(period), float(depth))}


@dataclass
class Case:
    """One single-domain problem: mesh, physics, boundaries, controls, fields.

    Arrays are float64 with shape (nz, ny, nx) (x fastest in memory); U has
    shape (3, nz, ny, nx).  ``bc`` lists the six domain faces in the order
    x-, x+, y-, y+, z-, z+.
    """
    name: str
    shape: tuple
    h: tuple
    fluids: dict
    g: tuple
    bc: list
    phi: np.ndarray
    kinv: np.ndarray
    alpha: np.ndarray
    U: np.ndarray
    p_rgh: np.ndarray
    F: tuple | None = None
    c_alpha: float = 1.0
    kr: dict = field(default_factory=lambda: {"model": "brooks_corey", "m": 2.0})
    pc: dict = field(default_factory=lambda: {"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})
    dt: float = 1e-5
    n_corr: int = 2
    mom_maxit: int = 100        # sweep cap of the momentum predictor solve
    mom_tol: float = 1e-14      # predictor: ||B + N U - D U|| <= mom_tol ||B||
    n_alpha_sub: int = 1        # saturation sub-cycles per step
    transpose_visc: bool = True
    mules_iter: int = 3
    p_tol: float = 1e-13
    p_maxit: int = 2000
    precision: str = "fp64"
    steps: int = 1
    t0: float = 0.0
    sigma: float = 0.0
    contact_angle: float = 0.0  # radians, at clear/porous faces; 0 = not imposed
    target_courant: float = 0.0  # > 0: CFL-adaptive time step (dt is the first)
    dt_max: float = 0.0          # cap of the adaptive time step

    @property
    def ncells(self) -> int:
        return int(np.prod(self.shape))

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


def _zeros(shape):
    nx, ny, nz = shape
    return np.zeros((nz, ny, nx))


def _blank_state(shape):
    nx, ny, nz = shape
    return _zeros(shape), np.zeros((3, nz, ny, nx)), _zeros(shape)


# --------------------------------------------------------------- 2D layered


def layered_2d(n=64, h=1e-3, dt=1e-5, U_in=1e-3, steps=20, name="layered_2d_64"):
    """2D n x n, lower half porous (phi 0.5, k 1e-12 m^2), upper half clear.

    Water (wetting) enters over the full height of the left side into air;
    fixed-pressure outlet on the right, walls top and bottom, gravity -y.
    Brooks-Corey k_r (m = 2) and p_c (entry 1e3 Pa, beta 0.5).
    """
    shape = (n, n, 1)
    phi = np.ones((1, n, n))
    kinv = np.zeros((1, n, n))
    phi[:, : n // 2, :] = 0.5
    kinv[:, : n // 2, :] = 1e12
    alpha, U, prgh = _blank_state(shape)
    bc = [inlet((U_in, 0, 0), 1.0), outlet(0.0, 0.0), wall(), wall(), empty(), empty()]
    return Case(name=name, shape=shape, h=(h, h, h), fluids=fluids(WATER, AIR),
                g=(0.0, -GRAVITY, 0.0), bc=bc, phi=phi, kinv=kinv, alpha=alpha, U=U,
                p_rgh=prgh, dt=dt, steps=steps,
                kr={"model": "brooks_corey", "m": 2.0},
                pc={"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})


def layered_2d_stress(n=64):
    """Limiter-stress variant: 100x the inlet speed and dt (Courant ~0.1-0.2)."""
    return layered_2d(n=n, dt=1e-3, U_in=0.1, name=f"layered_2d_{n}_stress")


# ------------------------------------------------------ 3D fractured matrix


def gaussian_field(shape, seed, corr_cells=8.0):
    """White noise N(0,1) smoothed by a periodic Gaussian kernel of standard
    deviation corr_cells (FFT), then standardised to mean 0 and std 1."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.fftfreq(nx)[None, None, :]
    s = corr_cells
    filt = np.exp(-2.0 * (np.pi * s) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    f = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    sd = f.std()
    return (f - f.mean()) / (sd if sd > 0 else 1.0)


def porous_matrix(shape, seed_k, seed_phi, log10k_mean=-13.0, log10k_sigma=0.5,
                  phi_range=(0.2, 0.4), corr_cells=8.0):
    g = gaussian_field(shape, seed_k, corr_cells)
    k = 10.0 ** (log10k_mean + log10k_sigma * g)
    rng = np.random.default_rng(seed_phi)
    nx, ny, nz = shape
    phi = rng.uniform(phi_range[0], phi_range[1], size=(nz, ny, nx))
    return phi, 1.0 / k


def _cell_centres(shape, h):
    nx, ny, nz = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h[2], (np.arange(ny) + 0.5) * h[1],
                          (np.arange(nx) + 0.5) * h[0], indexing="ij")
    return x, y, z


def slab_fracture_mask(shape, h, half_width_cells=4):
    """Solid-free slab |y - L_y/2| < half_width, spanning x and z."""
    x, y, z = _cell_centres(shape, h)
    Ly = shape[1] * h[1]
    return np.abs(y - 0.5 * Ly) < half_width_cells * h[1]


def random_plane_fractures(shape, h, n_frac, seed, half_width_cells=4):
    """n_frac planes: normals uniform on the sphere, centres uniform in the
    middle half of the box; cells within half_width of a plane are clear."""
    rng = np.random.default_rng(seed)
    x, y, z = _cell_centres(shape, h)
    L = np.array([shape[0] * h[0], shape[1] * h[1], shape[2] * h[2]])
    mask = np.zeros(x.shape, dtype=bool)
    for _ in range(n_frac):
        nrm = rng.standard_normal(3)
        nrm /= np.linalg.norm(nrm)
        c = rng.uniform(0.25, 0.75, size=3) * L
        d = nrm[0] * (x - c[0]) + nrm[1] * (y - c[1]) + nrm[2] * (z - c[2])
        mask |= np.abs(d) < half_width_cells * h[0]
    return mask


def fractured_3d(n=128, h=1e-4, dt=1e-5, seed_k=1, seed_phi=2, fractures="slab",
                 frac_seed=5, n_frac=3, steps=100, U_in=1e-3, name=None, shape=None):
    """3D fractured microporous matrix: water displacing oil.

    log10 k = -13 + 0.5 g (g: 8-cell-correlated Gaussian field), phi ~ U[0.2,0.4];
    fractures (phi = 1, k^-1 = 0) 8 cells wide: one slab normal to y, or
    ``n_frac`` random planes.  Inlet on x- (U_in, alpha = 1), outlet on x+,
    walls elsewhere, gravity -y; constitutive models as the 2D layered case.
    """
    shape = tuple(shape) if shape is not None else (n, n, n)
    hh = (h, h, h)
    phi, kinv = porous_matrix(shape, seed_k, seed_phi)
    if fractures == "slab":
        m = slab_fracture_mask(shape, hh)
    elif fractures == "planes":
        m = random_plane_fractures(shape, hh, n_frac, frac_seed)
    else:
        m = np.zeros(phi.shape, dtype=bool)
    phi[m] = 1.0
    kinv[m] = 0.0
    alpha, U, prgh = _blank_state(shape)
    bc = [inlet((U_in, 0, 0), 1.0), outlet(0.0, 0.0), wall(), wall(), wall(), wall()]
    nm = name or f"fractured_3d_{shape[0]}x{shape[1]}x{shape[2]}_{fractures}"
    return Case(name=nm, shape=shape, h=hh, fluids=fluids(WATER, OIL),
                g=(0.0, -GRAVITY, 0.0), bc=bc, phi=phi, kinv=kinv, alpha=alpha, U=U,
                p_rgh=prgh, dt=dt, steps=steps,
                kr={"model": "brooks_corey", "m": 2.0},
                pc={"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})


# ------------------------------------------- Darcy-scale heterogeneous reservoir


def reservoir_2d(nx=2000, ny=800, size=(1.0, 0.4), blocks=(4, 4), seed=8, U_in=1e-4,
                 phi=0.5, dt=0.5, steps=10, name=None):
    """2D heterogeneous oil reservoir flooded with water (shaped after the
    paper's Darcy-scale drainage case, Sec. 4.1.4): 1 m x 0.4 m, a grid of
    blocks x blocks of 0.25 m x 0.1 m with k0 ~ U[1e-13, 4e-13] m^2 per block
    (seeded), phi = 0.5 (not given in the paper), Van Genuchten k_r (m = 0.5)
    and no capillary pressure, inlet U_in at x-, fixed p = 0 at x+, walls
    top and bottom, no gravity (a horizontal section)."""
    shape = (nx, ny, 1)
    h = (size[0] / nx, size[1] / ny, size[0] / nx)
    rng = np.random.default_rng(seed)
    k_block = rng.uniform(1e-13, 4e-13, size=(blocks[1], blocks[0]))
    x, y, _ = _cell_centres(shape, h)
    bi = np.minimum((x / (size[0] / blocks[0])).astype(int), blocks[0] - 1)
    bj = np.minimum((y / (size[1] / blocks[1])).astype(int), blocks[1] - 1)
    kinv = 1.0 / k_block[bj, bi]
    alpha, U, prgh = _blank_state(shape)
    bc = [inlet((U_in, 0, 0), 1.0), outlet(0.0, 0.0), wall(), wall(), empty(), empty()]
    return Case(name=name or f"reservoir_2d_{nx}x{ny}", shape=shape, h=h,
                fluids=fluids(WATER, OIL), g=(0.0, 0.0, 0.0), bc=bc,
                phi=np.full((1, ny, nx), phi), kinv=kinv, alpha=alpha, U=U, p_rgh=prgh,
                dt=dt, steps=steps, kr={"model": "van_genuchten", "m": 0.5},
                pc={"model": "van_genuchten", "pc0": 0.0, "exp": 0.5})


# ------------------------------------------------------------ clear-fluid drop


def droplet(shape=(64, 64, 1), h=1e-4, radius_cells=16.0, width_cells=1.0, centre=None,
            sigma=0.07, dt=1e-5, porous_rows=0, gravity=False, steps=5, name=None,
            contact_angle=0.0):
    """A water drop in air inside a closed box (walls; z empty when nz = 1).

    alpha = (1 - tanh((r - R) / w)) / 2 around ``centre`` (cell units, the
    box centre by default), R = radius_cells h, w = width_cells h;
    sigma = 0.07 N/m (water-air).  ``porous_rows`` > 0 puts a porous floor
    of that many cell rows (phi 0.5, k 1e-12 m^2, Brooks-Corey models as the
    2D layered case) under the drop; gravity -y when ``gravity``;
    ``contact_angle`` (radians, 0 = none) is imposed on the floor.
    """
    shape = tuple(shape)
    nx, ny, nz = shape
    hh = (h, h, h)
    x, y, z = _cell_centres(shape, hh)
    c = centre if centre is not None else (nx / 2, ny / 2, nz / 2)
    r2 = (x - c[0] * h) ** 2 + (y - c[1] * h) ** 2
    if nz > 1:
        r2 = r2 + (z - c[2] * h) ** 2
    alpha = 0.5 * (1.0 - np.tanh((np.sqrt(r2) - radius_cells * h) / (width_cells * h)))
    phi = np.ones((nz, ny, nx))
    kinv = np.zeros((nz, ny, nx))
    if porous_rows > 0:
        phi[:, :porous_rows, :] = 0.5
        kinv[:, :porous_rows, :] = 1e12
    U = np.zeros((3, nz, ny, nx))
    prgh = _zeros(shape)
    zb = [empty(), empty()] if nz == 1 else [wall(), wall()]
    bc = [wall(), wall(), wall(), wall()] + zb
    nm = name or f"droplet_{nx}x{ny}x{nz}"
    return Case(name=nm, shape=shape, h=hh, fluids=fluids(WATER, AIR),
                g=(0.0, -GRAVITY if gravity else 0.0, 0.0), bc=bc, phi=phi, kinv=kinv,
                alpha=alpha, U=U, p_rgh=prgh, dt=dt, steps=steps, sigma=sigma,
                contact_angle=contact_angle,
                kr={"model": "brooks_corey", "m": 2.0},
                pc={"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})


def capillary_rise(n_tube=40, ny=400, width=1e-3, height=20e-3, wall_cells=2,
                   theta_deg=45.0, h0=8e-3, sigma=0.07, dt=2e-6, steps=30000, wall_alpha=None,
                   name=None):
    """Water rising in an air-filled 2D tube (the pore-scale capillary rise
    of Sec. 4.2): a ``width`` x ``height`` slit of n_tube x ny clear cells
    between porous walls of ``wall_cells`` columns each (k^-1 = 1e20 m^-2,
    phi 0.5: impermeable), contact angle ``theta_deg`` on the clear/porous
    faces, gravity -y.  The bottom face is a water reservoir (fixed p_rgh =
    0, inflow carries alpha = 1), the top face is open to the air (fixed
    p_rgh = 0, inflow carries alpha = 0).  The meniscus starts flat at
    ``h0`` (a tanh profile one cell wide) in the tube and, unless
    ``wall_alpha`` gives their saturation, in the walls (whose saturation
    cannot change).  The
    Jurin height 2 sigma cos(theta) / (rho_l g width) is 10.1 mm for the
    defaults."""
    nx = n_tube + 2 * wall_cells
    hh = (width / n_tube, height / ny, width / n_tube)
    shape = (nx, ny, 1)
    x, y, z = _cell_centres(shape, hh)
    alpha = 0.5 * (1.0 - np.tanh((y - h0) / hh[1]))
    phi = np.ones((1, ny, nx))
    kinv = np.zeros((1, ny, nx))
    phi[:, :, :wall_cells] = phi[:, :, nx - wall_cells:] = 0.5
    kinv[:, :, :wall_cells] = kinv[:, :, nx - wall_cells:] = 1e20
    if wall_alpha is not None:
        alpha[:, :, :wall_cells] = alpha[:, :, nx - wall_cells:] = wall_alpha
    U = np.zeros((3, 1, ny, nx))
    bc = [wall(), wall(), outlet(0.0, 1.0), outlet(0.0, 0.0), empty(), empty()]
    nm = name or f"capillary_rise_{n_tube}x{ny}"
    return Case(name=nm, shape=shape, h=hh, fluids=fluids(WATER, AIR),
                g=(0.0, -GRAVITY, 0.0), bc=bc, phi=phi, kinv=kinv, alpha=alpha, U=U,
                p_rgh=_zeros(shape), dt=dt, steps=steps, sigma=sigma,
                contact_angle=float(np.deg2rad(theta_deg)),
                kr={"model": "brooks_corey", "m": 2.0},
                pc={"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})


ETHANOL = {"rho": 789.0, "mu": 1.2e-3}


def taylor_film(nx=280, ny=116, length=800e-6, width=100e-6, wall_cells=2, U_in=0.4,
                sigma=0.022, theta_deg=20.0, dt=2e-8, steps=30000, name=None):
    """Air driving ethanol out of a 2D micro-channel (the Taylor-film case of
    Sec. 4.2): a ``length`` x ``width`` channel of nx x ny clear cells
    between impermeable porous walls of ``wall_cells`` rows (k^-1 =
    1e20 m^-2, phi 0.5, saturated with ethanol), contact angle
    ``theta_deg``, no gravity.  Air enters at x- with U_in (inlet alpha =
    0), the outlet at x+ holds p = 0 (ethanol on backflow); the channel is
    full of ethanol moving at U_in except an air plug over the first tenth
    (a one-cell tanh).  sigma = 0.022 N/m (ethanol-air, not given in the
    paper).  The film left on the walls is R 1.34 Ca^(2/3) / (1 + 3.35
    Ca^(2/3)) with R the half-width and Ca = mu U / sigma: 4.15 um here."""
    nyt = ny + 2 * wall_cells
    hh = (length / nx, width / ny, length / nx)
    shape = (nx, nyt, 1)
    x, y, z = _cell_centres(shape, hh)
    alpha = 0.5 * (1.0 + np.tanh((x - 0.1 * length) / hh[0]))
    phi = np.ones((1, nyt, nx))
    kinv = np.zeros((1, nyt, nx))
    phi[:, :wall_cells, :] = phi[:, nyt - wall_cells:, :] = 0.5
    kinv[:, :wall_cells, :] = kinv[:, nyt - wall_cells:, :] = 1e20
    alpha[:, :wall_cells, :] = alpha[:, nyt - wall_cells:, :] = 1.0
    U = np.zeros((3, 1, nyt, nx))
    U[0, :, wall_cells:nyt - wall_cells, :] = U_in
    bc = [inlet((U_in, 0.0, 0.0), 0.0), outlet(0.0, 1.0), wall(), wall(), empty(), empty()]
    nm = name or f"taylor_film_{nx}x{ny}"
    return Case(name=nm, shape=shape, h=hh, fluids=fluids(ETHANOL, AIR), g=(0.0, 0.0, 0.0),
                bc=bc, phi=phi, kinv=kinv, alpha=alpha, U=U, p_rgh=_zeros(shape), dt=dt,
                steps=steps, sigma=sigma, contact_angle=float(np.deg2rad(theta_deg)),
                kr={"model": "brooks_corey", "m": 2.0},
                pc={"model": "brooks_corey", "pc0": 1e3, "exp": 0.5})


def fractured_128():
    """128^3, one slab fracture, k seed 1, phi seed 2, 100 steps."""
    return fractured_3d(n=128, seed_k=1, seed_phi=2, fractures="slab", steps=100,
                        name="fractured_3d_128_slab")


def fractured_256(precision="mixed", p_tol=1e-8):
    """256^3, three random planar fractures (seed 5), k seed 3, phi seed 4."""
    c = fractured_3d(n=256, seed_k=3, seed_phi=4, fractures="planes", frac_seed=5,
                     n_frac=3, steps=12, name="fractured_3d_256_planes")
    return c.replace(precision=precision, p_tol=p_tol)


def batch_sizes(n_samples=512, seed=6, lo=32, hi=96):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n_samples)


def batch_cases(n_samples=512, seed=6, lo=32, hi=96, precision="fp64", p_tol=1e-13):
    """Independent cubic porous samples of edge U{lo..hi}; sample s has k seed
    1000+s and phi seed 2000+s, no fracture."""
    out = []
    for s, n in enumerate(batch_sizes(n_samples, seed, lo, hi)):
        c = fractured_3d(n=int(n), seed_k=1000 + s, seed_phi=2000 + s, fractures=None,
                         steps=12, name=f"sample_{s}_{n}")
        out.append(c.replace(precision=precision, p_tol=p_tol))
    return out


# ---------------------------------------------------------- 2D wave flume


def wave_flume(nx=2048, ny=512, h=5e-3, dt=1e-3, amplitude=0.05, period=1.5, depth=0.3,
               x_barrier=7.0, crest_height=0.4, crest_width=0.4, slope=2.0, steps=2000,
               name=None):
    """2D wave flume after the paper's coastal-barrier application (Sec. 4.2):
    still water of the given depth over the whole length (barrier pores
    included), a trapezoidal porous barrier (porosity 0.5, k = 1e-8 m^2,
    Van Genuchten k_r and p_c with m = 0.8, p_c0 = 1e3 Pa) centred at
    x_barrier with the given crest height and width and side slopes of
    slope:1 (horizontal:vertical), a linear-wave inlet at x-, a wall at x+
    and at the bottom, and an open top (p = 0, air on backflow).  Water
    under air.  The paper's geometry exists only as a figure; these sizes
    are a stand-in (full size: 10.24 m x 2.56 m, 5 mm cells)."""
    shape = (nx, ny, 1)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)  # (ny, nx)
    half = 0.5 * crest_width + slope * (crest_height - Y)
    barrier = (Y < crest_height) & (np.abs(X - x_barrier) < half)
    phi = np.where(barrier, 0.5, 1.0)[None]
    kinv = np.where(barrier, 1e8, 0.0)[None]
    alpha = np.where(Y < depth, 1.0, 0.0)[None]
    _, U, prgh = _blank_state(shape)
    bc = [wave(amplitude, period, depth), wall(), wall(), outlet(0.0, 0.0), empty(), empty()]
    nm = name or f"wave_flume_{nx}x{ny}_A{amplitude:.4f}"
    return Case(name=nm, shape=shape, h=(h, h, h), fluids=fluids(WATER, AIR),
                g=(0.0, -GRAVITY, 0.0), bc=bc, phi=phi, kinv=kinv, alpha=alpha, U=U,
                p_rgh=prgh, dt=dt, steps=steps,
                kr={"model": "van_genuchten", "m": 0.8},
                pc={"model": "van_genuchten", "pc0": 1e3, "exp": 0.8})


def flume_amplitudes(n=16, seed=7, a0=0.05):
    """Wave amplitudes a0 (0.75 + 0.5 u), u ~ U[0, 1) seeded."""
    rng = np.random.default_rng(seed)
    return a0 * (0.75 + 0.5 * rng.uniform(0.0, 1.0, size=n))


def flume_batch(n=16, seed=7, precision="mixed", p_tol=1e-8, **kw):
    """The flume with n seeded wave amplitudes (one sample each)."""
    return [wave_flume(amplitude=float(a), **kw).replace(precision=precision, p_tol=p_tol)
            for a in flume_amplitudes(n, seed)]
