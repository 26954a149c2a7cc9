"""Seeded synthetic problem definitions (inputs only, no method arithmetic).

Both the GPU library and the CPU oracle take these as inputs.  The shapes,
sizes and value distributions follow the paper's workloads (Sec. 3):
log-spaced frequency groups (Sec. 3, group set-up), opacities of the form
kappa * nu^-3 (Eq. sigmaMarsharkMF without the temperature factor), cold
initial state with a Planckian incident boundary (Sec. 3.1), sharp opacity
jumps (Sec. 3.2, 3.3), and a 2-D block-structured medium with a central
source (Sec. 3.5, whose block layout is not printed, so a checkerboard
lattice stands in for it).  Nothing here comes from the paper's figures.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

BC_VACUUM, BC_PLANCK, BC_REFLECT = 0, 1, 2
FLAG_GROUP_SIGMA = 1
FLAG_SI_LINEARIZED = 8
FLAG_SLOPES = 16
FLAG_WAVE_ITER = 32
FLAG_BOUNDARY_PARTICLES = 64


@dataclass
class Problem:
    name: str
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc: List[int]            # XLO, XHI, YLO, YHI
    bcT: List[float]
    nu_edges: np.ndarray     # G+1 ascending
    kappa: np.ndarray        # [ncell, G]
    cv: np.ndarray           # [ncell]
    T0: np.ndarray           # [ncell]
    Tr0: np.ndarray          # [ncell]
    pinned: np.ndarray       # [ncell] uint8
    dt: float
    steps: int
    w_ref: float
    nu_power: float = 3.0
    c: float = 1.0
    a: float = 1.0
    eps: float = 1.0
    n_cap: int = 1 << 20
    seed: int = 0
    pool_cap: int = 1 << 20
    si_max_iters: int = 200
    si_tol: float = 1e-13
    flags: int = 0
    tau_num_C: float = 0.0       # > 0: numerical collision time in thin-thick-joint cells
    tau_num_jump: float = 10.0   # opacity ratio across a face that makes its cells joint
    T_power: float = 0.0         # sigma(nu, T) = kappa nu^-p T^-T_power
    opacity_stim: int = 0        # 1: sigma also carries (1 - e^{-nu/T})
    olson_H: Optional[np.ndarray] = None    # [ncell]: H > 0 gives a T^3 H [1 + alpha + (T + chi) alpha']
    olson_chi: Optional[np.ndarray] = None  # [ncell]
    source: Optional[np.ndarray] = None     # [ncell, G] volumetric source rate (rho units per unit time)
    source_shape: Optional[np.ndarray] = None   # [ncell] f(x): a Planckian source (c/eps^2) f(x) phi_g(source_T)
    source_T: float = 0.0
    source_t_off: float = float("inf")      # the source acts in steps starting before this time
    opacity_table: Optional[dict] = None    # {"mat": [ncell], "nu": [nnu], "T": [nT], "sigma": [nmat, nT, nnu]}

    @property
    def G(self) -> int:
        return len(self.nu_edges) - 1

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def log_edges(numin: float, numax: float, G: int) -> np.ndarray:
    """Log-spaced group edges numin * (numax/numin)^(j/G), j = 0..G."""
    j = np.arange(G + 1, dtype=np.float64)
    e = numin * (numax / numin) ** (j / G)
    e[0], e[-1] = numin, numax
    return e


def slab(nx: int, G: int, kappa_of_x, *, dt: float, steps: int, w_ref: float,
         numin: float = 0.01, numax: float = 10.0, T0: float = 1e-3, Tb: float = 1.0,
         bc_right: int = BC_VACUUM, pool_cap: int = 1 << 20, seed: int = 0,
         name: str = "slab", **kw) -> Problem:
    """1-D slab on [0,1]: Planckian incident left boundary at Tb, cold interior."""
    xc = (np.arange(nx) + 0.5) / nx
    kap = np.asarray(kappa_of_x(xc), dtype=np.float64)
    kappa = np.repeat(kap[:, None], G, axis=1).copy()
    return Problem(name=name, dim=1, nx=nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                   bc=[BC_PLANCK, bc_right, BC_VACUUM, BC_VACUUM], bcT=[Tb, 0.0, 0.0, 0.0],
                   nu_edges=log_edges(numin, numax, G), kappa=kappa,
                   cv=np.ones(nx), T0=np.full(nx, T0), Tr0=np.full(nx, T0),
                   pinned=np.zeros(nx, np.uint8), dt=dt, steps=steps, w_ref=w_ref,
                   pool_cap=pool_cap, seed=seed, **kw)


def c1_marshak_like(**kw) -> Problem:
    """100 cells x 10 groups, kappa = 1 (sigma = nu^-3), dt = 1e-3, 100 steps."""
    p = dict(dt=1e-3, steps=100, w_ref=2e-5, pool_cap=1 << 19, name="slab100_g10")
    p.update(kw)
    return slab(100, 10, lambda x: np.ones_like(x), **p)


def c2_two_material(nx: int = 2000, G: int = 64, **kw) -> Problem:
    """Two-material slab: kappa = 0.01 for x < 0.5, 1000 for x >= 0.5 (cell-centre rule)."""
    p = dict(dt=1e-4, steps=1000, w_ref=4e-6, pool_cap=1 << 25, name=f"slab{nx}_g{G}_jump")
    p.update(kw)
    return slab(nx, G, lambda x: np.where(x < 0.5, 0.01, 1000.0), **p)


def marshak(nx: int = 1000, G: int = 24, sigma0: float = 10.0, **kw) -> Problem:
    """Homogeneous Marshak wave stand-in (Sec. 3.1): [0, 5], sigma = sigma0 /
    (nu^3 sqrt(T)), C_v = 0.1, 24 log groups on [0.01, 100], Planckian wall at
    T = 1, reflective right wall, T0 = Tr0 = 1e-3, dt = dx / c."""
    p = dict(dt=5.0 / nx, steps=400, w_ref=1e-5, pool_cap=1 << 24, name=f"marshak{nx}_g{G}_s{sigma0:g}",
             numin=0.01, numax=100.0, bc_right=BC_REFLECT, T_power=0.5)
    p.update(kw)
    q = slab(nx, G, lambda x: np.full_like(x, sigma0), **p)
    return q.with_(x1=5.0, cv=np.full(nx, 0.1))


def larsen(nx: int = 200, G: int = 24, linearized: bool = False, **kw) -> Problem:
    """Larsen's three-region slab (Sec. 3.3) on [0, 4]: sigma = gamma0 (1 - e^{-nu/T})
    / nu^3 with gamma0 = 1 on [0, 2], 1000 on (2, 3] and 1 on (3, 4] (cell-centre
    rule), T0 = 1e-3, Planckian wall at T = 1 on the left and a free right
    boundary, 24 log groups on [0.01, 100], the numerical collision time of joint
    cells with C = 1e3.  The paper's units (cm, ns, keV, c = 29.98, a = 0.01372)
    are scaled to c = a = 1: time is measured as c t (so dt = dx / c = dx), the
    radiation density in units of a c, and the heat capacity becomes
    C_v / a = 0.05109 / 0.01372.  linearized: the linearized source iteration
    (same fixed point) instead of the literal one."""
    p = dict(dt=4.0 / nx, steps=400, w_ref=1e-5, pool_cap=1 << 24, name=f"larsen{nx}_g{G}",
             numin=0.01, numax=100.0, opacity_stim=1, tau_num_C=1e3, tau_num_jump=10.0,
             flags=FLAG_SI_LINEARIZED if linearized else 0)
    p.update(kw)
    q = slab(nx, G, lambda x: np.where((x > 0.5) & (x <= 0.75), 1000.0, 1.0), **p)
    return q.with_(x1=4.0, cv=np.full(nx, 0.05109 / 0.01372))


def thick_thin_joint(nx: int = 300, G: int = 24, **kw) -> Problem:
    """Thick-to-thin slab on [0, 1.5] with the numerical collision time of the
    joint cells on (Sec. 3.2, second case): kappa = 1000 for x <= 0.5 and 10
    beyond (cell-centre rule; the paper's 1/sqrt(T) factor dropped), 24 log
    groups on [0.01, 100], dt = dx / c, C = 1e5, reflective right wall."""
    p = dict(dt=1.5 / nx, steps=600, w_ref=4e-6, pool_cap=1 << 24, name=f"thick_thin{nx}_g{G}",
             numin=0.01, numax=100.0, bc_right=BC_REFLECT, tau_num_C=1e5, tau_num_jump=10.0)
    p.update(kw)
    q = slab(nx, G, lambda x: np.where(x <= 0.5 / 1.5, 1000.0, 10.0), **p)
    return q.with_(x1=1.5)


def c3_lattice(n: int = 256, G: int = 32, **kw) -> Problem:
    """2-D lattice on [0,7]^2: unit squares (a,b), absorber kappa=100 iff a+b odd,
    background kappa=1; cells with centres in [3,4]^2 pinned at T = 1; vacuum walls."""
    L = 7.0
    xc = (np.arange(n) + 0.5) * (L / n)
    X, Y = np.meshgrid(xc, xc, indexing="xy")     # [iy][ix]
    a = np.floor(X).astype(int)
    b = np.floor(Y).astype(int)
    kap = np.where((a + b) % 2 == 1, 100.0, 1.0).reshape(-1)
    src = ((X >= 3.0) & (X <= 4.0) & (Y >= 3.0) & (Y <= 4.0)).reshape(-1)
    ncell = n * n
    T0 = np.full(ncell, 1e-3)
    T0[src] = 1.0
    p = dict(dt=1e-3, steps=500, w_ref=1e-6, pool_cap=1 << 27, seed=0)
    p.update(kw)
    return Problem(name=f"lattice{n}x{n}_g{G}", dim=2, nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L,
                   bc=[BC_VACUUM] * 4, bcT=[0.0] * 4, nu_edges=log_edges(0.01, 10.0, G),
                   kappa=np.repeat(kap[:, None], G, axis=1).copy(), cv=np.ones(ncell), T0=T0,
                   Tr0=np.full(ncell, 1e-3), pinned=src.astype(np.uint8), **p)


def c5_lognormal(n: int = 128, G: int = 16, **kw) -> Problem:
    """2-D [0,1]^2, per-cell kappa = exp(1.5 Z), Z ~ N(0,1) (numpy default_rng(7)),
    Planckian left wall at T = 1, other walls vacuum."""
    rng = np.random.default_rng(7)
    Z = rng.standard_normal(n * n)
    kap = np.exp(1.5 * Z)
    ncell = n * n
    p = dict(dt=1e-3, steps=100, w_ref=1e-4, pool_cap=1 << 24, seed=0)
    p.update(kw)
    return Problem(name=f"lognormal{n}x{n}_g{G}", dim=2, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                   bc=[BC_PLANCK, BC_VACUUM, BC_VACUUM, BC_VACUUM], bcT=[1.0, 0.0, 0.0, 0.0],
                   nu_edges=log_edges(0.01, 10.0, G),
                   kappa=np.repeat(kap[:, None], G, axis=1).copy(), cv=np.ones(ncell),
                   T0=np.full(ncell, 1e-3), Tr0=np.full(ncell, 1e-3),
                   pinned=np.zeros(ncell, np.uint8), **p)


def c4_batch(n_inst: int = 512, nx_range=(64, 4096), groups=(16, 32, 64), steps: int = 200,
             dt: float = 1e-4, w_ref: float = 5e-4, key: int = 1) -> List[Problem]:
    """Independent 1-D slabs with uneven sizes: nx ~ U{64..4096}, G in {16,32,64},
    kappa_L, kappa_R ~ logU[1e-2, 1e3], jump position ~ U(0,1); instance seeds 0..n-1.
    Instance parameters come from numpy's Philox bit generator with the given key."""
    rng = np.random.Generator(np.random.Philox(key=key))
    out = []
    for k in range(n_inst):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        G = int(rng.choice(np.asarray(groups)))
        kl, kr = 10.0 ** rng.uniform(-2.0, 3.0, size=2)
        xj = float(rng.uniform(0.0, 1.0))
        pr = slab(nx, G, lambda x, kl=kl, kr=kr, xj=xj: np.where(x < xj, kl, kr),
                  dt=dt, steps=steps, w_ref=w_ref, seed=k, pool_cap=1 << 17,
                  name=f"inst{k}_nx{nx}_g{G}")
        out.append(pr)
    return out


def foam_kappa(nu: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Mass opacity (cm^2/g) of the carbon-hydrogen foam of Sec. 3.4 at photon
    energies nu and temperatures T (both keV), as printed: kappa[..., T, nu]."""
    n, t = np.meshgrid(np.asarray(nu, float), np.asarray(T, float), indexing="xy")
    k = np.minimum(1e7, 1e9 * t ** 2)
    mid = 3e6 * (0.008 / n) ** 2 / (1.0 + 200.0 * t ** 1.5)
    hi = (3e6 * (0.008 / n) ** 2 * (0.3 / n) ** 0.5 / (1.0 + 200.0 * t ** 1.5)
          + 4e4 * (0.3 / n) ** 2.5 / (1.0 + 8000.0 * t ** 2))
    return np.where(n <= 0.008, k, np.where(n <= 0.3, mid, hi))


def aluminium_kappa(nu: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Mass opacity (cm^2/g) of the aluminium blocks of Sec. 3.5, as printed."""
    n, t = np.meshgrid(np.asarray(nu, float), np.asarray(T, float), indexing="xy")
    low = np.minimum(1e7, 1e8 * t ** 2)
    a = 1e7 * (0.01 / n) ** 2 / (1.0 + 20.0 * t ** 1.5)
    b = 1e6 * (0.1 / n) ** 2 / (1.0 + 200.0 * t ** 2)
    c = 1e7 * (0.01 / n) ** 2 * (1.5 / n) ** 0.5 / (1.0 + 20.0 * t ** 1.5) + 1e5 * (1.5 / n) ** 2.5 / (1.0 + 1000.0 * t ** 2)
    return np.where(n <= 0.01, low, np.where(n <= 0.1, a, np.where(n <= 1.5, a + b, c)))


def opacity_nodes(breaks=(0.008, 0.01, 0.1, 0.3, 1.5), numin: float = 1e-3, numax: float = 200.0,
                  Tmin: float = 1e-3, Tmax: float = 2.0):
    """Table nodes: 24 per decade in nu, with a node just below and at every
    breakpoint of the printed piecewise opacities so that their jumps stay sharp,
    and 16 per decade in T."""
    nu = np.geomspace(numin, numax, int(round(24 * np.log10(numax / numin))) + 1)
    nu = np.unique(np.concatenate([nu, np.asarray(breaks), np.asarray(breaks) * (1.0 - 1e-9)]))
    T = np.geomspace(Tmin, Tmax, int(round(16 * np.log10(Tmax / Tmin))) + 1)
    return nu, T


def olson1d(nx: int = 128, G: int = 24, **kw) -> Problem:
    """Olson's 1-D foam problem (Sec. 3.4) on [0, 4.8] cm with a = c = 1: the
    foam's printed opacity times its density 0.001 g/cm^3, tabulated on
    opacity_nodes(); Olson's heat capacity with H = 0.1, chi = 0.1 (keV); T0 =
    Tr0 = 0.01 keV; reflecting walls; the source B(0.5 keV) e^{-693 x^3} (cell
    centres) on while c t < 2; 24 log groups on [0.01, 100] keV; dt = dx / c;
    the particle weight 1e-4 V; the linearized source iteration."""
    L = 4.8
    nu_n, T_n = opacity_nodes()
    p = dict(dt=L / nx, steps=int(round(4.0 / (L / nx))), w_ref=1e-4, pool_cap=1 << 24,
             name=f"olson1d_{nx}_g{G}", numin=0.01, numax=100.0, bc_right=BC_REFLECT,
             flags=FLAG_SI_LINEARIZED, si_max_iters=500)
    p.update(kw)
    q = slab(nx, G, lambda x: np.ones_like(x), T0=0.01, **p)
    xc = (np.arange(nx) + 0.5) * (L / nx)
    table = {"mat": np.zeros(nx, np.int32), "nu": nu_n, "T": T_n,
             "sigma": (1e-3 * foam_kappa(nu_n, T_n))[None, :, :].copy()}
    return q.with_(x1=L, bc=[BC_REFLECT, BC_REFLECT, BC_VACUUM, BC_VACUUM], bcT=[0.0] * 4,
                   kappa=np.zeros((nx, G)), cv=np.ones(nx), olson_H=np.full(nx, 0.1),
                   olson_chi=np.full(nx, 0.1), opacity_table=table,
                   source_shape=np.exp(-693.0 * xc ** 3), source_T=0.5, source_t_off=2.0)


# Aluminium blocks of the 2-D Olson stand-in (lower-left corners, side 0.5 cm): the
# paper's layout exists only as a figure, so a layout symmetric about y = x of the
# same kind (blocks around the source corner and along the diagonal) stands in.
OLSON2D_BLOCKS = ((1.0, 0.0), (0.0, 1.0), (1.5, 1.0), (1.0, 1.5), (2.5, 0.5), (0.5, 2.5), (2.5, 2.5))


def olson2d(n: int = 285, G: int = 24, **kw) -> Problem:
    """Olson's 2-D problem (Sec. 3.5) on [0, 3.8]^2 cm with a = c = 1: foam (as in
    olson1d) with aluminium blocks (the printed aluminium opacity times 0.001 g/cm^3;
    Olson's heat capacity with H = 0.5, chi = 0.3 keV) at OLSON2D_BLOCKS (cell-centre
    rule), both tabulated on opacity_nodes(); T0 = Tr0 = 0.01 keV; reflecting walls;
    the source B(0.5 keV) e^{-18.7 r^3}, r the distance of the cell centre from the
    origin, on while c t < 3; 24 log groups on [0.01, 100] keV; dt = dx / c; the
    particle weight 1e-4 V; the linearized source iteration."""
    L = 3.8
    h = L / n
    xc = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    al = np.zeros((n, n), bool)
    for (bx, by) in OLSON2D_BLOCKS:
        al |= (X >= bx) & (X < bx + 0.5) & (Y >= by) & (Y < by + 0.5)
    al = al.reshape(-1)
    ncell = n * n
    nu_n, T_n = opacity_nodes()
    table = {"mat": al.astype(np.int32), "nu": nu_n, "T": T_n,
             "sigma": np.stack([1e-3 * foam_kappa(nu_n, T_n), 1e-3 * aluminium_kappa(nu_n, T_n)])}
    p = dict(dt=h, steps=int(round(3.0 / h)), w_ref=1e-4, pool_cap=1 << 25, seed=0, flags=FLAG_SI_LINEARIZED,
             si_max_iters=500)
    p.update(kw)
    r = np.hypot(X, Y).reshape(-1)
    return Problem(name=f"olson2d_{n}x{n}_g{G}", dim=2, nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L,
                   bc=[BC_REFLECT] * 4, bcT=[0.0] * 4, nu_edges=log_edges(0.01, 100.0, G),
                   kappa=np.zeros((ncell, G)), cv=np.ones(ncell), T0=np.full(ncell, 0.01),
                   Tr0=np.full(ncell, 0.01), pinned=np.zeros(ncell, np.uint8),
                   olson_H=np.where(al, 0.5, 0.1), olson_chi=np.where(al, 0.3, 0.1), opacity_table=table,
                   source_shape=np.exp(-18.7 * r ** 3), source_T=0.5, source_t_off=3.0, **p)


def lattice_mid_run_state(prob: Problem, n_particles: int, seed: int = 5) -> dict:
    """A synthetic state of the lattice workload part-way through its run, at
    the particle count of its late steps: material temperatures that fall off
    from the pinned source (T0 per cell, pinned cells at 1), cold radiation
    outside the particles (Tr0 = 1e-3), and a pool of n_particles collisionless particles in the background
    (kappa = 1) squares within 3 of the centre, in the upper half of the
    groups, ordered by (cell, group), each at a uniform position in its cell,
    an isotropic direction, a frequency uniform in its group and weight w_ref V.
    rhop is the particles' weight per unit volume in each (cell, group) bin.
    Inputs only: both the GPU library and the oracle start from it."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    nx, ny, G = prob.nx, prob.ny, prob.G
    dx, dy = (prob.x1 - prob.x0) / nx, (prob.y1 - prob.y0) / ny
    xc = prob.x0 + (np.arange(nx) + 0.5) * dx
    yc = prob.y0 + (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    r = np.hypot(X - 0.5 * (prob.x0 + prob.x1), Y - 0.5 * (prob.y0 + prob.y1)).reshape(-1)
    T0 = np.maximum(0.5 * np.exp(-(r / 0.8) ** 2), 1e-3)
    T0[prob.pinned == 1] = 1.0
    Tr0 = np.full(nx * ny, 1e-3)
    thin = np.flatnonzero((prob.kappa[:, 0] <= 1.0) & (r <= 3.0) & (prob.pinned == 0))
    gh = G - G // 2                                   # groups G//2 .. G-1
    b = np.sort(rng.integers(0, thin.size * gh, size=n_particles))
    cell = thin[b // gh].astype(np.int32)
    g = (G // 2 + b % gh).astype(np.int32)
    del b
    ix, iy = cell % nx, cell // nx
    x = prob.x0 + (ix + rng.random(n_particles)) * dx
    y = prob.y0 + (iy + rng.random(n_particles)) * dy
    del ix, iy
    oz = 2.0 * rng.random(n_particles) - 1.0
    psi = 2.0 * np.pi * rng.random(n_particles)
    st = np.sqrt(1.0 - oz * oz)
    del oz
    nu_e = np.asarray(prob.nu_edges)
    nu = nu_e[g] + rng.random(n_particles) * (nu_e[g + 1] - nu_e[g])
    V = dx * dy
    w = np.full(n_particles, prob.w_ref * V)
    pool = dict(x=x, y=y, ox=st * np.cos(psi), oy=st * np.sin(psi), nu=nu, w=w,
                id=np.arange(n_particles, dtype=np.uint64), cell=cell, g=g)
    rhop = np.bincount(cell.astype(np.int64) * G + g, weights=w, minlength=nx * ny * G).reshape(nx * ny, G) / V
    return dict(T0=T0, Tr0=Tr0, pool=pool, rhop=rhop, births=n_particles)
