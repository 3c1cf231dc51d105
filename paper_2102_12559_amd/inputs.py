"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the bench.

This module holds no arithmetic of the lattice Boltzmann method itself: it only
produces run configurations (plain dicts), initial macroscopic fields and
velocity-set masks, all deterministic from a seed.  Random numbers come from
splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), implemented here from its published definition.

Units: cell spacing 1, velocities in units of sqrt(R T_L) with R = T_L = 1
(paper Sec. II.A, lattice temperature fixed to one for all velocity sets).
"""
from __future__ import annotations

import math

import numpy as np

# boundary kinds (same numeric values as the C-ABI and the oracle)
BC_PERIODIC = 0
BC_FIXED_EQ = 1      # ghost = lattice equilibrium of a fixed state (inlet, far field)
BC_OUTFLOW_ZG = 2    # ghost = copy of the boundary cell (zero gradient)
BC_DIFFUSE_WALL = 3  # diffuse-reflection wall

CRIT_NONE = 0
CRIT_MA = 1      # local Mach number above threshold -> high order
CRIT_PINEQ = 2   # |Pi_neq|_F / p above threshold -> high order
CRIT_KN = 3      # local Knudsen number lambda |grad rho| / rho above threshold -> high order

STORE_FP64 = 0
STORE_FP32 = 1
STORE_FP16_DEV = 2
STORE_BF16_DEV = 3

LIFT_GRAD = 0          # raw-moment completion with equilibrium moments
LIFT_GRAD_HERMITE = 1  # Hermite-coefficient completion
LIFT_MLP = 2           # raw completion + learned non-equilibrium correction

_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of splitmix64 started from `seed` (uint64 array)."""
    out = np.empty(count, dtype=np.uint64)
    s = seed & _MASK64
    for k in range(count):
        s = (s + 0x9E3779B97F4A7C15) & _MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out[k] = z ^ (z >> 31)
    return out


def uniform_pm1(seed: int, count: int) -> np.ndarray:
    """Uniform doubles in [-1, 1) from the top 53 bits of splitmix64."""
    if count == 0:
        return np.zeros(0)
    # vectorised splitmix64 (identical sequence to splitmix64())
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = (np.uint64(seed & _MASK64) + k * np.uint64(0x9E3779B97F4A7C15))
        z = s
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u01 = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u01 - 1.0


def base_config(**kw) -> dict:
    """A run configuration with every field defaulted; keyword args override."""
    cfg = dict(
        dim=2, nx=64, ny=64, nz=1,
        n_low=3, n_high=0,          # 1D Gauss-Hermite orders; n_high=0 -> one lattice
        thermal=0,                  # 1: f and g populations, ideal gas with Cv
        tau=0.6, cv=1.5, cfl=1.0,
        tau_mode=0, mu_exp=0.0, tau_ref_rho=1.0, tau_ref_T=1.0,
        rho0=1.0, T0=1.0,           # reference state of the deviation storage
        store=STORE_FP64, lift_mode=LIFT_GRAD,
        bc=[BC_PERIODIC] * 6,
        bc_state=[[1.0, 0.0, 0.0, 0.0, 1.0] for _ in range(6)],
        slot_state=[[1.0, 0.0, 0.0, 0.0, 1.0] for _ in range(6)],
        slot=[[0, 0, 0, 0] for _ in range(6)],
        slot_edge=[0.0] * 6,
        crit_kind=CRIT_NONE, crit_thr=0.0, crit_every=0,
    )
    cfg.update(kw)
    if cfg["dim"] == 2:
        cfg["nz"] = 1
    return cfg


# ---------------------------------------------------------------------------
# Convected vortex (paper Sec. IV.A.1 initial condition; also used in 3D as a
# columnar vortex along z).
# ---------------------------------------------------------------------------

def vortex_fields(nx, ny, nz=1, *, eps, rc, u0, ma_v=None, cs=1.0, rho0=1.0,
                  noise=1e-6, seed=0, xc=None, yc=None):
    """rho, u[dim], T fields of the Gaussian convected vortex.

    Velocity: u_x = U0 - eps (y-yc)/Rc exp(-r^2/(2Rc^2)),
              u_y = eps (x-xc)/Rc exp(-r^2/(2Rc^2)).
    Density:  rho = rho0 exp(-(Ma_v^2/2) exp(-r^2/Rc^2)), Ma_v = eps/cs.
    Uniform noise of amplitude `noise` is added to rho (splitmix64, `seed`).
    Cell centres sit at integer coordinates; the centre defaults to (nx/2, ny/2).
    Returns arrays shaped [nz, ny, nx] (rho, T) and [dim, nz, ny, nx] (u).
    """
    xc = nx / 2 if xc is None else xc
    yc = ny / 2 if yc is None else yc
    if ma_v is None:
        ma_v = eps / cs
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx = x - xc
    dy = y - yc
    r2 = dx * dx + dy * dy
    g = np.exp(-r2 / (2 * rc * rc))
    ux = u0 - eps * dy / rc * g
    uy = eps * dx / rc * g
    rho = rho0 * np.exp(-0.5 * ma_v * ma_v * np.exp(-r2 / (rc * rc)))
    rho = rho + noise * uniform_pm1(seed, rho.size).reshape(rho.shape)
    dim = 2 if nz == 1 else 3
    u = np.zeros((dim,) + rho.shape)
    u[0] = ux
    u[1] = uy
    T = np.ones_like(rho)
    return rho.astype(np.float64), u, T


def disk_mask(nx, ny, nz=1, *, radius, xc=None, yc=None):
    """uint8 velocity-set mask [nz, ny, nx]: 1 (high order) inside the disk."""
    xc = nx / 2 if xc is None else xc
    yc = ny / 2 if yc is None else yc
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (((x - xc) ** 2 + (y - yc) ** 2) <= radius * radius).astype(np.uint8)


def vortex_c1():
    """Athermal convected vortex on a 64x64 periodic grid, FP64, 200 steps.

    D2Q9 everywhere except a fixed D2Q16 disk of radius 12 cells at the centre;
    BGK tau 0.6; eps 0.07, core radius 8, advection Ma 0.5; 1e-6 noise on rho.
    """
    nx = ny = 64
    cfg = base_config(dim=2, nx=nx, ny=ny, n_low=3, n_high=4, tau=0.6,
                      store=STORE_FP64)
    rho, u, T = vortex_fields(nx, ny, eps=0.07, rc=8.0, u0=0.5)
    mask = disk_mask(nx, ny, radius=12.0)
    return dict(cfg=cfg, rho=rho, u=u, T=T, mask=mask, steps=200)


# ---------------------------------------------------------------------------
# Jet (compressible, thermal two-population model)
# ---------------------------------------------------------------------------

def gamma_of(cv):
    return (cv + 1.0) / cv


def jet_c2(nx=1024, ny=512, slot_w=32, ma=0.6, tau=0.52, store=STORE_FP32,
           crit_thr=0.4, crit_every=20, n_high=6, edge=4.0, thermal=0):
    """Slot jet at Mach `ma` into quiescent gas (rho = T = 1).

    x-low face: equilibrium ghost at rest except the slot rows
    [ny/2 - slot_w/2, ny/2 + slot_w/2), which hold the inlet state
    (rho 1, u_x = ma * c_s, T 1), blended with tanh edges of `edge` cells.
    Other faces: zero-gradient outflow.  D2Q9 plus the high-order set where the
    local Mach number exceeds `crit_thr`, re-evaluated every `crit_every` steps.

    Defaults follow the paper's own jet (Sec. IV.A.2: athermal, jet Mach
    number 0.6) with D2Q36 as the high-order set and smoothed slot edges: in
    the lattice frame with BGK at tau = 0.52 every thermal variant, every
    D2Q16 variant and every Mach-1.2 slot diverged within 250 to 8000 steps;
    this one runs the 20000 steps.
    """
    cv = 1.5
    cs = math.sqrt(gamma_of(cv) * 1.0)
    lo = ny // 2 - slot_w // 2
    if not thermal:
        cs = 1.0
    cfg = base_config(dim=2, nx=nx, ny=ny, n_low=3, n_high=n_high, thermal=thermal,
                      tau=tau, cv=cv, store=store,
                      crit_kind=CRIT_MA, crit_thr=crit_thr, crit_every=crit_every)
    cfg["bc"] = [BC_FIXED_EQ, BC_OUTFLOW_ZG, BC_OUTFLOW_ZG, BC_OUTFLOW_ZG,
                 BC_PERIODIC, BC_PERIODIC]
    cfg["slot"][0] = [lo, lo + slot_w, 0, 0]
    cfg["slot_state"][0] = [1.0, ma * cs, 0.0, 0.0, 1.0]
    cfg["slot_edge"][0] = edge
    rho = np.ones((1, ny, nx))
    u = np.zeros((2, 1, ny, nx))
    T = np.ones((1, ny, nx))
    mask = np.zeros((1, ny, nx), dtype=np.uint8)
    return dict(cfg=cfg, rho=rho, u=u, T=T, mask=mask, steps=20000)


# ---------------------------------------------------------------------------
# Shock structure (Rankine-Hugoniot end states, hard-sphere viscosity)
# ---------------------------------------------------------------------------

def rankine_hugoniot(ma1, gamma, rho1=1.0, T1=1.0):
    """Downstream (rho2, u2, T2) and upstream u1 of a normal shock.

    Textbook normal-shock relations of an ideal gas (p = rho T, R = 1):
      rho2/rho1 = (g+1) M^2 / ((g-1) M^2 + 2)
      p2/p1     = 1 + 2g/(g+1) (M^2 - 1)
    with u1 = M sqrt(g T1) and u2 = u1 rho1 / rho2.
    """
    g = gamma
    m2 = ma1 * ma1
    r = (g + 1) * m2 / ((g - 1) * m2 + 2)
    pr = 1 + 2 * g / (g + 1) * (m2 - 1)
    u1 = ma1 * math.sqrt(g * T1)
    rho2 = rho1 * r
    T2 = T1 * pr / r
    u2 = u1 / r
    return dict(rho1=rho1, u1=u1, T1=T1, rho2=rho2, u2=u2, T2=T2)


def hard_sphere_tau(lam_cells, rho, T, gamma, dt):
    """BGK tau from a hard-sphere mean free path of `lam_cells` cells.

    mean free path lam = 16/(5 sqrt(2 pi g)) * mu a / p, a = sqrt(g T), p = rho T,
    so mu = lam p 5 sqrt(2 pi g) / (16 a); tau = mu / (rho T dt) + 1/2.
    """
    a = math.sqrt(gamma * T)
    p = rho * T
    mu = lam_cells * p * 5.0 * math.sqrt(2 * math.pi * gamma) / (16.0 * a)
    return mu / (rho * T * dt) + 0.5


def shock_frame(ma1, gamma=5.0 / 3.0):
    """Global constant frame of the shock runs: the mean of the two end
    states' velocities and temperatures, u_ref = ((u1 + u2)/2, 0, 0),
    T_ref = (T1 + T2)/2."""
    rh = rankine_hugoniot(ma1, gamma)
    return (0.5 * (rh["u1"] + rh["u2"]), 0.0, 0.0), 0.5 * (rh["T1"] + rh["T2"])


def shock_c3(ma1=2.0, nx=8192, ny=4, store=STORE_FP64, n_high=6, lam=2.0,
             crit_thr=1e-3, crit_every=5, dt=None, frame=False):
    """Quasi-1D normal shock: RH states at the x ends, step at the centre.

    D2Q9 far field, D2Q36 where |Pi_neq|/p exceeds the threshold; viscosity
    mu ~ T^0.5 (hard spheres) with tau set by a mean free path of `lam` cells
    upstream.  `dt` must be the time step of the lattice pair in the run's
    frame (CFL / the largest particle speed).  frame=True runs in the global
    constant frame of shock_frame(); otherwise in the lattice frame.
    The run starts all low order (the step is an equilibrium on both sides,
    so the criterion sees nothing at step 0); the criterion runs every 5
    steps because the D2Q9 shock diverges within about 15 steps.
    """
    cv = 1.5
    g = gamma_of(cv)
    rh = rankine_hugoniot(ma1, g)
    if dt is None:
        raise ValueError("dt of the lattice pair is required")
    tau1 = hard_sphere_tau(lam, rh["rho1"], rh["T1"], g, dt)
    cfg = base_config(dim=2, nx=nx, ny=ny, n_low=3, n_high=n_high, thermal=1,
                      tau=tau1, cv=cv, tau_mode=1, mu_exp=0.5,
                      tau_ref_rho=rh["rho1"], tau_ref_T=rh["T1"], store=store,
                      crit_kind=CRIT_PINEQ, crit_thr=crit_thr, crit_every=crit_every)
    cfg["bc"] = [BC_FIXED_EQ, BC_FIXED_EQ, BC_PERIODIC, BC_PERIODIC,
                 BC_PERIODIC, BC_PERIODIC]
    cfg["bc_state"][0] = [rh["rho1"], rh["u1"], 0.0, 0.0, rh["T1"]]
    cfg["bc_state"][1] = [rh["rho2"], rh["u2"], 0.0, 0.0, rh["T2"]]
    if frame:
        cfg["u_ref"], cfg["T_ref"] = shock_frame(ma1, g)
    x = np.arange(nx)
    left = (x < nx // 2)[None, None, :].repeat(ny, axis=1)
    rho = np.where(left, rh["rho1"], rh["rho2"]).astype(np.float64)
    T = np.where(left, rh["T1"], rh["T2"]).astype(np.float64)
    u = np.zeros((2, 1, ny, nx))
    u[0] = np.where(left, rh["u1"], rh["u2"])
    mask = np.zeros((1, ny, nx), dtype=np.uint8)
    return dict(cfg=cfg, rho=rho, u=u, T=T, mask=mask, steps=50000, rh=rh)


# ---------------------------------------------------------------------------
# Planar Couette flow between diffuse walls
# ---------------------------------------------------------------------------

def couette_c4(N=64, kn=0.1, nx=8, band=4, uw=0.1, store=STORE_FP32, dt=None,
               n_high=6, lift_mode=LIFT_GRAD, thermal=0):
    """8 x N channel, x periodic, diffuse walls at y = -1/2 and y = N - 1/2.

    Walls move with u_x = -uw (bottom) and +uw (top), T_w = 1.  D2Q9 in the
    bulk, the high-order lattice in `band` rows next to each wall.  BGK tau
    from a hard-sphere mean free path lam = Kn * N cells at rho = T = 1.
    """
    cv = 1.5
    g = gamma_of(cv)
    if dt is None:
        raise ValueError("dt of the lattice pair is required")
    tau = hard_sphere_tau(kn * N, 1.0, 1.0, g, dt)
    cfg = base_config(dim=2, nx=nx, ny=N, n_low=3, n_high=n_high, thermal=thermal,
                      tau=tau, cv=cv, store=store, lift_mode=lift_mode)
    cfg["bc"] = [BC_PERIODIC, BC_PERIODIC, BC_DIFFUSE_WALL, BC_DIFFUSE_WALL,
                 BC_PERIODIC, BC_PERIODIC]
    cfg["bc_state"][2] = [1.0, -uw, 0.0, 0.0, 1.0]
    cfg["bc_state"][3] = [1.0, +uw, 0.0, 0.0, 1.0]
    rho = np.ones((1, N, nx))
    u = np.zeros((2, 1, N, nx))
    T = np.ones((1, N, nx))
    mask = np.zeros((1, N, nx), dtype=np.uint8)
    if n_high:
        mask[:, :band, :] = 1
        mask[:, N - band:, :] = 1
    return dict(cfg=cfg, rho=rho, u=u, T=T, mask=mask, steps=None)


# ---------------------------------------------------------------------------
# 3D convected vortex + shear layer
# ---------------------------------------------------------------------------

def vortex_shear_3d(n=256, store=STORE_FP16_DEV, eps=0.05, ma=0.6, rc=16.0,
                    slab_lo=None, slab_hi=None, width=4.0, noise=1e-6, seed=0,
                    crit_thr=0.4, crit_every=20, lift_mode=LIFT_GRAD):
    """n^3 periodic box: columnar Gaussian vortex along z plus a shear slab.

    u_x = Ma c_s * (tanh((y - lo)/w) - tanh((y - hi)/w)) / 2 + vortex u_x,
    vortex with strength eps and core radius rc centred in (x, y); rho from the
    vortex density law; noise on rho.  D3Q27 bulk, D3Q64 where Ma > crit_thr.
    """
    lo = (96 / 256) * n if slab_lo is None else slab_lo
    hi = (160 / 256) * n if slab_hi is None else slab_hi
    rho, u, T = vortex_fields(n, n, n, eps=eps, rc=rc, u0=0.0, noise=noise, seed=seed)
    y = np.arange(n)[None, :, None]
    u[0] += ma * 0.5 * (np.tanh((y - lo) / width) - np.tanh((y - hi) / width))
    cfg = base_config(dim=3, nx=n, ny=n, nz=n, n_low=3, n_high=4, tau=0.6,
                      store=store, lift_mode=lift_mode, crit_kind=CRIT_MA,
                      crit_thr=crit_thr, crit_every=crit_every)
    mask = np.zeros((n, n, n), dtype=np.uint8)
    return dict(cfg=cfg, rho=rho, u=u, T=T, mask=mask, steps=2000)


# ---------------------------------------------------------------------------
# Smooth random flow (roofline runs and parity fixtures)
# ---------------------------------------------------------------------------

def smooth_random_flow(nx, ny, nz=1, *, umax=0.1, modes=3, seed=0, drho=0.01,
                       dT=0.0):
    """Periodic random-phase flow: sums of low Fourier modes, |u| <= umax."""
    dim = 2 if nz == 1 else 3
    r = uniform_pm1(seed, 4 * dim * modes * modes + 8 * modes)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((dim, nz, ny, nx))
    k = 0
    for a in range(dim):
        for m in range(1, modes + 1):
            for q in range(1, modes + 1):
                ph = math.pi * r[k]; k += 1
                amp = r[k]; k += 1
                u[a] += amp * np.sin(2 * math.pi * (m * x / nx + q * y / ny + (m * z / nz if dim == 3 else 0)) + ph)
    norm = np.max(np.sqrt((u * u).sum(axis=0)))
    u *= umax / max(norm, 1e-300)
    ph1, ph2 = math.pi * r[k], math.pi * r[k + 1]
    rho = 1.0 + drho * np.sin(2 * math.pi * x / nx + ph1) * np.cos(2 * math.pi * y / ny + ph2)
    T = 1.0 + dT * np.cos(2 * math.pi * x / nx + ph2) * np.sin(2 * math.pi * y / ny + ph1)
    return rho, u, T


def random_mask(nx, ny, nz=1, *, frac=0.1, seed=1, blob=6):
    """A mask of blobs (squares of side `blob`) covering about `frac` of cells."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    nb = max(1, int(round(frac * nx * ny * nz / float(blob ** (2 if nz == 1 else 3)))))
    r = uniform_pm1(seed, 3 * nb)
    for b in range(nb):
        x0 = int((r[3 * b] * 0.5 + 0.5) * nx) % nx
        y0 = int((r[3 * b + 1] * 0.5 + 0.5) * ny) % ny
        z0 = int((r[3 * b + 2] * 0.5 + 0.5) * nz) % nz if nz > 1 else 0
        xs = (x0 + np.arange(blob)) % nx
        ys = (y0 + np.arange(blob)) % ny
        zs = ((z0 + np.arange(blob)) % nz) if nz > 1 else np.array([0])
        m[np.ix_(zs, ys, xs)] = 1
    return m


def rect_zone_mask(nx, ny, frac=0.1):
    """The efficiency layout: two rectangular zones, the first `frac` of the
    columns (x) high order, the rest low order."""
    m = np.zeros((1, ny, nx), dtype=np.uint8)
    m[:, :, : max(1, int(round(frac * nx)))] = 1
    return m
