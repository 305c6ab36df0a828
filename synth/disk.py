"""Parametric protoplanetary-disk inputs on an (r, z/r) node grid.

Every array is produced in float64 and handed out as float32; the oracle
promotes those float32 values back to float64 exactly, so both sides read
bit-identical inputs.

Physics of the inputs (Methods, "Parametric Disk Modeling"):
  * surface density  Sigma(r) = Sigma0 (r/rc)^-gamma exp[-(r/rc)^(2-gamma)],
    Sigma0 fixed by the total gas mass;
  * two-layer temperature, T_mid and T_atm radial power laws blended by
    cos^(2 delta)(pi z / 2 z_q) below z_q(r) = z_q0 (r/r_scale)^1.3;
  * vertically Gaussian (isothermal-midplane) H2 density with scale height
    H = c_s,mid / Omega_K -- the configurations use this closed-form profile
    instead of integrating the hydrostatic equation numerically;
  * height-dependent Keplerian v_phi (the pressure term of the velocity
    equation is left out);
  * CO layer bounded below by the freeze-out surface (T = T_freeze) and above
    by the photodissociation surface (0.706 N_H2 = N_dissoc), Eq. co_layer,
    with the vertical column of Eq. column_density taken by the trapezoid rule
    downward from the top node.  Surfaces are returned as two height vectors
    per radial node; the renderer turns them into a soft mask.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# cgs constants used only to build inputs (CODATA 2018 / IAU 2015 nominal)
_G = 6.67430e-8
_MSUN = 1.98847e33
_AU = 1.495978707e13
_KB = 1.380649e-16
_H = 6.62607015e-27
_C = 2.99792458e10
_AMU = 1.66053906660e-24
_MH = 1.6735575e-24
_DEBYE = 1.0e-18
MU_GAS = 2.37


@dataclass
class GridSpec:
    nr: int
    nz: int
    r_min_au: float = 1.0
    r_max_au: float = 600.0
    zr_max: float = 0.5

    def r_nodes(self) -> np.ndarray:
        i = np.arange(self.nr, dtype=np.float64)
        return self.r_min_au * (self.r_max_au / self.r_min_au) ** (i / (self.nr - 1))

    def zr_nodes(self) -> np.ndarray:
        j = np.arange(self.nz, dtype=np.float64)
        return self.zr_max * j / (self.nz - 1)

    def outer_radius(self) -> float:
        """Radius one radial cell beyond the last node."""
        return self.r_max_au * (self.r_max_au / self.r_min_au) ** (1.0 / (self.nr - 1))

    def outer_zr(self) -> float:
        return self.zr_max * self.nz / (self.nz - 1)


@dataclass
class DiskParams:
    mstar_msun: float = 2.0
    mgas_msun: float = 0.09
    gamma: float = 1.0
    rc_au: float = 150.0
    t_mid0_k: float = 30.0
    t_atm_factor: float = 2.0
    t_ref_au: float = 100.0
    q: float = -0.5
    zq0_au: float = 70.0
    r_scale_au: float = 150.0
    delta: float = 2.0
    t_freeze_k: float = 20.0
    n_dissoc: float = 1.0e21
    noise_sigma: float = 0.1
    gaps: tuple = ()            # ((depth, width_au, center_au), ...)


@dataclass
class Camera:
    nx: int
    ny: int
    fov_au: float
    incl_deg: float = 45.0
    pa_deg: float = 0.0
    dist_pc: float = 100.0


@dataclass
class LineData:
    nu0_hz: float
    a_ul: float
    g_u: float
    g_l: float
    e_u_k: float
    e_l_k: float
    m_co_amu: float
    m_mol_amu: float
    lev_e_k: np.ndarray
    lev_g: np.ndarray


@dataclass
class Problem:
    grid: GridSpec
    ln_nh2: np.ndarray      # float32 [nr, nz]
    temp_k: np.ndarray      # float32 [nr, nz]
    vphi_kms: np.ndarray    # float32 [nr, nz]
    z_lo_au: np.ndarray     # float32 [nr]
    z_up_au: np.ndarray     # float32 [nr]
    camera: Camera
    v_kms: np.ndarray       # float64 [nch] channel velocities
    line: LineData
    nsamp: int
    x_co: float = 1.0e-4
    mask_width: float = 1.0
    v_turb: float = 0.05
    v_sys_kms: float = 0.0
    intensity_scale: float = 1.0
    mlp_w: Optional[np.ndarray] = None   # float32 flat weights (neural CO layer)
    meta: dict = field(default_factory=dict)

    @property
    def nch(self) -> int:
        return int(len(self.v_kms))

    @property
    def ray_samples(self) -> int:
        return self.camera.nx * self.camera.ny * self.nch * self.nsamp

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def co21_line(jmax: int = 100) -> LineData:
    """12CO J=2-1 as a rigid rotor: nu0 = 230.538 GHz, rotational constant
    B0 = nu0/4 so that E_2 - E_1 = h nu0 exactly; A_ul from the electric
    dipole formula with mu = 0.1101 D; levels J = 0..jmax, g_J = 2J+1."""
    nu0 = 230.538e9
    b0 = nu0 / 4.0
    j = np.arange(jmax + 1, dtype=np.float64)
    e_k = _H * b0 * j * (j + 1) / _KB
    g = 2 * j + 1
    mu = 0.1101 * _DEBYE
    ju = 2.0
    a_ul = 64 * np.pi ** 4 * nu0 ** 3 / (3 * _H * _C ** 3) * mu ** 2 * ju / (2 * ju + 1)
    return LineData(nu0_hz=nu0, a_ul=float(a_ul), g_u=5.0, g_l=3.0,
                    e_u_k=float(e_k[2]), e_l_k=float(e_k[1]),
                    m_co_amu=27.9949146, m_mol_amu=MU_GAS * _MH / _AMU,
                    lev_e_k=e_k, lev_g=g)


def _temperature(r, z, p: DiskParams):
    t_mid = p.t_mid0_k * (r / p.t_ref_au) ** p.q
    t_atm = p.t_atm_factor * t_mid
    zq = p.zq0_au * (r / p.r_scale_au) ** 1.3
    blend = np.cos(np.pi * np.minimum(z, zq) / (2 * zq)) ** (2 * p.delta)
    return t_atm + (t_mid - t_atm) * blend, t_mid


def _surface_density(r_au, p: DiskParams):
    rc = p.rc_au * _AU
    r = r_au * _AU
    sig0 = p.mgas_msun * _MSUN * (2 - p.gamma) / (2 * np.pi * rc ** 2)
    return sig0 * (r / rc) ** (-p.gamma) * np.exp(-(r / rc) ** (2 - p.gamma))


def _surfaces(zr, r, n, t, p: DiskParams, zr_max):
    """Freeze-out (lower) and photodissociation (upper) heights per radius."""
    nr, nz = n.shape
    z_lo = np.empty(nr)
    z_up = np.empty(nr)
    for i in range(nr):
        z = zr * r[i]
        col = np.zeros(nz)
        for jj in range(nz - 2, -1, -1):
            col[jj] = col[jj + 1] + 0.5 * (n[i, jj] + n[i, jj + 1]) * (z[jj + 1] - z[jj]) * _AU
        shield = 0.706 * col
        thr = p.n_dissoc
        if shield[0] <= thr:
            z_up[i] = -zr_max * r[i]
        else:
            jj = int(np.nonzero(shield > thr)[0].max())
            if jj == nz - 1:
                z_up[i] = z[-1]
            elif shield[jj + 1] > 0:
                f = (np.log(thr) - np.log(shield[jj])) / (np.log(shield[jj + 1]) - np.log(shield[jj]))
                z_up[i] = z[jj] + f * (z[jj + 1] - z[jj])
            else:
                f = (thr - shield[jj]) / (shield[jj + 1] - shield[jj])
                z_up[i] = z[jj] + f * (z[jj + 1] - z[jj])
        tc = t[i]
        if tc[0] > p.t_freeze_k:
            z_lo[i] = -zr_max * r[i]
        else:
            warm = np.nonzero(tc > p.t_freeze_k)[0]
            if len(warm) == 0:
                z_lo[i] = 2 * zr_max * r[i]
            else:
                jj = int(warm[0]) - 1
                f = (p.t_freeze_k - tc[jj]) / (tc[jj + 1] - tc[jj])
                z_lo[i] = z[jj] + f * (z[jj + 1] - z[jj])
    return z_lo, z_up


def make_disk(grid: GridSpec, p: DiskParams, seed: int):
    """Fields on the node grid: (ln n_H2 [cm^-3], T [K], v_phi [km/s],
    z_lo [au], z_up [au]), float32, with median-one lognormal node noise on
    n_H2 and T drawn after the surfaces are extracted."""
    r = grid.r_nodes()
    zr = grid.zr_nodes()
    R, ZR = np.meshgrid(r, zr, indexing="ij")
    Z = ZR * R
    t, t_mid = _temperature(R, Z, p)
    cs2 = _KB * t_mid / (MU_GAS * _MH)
    omega2 = _G * p.mstar_msun * _MSUN / (R * _AU) ** 3
    h = np.sqrt(cs2 / omega2) / _AU
    sig = _surface_density(R, p)
    rho = sig / (np.sqrt(2 * np.pi) * h * _AU) * np.exp(-Z ** 2 / (2 * h ** 2))
    for depth, width, center in p.gaps:
        rho = rho * (1 - depth * np.exp(-(R - center) ** 2 / (2 * width ** 2)))
    n = rho / (MU_GAS * _MH)
    z_lo, z_up = _surfaces(zr, r, n, t, p, grid.zr_max)
    vphi = np.sqrt(_G * p.mstar_msun * _MSUN / (R * _AU)) * (1 + ZR ** 2) ** -0.75 / 1e5
    rng = np.random.Generator(np.random.PCG64(seed))
    ln_n = np.log(n)
    if p.noise_sigma > 0:
        ln_n = ln_n + p.noise_sigma * rng.standard_normal(ln_n.shape)
        t = t * np.exp(p.noise_sigma * rng.standard_normal(t.shape))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return f32(ln_n), f32(t), f32(vphi), f32(z_lo), f32(z_up)


def default_fov(grid: GridSpec) -> float:
    rc = grid.outer_radius()
    zc = grid.outer_zr() * rc
    return 2.0 * float(np.hypot(rc, zc))


def channels(nch: int, dv: float, v_sys: float = 0.0) -> np.ndarray:
    c = np.arange(nch, dtype=np.float64)
    return v_sys + (c - (nch - 1) / 2.0) * dv


def make_problem(grid: GridSpec, p: DiskParams, seed: int, *, nx: int, ny: int, nch: int,
                 dv: float, nsamp: int, incl: float = 45.0, pa: float = 0.0,
                 dist: float = 100.0, v_sys: float = 0.0, fov: Optional[float] = None,
                 intensity_scale: float = 1.0, meta=None) -> Problem:
    ln_n, t, vphi, z_lo, z_up = make_disk(grid, p, seed)
    cam = Camera(nx=nx, ny=ny, fov_au=default_fov(grid) if fov is None else fov,
                 incl_deg=incl, pa_deg=pa, dist_pc=dist)
    return Problem(grid=grid, ln_nh2=ln_n, temp_k=t, vphi_kms=vphi, z_lo_au=z_lo, z_up_au=z_up,
                   camera=cam, v_kms=channels(nch, dv, v_sys), line=co21_line(), nsamp=nsamp,
                   v_sys_kms=v_sys, intensity_scale=intensity_scale,
                   meta=dict(meta or {}, seed=seed, params=dataclasses.asdict(p)))


def rj_kelvin_scale(line: LineData) -> float:
    """Factor turning cgs specific intensity into Rayleigh-Jeans brightness
    temperature [K] at nu0 (c^2 / 2 k nu0^2)."""
    return _C ** 2 / (2 * _KB * line.nu0_hz ** 2)


# ---------------------------------------------------------------- configs
def config1(seed: int = 1, **over) -> Problem:
    """64x64 px, 16 channels x 0.2 km/s about v_sys = 0, 128 samples, 128x64 grid."""
    kw = dict(nx=64, ny=64, nch=16, dv=0.2, nsamp=128, incl=45.0)
    kw.update(over)
    grid = GridSpec(nr=kw.pop("nr", 128), nz=kw.pop("nz", 64))
    return make_problem(grid, DiskParams(), seed, meta={"config": "plain-64x64x16"}, **kw)


def config2_params(seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    mstar = rng.uniform(1.0, 2.5)
    incl = rng.uniform(20.0, 60.0)
    q = rng.uniform(-0.7, -0.3)
    gaps = []
    for _ in range(3):
        depth = rng.uniform(0.2, 0.8)
        width = rng.uniform(10.0, 40.0)
        center = float(np.exp(rng.uniform(np.log(20.0), np.log(400.0))))
        gaps.append((depth, width, center))
    return DiskParams(mstar_msun=mstar, q=q, gaps=tuple(gaps)), incl


def config2(seed: int = 2000, **over) -> Problem:
    """512x512 px, 64 channels x 0.1 km/s, 512 samples, 256x128 grid, seeded
    M* in [1, 2.5], inclination in [20, 60] deg, q in [-0.7, -0.3], 3 gaps."""
    p, incl = config2_params(seed)
    kw = dict(nx=512, ny=512, nch=64, dv=0.1, nsamp=512, incl=incl)
    kw.update(over)
    grid = GridSpec(nr=kw.pop("nr", 256), nz=kw.pop("nz", 128))
    return make_problem(grid, p, seed + 1, meta={"config": "full-512x512x64"}, **kw)


def config3(seed: int = 3, **over) -> Problem:
    """Forward + adjoint case: 256x256 px, 48 channels x 0.1 km/s, 256 samples."""
    kw = dict(nx=256, ny=256, nch=48, dv=0.1, nsamp=256, incl=45.0)
    kw.update(over)
    grid = GridSpec(nr=kw.pop("nr", 256), nz=kw.pop("nz", 128))
    return make_problem(grid, DiskParams(), seed, meta={"config": "adjoint-256x256x48"}, **kw)


def perturb_surfaces(prob: Problem, seed: int = 30, amp: float = 0.1) -> Problem:
    """Same disk with z_s(r) (1 + amp g_s(r)); g_s is a sum of three Gaussian
    bumps in ln r with amplitudes drawn from U[-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lr = np.log(prob.grid.r_nodes())
    g = np.zeros_like(lr)
    for _ in range(3):
        a = rng.uniform(-1.0, 1.0)
        mu = rng.uniform(np.log(20.0), np.log(400.0))
        g += a * np.exp(-(lr - mu) ** 2 / (2 * 0.25 ** 2))
    fac = 1.0 + amp * g
    return prob.replace(z_lo_au=np.float32(prob.z_lo_au * fac), z_up_au=np.float32(prob.z_up_au * fac))


def config3_target_disk(prob: Problem, seed: int = 30) -> Problem:
    return perturb_surfaces(prob, seed)


def add_noise(cube: np.ndarray, frac: float = 0.05, seed: int = 31) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    peak = float(np.max(np.abs(cube)))
    return (cube + frac * peak * rng.standard_normal(cube.shape)).astype(np.float32)


def config4(seed: int = 4, **over) -> Problem:
    """Neural CO layer: config-3 disk, 256x256 px x 32 channels x 256 samples."""
    from .mlp import make_mlp_weights
    kw = dict(nx=256, ny=256, nch=32, dv=0.1, nsamp=256, incl=45.0)
    kw.update(over)
    grid = GridSpec(nr=kw.pop("nr", 256), nz=kw.pop("nz", 128))
    prob = make_problem(grid, DiskParams(), 3, meta={"config": "neural-256x256x32"}, **kw)
    return prob.replace(mlp_w=make_mlp_weights(seed))


def small_problem(nx=16, ny=12, nch=8, nsamp=48, nr=24, nz=12, seed=7, incl=45.0, dv=0.25,
                  pa=0.0, v_sys=0.0, mlp_seed=None, **extra) -> Problem:
    """Config-1 family at a size the oracle finishes in well under a second."""
    grid = GridSpec(nr=nr, nz=nz)
    prob = make_problem(grid, DiskParams(), seed, nx=nx, ny=ny, nch=nch, dv=dv, nsamp=nsamp,
                        incl=incl, pa=pa, v_sys=v_sys, meta={"config": "small"}, **extra)
    if mlp_seed is not None:
        from .mlp import make_mlp_weights
        prob = prob.replace(mlp_w=make_mlp_weights(mlp_seed))
    return prob


def slab_problem(temp=40.0, ln_n=np.log(1e6), nsamp=64, m=24, nch=9, dv=0.1, nx=8, ny=8,
                 nr=32, nz=16, x_co=1e-4, width=1e-3) -> Problem:
    """Isothermal uniform slab viewed face-on.  z_up is placed on a segment
    boundary of every chord so each sample is fully inside or outside the
    layer; with a very narrow mask the layer is |z| < H exactly."""
    grid = GridSpec(nr=nr, nz=nz)
    rc = grid.outer_radius()
    zc = grid.outer_zr() * rc
    h = zc * (1.0 - 2.0 * m / nsamp)
    ln = np.full((nr, nz), ln_n, np.float32)
    tt = np.full((nr, nz), temp, np.float32)
    vp = np.zeros((nr, nz), np.float32)
    zlo = np.full(nr, -1.0, np.float32)
    zup = np.full(nr, h, np.float32)
    h32 = float(np.float32(h))
    cam = Camera(nx=nx, ny=ny, fov_au=2 * rc, incl_deg=0.0)
    return Problem(grid=grid, ln_nh2=ln, temp_k=tt, vphi_kms=vp, z_lo_au=zlo, z_up_au=zup,
                   camera=cam, v_kms=channels(nch, dv), line=co21_line(), nsamp=nsamp,
                   x_co=x_co, mask_width=width, meta={"config": "slab", "H_au": h32})


def ring_problem(r0=100.0, width=2.0, vphi=5.0, incl=40.0, nx=24, ny=24, nch=81, dv=0.1,
                 nsamp=400, nr=256, nz=16, x_co=1e-12, temp=40.0) -> Problem:
    """Optically thin narrow ring of gas at radius r0 (Gaussian in r of the
    given width, uniform in z/r), uniform v_phi and T."""
    grid = GridSpec(nr=nr, nz=nz, r_min_au=10.0, r_max_au=400.0, zr_max=5.0)
    r = grid.r_nodes()
    ln = np.log(1e8) - (r[:, None] - r0) ** 2 / (2 * width ** 2) + np.zeros((nr, nz))
    tt = np.full((nr, nz), temp)
    vp = np.full((nr, nz), vphi)
    zlo = -np.ones(nr) * 1e3
    zup = np.ones(nr) * 1e3
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    cam = Camera(nx=nx, ny=ny, fov_au=2.6 * r0, incl_deg=incl)
    return Problem(grid=grid, ln_nh2=f32(ln), temp_k=f32(tt), vphi_kms=f32(vp), z_lo_au=f32(zlo),
                   z_up_au=f32(zup), camera=cam, v_kms=channels(nch, dv), line=co21_line(),
                   nsamp=nsamp, x_co=x_co, meta={"config": "ring", "r0": r0})
