"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds the problem configurations (nondimensional groups, grid sizes, time step)
and the initial-state generators. It contains none of the solver's arithmetic: no stencil,
no transform, no time-integration constant. The initial phase field is the equilibrium
tanh profile of a droplet sitting on the bottom wall (the wetting set-ups of Sec. 4.3 of
the paper: a half-circle or half-sphere at 90 degrees on the wall), optionally plus
uniform noise drawn from a counter-based SplitMix64 stream (Steele, Lea and Flood 2014),
so that every consumer regenerates bit-identical inputs from the seed alone.

Array layout everywhere: ``[z][y][x]`` with x contiguous; z is wall-normal, x and y are
periodic. A 2D case has one coarse and one fine cell in y.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Config", "CONFIGS", "config", "initial_phi", "splitmix64_uniform", "fine_shape",
           "coarse_shape", "droplet_state", "adjoint_seed"]


@dataclasses.dataclass
class Config:
    """One problem set-up. Sizes are coarse-grid cell counts; the phase-field grid is
    ``refine`` times as fine in x and z, and in y when ny > 1 (refine 1: one grid)."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    re: float
    ca: float
    cn: float
    pe: float
    wi: float = 1.0
    beta: float = 1.0
    theta_bottom_deg: float = 90.0
    theta_top_deg: float = 90.0
    rho_ratio: float = 1.0      # drop density / ambient density
    mu_ratio: float = 1.0       # drop total viscosity / ambient viscosity
    dt: float = 1e-4
    s_factor: float = 1.0
    a_ext: tuple = (0.0, 0.0, 0.0)
    viscoelastic: int = 0
    constitutive: int = 0       # 0: stress form, 1: log-conformation
    giesekus_alpha: float = 0.0
    refine: int = 2             # phase-field grid: 2 dual resolution, 1 single resolution
    advection: int = 0          # 0: second-order central flux, 1: fifth-order WENO-Z
    d_w: float = 0.0             # wall relaxation D_w of eq. NS15
    u_wall_bottom: tuple = (0.0, 0.0)   # tangential wall velocity (x, y) at z = 0
    u_wall_top: tuple = (0.0, 0.0)      # tangential wall velocity (x, y) at z = lz
    check_finite_every: int = 0          # library option: finite checks every n steps (0: none)
    steps: int = 10
    radius: float = 0.25
    centre: tuple | None = None  # (x, y) of the drop foot on the bottom wall
    noise: float = 0.0
    seed: int = 0

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    @property
    def ndim(self) -> int:
        return 2 if self.ny == 1 else 3


def _c(**kw) -> Config:
    return Config(**kw)


CONFIGS: dict[str, Config] = {
    # 2D Newtonian spreading, 64x32 coarse / 128x64 fine on a 2x1 box.
    "C1": _c(name="C1", nx=64, ny=1, nz=32, lx=2.0, ly=2.0 / 64, lz=1.0, re=10.0, ca=0.1,
             cn=0.01, pe=1000.0, theta_bottom_deg=60.0, dt=1e-4, steps=100, radius=0.3,
             noise=1e-3, seed=1),
    # 3D Newtonian drop, density ratio 1000 and viscosity ratio 100.
    "C2": _c(name="C2", nx=128, ny=128, nz=64, lx=2.0, ly=2.0, lz=1.0, re=100.0, ca=1.0,
             cn=0.01, pe=300.0, theta_bottom_deg=90.0, rho_ratio=1000.0, mu_ratio=100.0,
             dt=1e-4, steps=500, radius=0.25),
    # 3D Oldroyd-B drop on a wall.
    "C3": _c(name="C3", nx=128, ny=128, nz=64, lx=2.0, ly=2.0, lz=1.0, re=1.0, ca=1.0,
             cn=0.01, pe=300.0, wi=1.0, beta=0.5, theta_bottom_deg=120.0, dt=5e-5,
             steps=1000, radius=0.25, viscoelastic=1),
    # 2D viscoelastic drop used for the gradient case.
    "C4": _c(name="C4", nx=256, ny=1, nz=128, lx=2.0, ly=2.0 / 256, lz=1.0, re=10.0, ca=0.1,
             cn=0.01, pe=500.0, wi=0.5, beta=0.5, theta_bottom_deg=70.0, dt=1e-4,
             steps=2000, radius=0.3, viscoelastic=1),
    # Large 3D viscoelastic run: 67.1M fine cells.
    "C5": _c(name="C5", nx=256, ny=256, nz=128, lx=2.0, ly=2.0, lz=1.0, re=1.0, ca=1.0,
             cn=0.01, pe=300.0, wi=2.0, beta=0.3, theta_bottom_deg=45.0, rho_ratio=100.0,
             mu_ratio=10.0, dt=5e-5, steps=200, radius=0.25, viscoelastic=1),
    # C2 and C3 at a single resolution: everything on the 256x256x128 grid that carries the
    # phase field of C2 / C3 (the baselines of the dual-resolution comparison).
    "C2S": _c(name="C2S", nx=256, ny=256, nz=128, lx=2.0, ly=2.0, lz=1.0, re=100.0, ca=1.0,
              cn=0.01, pe=300.0, theta_bottom_deg=90.0, rho_ratio=1000.0, mu_ratio=100.0,
              dt=1e-4, steps=500, radius=0.25, refine=1),
    "C3S": _c(name="C3S", nx=256, ny=256, nz=128, lx=2.0, ly=2.0, lz=1.0, re=1.0, ca=1.0,
              cn=0.01, pe=300.0, wi=1.0, beta=0.5, theta_bottom_deg=120.0, dt=5e-5,
              steps=1000, radius=0.25, viscoelastic=1, refine=1),
    # C3 with the log-conformation update of the paper and a Giesekus term.
    "C3L": _c(name="C3L", nx=128, ny=128, nz=64, lx=2.0, ly=2.0, lz=1.0, re=1.0, ca=1.0,
              cn=0.01, pe=300.0, wi=1.0, beta=0.5, theta_bottom_deg=120.0, dt=5e-5,
              steps=1000, radius=0.25, viscoelastic=1, constitutive=1, giesekus_alpha=0.2),
    # C2 with relaxed walls (eq. NS15 with D_w = 0.1): the Robin form of the wall-normal pass.
    "C2R": _c(name="C2R", nx=128, ny=128, nz=64, lx=2.0, ly=2.0, lz=1.0, re=100.0, ca=1.0,
              cn=0.01, pe=300.0, theta_bottom_deg=90.0, rho_ratio=1000.0, mu_ratio=100.0,
              dt=1e-4, steps=500, radius=0.25, d_w=0.1),
    # C3L with the fifth-order WENO-Z advection of the phase field and of the log-conformation:
    # the full scheme of the paper's three-dimensional viscoelastic runs.
    "C3P": _c(name="C3P", nx=128, ny=128, nz=64, lx=2.0, ly=2.0, lz=1.0, re=1.0, ca=1.0,
              cn=0.01, pe=300.0, wi=1.0, beta=0.5, theta_bottom_deg=120.0, dt=5e-5,
              steps=1000, radius=0.25, viscoelastic=1, constitutive=1, giesekus_alpha=0.2,
              advection=1),
}


def config(name: str, **overrides) -> Config:
    return CONFIGS[name].replace(**overrides)


def coarse_shape(cfg: Config) -> tuple[int, int, int]:
    return (cfg.nz, cfg.ny, cfg.nx)


def fine_shape(cfg: Config) -> tuple[int, int, int]:
    r = cfg.refine
    return (r * cfg.nz, 1 if cfg.ny == 1 else r * cfg.ny, r * cfg.nx)


_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """The first ``n`` outputs of a SplitMix64 stream started at ``seed``, mapped to
    doubles in [0, 1) from their top 53 bits. Output ``c`` is the mixer applied to
    ``seed + (c + 1) * golden_gamma`` (mod 2**64)."""
    with np.errstate(over="ignore"):
        c = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + c * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def initial_phi(cfg: Config) -> np.ndarray:
    """Fine-grid phase field: +1 inside a drop of radius ``cfg.radius`` whose centre sits on
    the bottom wall, with the equilibrium profile tanh(d / (sqrt(2) Cn)) across the
    interface (d = signed distance to the circle / sphere), plus U(-noise, +noise)."""
    nzf, nyf, nxf = fine_shape(cfg)
    hx, hz = cfg.lx / nxf, cfg.lz / nzf
    hy = cfg.ly / nyf
    cx, cy = cfg.centre if cfg.centre is not None else (0.5 * cfg.lx, 0.5 * cfg.ly)
    x = (np.arange(nxf) + 0.5) * hx
    y = (np.arange(nyf) + 0.5) * hy
    z = (np.arange(nzf) + 0.5) * hz
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    if cfg.ny == 1:
        r = np.sqrt((xx - cx) ** 2 + zz ** 2)
    else:
        r = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2 + zz ** 2)
    phi = np.tanh((cfg.radius - r) / (math.sqrt(2.0) * cfg.cn))
    if cfg.noise > 0.0:
        phi = phi + cfg.noise * (2.0 * splitmix64_uniform(cfg.seed, phi.size).reshape(phi.shape) - 1.0)
    return np.ascontiguousarray(phi)


def droplet_state(cfg: Config) -> dict:
    """Full initial state as FP64 numpy arrays: both time levels equal (the first step is a
    one-level start), velocity, pressure and polymer stress zero, log-conformation zero."""
    phi = initial_phi(cfg)
    cs = coarse_shape(cfg)
    z = lambda: np.zeros(cs)
    return {
        "phi": [phi.copy(), phi.copy()],
        "u": [z(), z()], "v": [z(), z()], "w": [z(), z()],
        "p": [z(), z()],
        "tau": [[z() for _ in range(6)], [z() for _ in range(6)]],
        "theta": [z() for _ in range(6)],  # log-conformation (c = I)
        "step": 0,
    }


def adjoint_seed(cfg: Config, seed: int) -> dict:
    """A state-shaped set of arrays with entries uniform in [-1, 1) from the SplitMix64 stream
    of ``seed`` (fields in the order phi, u, v, w, p, tau; level n before n-1), used as the
    adjoint of a state in reverse-step tests. The polymer part is zero for a Newtonian case."""
    fs, cs = fine_shape(cfg), coarse_shape(cfg)
    shapes = [fs, fs] + [cs] * 8 + ([cs] * 12 if cfg.viscoelastic else [])
    n = sum(int(np.prod(s)) for s in shapes)
    r = 2.0 * splitmix64_uniform(seed, n) - 1.0
    out, pos = [], 0
    for s in shapes:
        m = int(np.prod(s))
        out.append(np.ascontiguousarray(r[pos:pos + m].reshape(s)))
        pos += m
    lam = {"phi": out[0:2], "u": out[2:4], "v": out[4:6], "w": out[6:8], "p": out[8:10]}
    if cfg.viscoelastic:
        lam["tau"] = [out[10:16], out[16:22]]
    else:
        lam["tau"] = [[np.zeros(cs) for _ in range(6)] for _ in range(2)]
    lam["step"] = 0
    return lam
