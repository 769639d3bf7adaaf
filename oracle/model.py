"""Nondimensional model and the scheme constants (oracle; test infrastructure only).

Scales (the paper gives none; these follow its wetting cases, Sec. 4.3): drop density and
total drop viscosity, the wall gap as length, a velocity U. Then

* Re = rho_d U L / mu_d, Ca = mu_d U / sigma, Cn = eta / L,
  Pe = 2 sqrt(2) U L eta / (3 M sigma)  (Sec. 4.1 definitions),
* the mixing energy of eq. NS7 and the mobility combine to M lambda / eta^2 = 1 / Pe, so
  with eta -> Cn, lambda -> Cn^2, M -> 1/Pe the chemical potential of eq. NS5 becomes
  G = phi^3 - phi - Cn^2 lap(phi),
* the capillary force G grad(phi) of eq. NS2, divided by rho_d U^2 / L, carries
  K_sigma = 3 / (2 sqrt(2) Re Ca Cn),
* the polymer stress is scaled by mu_d U / L, so the Giesekus law (eq. NS4) reads
  tau + Wi tau_upper-convected + alpha Wi/(1 - beta) tau.tau = (1 - beta)(grad u + grad u^T)
  (alpha = 0: Oldroyd-B), i.e. tau = (1 - beta)/Wi (c - I) with the conformation law of
  eq. NS18, and enters momentum as (1 / (Re rho)) div[(1 + phi)/2 tau]  (second approach,
  eq. NS12).

The Dong splitting constants follow eqs. NS29-NS30 with the stabilisation
S = s_factor * Cn * sqrt(4 gamma0 Pe / dt), s_factor >= 1; the projection constants follow
the text after eq. NS39: rho0 = min density, nu_m = max solvent viscosity / (Re rho0).
"""
from __future__ import annotations

import dataclasses
import math


@dataclasses.dataclass
class Params:
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
    rho_ratio: float = 1.0
    mu_ratio: float = 1.0
    dt: float = 1e-4
    s_factor: float = 1.0
    a_ext: tuple = (0.0, 0.0, 0.0)
    viscoelastic: int = 0
    constitutive: int = 0          # 0: stress form, 1: log-conformation (lcr.py)
    giesekus_alpha: float = 0.0    # Giesekus mobility; 0 is Oldroyd-B
    refine: int = 2                # phase-field grid refinement: 2 dual resolution, 1 single
    advection: int = 0             # 0: second-order central flux, 1: fifth-order WENO-Z (weno.py)
    d_w: float = 0.0               # wall relaxation D_w of eq. NS15 (0: static contact angle)
    u_wall_bottom: tuple = (0.0, 0.0)  # wall velocity (x, y) at z = 0 (eq. NS13, u = u_w)
    u_wall_top: tuple = (0.0, 0.0)     # wall velocity (x, y) at z = lz

    @classmethod
    def from_config(cls, cfg) -> "Params":
        names = {f.name for f in dataclasses.fields(cls)}
        return cls(**{k: getattr(cfg, k) for k in names})

    # --- grid ---------------------------------------------------------------------------
    def walls(self, comp: int):
        """(bottom, top) wall values of the tangential velocity component comp (0: u, 1: v)."""
        return (float(self.u_wall_bottom[comp]), float(self.u_wall_top[comp]))

    @property
    def moving_walls(self) -> bool:
        return any(float(x) != 0.0 for x in tuple(self.u_wall_bottom) + tuple(self.u_wall_top))

    @property
    def ry(self) -> int:
        """Refinement factor in y (1 for a 2D case with a single y cell)."""
        return 1 if self.ny == 1 else self.refine

    @property
    def h(self):
        return (self.lx / self.nx, self.ly / self.ny, self.lz / self.nz)

    @property
    def hf(self):
        r = self.refine
        return (self.lx / (r * self.nx), self.ly / (self.ry * self.ny), self.lz / (r * self.nz))

    @property
    def fine_shape(self):
        r = self.refine
        return (r * self.nz, self.ry * self.ny, r * self.nx)

    @property
    def coarse_shape(self):
        return (self.nz, self.ny, self.nx)


@dataclasses.dataclass
class Constants:
    gamma0: float
    S: float        # stabilisation (eq. NS30 bound times s_factor)
    alpha: float    # eq. NS29
    c_psi: float    # alpha + S / Cn^2, the shift of eq. NS26
    rho1: float
    rho2: float
    mu1: float      # drop solvent viscosity
    mu2: float      # ambient viscosity
    rho0: float
    nu_m: float
    k_sigma: float
    c_j: float      # J = -c_j grad G


def constants(P: Params, first: bool) -> Constants:
    """Scheme constants for one step; ``first`` selects the one-level start (gamma0 = 1)."""
    g0 = 1.0 if first else 1.5
    cn2 = P.cn * P.cn
    S = P.s_factor * P.cn * math.sqrt(4.0 * g0 * P.pe / P.dt)
    # eq. NS29 with M lambda = Cn^2 / Pe and eta = Cn. With S equal to s_factor times the
    # bound of eq. NS30, the discriminant 1 - 4 gamma0 eta^4 / (M lambda dt S^2) is exactly
    # 1 - 1 / s_factor^2; it is evaluated in that form so that s_factor = 1 gives a double
    # root without a rounding residue under the square root.
    disc = 1.0 - 1.0 / (P.s_factor * P.s_factor)
    alpha = -(S / (2.0 * cn2)) * (1.0 + math.sqrt(disc))
    c_psi = alpha + S / cn2
    rho1, rho2 = 1.0, 1.0 / P.rho_ratio
    mu1 = P.beta if P.viscoelastic else 1.0
    mu2 = 1.0 / P.mu_ratio
    rho0 = min(rho1, rho2)
    nu_m = max(mu1, mu2) / (P.re * rho0)
    k_sigma = 3.0 / (2.0 * math.sqrt(2.0) * P.re * P.ca * P.cn)
    c_j = 0.5 * (rho1 - rho2) / P.pe
    return Constants(g0, S, alpha, c_psi, rho1, rho2, mu1, mu2, rho0, nu_m, k_sigma, c_j)
