"""Log-conformation polymer update (oracle; test infrastructure only).

The conformation tensor c (tau_p = (1 - beta)/Wi (c - I) in the scaling of model.py) is
advanced through its logarithm Theta = log c (Sec. 2.2, eqs. NS17-NS24), with the Giesekus
relaxation [I + alpha (c - I)](c - I) / Wi (alpha = 0: Oldroyd-B), in the order of
Sec. 3.2.3 (eqs. NS40-NS46): two stages of the TVD Runge-Kutta scheme with u^{n+1} fixed, each
stage diagonalising its own Theta, then tau^{n+1} from the diagonalised Theta^{n+1}.

Readings (the paper is silent or garbled here):

* Sign of the relaxation. The right-hand sides of eqs. NS18, NS22 and NS41 are printed with a
  plus sign; with it c would move away from I. The c equation used is
  dc/dt + u.grad c - K c - c K^T = -(1/Wi) [I + alpha (c - I)](c - I),  K_ij = du_i/dx_j,
  and its image for Theta is -(1/Wi) e^{-Theta} [I + alpha (e^Theta - I)](e^Theta - I).
* Frames. The paper's grad u has entries du_j/dx_i, so its (grad u)^T in eq. NS23 is K:
  M = R^T K R with R the eigenvectors of Theta (equal to those of c).
* Equal eigenvalues. omega_ij = (lam_j m_ij + lam_i m_ji)/(lam_j - lam_i) (eq. NS24) is
  singular when lam_i = lam_j; the paper gives the rule for tau_p = 0 only (Omega = 0,
  B = sym K). Only the product omega_ij (theta_j - theta_i) enters RH, through the
  commutator Omega Theta - Theta Omega, and it has the finite limit m_ij + m_ji. The oracle
  forms that product as (lam_j m_ij + lam_i m_ji) (theta_j - theta_i)/(lam_j - lam_i), the
  last ratio evaluated as exp(-theta_i) d / expm1(d), d = theta_j - theta_i (its value 1 at
  d = 0): the paper's expression for distinct eigenvalues, its limit for equal ones, which for
  c = I is the paper's rule.
* Advection: the stress form's flux form, second-order central or (P.advection = 1) the
  paper's WENO-Z (weno.py), zero wall flux.
"""
from __future__ import annotations

import numpy as np

from . import discrete as D
from . import weno
from .model import Params

XX, YY, ZZ, XY, XZ, YZ = range(6)
_PAIRS = ((0, 0, XX), (1, 1, YY), (2, 2, ZZ), (0, 1, XY), (0, 2, XZ), (1, 2, YZ))


def to_matrix(comps):
    """Six symmetric components (xx, yy, zz, xy, xz, yz), each an array, -> (..., 3, 3)."""
    shape = np.shape(comps[0])
    m = np.empty(shape + (3, 3))
    for a, b, c in _PAIRS:
        m[..., a, b] = comps[c]
        m[..., b, a] = comps[c]
    return m


def from_matrix(m):
    return [np.ascontiguousarray(m[..., a, b]) for a, b, _ in _PAIRS]


def eig(theta_m):
    """Theta = R diag(theta) R^T (eq. NS43 / NS45): eigenvalues theta_i, columns of R."""
    return np.linalg.eigh(theta_m)


def source(theta_m, K, wi, alpha):
    """The non-advective part of RH (eq. NS41) at every point: Omega Theta - Theta Omega + 2 B
    minus the relaxation, for Theta (..., 3, 3) and K = grad u with K_ij = du_i/dx_j."""
    th, R = eig(theta_m)
    lam = np.exp(th)
    RT = np.swapaxes(R, -1, -2)
    M = RT @ K @ R                                       # eq. NS23
    # commutator in the eigenframe: entry (i, j) = omega_ij (theta_j - theta_i), eq. NS24
    C = np.zeros_like(M)
    for i in range(3):
        for j in range(3):
            if i == j:
                continue
            d = th[..., j] - th[..., i]
            ratio = np.exp(-th[..., i]) * np.where(d == 0.0, 1.0, d / np.where(d == 0.0, 1.0, np.expm1(d)))
            C[..., i, j] = (lam[..., j] * M[..., i, j] + lam[..., i] * M[..., j, i]) * ratio
    # 2 B: B = R diag(m_ii) R^T
    Bd = np.zeros_like(M)
    for i in range(3):
        Bd[..., i, i] = 2.0 * M[..., i, i]
    # relaxation e^{-Theta}[I + alpha (e^Theta - I)](e^Theta - I), diagonal in the eigenframe:
    # (1 - e^{-theta})(1 + alpha (e^theta - 1))
    rel = -np.expm1(-th) * (1.0 + alpha * np.expm1(th))
    Rd = np.zeros_like(M)
    for i in range(3):
        Rd[..., i, i] = rel[..., i] / wi
    return R @ (C + Bd - Rd) @ RT


def conformation(theta_m):
    """c = R diag(exp(theta)) R^T (eq. NS46)."""
    th, R = eig(theta_m)
    return (R * np.exp(th)[..., None, :]) @ np.swapaxes(R, -1, -2)


def stress(P: Params, theta_comps):
    """tau_p = (1 - beta)/Wi (c - I) (eq. NS17 in the scaling of model.py), with
    c - I = R diag(exp(theta) - 1) R^T (eq. NS46) and exp(theta) - 1 evaluated by expm1."""
    th, R = eig(to_matrix(theta_comps))
    cm = (R * np.expm1(th)[..., None, :]) @ np.swapaxes(R, -1, -2)
    return [(1.0 - P.beta) / P.wi * x for x in from_matrix(cm)]


def advection(P: Params, q, u, v, w):
    """-div(u q) in flux form with face-mean values (or the WENO-Z face values) and zero wall
    flux, as the stress form."""
    if P.advection == 1:
        return -weno.divergence(q, u, v, w, P.h, D)
    hx, hy, hz = P.h
    fx = u * 0.5 * (q + D.xp(q))
    fy = v * 0.5 * (q + D.yp(q))
    fz = w * 0.5 * (q + D.zp_neu(q))
    fz[-1] = 0.0
    return -((fx - D.xm(fx)) / hx + (fy - D.ym(fy)) / hy + (fz - D.zm_face(fz)) / hz)


def rhs(P: Params, theta, u, v, w, L):
    """RH of eq. NS41 for the six components of Theta; L[a][b] = du_b/dx_a at centres."""
    K = np.empty(np.shape(theta[0]) + (3, 3))
    for a in range(3):
        for b in range(3):
            K[..., b, a] = L[a][b]
    src = from_matrix(source(to_matrix(theta), K, P.wi, P.giesekus_alpha))
    return [advection(P, theta[c], u, v, w) + src[c] for c in range(6)]


def polymer(P: Params, theta_n, u, v, w, L):
    """Eqs. NS42-NS46: two TVD Runge-Kutta stages with u^{n+1} fixed, each diagonalising its
    own Theta; returns (Theta^{n+1}, tau_p^{n+1})."""
    rh0 = rhs(P, theta_n, u, v, w, L)
    t1 = [theta_n[c] + P.dt * rh0[c] for c in range(6)]
    rh1 = rhs(P, t1, u, v, w, L)
    t2 = [0.5 * theta_n[c] + 0.5 * (t1[c] + P.dt * rh1[c]) for c in range(6)]
    return t2, stress(P, t2)
