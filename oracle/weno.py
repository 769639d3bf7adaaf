"""Fifth-order WENO-Z advection (oracle; test infrastructure only).

The paper approximates the advection terms of eq. NS25 and of the polymer update (Sec. 3.2.3)
by the fifth-order WENO-Z scheme of Borges, Carmona, Costa and Don (2008). Written here from
that published method: at a face, the value is reconstructed from the five cell values of the
upwind-biased stencil as a convex combination of the three third-order candidates of Jiang and
Shu (1996), with the WENO-Z weights alpha_k = d_k (1 + tau5 / (beta_k + eps)), tau5 =
|beta_0 - beta_2|, exponent 1, ideal weights d = (1/10, 6/10, 3/10), eps = 1e-40. The face flux
is the face velocity times the value reconstructed on its upwind side, and the advection term
is the flux difference (conservative, like the central form it replaces).

Readings: the upwind side is taken from the sign of the face velocity (a zero velocity carries
no flux); beyond a wall the cell values are mirrored (the homogeneous Neumann extension of
cell-centred data, as the paper prescribes for the polymer at the walls), and the wall faces
carry no flux; x and y are periodic.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-40
D0, D1, D2 = 0.1, 0.6, 0.3


def candidates(vm2, vm1, v0, vp1, vp2):
    """The three third-order candidate values at the face between v0 and vp1."""
    q0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0
    q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0
    q2 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0
    return q0, q1, q2


def smoothness(vm2, vm1, v0, vp1, vp2):
    """Jiang-Shu smoothness indicators of the three candidate stencils."""
    b0 = 13.0 / 12.0 * (vm2 - 2.0 * vm1 + v0) ** 2 + 0.25 * (vm2 - 4.0 * vm1 + 3.0 * v0) ** 2
    b1 = 13.0 / 12.0 * (vm1 - 2.0 * v0 + vp1) ** 2 + 0.25 * (vm1 - vp1) ** 2
    b2 = 13.0 / 12.0 * (v0 - 2.0 * vp1 + vp2) ** 2 + 0.25 * (3.0 * v0 - 4.0 * vp1 + vp2) ** 2
    return b0, b1, b2


def reconstruct(vm2, vm1, v0, vp1, vp2):
    """Value at the face between v0 and vp1 from the side of v0 (upwind values vm2 .. vp2)."""
    q0, q1, q2 = candidates(vm2, vm1, v0, vp1, vp2)
    b0, b1, b2 = smoothness(vm2, vm1, v0, vp1, vp2)
    t5 = np.abs(b0 - b2)
    a0 = D0 * (1.0 + t5 / (b0 + EPS))
    a1 = D1 * (1.0 + t5 / (b1 + EPS))
    a2 = D2 * (1.0 + t5 / (b2 + EPS))
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def _shift(q, s, axis, wall):
    """q at index i + s along `axis`: periodic, or mirrored beyond the walls."""
    if not wall:
        return np.roll(q, -s, axis=axis)
    n = q.shape[axis]
    idx = np.arange(n) + s
    idx = np.where(idx < 0, -idx - 1, idx)
    idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
    return np.take(q, idx, axis=axis)


def face_flux(q, u, axis, wall):
    """u q_face at the faces i + 1/2 along `axis` (u given there), upwind WENO-Z value."""
    v = {s: _shift(q, s, axis, wall) for s in range(-2, 4)}
    pos = reconstruct(v[-2], v[-1], v[0], v[1], v[2])
    neg = reconstruct(v[3], v[2], v[1], v[0], v[-1])
    return u * np.where(u > 0.0, pos, neg)


def divergence(q, u, v, w, h, D):
    """div(u q) with WENO-Z face values: x, y periodic; no flux through the walls (the top
    z face of the last cell is the wall, the bottom wall face is implicit)."""
    hx, hy, hz = h
    fx = face_flux(q, u, 2, False)
    fy = face_flux(q, v, 1, False)
    fz = face_flux(q, w, 0, True)
    fz[-1] = 0.0
    return (fx - D.xm(fx)) / hx + (fy - D.ym(fy)) / hy + (fz - D.zm_face(fz)) / hz
