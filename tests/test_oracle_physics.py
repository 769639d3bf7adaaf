"""Physics pins of the FP64 oracle: the capillary scaling through the Laplace pressure jump of
a free drop, and the static wetting condition through the equilibrium cap of a drop on a
wall (closed form of eq. NS48 and the cap angle)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W
from oracle import model
from oracle import step as S


def _drop_state(cfg, P, xc, zc, R):
    st = W.droplet_state(cfg)
    nzf, nyf, nxf = P.fine_shape
    hx, _, hz = P.hf
    x = (np.arange(nxf) + 0.5) * hx
    z = (np.arange(nzf) + 0.5) * hz
    zz, xx = np.meshgrid(z, x, indexing="ij")
    r = np.sqrt((xx - xc) ** 2 + (zz - zc) ** 2)
    phi = np.tanh((R - r) / (math.sqrt(2.0) * cfg.cn))[:, None, :]
    st["phi"] = [phi.copy(), phi.copy()]
    return st


def test_laplace_pressure_jump_free_drop():
    """2D drop of radius R in the middle of the box: p_in - p_out = sigma / R, i.e.
    1 / (Re Ca R) in these units (K_sigma and the capillary force G grad(phi))."""
    R = 0.25
    cfg = W.Config(name="laplace", nx=64, ny=1, nz=64, lx=1.0, ly=1.0 / 64, lz=1.0, re=10.0,
                   ca=1.0, cn=0.02, pe=150.0, dt=1e-3, radius=R)
    P = model.Params.from_config(cfg)
    st = _drop_state(cfg, P, 0.5, 0.5, R)
    st = S.run(P, st, 200)
    p = st["p"][0][:, 0, :]
    nz, nx = p.shape
    p_in = p[nz // 2 - 2:nz // 2 + 2, nx // 2 - 2:nx // 2 + 2].mean()
    p_out = np.mean([p[1, 1], p[1, -2], p[-2, 1], p[-2, -2]])
    jump = (p_in - p_out) * cfg.re * cfg.ca * R
    assert abs(jump - 1.0) < 0.03, jump
    o = S.observables(P, st)
    assert o["kinetic_energy"] < 1e-8


def _cap_measure(P, st):
    phi = st["phi"][0][:, 0, :]
    hx, _, hz = P.hf
    col = phi[:, phi.shape[1] // 2]
    k = int(np.where(col < 0)[0][0])
    z0, z1 = (k - 0.5) * hz, (k + 0.5) * hz
    H = z0 + (z1 - z0) * col[k - 1] / (col[k - 1] - col[k])
    w = phi[0]
    cross = []
    for i in np.where(np.diff(np.sign(w)) != 0)[0]:
        xa, xb = (i + 0.5) * hx, (i + 1.5) * hx
        cross.append(xa + (xb - xa) * w[i] / (w[i] - w[i + 1]))
    L = cross[-1] - cross[0]
    area = float(np.sum(0.5 * (1.0 + phi))) * hx * hz
    return H, L, area


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_equilibrium_cap(theta):
    """A half-circle drop (90 deg) relaxes on a wall with static angle theta (eqs. NS15-NS16,
    D_w = 0). At equilibrium the cap angle 2 atan(2H/L) equals theta, and height and
    wetted length follow eq. NS48 for the drop's own area (within the shrinkage of a diffuse
    interface of width Cn/R0 = 0.1)."""
    R0 = 0.4
    cfg = W.Config(name="cap", nx=64, ny=1, nz=32, lx=2.0, ly=2.0 / 64, lz=1.0, re=10.0, ca=1.0,
                   cn=0.04, pe=75.0, dt=1e-2, radius=R0, theta_bottom_deg=theta,
                   rho_ratio=1.1, mu_ratio=1.1)
    P = model.Params.from_config(cfg)
    st = S.run(P, W.droplet_state(cfg), 2000)
    assert S.observables(P, st)["kinetic_energy"] < 1e-8
    H, L, area = _cap_measure(P, st)
    fit = math.degrees(2.0 * math.atan(2.0 * H / L))
    assert abs(fit - theta) < 2.0, fit
    t = math.radians(theta)
    # eq. NS48 written for the area A of the drop: R^2 (t - sin t cos t) = A
    R = math.sqrt(area / (t - math.sin(t) * math.cos(t)))
    assert H == pytest.approx(R * (1 - math.cos(t)), rel=0.08)
    assert L == pytest.approx(2 * R * math.sin(t), rel=0.08)
    # with the nominal area pi R0^2 / 2 eq. NS48 reads as printed
    fac = math.sqrt(math.pi / (2 * (t - math.sin(t) * math.cos(t))))
    assert H == pytest.approx(R0 * (1 - math.cos(t)) * fac, rel=0.12)
    assert L == pytest.approx(2 * R0 * math.sin(t) * fac, rel=0.12)
