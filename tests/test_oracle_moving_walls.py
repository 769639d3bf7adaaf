"""Pins of the oracle's wall data: moving no-slip walls (eq. NS13, u = u_w) and inhomogeneous
wall data of the constant-coefficient solves.

* The solves with wall data satisfy their stencil cell by cell, with the ghosts written out
  explicitly by loops (Neumann: adjacent + hz g; no-slip: 2 u_w - adjacent; face-located:
  the wall value itself).
* Plane Couette flow: between walls moving with different velocities in x and y, the linear
  profile is an exact steady state of the discrete step (the no-slip ghost makes the
  discrete Laplacian of a linear profile vanish); with an Oldroyd-B drop phase the steady
  stresses tau_xz = (1-beta) g_x, tau_yz = (1-beta) g_y, tau_xx = 2 Wi (1-beta) g_x^2,
  tau_yy = 2 Wi (1-beta) g_y^2, tau_xy = 2 Wi (1-beta) g_x g_y make it a steady state too.
* Started from rest, the flow reaches that profile.
"""
from __future__ import annotations

import types
from pathlib import Path

import numpy as np
import pytest

from oracle import discrete as D
from oracle import model
from oracle import step as S


# --------------------------------------------------------------------------------------
# constant-coefficient solves with wall data
# --------------------------------------------------------------------------------------


def _loop_residual(x, rhs, coeff, shift, kind, h, walls):
    """coeff * L x - shift * x - rhs, cell by cell, with explicit ghosts."""
    nz, ny, nx = x.shape
    hx, hy, hz = h
    gb, gt = walls
    out = np.zeros_like(x)
    nzu = nz - 1 if kind == "wface" else nz
    for k in range(nzu):
        for j in range(ny):
            for i in range(nx):
                c = x[k, j, i]
                s = (x[k, j, (i + 1) % nx] - 2 * c + x[k, j, (i - 1) % nx]) / hx ** 2
                s += (x[k, (j + 1) % ny, i] - 2 * c + x[k, (j - 1) % ny, i]) / hy ** 2
                if kind == "neumann":
                    up = x[k + 1, j, i] if k + 1 < nz else c + hz * gt[j, i]
                    dn = x[k - 1, j, i] if k > 0 else c + hz * gb[j, i]
                elif kind == "dirichlet":
                    up = x[k + 1, j, i] if k + 1 < nz else 2 * gt[j, i] - c
                    dn = x[k - 1, j, i] if k > 0 else 2 * gb[j, i] - c
                else:  # face-located: faces k = 0..nz-2 inside, wall faces at z = 0, lz
                    up = x[k + 1, j, i] if k + 1 < nz - 1 else gt[j, i]
                    dn = x[k - 1, j, i] if k > 0 else gb[j, i]
                s += (up - 2 * c + dn) / hz ** 2
                out[k, j, i] = coeff * s - shift * c - rhs[k, j, i]
    return out


@pytest.mark.parametrize("kind,shift", [("neumann", 2.5), ("neumann", 0.0), ("dirichlet", 4.0),
                                        ("wface", 3.0)])
@pytest.mark.parametrize("shape", [(6, 4, 8), (5, 1, 8)])
def test_helmholtz_with_wall_data(kind, shift, shape):
    rng = np.random.default_rng(23)
    h = (0.13, 0.21, 0.17)
    coeff = 0.8
    rhs = rng.standard_normal(shape)
    gb = rng.standard_normal(shape[1:])
    gt = rng.standard_normal(shape[1:])
    if kind == "neumann" and shift == 0.0:
        # solvable only if the data balance: sum(rhs) = coeff * (sum of the boundary fluxes)
        rhs += coeff * (gb.sum() + gt.sum()) / (shape[0] * h[2] * gb.size) - rhs.mean()
    x = D.helmholtz(rhs, coeff, shift, kind, h, walls=(gb, gt))
    res = _loop_residual(x, rhs, coeff, shift, kind, h, (gb, gt))
    assert np.max(np.abs(res)) <= 1e-11 * np.max(np.abs(rhs)) * max(1.0, coeff / min(h) ** 2)
    if kind == "wface":
        assert np.array_equal(x[-1], gt)
    if kind == "neumann" and shift == 0.0:
        assert abs(x.mean()) < 1e-13 * np.max(np.abs(x))
    # zero wall data: the homogeneous solve, bit for bit
    z = np.zeros(shape[1:])
    x0 = D.helmholtz(rhs, coeff, shift, kind, h, walls=(z, z))
    xh = D.helmholtz(rhs, coeff, shift, kind, h)
    assert np.array_equal(x0[:-1] if kind == "wface" else x0, xh[:-1] if kind == "wface" else xh)


# --------------------------------------------------------------------------------------
# plane Couette flow
# --------------------------------------------------------------------------------------

UB, UT = (0.3, -0.4), (1.1, 0.6)


def _couette_params(ny, viscoelastic, dt=1e-3, **kw):
    base = dict(nx=8, ny=ny, nz=12, lx=1.0, ly=0.5 if ny > 1 else 1.0 / 8, lz=1.0, re=2.0,
                ca=0.5, cn=0.05, pe=50.0, dt=dt, rho_ratio=3.0, mu_ratio=2.0, wi=0.8, beta=0.4,
                viscoelastic=viscoelastic,
                u_wall_bottom=UB if ny > 1 else (UB[0], 0.0),
                u_wall_top=UT if ny > 1 else (UT[0], 0.0))
    base.update(kw)
    return model.Params(**base)


def _couette_state(P, phase, step, stresses):
    cs = P.coarse_shape
    z = (np.arange(P.nz) + 0.5) * P.h[2] / P.lz
    gx = (P.u_wall_top[0] - P.u_wall_bottom[0]) / P.lz
    gy = (P.u_wall_top[1] - P.u_wall_bottom[1]) / P.lz
    u = np.broadcast_to((P.u_wall_bottom[0] + gx * z * P.lz)[:, None, None], cs).copy()
    v = np.broadcast_to((P.u_wall_bottom[1] + gy * z * P.lz)[:, None, None], cs).copy()
    zero = lambda: np.zeros(cs)
    tau = [zero() for _ in range(6)]
    if stresses:
        c = 1.0 - P.beta
        full = lambda val: np.full(cs, val)
        tau = [full(2 * P.wi * c * gx * gx), full(2 * P.wi * c * gy * gy), zero(),
               full(2 * P.wi * c * gx * gy), full(c * gx), full(c * gy)]
    phi = np.full(P.fine_shape, float(phase))
    return {"phi": [phi, phi.copy()], "u": [u, u.copy()], "v": [v, v.copy()],
            "w": [zero(), zero()], "p": [zero(), zero()],
            "tau": [tau, [t.copy() for t in tau]], "step": step}


@pytest.mark.parametrize("step", [0, 3], ids=["first", "bdf2"])
@pytest.mark.parametrize("ny,viscoelastic,phase", [(4, 0, -1.0), (1, 0, 1.0), (4, 1, 1.0),
                                                   (1, 1, 1.0), (4, 1, -1.0)])
def test_couette_steady_state(step, ny, viscoelastic, phase, mod=S):
    P = _couette_params(ny, viscoelastic)
    st = _couette_state(P, phase, step, bool(viscoelastic))
    new = mod.step(P, st)
    scale = max(abs(x) for x in UB + UT)
    for f in ("u", "v"):
        assert np.max(np.abs(new[f][0] - st[f][0])) <= 1e-12 * scale, f
    assert np.max(np.abs(new["w"][0])) <= 1e-12 * scale
    assert np.max(np.abs(new["p"][0] - new["p"][0].mean())) <= 1e-10 * scale
    if viscoelastic:
        tmax = max(np.max(np.abs(t)) for t in st["tau"][0])
        for m in range(6):
            assert np.max(np.abs(new["tau"][0][m] - st["tau"][0][m])) <= 1e-12 * tmax, m


def test_couette_start_up():
    """From rest the flow settles on the linear profile (the slowest mode decays as
    exp(-pi^2 nu t / lz^2); after t = 4 it is below 1e-15 of the wall speed)."""
    P = _couette_params(4, 0, dt=0.02, rho_ratio=1.0, mu_ratio=1.0, re=1.0)
    target = _couette_state(P, -1.0, 0, False)
    st = _couette_state(P, -1.0, 0, False)
    for f in ("u", "v"):
        st[f] = [np.zeros(P.coarse_shape), np.zeros(P.coarse_shape)]
    st = S.run(P, st, 200)
    for f in ("u", "v"):
        assert np.max(np.abs(st[f][0] - target[f][0])) < 1e-9, f


def _mutant(old, new):
    src = Path(S.__file__).read_text()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle._step_mutant")
    mod.__package__ = "oracle"
    mod.__file__ = S.__file__
    exec(compile(src.replace(old, new), S.__file__ + "<mutant>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("old,new", [
    # the wall velocity left out of the implicit Helmholtz solve of eq. NS36
    ("walls = (lambda c: P.walls(c)) if P.moving_walls else (lambda c: None)",
     "walls = lambda c: None"),
    # the explicit viscous Laplacian with walls at rest
    ("D.lap_dirichlet(us, P.h, uw)", "D.lap_dirichlet(us, P.h)"),
], ids=["implicit-wall-data", "explicit-laplacian"])
def test_couette_catches_planted_mistake(old, new):
    with pytest.raises(AssertionError):
        test_couette_steady_state(3, 4, 0, -1.0, mod=_mutant(old, new))


@pytest.mark.parametrize("old,new", [
    # the wall advection of eq. NS34 left out, or with the wrong sign
    ("            bR[layer] -= (P.d_w / hz) * adv\n", "            pass\n"),
    ("            bR[layer] -= (P.d_w / hz) * adv\n", "            bR[layer] += (P.d_w / hz) * adv\n"),
    # the other wall's velocity
    ("            adv = P.walls(0)[side] * dx + P.walls(1)[side] * dy\n",
     "            adv = P.walls(0)[1 - side] * dx + P.walls(1)[1 - side] * dy\n"),
    # x and y derivatives exchanged
    ("            adv = P.walls(0)[side] * dx + P.walls(1)[side] * dy\n",
     "            adv = P.walls(0)[side] * dy + P.walls(1)[side] * dx\n"),
], ids=["dropped", "sign", "other-wall", "swapped-axes"])
def test_relaxed_moving_walls_catch_planted_mistake(old, new):
    """The cell-by-cell NS25/NS34 residual with moving, relaxed walls sees each mistake."""
    from tests import test_oracle_pins as pins
    with pytest.raises(AssertionError):
        pins.test_ch_solves_unsplit_equation(2, False, 0.05, True, mod=_mutant(old, new))


def test_relaxed_moving_walls_couette_and_mass():
    """Relaxed walls with moving walls: a flat phase field has no tangential gradient on the
    walls, so plane Couette flow stays on its linear profile as with static walls; a drop
    conserves its mass to round-off. The differentiable step still refuses the combination."""
    P = _couette_params(4, 0, d_w=0.1)
    st = _couette_state(P, -1.0, 3, False)
    new = S.step(P, st)
    scale = max(abs(x) for x in UB + UT)
    for f in ("u", "v"):
        assert np.max(np.abs(new[f][0] - st[f][0])) <= 1e-12 * scale, f
    assert np.max(np.abs(new["phi"][0] - st["phi"][0])) <= 1e-13
    import workloads as W
    cfg = W.config("C2", nx=8, ny=4, nz=8, lx=1.0, ly=0.5, lz=0.5, radius=0.25, noise=1e-3, seed=3,
                   d_w=0.2, u_wall_bottom=(0.5, -0.3), u_wall_top=(-0.4, 0.2))
    P = model.Params.from_config(cfg)
    st = W.droplet_state(cfg)
    m0 = np.sum(st["phi"][0])
    for _ in range(4):
        st = S.step(P, st)
    assert abs(np.sum(st["phi"][0]) - m0) < 1e-11 * np.sum(np.abs(st["phi"][0]))
    from oracle import adjoint as A
    with pytest.raises(NotImplementedError):
        A.step(P, st, None, None, None)
