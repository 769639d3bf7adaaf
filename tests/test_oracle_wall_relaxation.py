"""Pins of the oracle's wall relaxation (eq. NS15 with D_w > 0, discretised as eq. NS34)
against things other than itself. The cell-by-cell residual of the unsplit eq. NS25 with the
relaxed ghost, and the Robin solve against a dense loop-built operator, are in
test_oracle_pins.py; here:

* mass is conserved: the outer operator keeps zero-flux walls whatever D_w;
* second order in time with a wall term strong enough to change the solution at O(1): the
  implicit wall derivative is the BDF2 one of eq. NS31, so halving dt divides the error by
  four;
* the limit of large D_w: the wall condition forces (d phi / dt) = 0 on the wall-adjacent
  cells, which then keep their initial values while the interior moves;
* relaxation retards the wall: the change of the wall-adjacent layer over a fixed time
  decreases monotonically with D_w (the paper's statement about eq. NS15), and D_w -> 0
  approaches the static-angle step.
"""
from __future__ import annotations

import math

import numpy as np

import workloads as W
from oracle import model
from oracle import step as S


def _drop(d_w, dt=2e-4, **kw):
    base = dict(nx=16, ny=1, nz=8, lx=2.0, ly=2.0 / 16, lz=1.0, re=10.0, ca=0.1, cn=0.05,
                pe=10.0, dt=dt, theta_bottom_deg=45.0, theta_top_deg=120.0, d_w=d_w)
    base.update(kw)
    return model.Params(**base)


def _state(P, radius=0.5, seed=3):
    cfg = W.config("C1", nx=P.nx, ny=P.ny, nz=P.nz, lx=P.lx, ly=P.ly, lz=P.lz, radius=radius,
                   noise=0.0, seed=seed)
    return W.droplet_state(cfg)


def _ch_only(P, st, nsteps):
    """Cahn-Hilliard steps with the fluid at rest (the wall dynamics in isolation)."""
    st = dict(st)
    for _ in range(nsteps):
        C = model.constants(P, st["step"] == 0)
        phi, _, _, _ = S.cahn_hilliard(P, st, C)
        st = dict(st, phi=[phi, st["phi"][0]], step=st["step"] + 1)
    return st


def test_mass_conserved_with_relaxation():
    P = _drop(0.3)
    st = _state(P)
    m0 = float(np.sum(st["phi"][0]))
    out = S.run(P, st, 6)
    assert abs(float(np.sum(out["phi"][0])) - m0) < 1e-12 * float(np.sum(np.abs(out["phi"][0])))


def test_second_order_in_time():
    """Self-convergence at fixed S (the stabilisation is held constant across dt, as in the
    linear-mode test of the static scheme): errors against a 16x finer dt shrink by ~4. With
    D_w = 2 the final phase field differs from the static one by 0.3."""
    T, d_w = 0.02, 2.0
    P0 = _drop(d_w, dt=T / 1280)
    s_fixed = 1.2 * P0.cn * math.sqrt(4 * 1.5 * P0.pe / P0.dt)   # the bound at the smallest dt

    def run(n, dw=d_w):
        dt = T / n
        sf = s_fixed / (P0.cn * math.sqrt(4 * 1.5 * P0.pe / dt))
        assert sf >= 1.0
        P = _drop(dw, dt=dt, s_factor=sf)
        return _ch_only(P, _state(P), n)["phi"][0]

    ref = run(1280)
    errs = [float(np.max(np.abs(run(n) - ref))) for n in (80, 160, 320)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.6 and 3.6 < r2 < 4.6, errs
    assert float(np.max(np.abs(ref - run(1280, 0.0)))) > 100 * errs[0]


def test_large_relaxation_freezes_the_wall_layer():
    P = _drop(1e9)
    st = _state(P)
    out = _ch_only(P, st, 8)
    wall = [0, -1]
    dwall = float(np.max(np.abs(out["phi"][0][wall] - st["phi"][0][wall])))
    dint = float(np.max(np.abs(out["phi"][0][1:-1] - st["phi"][0][1:-1])))
    assert dint > 1e-3
    assert dwall < 1e-6 * dint


def test_relaxation_retards_the_wall_and_vanishes_at_zero():
    changes = []
    for d_w in (0.0, 0.01, 0.1, 1.0):
        P = _drop(d_w)
        st = _state(P)
        out = _ch_only(P, st, 10)
        changes.append(float(np.max(np.abs(out["phi"][0][0] - st["phi"][0][0]))))
    assert all(a > b for a, b in zip(changes, changes[1:])), changes
    # D_w -> 0 is continuous with the static scheme
    P, P0 = _drop(1e-9), _drop(0.0)
    a = _ch_only(P, _state(P), 4)["phi"][0]
    b = _ch_only(P0, _state(P0), 4)["phi"][0]
    assert float(np.max(np.abs(a - b))) < 1e-6
