"""Pins of the oracle's adjoint (oracle/adjoint.py) against things other than itself:

* its differentiable step reproduces the NumPy oracle step (independent code, pinned by
  test_oracle_pins.py and test_oracle_physics.py) to round-off;
* its state adjoint satisfies <lam, J v> = <J^T lam, v> with J v taken by central
  differences of the NumPy oracle step along seeded directions v;
* its parameter gradients through many steps equal central differences of the NumPy oracle
  trajectory in the bottom static angle, Pe and Wi;
* all three also with relaxed walls (D_w > 0) and with WENO-Z advection, the first two also
  with the Giesekus term of the stress form and with moving walls, whose NumPy steps are
  pinned separately (test_oracle_wall_relaxation.py, test_oracle_weno.py, test_oracle_lcr.py,
  test_oracle_moving_walls.py).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import model
from oracle import step as S

FIELDS = ("phi", "u", "v", "w", "p")

CASES = [("C4", dict(nx=16, nz=8, noise=1e-2)), ("C1", dict(nx=16, nz=8, noise=1e-2)),
         ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2)), ("C2", dict(nx=8, ny=4, nz=8, noise=0.0))]
# relaxed walls (D_w > 0, eqs. NS15, NS33, NS34): 2D Oldroyd-B, 3D Oldroyd-B with strong
# relaxation, 3D Newtonian with the C2R value
RELAXED = [("C4", dict(nx=16, nz=8, noise=1e-2, d_w=0.5)), ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2, d_w=2.0)),
           ("C2", dict(nx=8, ny=4, nz=8, noise=0.0, d_w=0.1))]
RELAXED_IDS = ["C4-dw0.5", "C3-dw2", "C2-dw0.1"]
# WENO-Z advection of the phase field and of the stress (advection 1, Sec. 3.2.3)
WENO = [("C4", dict(nx=16, nz=8, noise=1e-2, advection=1)), ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2, advection=1)),
        ("C2", dict(nx=8, ny=4, nz=8, noise=0.0, advection=1)),
        ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2, advection=1, d_w=0.5))]
WENO_IDS = ["C4-weno", "C3-weno", "C2-weno", "C3-weno-dw0.5"]
# Giesekus in the stress form (eq. NS4 with alpha > 0): 2D and 3D, the latter with WENO-Z
GIESEKUS = [("C4", dict(nx=16, nz=8, noise=1e-2, giesekus_alpha=0.3)),
            ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2, giesekus_alpha=0.2, advection=1))]
GIESEKUS_IDS = ["C4-giesekus", "C3-giesekus-weno"]
# moving walls (eq. NS13, u = u_w on the walls): 2D, 3D Oldroyd-B, 3D Newtonian with contrast
MOVING = [("C4", dict(nx=16, nz=8, noise=1e-2, u_wall_bottom=(0.3, 0.0), u_wall_top=(-0.5, 0.0))),
          ("C3", dict(nx=8, ny=4, nz=8, noise=1e-2, u_wall_bottom=(0.2, -0.1), u_wall_top=(-0.3, 0.4))),
          ("C2", dict(nx=8, ny=4, nz=8, noise=1e-4, u_wall_top=(0.5, 0.2)))]
MOVING_IDS = ["C4-moving", "C3-moving", "C2-moving"]


def _flat(st, ve):
    xs = [st[f][l] for f in FIELDS for l in range(2)]
    if ve:
        xs += [st["tau"][l][c] for l in range(2) for c in range(6)]
    return xs


@pytest.mark.parametrize("name,kw", CASES + RELAXED + WENO + GIESEKUS + MOVING,
                         ids=[c[0] for c in CASES] + RELAXED_IDS + WENO_IDS + GIESEKUS_IDS + MOVING_IDS)
def test_differentiable_step_equals_numpy_step(name, kw):
    import torch
    cfg = W.config(name, **kw)
    P = model.Params.from_config(cfg)
    st = W.droplet_state(cfg)
    th = torch.tensor(math.radians(P.theta_bottom_deg), dtype=torch.float64)
    pe = torch.tensor(P.pe, dtype=torch.float64)
    wi = torch.tensor(P.wi, dtype=torch.float64)
    for _ in range(3):
        ref = S.step(P, st)
        got = OA.step(P, OA.to_torch(st), th, pe, wi)
        for a, b in zip(_flat(ref, P.viscoelastic), OA.flat(got)[:len(_flat(ref, P.viscoelastic))]):
            scale = max(float(np.max(np.abs(a))), 1e-300)
            assert float(np.max(np.abs(b.numpy() - a))) <= 1e-10 * scale
        st = ref


def _perturbed(st, v, eps, ve):
    out = {f: [st[f][l] + eps * v[f][l] for l in range(2)] for f in FIELDS}
    out["tau"] = [[st["tau"][l][c] + (eps * v["tau"][l][c] if ve else 0.0) for c in range(6)]
                  for l in range(2)]
    out["step"] = st["step"]
    return out


def _inner(a, b, ve):
    return sum(float(np.sum(x * y)) for x, y in zip(_flat(a, ve), _flat(b, ve)))


@pytest.mark.parametrize("name,kw", CASES[:3] + RELAXED[:2] + WENO[:2] + WENO[3:] + GIESEKUS + MOVING[:2],
                         ids=[c[0] for c in CASES[:3]] + RELAXED_IDS[:2] + WENO_IDS[:2] + WENO_IDS[3:] + GIESEKUS_IDS
                         + MOVING_IDS[:2])
def test_state_adjoint_dot_product(name, kw):
    """<lam, (step(x + e v) - step(x - e v)) / 2e> = <adjoint_step(lam), v> (NumPy step for the
    directional derivative)."""
    cfg = W.config(name, **kw)
    P = model.Params.from_config(cfg)
    ve = bool(P.viscoelastic)
    st = S.run(P, W.droplet_state(cfg), 2)
    lam = W.adjoint_seed(cfg, 3)
    v = W.adjoint_seed(cfg, 4)
    for l in range(2):           # the top-wall w is identically zero in every state
        v["w"][l][-1] = 0.0
    adj, _ = OA.adjoint_step(P, st, lam)
    rhs = _inner(adj, v, ve)
    eps = 1e-6
    sp, sm = S.step(P, _perturbed(st, v, eps, ve)), S.step(P, _perturbed(st, v, -eps, ve))
    lhs = (_inner(lam, sp, ve) - _inner(lam, sm, ve)) / (2 * eps)
    assert abs(lhs - rhs) <= 1e-6 * max(abs(rhs), 1e-30), (lhs, rhs)


def test_parameter_gradients_vs_central_differences():
    """20 steps of a fast-spreading 2D viscoelastic drop: d(wetted radius)/d(theta, Pe, Wi)
    by reverse differentiation equals central differences (relative step 1e-4) of the NumPy
    oracle trajectory to 1e-7."""
    cfg = W.config("C4", nx=32, nz=16, cn=0.04, pe=75.0, dt=5e-3, noise=0.0)
    P = model.Params.from_config(cfg)
    st0 = W.droplet_state(cfg)
    N = 20
    _, g = OA.trajectory_gradient(P, st0, N, OA.wetted_radius)

    def J(P2):
        return S.observables(P2, S.run(P2, st0, N))["wetted_radius"]

    th0 = math.radians(P.theta_bottom_deg)
    for a, (x0, mk) in enumerate((
            (th0, lambda x: dataclasses.replace(P, theta_bottom_deg=math.degrees(x))),
            (P.pe, lambda x: dataclasses.replace(P, pe=x)),
            (P.wi, lambda x: dataclasses.replace(P, wi=x)))):
        e = 1e-4 * x0
        fd = (J(mk(x0 + e)) - J(mk(x0 - e))) / (2 * e)
        assert abs(fd - g[a]) <= 1e-7 * abs(g[a]), (a, fd, g[a])


def test_parameter_gradients_relaxed_walls_vs_central_differences():
    """The same check with relaxed walls (D_w = 0.5): 10 steps, d(wetted radius)/d(theta, Pe,
    Wi) by reverse differentiation against central differences of the NumPy oracle."""
    cfg = W.config("C4", nx=32, nz=16, cn=0.04, pe=75.0, dt=5e-3, noise=0.0, d_w=0.5)
    P = model.Params.from_config(cfg)
    st0 = W.droplet_state(cfg)
    N = 10
    _, g = OA.trajectory_gradient(P, st0, N, OA.wetted_radius)

    def J(P2):
        return S.observables(P2, S.run(P2, st0, N))["wetted_radius"]

    th0 = math.radians(P.theta_bottom_deg)
    for a, (x0, mk) in enumerate((
            (th0, lambda x: dataclasses.replace(P, theta_bottom_deg=math.degrees(x))),
            (P.pe, lambda x: dataclasses.replace(P, pe=x)),
            (P.wi, lambda x: dataclasses.replace(P, wi=x)))):
        e = 1e-4 * x0
        fd = (J(mk(x0 + e)) - J(mk(x0 - e))) / (2 * e)
        assert abs(fd - g[a]) <= 1e-7 * abs(g[a]), (a, fd, g[a])


def test_parameter_gradients_weno_vs_central_differences():
    """The same check with WENO-Z advection of the phase field and the stress: 10 steps. The
    WENO-Z weights are not differentiable where |beta_0 - beta_2| changes sign or a face
    velocity does, so J is smooth only piecewise in the parameters. dJ/dWi is small here
    ((Wi/J) dJ/dWi ~ 7e-5) and its central differences at relative steps 1e-5 .. 1e-3 scatter
    by up to 2e-6 relative around the reverse-mode value (measured) instead of converging:
    its bound is 5e-6; theta and Pe keep 1e-7."""
    cfg = W.config("C4", nx=32, nz=16, cn=0.04, pe=75.0, dt=5e-3, noise=0.0, advection=1)
    P = model.Params.from_config(cfg)
    st0 = W.droplet_state(cfg)
    N = 10
    _, g = OA.trajectory_gradient(P, st0, N, OA.wetted_radius)

    def J(P2):
        return S.observables(P2, S.run(P2, st0, N))["wetted_radius"]

    th0 = math.radians(P.theta_bottom_deg)
    for a, (x0, mk) in enumerate((
            (th0, lambda x: dataclasses.replace(P, theta_bottom_deg=math.degrees(x))),
            (P.pe, lambda x: dataclasses.replace(P, pe=x)),
            (P.wi, lambda x: dataclasses.replace(P, wi=x)))):
        e = 1e-4 * x0
        fd = (J(mk(x0 + e)) - J(mk(x0 - e))) / (2 * e)
        assert abs(fd - g[a]) <= (5e-6 if a == 2 else 1e-7) * abs(g[a]), (a, fd, g[a])


def test_newtonian_has_no_wi_gradient():
    cfg = W.config("C1", nx=16, nz=8, noise=1e-2)
    P = model.Params.from_config(cfg)
    _, g = OA.adjoint_step(P, W.droplet_state(cfg), W.adjoint_seed(cfg, 1))
    assert g[2] == 0.0 and g[0] != 0.0 and g[1] != 0.0
