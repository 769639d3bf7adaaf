"""Pins of the oracle's WENO-Z advection (oracle/weno.py) against things other than itself:

* the face value is the exact face value of the primitive for quadratic data (all three
  candidates agree, so the weights do not matter): for p(x) = x^2 sampled at x_j = j h, the
  face value at h/2 is h^2/4 - h^2/12 = h^2/6;
* the flux difference of a smooth periodic field converges to u q' at fifth order (both
  velocity signs), which a wrong candidate coefficient or smoothness indicator would break;
* at a jump the face values stay within the data (no new extrema) and pick the smooth side;
* the flux form conserves: the periodic sum of the divergence is zero, and the coupled step
  with WENO-Z advection conserves the phase-field mass;
* the mirror ghost at a wall: a field constant in z carries w q through every face, and a
  wall-bounded column equals the upper half of its even periodic extension (both walls).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W
from oracle import discrete as D
from oracle import model
from oracle import step as S
from oracle import weno


def _quadratic_with_averages(vals, h, cells):
    """Coefficients (c0, c1, c2) of p(x) = c0 + c1 x + c2 x^2 whose averages over the cells
    [(j - 1/2) h, (j + 1/2) h], j in `cells`, equal `vals` (a 3x3 solve)."""
    A = np.array([[1.0, j * h, (j * h) ** 2 + h * h / 12.0] for j in cells])
    return np.linalg.solve(A, np.array(vals, dtype=float))


def test_candidates_and_smoothness_from_the_stencil_polynomials():
    """Each candidate is the face value (x = h/2) of the quadratic with the stencil's three
    values as cell averages; each smoothness indicator is h int (p')^2 + h^3 int (p'')^2 over
    the cell [-h/2, h/2] (Jiang-Shu)."""
    rng = np.random.default_rng(13)
    h = 0.3
    for _ in range(5):
        v = list(rng.standard_normal(5))   # cells -2 .. 2
        q = weno.candidates(*v)
        b = weno.smoothness(*v)
        for k, cells in enumerate(((-2, -1, 0), (-1, 0, 1), (0, 1, 2))):
            c0, c1, c2 = _quadratic_with_averages([v[j + 2] for j in cells], h, cells)
            assert q[k] == pytest.approx(c0 + c1 * h / 2 + c2 * h * h / 4, rel=1e-12, abs=1e-12)
            # int_{-h/2}^{h/2} (c1 + 2 c2 x)^2 dx = h c1^2 + c2^2 h^3 / 3; (p'')^2 = 4 c2^2
            beta = h * (h * c1 * c1 + c2 * c2 * h ** 3 / 3.0) + h ** 3 * (4.0 * c2 * c2 * h)
            assert b[k] == pytest.approx(beta, rel=1e-12, abs=1e-14)


def test_flux_takes_the_upwind_side():
    q = np.zeros((1, 1, 8))
    q[..., 4:] = 1.0
    for sign in (1.0, -1.0):
        u = np.full((1, 1, 8), sign)
        F = weno.face_flux(q, u, 2, False)[0, 0]
        # face 3 | 4 (0 on the left, 1 on the right) and face 7 | 0 (1 left, 0 right)
        assert F[3] == pytest.approx(0.0 if sign > 0 else -1.0, abs=1e-12)
        assert F[7] == pytest.approx(1.0 if sign > 0 else 0.0, abs=1e-12)


def test_quadratic_face_value_exact():
    for h in (0.1, 0.37):
        v = [(s * h) ** 2 for s in (-2, -1, 0, 1, 2)]
        assert weno.reconstruct(*v) == pytest.approx(h * h / 6.0, rel=1e-14)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_fifth_order_convergence(sign):
    errs = []
    for n in (40, 80, 160):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        q = np.sin(2 * math.pi * x)
        u = np.full(n, sign)
        F = weno.face_flux(q[None, None, :], u[None, None, :], 2, False)[0, 0]
        div = (F - np.roll(F, 1)) / h
        errs.append(float(np.max(np.abs(div - sign * 2 * math.pi * np.cos(2 * math.pi * x)))))
    for a, b in zip(errs, errs[1:]):
        assert math.log2(a / b) > 4.7, errs


def test_jump_no_new_extrema():
    q = np.array([0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0])
    vals = [weno.reconstruct(*[q[(i + s) % 8] for s in (-2, -1, 0, 1, 2)]) for i in range(8)]
    assert all(-1e-30 <= v <= 1.0 + 1e-15 for v in vals), vals
    # the face between the last 0 and the first 1, seen from the left, takes the left value
    assert abs(vals[3]) < 1e-30


def test_periodic_sum_and_mirror_wall():
    rng = np.random.default_rng(12)
    q = rng.standard_normal((6, 4, 8))
    u = rng.standard_normal((6, 4, 8))
    z = np.zeros_like(q)
    div = weno.divergence(q, u, z, z, (0.1, 0.2, 0.3), D)
    assert abs(float(np.sum(div))) < 1e-12 * float(np.sum(np.abs(div)))
    # a field mirrored about the bottom wall face: the reconstruction at the first interior
    # face from below uses the mirror ghosts; for a field constant in z the z flux is w q
    qc = np.ones((6, 4, 8)) * 0.7
    w = rng.standard_normal((6, 4, 8))
    fz = weno.face_flux(qc, w, 0, True)
    assert np.max(np.abs(fz - 0.7 * w)) < 1e-15


def test_mirror_wall_equals_even_periodic_extension():
    """The mirror ghosts are the even extension: a wall-bounded column of n cells equals the
    upper half of the periodic column of 2n cells made of the column reflected below it, with
    the face velocities odd about the bottom wall (zero on both walls). The periodic branch uses
    true neighbours only, so this checks the ghost indices at both walls."""
    rng = np.random.default_rng(21)
    n = 8
    q = rng.standard_normal((n, 3, 4))
    w = rng.standard_normal((n, 3, 4))
    w[-1] = 0.0                                # top wall face
    fz = weno.face_flux(q, w, 0, True)
    fz[-1] = 0.0
    div_wall = fz - D.zm_face(fz)
    Q = np.concatenate([q[::-1], q], axis=0)  # Q[n + k] = q[k], Q[n - 1 - k] = q[k]
    Wp = np.zeros_like(Q)
    Wp[n:] = w                                 # face between Q[f], Q[f + 1]; Wp[2n - 1] = 0 (top)
    for f in range(n - 1):                     # the reflected faces; Wp[n - 1] = 0 (bottom wall)
        Wp[f] = -w[n - 2 - f]
    Fp = weno.face_flux(Q, Wp, 0, False)
    div_per = Fp - np.roll(Fp, 1, axis=0)
    assert np.max(np.abs(div_per[n:] - div_wall)) < 1e-13 * np.max(np.abs(div_wall))
    # and the lower half mirrors the upper one
    assert np.max(np.abs(div_per[:n][::-1] - div_wall)) < 1e-13 * np.max(np.abs(div_wall))


def test_coupled_step_conserves_mass_with_weno():
    cfg = W.config("C3", nx=16, ny=8, nz=8, lx=1.0, ly=0.5, lz=0.5, radius=0.2, noise=1e-2,
                   advection=1, giesekus_alpha=0.1)
    P = model.Params.from_config(cfg)
    st = W.droplet_state(cfg)
    m0 = S.observables(P, st)["mass"]
    st = S.run(P, st, 4)
    m1 = S.observables(P, st)["mass"]
    assert abs(m1 - m0) < 1e-12 * np.sum(np.abs(st["phi"][0])) * np.prod(P.hf)
    assert max(float(np.max(np.abs(t))) for t in st["tau"][0]) > 0
