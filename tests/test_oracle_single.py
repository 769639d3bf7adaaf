"""Pins of the oracle's single-resolution mode (refine = 1: the phase field on the flow grid),
the baseline of the dual-resolution comparison, against things other than itself:

* the transfers without refinement against loop-built means (a face: the mean of its two
  cells, an edge: of its four, the wall ghost equal to the adjacent cell) on a small field;
* the prolongation is the identity;
* Cahn-Hilliard mass is conserved over several coupled steps;
* over the first steps (velocity still small) the phase field of a single-resolution run
  equals that of the dual-resolution run with the same phase-field grid to within the
  velocity's influence.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import workloads as W
from oracle import discrete as D
from oracle import model
from oracle import step as S


def _loop_restrict(f, loc):
    """Mean over the 1, 2 or 4 (or 8) cells around the location, built by loops."""
    nz, ny, nx = f.shape
    lz, ly, lx = loc
    nzo = nz + 1 if lz == "f" else nz
    out = np.zeros((nzo, ny, nx))
    for m, j, i in itertools.product(range(nzo), range(ny), range(nx)):
        zs = [min(max(m - 1, 0), nz - 1), min(max(m, 0), nz - 1)] if lz == "f" else [m]
        ys = [j, (j + 1) % ny] if ly == "f" else [j]
        xs = [i, (i + 1) % nx] if lx == "f" else [i]
        vals = [f[a, b, c] for a in zs for b in ys for c in xs]
        out[m, j, i] = sum(vals) / len(vals)
    return out


@pytest.mark.parametrize("loc", ["ccc", "ccf", "cfc", "fcc", "cff", "fcf", "ffc"])
def test_single_resolution_transfer_against_loops(loc):
    rng = np.random.default_rng(8)
    f = rng.standard_normal((4, 4, 6))
    got = D.restrict(f, loc, 1, 1)
    assert np.max(np.abs(got - _loop_restrict(f, loc))) < 1e-15


def test_single_resolution_prolong_is_identity():
    rng = np.random.default_rng(9)
    u, v, w = (rng.standard_normal((4, 4, 8)) for _ in range(3))
    uf, vf, wf = D.prolong(u, v, w, 1, 1)
    assert np.array_equal(uf, u) and np.array_equal(vf, v) and np.array_equal(wf, w)


def test_single_resolution_conserves_mass():
    cfg = W.config("C2", nx=32, ny=16, nz=16, lx=2.0, ly=1.0, lz=1.0, radius=0.3, noise=1e-3,
                   refine=1)
    P = model.Params.from_config(cfg)
    st = W.droplet_state(cfg)
    m0 = S.observables(P, st)["mass"]
    st = S.run(P, st, 6)
    m1 = S.observables(P, st)["mass"]
    assert abs(m1 - m0) < 1e-12 * np.sum(np.abs(st["phi"][0])) * np.prod(P.hf)
    assert S.observables(P, st)["max_div"] < 1e-9


def test_single_matches_dual_phase_field_early():
    """Same phase-field grid (32x16x16), same initial field: the dual-resolution step runs the
    flow on the 16x8x8 grid, the single-resolution step on 32x16x16. While the velocity is
    small the phase-field updates agree to a small fraction of the change itself."""
    dual = W.config("C2", nx=16, ny=8, nz=8, lx=2.0, ly=1.0, lz=1.0, radius=0.3, noise=0.0,
                    dt=1e-4)
    single = dual.replace(nx=32, ny=16, nz=16, refine=1)
    assert W.fine_shape(dual) == W.fine_shape(single)
    s0 = W.droplet_state(dual)
    sd = S.run(model.Params.from_config(dual), s0, 3)
    ss = S.run(model.Params.from_config(single), W.droplet_state(single), 3)
    change = float(np.max(np.abs(sd["phi"][0] - s0["phi"][0])))
    diff = float(np.max(np.abs(sd["phi"][0] - ss["phi"][0])))
    assert change > 0
    assert diff < 0.05 * change, (diff, change)
