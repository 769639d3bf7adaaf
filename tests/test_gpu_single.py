"""GPU parity of the single-resolution mode (refine = 1: the phase field on the flow grid):
the HIP path through the C-ABI against the FP64 oracle on the same seeded inputs, 1e-10
relative per field in FP64."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W
from oracle import model
from oracle import step as S

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def drpf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_04577_amd as P
    P.lib()
    return P


def rel(a, b):
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)


def run_both(drpf, cfg, nsteps):
    import torch
    say(f"[gpu] single resolution {cfg.name} grid {cfg.nx}x{cfg.ny}x{cfg.nz} ve {cfg.viscoelastic} "
        f"constitutive {cfg.constitutive} steps {nsteps}")
    g = drpf.Grid(cfg, 64)
    assert g.fine_shape == g.coarse_shape
    st = g.state(W.droplet_state(cfg))
    g.step(st, nsteps)
    torch.cuda.synchronize()
    gh = st.to_host()
    oh = S.run(model.Params.from_config(cfg), W.droplet_state(cfg), nsteps)
    e = {k: rel(gh[k][0], oh[k][0]) for k in ("phi", "u", "w", "p")}
    if np.max(np.abs(oh["v"][0])) > 0:
        e["v"] = rel(gh["v"][0], oh["v"][0])
    if cfg.viscoelastic:
        e["tau"] = max(rel(gh["tau"][0][c], oh["tau"][0][c]) for c in range(6)
                       if np.max(np.abs(oh["tau"][0][c])) > 0)
    say(f"[gpu] errors {e}")
    return g, st, e


CASES = [
    ("3d-contrast", W.config("C2", nx=32, ny=16, nz=16, lx=2.0, ly=1.0, lz=1.0, radius=0.3,
                             noise=1e-3, seed=4, refine=1), 5),
    ("2d-newtonian", W.config("C1", nx=64, nz=32, ly=2.0 / 64, noise=1e-3, seed=1, refine=1), 8),
    ("3d-viscoelastic", W.config("C3", nx=32, ny=32, nz=16, lx=1.0, ly=1.0, lz=0.5, radius=0.2,
                                 noise=1e-3, seed=5, refine=1), 4),
    ("3d-all-terms", W.config("C5", nx=32, ny=16, nz=16, lx=1.0, ly=0.5, lz=0.5, radius=0.2,
                              theta_top_deg=100.0, a_ext=(0.3, -0.2, -1.0), s_factor=1.5,
                              noise=1e-3, seed=7, refine=1, constitutive=1, giesekus_alpha=0.2), 4),
]


@pytest.mark.parametrize("name,cfg,n", CASES, ids=[c[0] for c in CASES])
def test_single_resolution_matches_oracle(drpf, name, cfg, n):
    g, st, errs = run_both(drpf, cfg, n)
    for k, e in errs.items():
        assert e < TOL, (k, e)


def test_full_size_c2_single_resolution_one_step(drpf):
    """C2 on one 256x256x128 grid (the comparison baseline at the bench's size): one step,
    every field, plus mass and discrete incompressibility."""
    cfg = W.config("C2S")
    g, st, errs = run_both(drpf, cfg, 1)
    for k, e in errs.items():
        assert e < TOL, (k, e)
    assert g.observables(st)["max_div"] < 1e-8
