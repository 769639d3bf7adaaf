"""GPU cases at the largest extent the C-ABI accepts on each axis (coarse 1024 in x or y, 512
in z; phase-field lines of 2048 and 1024 points), each in a small volume so that the oracle
runs three steps in seconds. They exercise the launch shapes no benchmark workload reaches:
x transforms of 1024-point complex lines (one line per block), y transforms of 2048 points,
the fused coarse x-y transform of 4 x 1024 layers, and wall-normal passes over 1024 (CH) and
512 (NS) rows with a single mode per block, the latter with every option on (log-conformation,
Giesekus, WENO-Z, relaxed walls). FP64 against the oracle at 1e-10; the FP32 form runs the
same shapes and stays finite and close."""
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


def rel_family(gs, os_):
    """Per-component relative error with each denominator floored at 1e-3 of the family's
    largest component (components zero by symmetry hold only round-off on either side)."""
    fam = max(float(np.max(np.abs(o))) for o in os_)
    if fam == 0.0:
        return max(float(np.max(np.abs(g))) for g in gs)
    return max(float(np.max(np.abs(g - o))) / max(float(np.max(np.abs(o))), 1e-3 * fam)
               for g, o in zip(gs, os_))


DENS = dict(rho_ratio=10.0, mu_ratio=5.0)
CASES = [
    ("x-max-2d", W.config("C1", nx=1024, nz=4, lx=4.0, ly=4.0 / 1024, lz=0.5, radius=0.2,
                          noise=1e-3, seed=11)),
    ("x-max-3d", W.config("C2", nx=1024, ny=4, nz=4, lx=4.0, ly=0.5, lz=0.5, radius=0.2,
                          noise=1e-3, seed=12, **DENS)),
    ("y-max", W.config("C2", nx=4, ny=1024, nz=4, lx=0.5, ly=4.0, lz=0.5, radius=0.2, noise=1e-3,
                       seed=13, **DENS)),
    ("z-max", W.config("C2", nx=4, ny=4, nz=512, lx=0.5, ly=0.5, lz=4.0, radius=0.2, noise=1e-3,
                       seed=14, theta_bottom_deg=60.0, **DENS)),
    ("z-max-all-options", W.config("C3", nx=4, ny=4, nz=512, lx=0.5, ly=0.5, lz=4.0, radius=0.2,
                                   noise=1e-3, seed=15, wi=0.5, constitutive=1,
                                   giesekus_alpha=0.2, advection=1, d_w=0.1,
                                   theta_bottom_deg=60.0)),
]


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_largest_extents_match_oracle(drpf, name, cfg):
    import torch
    n = 3
    say(f"[gpu] extents {name}: coarse {cfg.nx}x{cfg.ny}x{cfg.nz}, fine {W.fine_shape(cfg)[::-1]}")
    g = drpf.Grid(cfg, 64)
    st = g.state(W.droplet_state(cfg))
    g.step(st, n)
    torch.cuda.synchronize()
    gh = st.to_host()
    oh = S.run(model.Params.from_config(cfg), W.droplet_state(cfg), n)
    e = {k: rel(gh[k][0], oh[k][0]) for k in ("phi", "p")}
    e["vel"] = rel_family([gh[k][0] for k in "uvw"], [oh[k][0] for k in "uvw"])
    if cfg.viscoelastic:
        e["tau"] = rel_family(gh["tau"][0], oh["tau"][0])
    if cfg.constitutive == 1:
        e["theta"] = rel_family(gh["theta"], oh["theta"])
    say(f"[gpu] errors {e}")
    for k, v in e.items():
        assert v < TOL, (name, k, v)
    g32 = drpf.Grid(cfg, 32)
    s32 = g32.state(W.droplet_state(cfg))
    g32.step(s32, n)
    torch.cuda.synchronize()
    h32 = s32.to_host()
    assert all(np.all(np.isfinite(h32[k][0])) for k in ("phi", "u", "v", "w", "p"))
    assert rel(h32["phi"][0], gh["phi"][0]) < 1e-4
