"""GPU edge cases: the smallest grids the C-ABI accepts (coarse 4 x 4 x 4 and 4 x 1 x 4, fine
8 x 8 x 8 and 8 x 1 x 8), where every launcher takes its smallest tiles (blocks below one
wavefront, single-line wall-normal tiles, a two-point x transform), against the FP64 oracle at
1e-10, with the default scheme and with every option on; and a zero-step call, which must leave
the state as it is."""
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


MIN3 = W.config("C2", nx=4, ny=4, nz=4, lx=1.0, ly=1.0, lz=1.0, radius=0.4, noise=1e-3, seed=3,
                theta_bottom_deg=70.0, theta_top_deg=110.0, rho_ratio=10.0, mu_ratio=5.0)
MIN2 = W.config("C1", nx=4, nz=4, lx=1.0, ly=0.25, lz=1.0, radius=0.4, noise=1e-3, seed=2)
ALL3 = W.config("C3", nx=4, ny=4, nz=4, lx=1.0, ly=1.0, lz=1.0, radius=0.4, noise=1e-3, seed=5,
                wi=0.5, constitutive=1, giesekus_alpha=0.2, advection=1, d_w=0.1,
                theta_bottom_deg=60.0)

CASES = [
    ("3d-minimum", MIN3, 4),
    ("2d-minimum", MIN2, 4),
    ("3d-minimum-all-options", ALL3, 4),
    ("3d-minimum-single", MIN3.replace(refine=1), 4),
]


@pytest.mark.parametrize("name,cfg,n", CASES, ids=[c[0] for c in CASES])
def test_smallest_grids_match_oracle(drpf, name, cfg, n):
    import torch
    say(f"[gpu] edge {name}: coarse {cfg.nx}x{cfg.ny}x{cfg.nz} refine {cfg.refine} steps {n}")
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
    # the FP32 form runs the same launch shapes and stays finite
    g32 = drpf.Grid(cfg, 32)
    s32 = g32.state(W.droplet_state(cfg))
    g32.step(s32, n)
    torch.cuda.synchronize()
    h32 = s32.to_host()
    assert all(np.all(np.isfinite(h32[k][0])) for k in ("phi", "u", "v", "w", "p"))
    assert rel(h32["phi"][0], gh["phi"][0]) < 1e-4


def test_zero_steps_leave_the_state(drpf):
    import torch
    cfg = MIN3
    g = drpf.Grid(cfg, 64)
    st = g.state(W.droplet_state(cfg))
    g.step(st, 2)
    torch.cuda.synchronize()
    before = st.to_host()
    g.step(st, 0)
    torch.cuda.synchronize()
    after = st.to_host()
    assert after["step"] == before["step"]
    for k in ("phi", "u", "v", "w", "p"):
        for lvl in range(2):
            assert np.array_equal(after[k][lvl], before[k][lvl]), (k, lvl)
