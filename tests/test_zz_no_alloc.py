"""The allocation-free Helmholtz entry point (drpf_helmholtz_solve_static) against
drpf_helmholtz_solve through the C-ABI: the same kernels on the same inputs give the same bits,
with and without wall data, on two calls in a row (the second on a smaller grid), plus the
oracle's solve at 1e-12 and the size limit of the static scratch."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W
from oracle import discrete as D
from oracle import model

pytestmark = pytest.mark.gpu


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


BIG = W.config("C2", nx=64, ny=16, nz=16, lx=2.0, ly=0.5, lz=0.5)
SMALL = W.config("C2", nx=16, ny=4, nz=8, lx=1.0, ly=0.25, lz=0.5)
KINDS = {"neumann": "neumann", "dirichlet": "dirichlet", "face_dirichlet": "wface"}


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("bc,coeff,shift,walls", [("neumann", 1.0, 0.0, False), ("neumann", 0.7, 37.0, True),
                                                  ("dirichlet", 0.3, 5.0, True),
                                                  ("face_dirichlet", 2.0, 11.0, True)])
def test_static_solve_matches_workspace_solve(drpf, precision, bc, coeff, shift, walls):
    import torch
    dt = torch.float64 if precision == 64 else torch.float32
    rng = np.random.default_rng(41)
    for cfg in (BIG, SMALL):  # two calls in a row, the second on a smaller input
        for which in ("fine", "coarse"):
            say(f"[gpu] static helmholtz fp{precision} {bc} walls {walls} {which} coarse {cfg.nx}x{cfg.ny}x{cfg.nz}")
            g = drpf.Grid(cfg, precision)
            shape = g.fine_shape if which == "fine" else g.coarse_shape
            rhs = rng.standard_normal(shape) + 0.4
            if bc == "face_dirichlet":
                rhs[-1] = 0.0
            wall = rng.standard_normal((2,) + shape[1:]) if walls else None
            rt = torch.tensor(rhs, device="cuda", dtype=dt)
            wt = torch.tensor(wall, device="cuda", dtype=dt) if walls else None
            a = g.helmholtz_solve_static(rt, which, bc, coeff, shift, wall=wt)
            b = g.helmholtz_solve(rt, which, bc, coeff, shift, wall=wt)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (cfg.nx, which)
            if precision == 64:
                P = model.Params.from_config(cfg)
                h = P.hf if which == "fine" else P.h
                ref = D.helmholtz(rhs, coeff, shift, KINDS[bc], h,
                                  walls=(wall[0], wall[1]) if walls else None)
                err = float(np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref)))
                assert err < 1e-12, err
            del g


def test_static_scratch_limit(drpf):
    """A solve whose spectral buffer exceeds the 32 MiB scratch is refused with a clear error;
    one that fits on the same grid runs."""
    import torch
    from paper_2111_04577_amd import binding as B
    cfg = W.config("C2")  # fine 256x256x128: (129 * 256 * 128) complex FP64 = 67.6 MB
    say("[gpu] static helmholtz size limit on C2")
    g = drpf.Grid(cfg, 64)
    rhs = torch.zeros(g.fine_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(B.DrpfError) as e:
        g.helmholtz_solve_static(rhs, "fine", "neumann", 1.0, 1.0)
    assert e.value.code == B.DRPF_EWORKSPACE
    assert "static limit" in str(e.value)
    rc = torch.ones(g.coarse_shape, dtype=torch.float64, device="cuda")
    x = g.helmholtz_solve_static(rc, "coarse", "neumann", 1.0, 2.0)
    torch.cuda.synchronize()
    assert torch.allclose(x, torch.full_like(x, -0.5), rtol=1e-13, atol=0)
