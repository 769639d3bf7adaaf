"""GPU tests of the C-ABI's wall data, finite checks and state layout, against the oracle:

* drpf_helmholtz_solve with inhomogeneous wall data (Neumann derivative, no-slip value, face
  value) against the oracle's solve with the same data (1e-12);
* moving walls (eq. NS13, u = u_w) in the coupled step against the oracle (1e-10): 3D with
  density and viscosity contrast, Oldroyd-B, 2D, the log-conformation form with WENO-Z, and a
  single resolution; the plane Couette steady state in both precision forms;
* check_finite_every: a non-finite phase field stops drpf_step with DRPF_ENONFINITE at the
  first check after it, and checks on a finite run change nothing;
* drpf_state_layout against the staggered placement of every field.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W
from oracle import discrete as D
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


# ---------------------------------------------------------------------------------------
# Helmholtz solves with wall data
# ---------------------------------------------------------------------------------------

SMALL3D = W.config("C2", nx=32, ny=8, nz=8, lx=2.0, ly=0.5, lz=0.5, noise=1e-3, seed=3)
SMALL2D = W.config("C1", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=2)


@pytest.mark.parametrize("cfg", [SMALL3D, SMALL2D], ids=["3d", "2d"])
@pytest.mark.parametrize("which", ["fine", "coarse"])
@pytest.mark.parametrize("bc,coeff,shift", [("neumann", 1.0, 0.0), ("neumann", 0.7, 37.0),
                                             ("dirichlet", 0.3, 5.0), ("face_dirichlet", 2.0, 11.0)])
def test_helmholtz_wall_data(drpf, cfg, which, bc, coeff, shift):
    import torch
    say(f"[gpu] helmholtz wall data {cfg.name} {which} {bc}")
    g = drpf.Grid(cfg, 64)
    shape = g.fine_shape if which == "fine" else g.coarse_shape
    P = model.Params.from_config(cfg)
    h = P.hf if which == "fine" else P.h
    rng = np.random.default_rng(29)
    rhs = rng.standard_normal(shape)
    wall = rng.standard_normal((2,) + shape[1:])
    if bc == "face_dirichlet":
        rhs[-1] = 0.0
    kind = {"neumann": "neumann", "dirichlet": "dirichlet", "face_dirichlet": "wface"}[bc]
    x = g.helmholtz_solve(torch.tensor(rhs, device="cuda"), which, bc, coeff, shift,
                          wall=torch.tensor(wall, device="cuda"))
    torch.cuda.synchronize()
    ref = D.helmholtz(rhs, coeff, shift, kind, h, walls=(wall[0], wall[1]))
    assert rel(x.cpu().numpy(), ref) < 1e-12
    if bc == "face_dirichlet":
        assert np.array_equal(x[-1].cpu().numpy(), wall[1])


# ---------------------------------------------------------------------------------------
# moving walls in the coupled step
# ---------------------------------------------------------------------------------------

UWB, UWT = (0.3, -0.2), (-0.6, 0.45)
MOVING = [
    ("3d-contrast", W.config("C2", nx=32, ny=8, nz=8, lx=2.0, ly=0.5, lz=0.5, radius=0.2,
                             noise=1e-3, seed=4, u_wall_bottom=UWB, u_wall_top=UWT), 5),
    ("3d-oldroyd-b", W.config("C3", nx=16, ny=16, nz=8, lx=1.0, ly=1.0, lz=0.5, radius=0.2,
                              noise=1e-3, seed=5, u_wall_bottom=UWB, u_wall_top=UWT), 5),
    ("2d-viscoelastic", W.config("C4", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=6,
                                 u_wall_bottom=(0.5, 0.1), u_wall_top=(-0.25, 0.2)), 8),
    ("3d-lcr-weno", W.config("C3L", nx=16, ny=8, nz=8, lx=1.0, ly=0.5, lz=0.5, radius=0.2,
                             noise=1e-3, seed=8, advection=1, u_wall_bottom=UWB,
                             u_wall_top=UWT), 4),
    ("3d-single-resolution", W.config("C3S", nx=16, ny=16, nz=8, lx=1.0, ly=1.0, lz=0.5,
                                      radius=0.2, noise=1e-3, seed=9, u_wall_bottom=UWB,
                                      u_wall_top=UWT), 4),
]


def field_errors(gh, oh, viscoelastic):
    errs = {f: rel(gh[f][0], oh[f][0]) for f in ("phi", "u", "v", "w", "p")}
    if viscoelastic:
        errs["tau"] = max(rel(gh["tau"][0][c], oh["tau"][0][c]) for c in range(6)
                          if np.max(np.abs(oh["tau"][0][c])) > 0)
    return errs


@pytest.mark.parametrize("name,cfg,n", MOVING, ids=[c[0] for c in MOVING])
def test_moving_walls_match_oracle(drpf, name, cfg, n):
    import torch
    say(f"[gpu] moving walls {name} {n} steps")
    P = model.Params.from_config(cfg)
    oh = S.run(P, W.droplet_state(cfg), n)
    g = drpf.Grid(cfg, 64)
    st = g.state(W.droplet_state(cfg))
    g.step(st, n)
    torch.cuda.synchronize()
    errs = field_errors(st.to_host(), oh, cfg.viscoelastic)
    say(f"[gpu] {name} errors {errs}")
    for k, e in errs.items():
        assert e < TOL, (k, e)
    # the wall motion is felt: the same case at rest differs far beyond the tolerance
    rest = S.run(model.Params.from_config(cfg.replace(u_wall_bottom=(0.0, 0.0),
                                                     u_wall_top=(0.0, 0.0))),
                 W.droplet_state(cfg), n)
    assert rel(rest["u"][0], oh["u"][0]) > 1e-3


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 1e-5)])
@pytest.mark.parametrize("viscoelastic", [0, 1])
def test_couette_steady_state(drpf, precision, tol, viscoelastic):
    """The linear profile between the moving walls (with the Oldroyd-B steady stresses when
    viscoelastic) is a fixed point of the GPU step."""
    import torch
    cfg = W.config("C3" if viscoelastic else "C2", nx=16, ny=8, nz=16, lx=1.0, ly=0.5, lz=1.0,
                   rho_ratio=3.0, mu_ratio=2.0, u_wall_bottom=(0.3, -0.4), u_wall_top=(1.1, 0.6))
    say(f"[gpu] couette fp{precision} viscoelastic {viscoelastic}")
    P = model.Params.from_config(cfg)
    cs = P.coarse_shape
    z = (np.arange(P.nz) + 0.5) * P.h[2]
    gx = (cfg.u_wall_top[0] - cfg.u_wall_bottom[0]) / cfg.lz
    gy = (cfg.u_wall_top[1] - cfg.u_wall_bottom[1]) / cfg.lz
    u = np.broadcast_to((cfg.u_wall_bottom[0] + gx * z)[:, None, None], cs).copy()
    v = np.broadcast_to((cfg.u_wall_bottom[1] + gy * z)[:, None, None], cs).copy()
    zero = lambda: np.zeros(cs)
    tau = [zero() for _ in range(6)]
    if viscoelastic:
        c = 1.0 - cfg.beta
        tau = [np.full(cs, 2 * cfg.wi * c * gx * gx), np.full(cs, 2 * cfg.wi * c * gy * gy), zero(),
               np.full(cs, 2 * cfg.wi * c * gx * gy), np.full(cs, c * gx), np.full(cs, c * gy)]
    phase = 1.0 if viscoelastic else -1.0
    phi = np.full(P.fine_shape, phase)
    host = {"phi": [phi, phi.copy()], "u": [u, u.copy()], "v": [v, v.copy()], "w": [zero(), zero()],
            "p": [zero(), zero()], "tau": [tau, [t.copy() for t in tau]], "step": 3,
            "theta": [zero() for _ in range(6)]}
    g = drpf.Grid(cfg, precision)
    st = g.state(host)
    g.step(st, 3)
    torch.cuda.synchronize()
    out = st.to_host()
    scale = 1.1
    for f, ref in (("u", u), ("v", v)):
        assert np.max(np.abs(out[f][0] - ref)) <= tol * scale, f
    assert np.max(np.abs(out["w"][0])) <= tol * scale
    if viscoelastic:
        tmax = max(np.max(np.abs(t)) for t in tau)
        for m in range(6):
            assert np.max(np.abs(out["tau"][0][m] - tau[m])) <= tol * tmax, m


# ---------------------------------------------------------------------------------------
# finite checks
# ---------------------------------------------------------------------------------------


def test_check_finite_stops_the_step(drpf):
    import torch
    from paper_2111_04577_amd import binding as B
    cfg = W.config("C1", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=1, check_finite_every=2)
    say("[gpu] check_finite_every: planted NaN")
    host = W.droplet_state(cfg)
    host["phi"][0][3, 0, 5] = np.nan
    host["phi"][1][3, 0, 5] = np.nan
    g = drpf.Grid(cfg, 64)
    st = g.state(host)
    with pytest.raises(B.DrpfError) as e:
        g.step(st, 5)
    assert e.value.code == B.DRPF_ENONFINITE
    assert st.step == 2
    assert "after step 2" in str(e.value)


@pytest.mark.parametrize("precision", [64, 32])
def test_check_finite_changes_nothing(drpf, precision):
    import torch
    cfg = W.config("C3", nx=16, ny=8, nz=8, lx=1.0, ly=0.5, lz=0.5, radius=0.2, noise=1e-3, seed=5)
    say(f"[gpu] check_finite_every on a finite run, fp{precision}")
    outs = []
    for every in (0, 1):
        g = drpf.Grid(cfg.replace(check_finite_every=every), precision)
        st = g.state(W.droplet_state(cfg))
        g.step(st, 4)
        torch.cuda.synchronize()
        assert st.step == 4
        outs.append(st.to_host())
    for f in ("phi", "u", "v", "w", "p"):
        assert np.array_equal(outs[0][f][0], outs[1][f][0]), f


# ---------------------------------------------------------------------------------------
# state layout
# ---------------------------------------------------------------------------------------


@pytest.mark.parametrize("cfg,precision", [
    (W.config("C3L", nx=16, ny=8, nz=4, lx=1.0, ly=0.5, lz=0.25), 32),
    (W.config("C1", nx=32, nz=16, ly=2.0 / 32), 64),
    (W.config("C2S", nx=16, ny=8, nz=8, lx=1.0, ly=0.5, lz=0.5), 64),
], ids=["3d-lcr-fp32", "2d-fp64", "single-resolution"])
def test_state_layout(drpf, cfg, precision):
    g = drpf.Grid(cfg, precision)
    L = g.layout()
    es = 4 if precision == 32 else 8
    assert L["elem_bytes"] == es
    P = model.Params.from_config(cfg)
    fz, fy, fx = P.fine_shape
    cz, cy, cx = P.coarse_shape
    hf, hc = P.hf, P.h
    expect = {
        "phi": ((fx, fy, fz), hf, (0.5, 0.5, 0.5), 3),
        "u": ((cx, cy, cz), hc, (1.0, 0.5, 0.5), 2),
        "v": ((cx, cy, cz), hc, (0.5, 1.0, 0.5), 2),
        "w": ((cx, cy, cz), hc, (0.5, 0.5, 1.0), 2),
        "p": ((cx, cy, cz), hc, (0.5, 0.5, 0.5), 2),
        "tau": ((cx, cy, cz), hc, (0.5, 0.5, 0.5), 12 if cfg.viscoelastic else 0),
        "theta": ((cx, cy, cz), hc, (0.5, 0.5, 0.5), 6 if cfg.constitutive == 1 else 0),
    }
    total = 0
    for f, (n, h, off, arrays) in expect.items():
        e = L[f]
        assert e["n"] == n, f
        assert e["stride"] == (1, n[0], n[0] * n[1]), f
        assert e["elems"] == n[0] * n[1] * n[2], f
        assert e["arrays"] == arrays, f
        for a in range(3):
            assert e["spacing"][a] == pytest.approx(h[a], rel=1e-15), f
            assert e["origin"][a] == pytest.approx(off[a] * h[a], rel=1e-15), f
        total += arrays * e["elems"] * es
    assert L["state_bytes"] == total
    # the binding's own state buffer holds exactly these arrays
    st = g.state(W.droplet_state(cfg))
    assert st.flat.numel() * st.flat.element_size() == total
