"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the same seeded
inputs. FP64 results must agree to 1e-10 relative per field (max |gpu - oracle| divided by
max |oracle|); linear operators to 1e-12; transfers to a few ulps."""
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


def field_errors(gh, oh, viscoelastic):
    errs = {"phi": rel(gh["phi"][0], oh["phi"][0]), "u": rel(gh["u"][0], oh["u"][0]),
            "w": rel(gh["w"][0], oh["w"][0]), "p": rel(gh["p"][0], oh["p"][0])}
    if np.max(np.abs(oh["v"][0])) > 0:
        errs["v"] = rel(gh["v"][0], oh["v"][0])
    else:
        errs["v"] = float(np.max(np.abs(gh["v"][0])))
    if viscoelastic:
        errs["tau"] = max(rel(gh["tau"][0][c], oh["tau"][0][c]) for c in range(6)
                          if np.max(np.abs(oh["tau"][0][c])) > 0)
    return errs


def run_both(drpf, cfg, nsteps, precision=64):
    import torch
    say(f"[gpu] config {cfg.name} coarse {cfg.nx}x{cfg.ny}x{cfg.nz} steps {nsteps} fp{precision}")
    g = drpf.Grid(cfg, precision)
    st = g.state(W.droplet_state(cfg))
    g.step(st, nsteps)
    torch.cuda.synchronize()
    gh = st.to_host()
    P = model.Params.from_config(cfg)
    oh = S.run(P, W.droplet_state(cfg), nsteps)
    return g, st, gh, oh


# ---------------------------------------------------------------------------------------
# linear building blocks
# ---------------------------------------------------------------------------------------

SMALL3D = W.config("C2", nx=32, ny=8, nz=8, lx=2.0, ly=0.5, lz=0.5, noise=1e-3, seed=3)
SMALL2D = W.config("C1", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=2)


@pytest.mark.parametrize("cfg", [SMALL3D, SMALL2D], ids=["3d", "2d"])
@pytest.mark.parametrize("which", ["fine", "coarse"])
@pytest.mark.parametrize("bc,coeff,shift,offset", [
    ("neumann", 1.0, 0.0, 0.0), ("neumann", 1.0, 0.0, 0.75), ("neumann", 0.7, 37.0, 0.0),
    ("dirichlet", 0.3, 5.0, 0.0), ("face_dirichlet", 2.0, 11.0, 0.0)])
def test_helmholtz_solve(drpf, cfg, which, bc, coeff, shift, offset):
    """Against the oracle's exact solve; the singular Neumann Poisson problem (shift 0) with a
    right-hand side of non-zero mean (offset) returns the pseudo-inverse's zero-mean
    solution, as the oracle does."""
    import torch
    say(f"[gpu] helmholtz {cfg.name} {which} {bc} offset {offset}")
    g = drpf.Grid(cfg, 64)
    shape = g.fine_shape if which == "fine" else g.coarse_shape
    P = model.Params.from_config(cfg)
    h = P.hf if which == "fine" else P.h
    rng = np.random.default_rng(17)
    rhs = rng.standard_normal(shape)
    if bc == "neumann" and shift == 0.0:
        rhs += offset - rhs.mean()
    if bc == "face_dirichlet":
        rhs[-1] = 0.0
    x = g.helmholtz_solve(torch.tensor(rhs, device="cuda"), which, bc, coeff, shift)
    torch.cuda.synchronize()
    kind = {"neumann": "neumann", "dirichlet": "dirichlet", "face_dirichlet": "wface"}[bc]
    ref = D.helmholtz(rhs, coeff, shift, kind, h)
    assert rel(x.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("cfg", [SMALL3D, SMALL2D], ids=["3d", "2d"])
def test_prolong_restrict(drpf, cfg):
    import torch
    say(f"[gpu] transfers {cfg.name}")
    g = drpf.Grid(cfg, 64)
    rng = np.random.default_rng(5)
    cs = g.coarse_shape
    u, v, w = (rng.standard_normal(cs) for _ in range(3))
    w[-1] = 0.0
    if cfg.ny == 1:
        v[:] = 0.0
    P = model.Params.from_config(cfg)
    uf, vf, wf = g.prolong(*(torch.tensor(a, device="cuda") for a in (u, v, w)))
    ru, rv, rw = D.prolong(u, v, w, P.ry)
    for a, b in ((uf, ru), (vf, rv), (wf, rw)):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-15 * max(1.0, np.max(np.abs(b)))
    f = rng.standard_normal(g.fine_shape)
    ft = torch.tensor(f, device="cuda")
    for loc, code in (("ccc", "center"), ("ccf", "face_x"), ("cfc", "face_y"), ("fcc", "face_z"),
                      ("cff", "edge_xy"), ("fcf", "edge_xz"), ("ffc", "edge_yz")):
        out = g.restrict(ft, code).cpu().numpy()
        ref = D.restrict(f, loc, P.ry)
        assert out.shape == ref.shape, code
        assert np.max(np.abs(out - ref)) <= 4e-16 * np.max(np.abs(ref)) + 1e-300, code


# ---------------------------------------------------------------------------------------
# coupled step
# ---------------------------------------------------------------------------------------

STEP_CASES = [
    ("2d-newtonian", W.config("C1", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=1), 8),
    ("3d-contrast", W.config("C2", nx=32, ny=8, nz=8, lx=2.0, ly=0.5, lz=0.5, radius=0.2,
                             noise=1e-3, seed=4), 5),
    ("3d-viscoelastic", W.config("C3", nx=16, ny=16, nz=8, lx=1.0, ly=1.0, lz=0.5, radius=0.2,
                                 noise=1e-3, seed=5), 5),
    ("2d-viscoelastic", W.config("C4", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=6), 8),
    ("3d-all-terms", W.config("C5", nx=16, ny=8, nz=8, lx=1.0, ly=0.5, lz=0.5, radius=0.2,
                              theta_top_deg=100.0, a_ext=(0.3, -0.2, -1.0), s_factor=1.5,
                              noise=1e-3, seed=7), 4),
]


@pytest.mark.parametrize("name,cfg,n", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_step_matches_oracle(drpf, name, cfg, n):
    g, st, gh, oh = run_both(drpf, cfg, n)
    assert st.step == n
    errs = field_errors(gh, oh, cfg.viscoelastic)
    say(f"[gpu] {name} errors {errs}")
    for k, e in errs.items():
        assert e < TOL, (k, e)
    # level n-1 too
    assert rel(gh["phi"][1], oh["phi"][1]) < TOL


def test_first_step_intermediates(drpf):
    """Restricted set and momentum right-hand side after one step (diagnostic)."""
    import torch
    cfg = STEP_CASES[4][1]
    say("[gpu] first-step intermediates")
    g = drpf.Grid(cfg, 64)
    st = g.state(W.droplet_state(cfg))
    g.step(st, 1)
    torch.cuda.synchronize()
    P = model.Params.from_config(cfg)
    _, parts = S.step(P, W.droplet_state(cfg), return_parts=True)
    R = parts["R"]
    names = ["phi_c", "G_c", "G_x", "G_y", "G_z", "rinv_x", "rinv_y", "rinv_z", "mu_c", "mu_xy",
             "mu_xz", "mu_yz"]
    for idx, nm in enumerate(names):
        ref = R[nm]
        if nm in ("G_z", "rinv_z"):
            ref = ref[1:]   # the library stores z faces k = 0..nz-1
        got = g.debug_field(idx)
        assert rel(got, ref) < 1e-12, nm
    C = model.constants(P, True)
    ru, rv, rw = S.momentum_rhs(P, W.droplet_state(cfg), R, C)
    for idx, ref in zip((12, 13, 14), (ru, rv, rw)):
        assert rel(g.debug_field(idx), ref) < 1e-11, idx


def test_c1_hundred_steps(drpf):
    cfg = W.config("C1")
    g, st, gh, oh = run_both(drpf, cfg, cfg.steps)
    errs = field_errors(gh, oh, False)
    say(f"[gpu] C1 100 steps errors {errs}")
    for k, e in errs.items():
        assert e < TOL, (k, e)
    o_g = g.observables(st)
    o_o = S.observables(model.Params.from_config(cfg), oh)
    for k in ("mass", "wetted_radius", "centroid_height", "kinetic_energy"):
        assert o_g[k] == pytest.approx(o_o[k], rel=1e-10, abs=1e-14), k
    assert o_g["max_div"] < 1e-9


# Stated per-field bounds of the FP32 form (storage, stencils, transforms and the CH and
# velocity solves in FP32; the pressure Poisson, its zero mode and the mass sums in FP64)
# against the FP64 oracle: max |x - x_ref| / max |x_ref| after the stated number of steps.
# Each is about twice the error measured with the current kernels (which are deterministic):
# C2 20 steps phi 1.1e-5, u 5.4e-5, v 4.6e-5, w 1.8e-4, p 3.5e-5; C3 20 steps phi 1.5e-5,
# u 3.6e-5, v 2.5e-5, w 9.1e-5, p 5.6e-5, tau 3.1e-5; C5 2 steps phi 1.5e-6, u 6.1e-5,
# v 7.2e-5, w 2.2e-4, p 4.5e-5, tau 8.5e-5.
FP32_BOUND = {
    "C2": {"phi": 2e-5, "u": 1e-4, "v": 1e-4, "w": 4e-4, "p": 1e-4},
    "C3": {"phi": 3e-5, "u": 1e-4, "v": 1e-4, "w": 2e-4, "p": 2e-4, "tau": 1e-4},
    "C5": {"phi": 4e-6, "u": 2e-4, "v": 2e-4, "w": 4e-4, "p": 2e-4, "tau": 2e-4},
}
FULL_STEPS = {"C2": 20, "C3": 20, "C5": 2}


def run_forms(drpf, cfg, nsteps):
    """The oracle once, then the GPU FP64 and FP32 forms from the same input."""
    import torch
    P = model.Params.from_config(cfg)
    oh = W.droplet_state(cfg)
    for n in range(nsteps):
        oh = S.step(P, oh)
        say(f"[gpu] oracle {cfg.name} step {n + 1} of {nsteps}")
    out = {}
    for prec in (64, 32):
        say(f"[gpu] config {cfg.name} coarse {cfg.nx}x{cfg.ny}x{cfg.nz} steps {nsteps} fp{prec}")
        g = drpf.Grid(cfg, prec)
        st = g.state(W.droplet_state(cfg))
        g.step(st, nsteps)
        torch.cuda.synchronize()
        out[prec] = (st.to_host(), g.observables(st))
        del g, st
        torch.cuda.empty_cache()
    return P, oh, out


def check_forms(cfg, P, oh, out, nsteps):
    e64 = field_errors(out[64][0], oh, cfg.viscoelastic)
    e32 = field_errors(out[32][0], oh, cfg.viscoelastic)
    say(f"[gpu] {cfg.name} {nsteps} steps fp64 errors {e64}")
    say(f"[gpu] {cfg.name} {nsteps} steps fp32 errors {e32}")
    for k, e in e64.items():
        assert e < TOL, ("fp64", k, e)
    for k, e in e32.items():
        assert e < FP32_BOUND[cfg.name][k], ("fp32", k, e, FP32_BOUND[cfg.name][k])
    m0 = S.observables(P, W.droplet_state(cfg))["mass"]
    scale = np.sum(np.abs(oh["phi"][0])) * np.prod(P.hf)
    assert abs(out[64][1]["mass"] - m0) < 1e-12 * scale
    assert abs(out[32][1]["mass"] - m0) < 1e-6 * scale
    assert out[64][1]["max_div"] < 1e-8


@pytest.mark.timeout(900)
def test_full_size_c2_both_forms(drpf):
    """Launch configuration of the benchmark's Newtonian workload (128x128x64 coarse,
    256x256x128 fine, density ratio 1000, viscosity ratio 100): 20 steps against the oracle,
    the FP64 form at 1e-10 and the FP32 form at its stated per-field bounds; mass
    conservation and discrete incompressibility."""
    cfg = W.config("C2")
    n = FULL_STEPS["C2"]
    check_forms(cfg, *run_forms(drpf, cfg, n), n)


@pytest.mark.timeout(900)
def test_full_size_c3_both_forms(drpf):
    """The 3D Oldroyd-B set-up at full size (128x128x64 coarse, 256x256x128 fine, the
    z-marching momentum launch and the polymer stages at scale): 20 steps against the oracle,
    every field including the six stress components, in both forms."""
    cfg = W.config("C3")
    n = FULL_STEPS["C3"]
    check_forms(cfg, *run_forms(drpf, cfg, n), n)


@pytest.mark.timeout(900)
def test_full_size_c5_both_forms(drpf):
    """The largest set-up (256x256x128 coarse, 512x512x256 = 67.1M fine cells, Oldroyd-B,
    density and viscosity contrast; coarse x and y transforms in separate passes): two steps,
    so that the second-order (BDF2) step runs at these launch shapes, against the oracle in
    both forms."""
    cfg = W.config("C5")
    n = FULL_STEPS["C5"]
    check_forms(cfg, *run_forms(drpf, cfg, n), n)


def test_deterministic(drpf):
    import torch
    cfg = STEP_CASES[1][1]
    say("[gpu] determinism")
    outs = []
    for _ in range(2):
        g = drpf.Grid(cfg, 64)
        st = g.state(W.droplet_state(cfg))
        g.step(st, 3)
        torch.cuda.synchronize()
        outs.append(st.to_host())
    for f in ("phi", "u", "v", "w", "p"):
        assert np.array_equal(outs[0][f][0], outs[1][f][0]), f


def test_checkpoint_resume_bitwise(drpf):
    """2N straight steps equal N steps, a host round trip of the state, and N more."""
    import torch
    cfg = STEP_CASES[3][1]
    say("[gpu] checkpoint/resume")
    g = drpf.Grid(cfg, 64)
    a = g.state(W.droplet_state(cfg))
    g.step(a, 6)
    torch.cuda.synchronize()
    b = g.state(W.droplet_state(cfg))
    g.step(b, 3)
    torch.cuda.synchronize()
    saved = b.to_host()
    c = g.state(saved)
    g.step(c, 3)
    torch.cuda.synchronize()
    ha, hc = a.to_host(), c.to_host()
    for f in ("phi", "u", "v", "w", "p"):
        assert np.array_equal(ha[f][0], hc[f][0]), f
    for m in range(6):
        assert np.array_equal(ha["tau"][0][m], hc["tau"][0][m])


def test_observables_nonfinite(drpf):
    import torch
    cfg = STEP_CASES[0][1]
    g = drpf.Grid(cfg, 64)
    host = W.droplet_state(cfg)
    host["phi"][0][3, 0, 5] = np.nan
    st = g.state(host)
    o = g.observables(st)
    assert not o["finite"]
