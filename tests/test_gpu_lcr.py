"""GPU parity of the log-conformation polymer update and of the Giesekus term (stress form):
the HIP path through the C-ABI against the FP64 oracle (oracle/lcr.py, oracle/step.py) on the
same seeded inputs, 1e-10 relative per field in FP64 (Theta and tau included)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W
from oracle import lcr
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


def initial(cfg, theta_amp=0.0, seed=11):
    """The droplet state; with theta_amp > 0 a seeded log-conformation field, entries
    theta_amp * U(-1, 1), and the matching stress at both levels."""
    st = W.droplet_state(cfg)
    if theta_amp > 0:
        cs = W.coarse_shape(cfg)
        n = int(np.prod(cs))
        r = 2.0 * W.splitmix64_uniform(seed, 6 * n) - 1.0
        st["theta"] = [theta_amp * r[m * n:(m + 1) * n].reshape(cs) for m in range(6)]
        tau = lcr.stress(model.Params.from_config(cfg), st["theta"])
        st["tau"] = [[t.copy() for t in tau], [t.copy() for t in tau]]
    return st


def errors(gh, oh, lcr_form):
    e = {k: rel(gh[k][0], oh[k][0]) for k in ("phi", "u", "w", "p")}
    if np.max(np.abs(oh["v"][0])) > 0:
        e["v"] = rel(gh["v"][0], oh["v"][0])
    e["tau"] = max(rel(gh["tau"][0][c], oh["tau"][0][c]) for c in range(6)
                   if np.max(np.abs(oh["tau"][0][c])) > 0)
    if lcr_form:
        e["theta"] = max(rel(gh["theta"][c], oh["theta"][c]) for c in range(6)
                         if np.max(np.abs(oh["theta"][c])) > 0)
    return e


def run_both(drpf, cfg, nsteps, theta_amp=0.0, precision=64):
    import torch
    say(f"[gpu] {cfg.name} coarse {cfg.nx}x{cfg.ny}x{cfg.nz} constitutive {cfg.constitutive} "
        f"alpha {cfg.giesekus_alpha} theta_amp {theta_amp} steps {nsteps} fp{precision}")
    g = drpf.Grid(cfg, precision)
    st = g.state(initial(cfg, theta_amp))
    g.step(st, nsteps)
    torch.cuda.synchronize()
    gh = st.to_host()
    oh = S.run(model.Params.from_config(cfg), initial(cfg, theta_amp), nsteps)
    return gh, oh


C3S = W.config("C3", nx=16, ny=16, nz=8, lx=1.0, ly=1.0, lz=0.5, radius=0.2, noise=1e-3, seed=5,
               wi=0.5)
C4S = W.config("C4", nx=32, nz=16, ly=2.0 / 32, noise=1e-3, seed=6)

CASES = [
    ("3d-lcr-oldroyd", C3S.replace(constitutive=1), 5, 0.0),
    ("3d-lcr-giesekus", C3S.replace(constitutive=1, giesekus_alpha=0.3), 5, 0.0),
    ("3d-lcr-random-theta", C3S.replace(constitutive=1, giesekus_alpha=0.2), 3, 0.5),
    ("2d-lcr-giesekus", C4S.replace(constitutive=1, giesekus_alpha=0.25), 6, 0.3),
    ("3d-stress-giesekus", C3S.replace(giesekus_alpha=0.3), 5, 0.0),
    ("2d-stress-giesekus", C4S.replace(giesekus_alpha=0.4), 6, 0.0),
]


@pytest.mark.parametrize("name,cfg,n,amp", CASES, ids=[c[0] for c in CASES])
def test_polymer_forms_match_oracle(drpf, name, cfg, n, amp):
    gh, oh = run_both(drpf, cfg, n, amp)
    errs = errors(gh, oh, cfg.constitutive == 1)
    say(f"[gpu] {name} errors {errs}")
    for k, e in errs.items():
        assert e < TOL, (k, e)


def test_full_size_c3_log_conformation_two_steps(drpf):
    """The C3 launch configuration (128x128x64 coarse) in the log-conformation form with a
    Giesekus term and a seeded Theta: two steps, every field, Theta and tau."""
    cfg = W.config("C3", constitutive=1, giesekus_alpha=0.2)
    gh, oh = run_both(drpf, cfg, 2, theta_amp=0.3)
    errs = errors(gh, oh, True)
    say(f"[gpu] C3 log-conformation full-size errors {errs}")
    for k, e in errs.items():
        assert e < TOL, (k, e)


def test_fp32_log_conformation_tracks_fp64(drpf):
    """The FP32 form (FP64 eigensolves) stays within FP32 round-off growth of the FP64 run."""
    import torch
    cfg = C3S.replace(constitutive=1, giesekus_alpha=0.2)
    outs = {}
    for prec in (64, 32):
        g = drpf.Grid(cfg, prec)
        st = g.state(initial(cfg, 0.3))
        g.step(st, 20)
        torch.cuda.synchronize()
        outs[prec] = st.to_host()
    for c in range(6):
        assert np.all(np.isfinite(outs[32]["theta"][c]))
        assert rel(outs[32]["theta"][c], outs[64]["theta"][c]) < 1e-4, c
        assert rel(outs[32]["tau"][0][c], outs[64]["tau"][0][c]) < 1e-3, c
