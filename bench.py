#!/usr/bin/env python3
"""Benchmark of the dual-resolution phase-field step on one MI355X.

Workload (headline): the largest single-GPU set-up, a 3D Oldroyd-B drop with density ratio 100
and viscosity ratio 10 (coarse 256x256x128, fine 512x512x256 = 67.1M phase-field cells, Wi 2,
beta 0.3, Cn 0.01, Re 1, static angle 45 deg, dt 5e-5), synthetic initial state
(hemispherical drop on the bottom wall, zero flow and stress). Inputs are resident in HBM
before timing starts.

Timed: K whole coupled steps (Cahn-Hilliard fine solve, restriction, Navier-Stokes
projection, polymer stress) after W warm-up steps, bracketed by synchronisations and HIP
events on the stream the library launches on. Both precision forms are timed: the FP32 form
(FP64 kept for the pressure Poisson wall-normal solve, its zero mode and the mass sums) is the
headline value, the FP64 form is reported beside it; the workload's own protocol (10 warm-up,
200 timed steps) is timed too when K and W differ from it.

Accuracy beside the rate: the FP32 and FP64 forms against the FP64 oracle after the steps of
the oracle's timed sample (the CPU baseline runs the oracle on the same workload), and the
FP32 form against the FP64 form over long runs of smaller workloads.

Per-kernel durations come from HIP events recorded by the library after every launch
(drpf_profile_begin / drpf_profile_end) in a second pass of K steps; the roofline entry is
for the kernel with the largest share of that time.

Prints ONE JSON line. ``--gpus N`` with N > 1 exits: the library targets one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="C5")
    ap.add_argument("--precision", choices=["both", "32", "64"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="steps of the oracle sample (each leg); also the step count of the accuracy check")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-protocol", action="store_true",
                    help="skip the workload's own 10 + 200 step timing (short profiled runs)")
    ap.add_argument("--others", default="C2,C3,C3L,C3P,C2R,C2S,C3S",
                    help="further workloads timed in both forms beside the headline one ('' for none)")
    ap.add_argument("--other-steps", type=int, default=100)
    ap.add_argument("--no-error", action="store_true",
                    help="skip the FP32-vs-FP64 per-field error runs (C2 500 steps, C3, C3L and C3P 1000 steps)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run only the gradient case and print its JSON object")
    ap.add_argument("--adjoint-config", default="C4")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="steps of the gradient case (default: the config's own, 2000 for C4)")
    ap.add_argument("--adjoint-every", type=int, default=50)
    ap.add_argument("--ingest-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON", "WORKLOAD"),
                    help="turn rocprofv3 --pmc counter CSVs of one workload into the traffic summary and exit")
    return ap.parse_args()


# ---------------------------------------------------------------------------------------
# algorithmic bytes per launch: every kernel reads its inputs once and writes its outputs
# once (spectral buffers count as complex arrays of (nx/2+1) ny nz entries)
# ---------------------------------------------------------------------------------------

def grid_sizes(cfg):
    r = 1 if cfg.refine == 1 else 2  # single resolution: the phase field on the flow grid
    ry = 1 if cfg.ny == 1 else r
    F = dict(nx=r * cfg.nx, ny=ry * cfg.ny, nz=r * cfg.nz)
    C = dict(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz)
    for d in (F, C):
        d["cells"] = d["nx"] * d["ny"] * d["nz"]
        d["spec"] = (d["nx"] // 2 + 1) * d["ny"] * d["nz"]
    return F, C


def alg_bytes(kernel, cfg, es):
    F, C = grid_sizes(cfg)
    nf, nc = F["cells"], C["cells"]
    sf, sc = F["spec"] * 2, C["spec"] * 2   # complex -> 2 words
    ne = C["nx"] * C["ny"] * (C["nz"] + 1)
    ve = cfg.viscoelastic
    words = {
        # with WENO-Z the advection arrives precomputed (read once) instead of the velocities
        "ch_rhs": 4 * nf if cfg.advection == 1 else 3 * nf + 6 * nc,
        "weno_adv_fine": 3 * nf + 6 * nc if cfg.advection == 1 else 0,
        "fft_x_fwd_fine": nf + sf,
        "fft_y_fwd_fine": 2 * sf if F["ny"] > 1 else 0,
        "zpass_ch": 2 * sf,
        "fft_y_inv_fine": 2 * sf if F["ny"] > 1 else 0,
        "fft_x_inv_fine": sf + nf,
        # single resolution: G and phi at the cells (2 N_c written), then faces and edges from
        # them (2 N_c read back) in a second kernel, both under this timing id
        "restrict_g": 3 * nf + (12 if cfg.refine == 1 else 10) * nc + 2 * ne,
        "momentum_rhs": (8 + 10 + 12 * ve + 3) * nc + 2 * ne,
        "fft_x_fwd_coarse": 3 * nc + 3 * sc,
        "fft_y_fwd_coarse": 6 * sc if C["ny"] > 1 else 0,
        "zpass_ns": 7 * sc,
        "fft_y_inv_coarse": 8 * sc if C["ny"] > 1 else 0,
        "fft_x_inv_coarse": 4 * sc + 5 * nc,
        # the x and y passes in one kernel: the spectral round trip between them is gone
        "fft_xy_fwd_coarse": 3 * nc + 3 * sc,
        "fft_xy_inv_coarse": 4 * sc + 5 * nc,
        # log-conformation: stage 2 also writes tau from the new Theta
        "polymer_stage1": 15 * nc if ve else 0,
        "polymer_stage2": (27 if cfg.constitutive == 1 else 21) * nc if ve else 0,
        # both stages in one pass: u, v, w and tau^n read, tau^{n+1} written
        "polymer_rk2": 15 * nc if ve else 0,
    }
    return words[kernel] * es


KERNEL_SOURCE = {
    "ch_rhs": "stencil_ch.hip", "restrict_g": "stencil_ch.hip", "weno_adv_fine": "stencil_ch.hip",
    "momentum_rhs": "stencil_ns.hip",
    "polymer_stage1": "stencil_ns.hip", "polymer_stage2": "stencil_ns.hip", "polymer_rk2": "stencil_ns.hip",
    "zpass_ch": "tridiag.hip", "zpass_ns": "tridiag.hip",
}


def source_sha(kernel):
    """Hash of the kernel's source file and of every shared header it may include."""
    csrc = os.path.join(ROOT, "paper_2111_04577_amd", "csrc")
    names = [KERNEL_SOURCE.get(kernel, "fft.hip")] + sorted(f for f in os.listdir(csrc) if f.endswith(".hpp"))
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(csrc, n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_entry(kernel, precision, workload):
    """HBM bytes per launch of a kernel on a workload from the committed counter summary, if
    it was taken on that workload and on the current source of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(f"{kernel}/fp{precision}/{workload}")
    if not e or e.get("source_sha") != source_sha(kernel):
        return None
    return e.get("bytes_per_launch")


# ---------------------------------------------------------------------------------------

def time_form(drpf, W, cfg, precision, steps, warmup):
    import torch
    g = drpf.Grid(cfg, precision)
    st = g.state(W.droplet_state(cfg))
    g.step(st, warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(st, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # per-kernel pass (HIP events after every launch, same stream)
    g.profile_begin(steps * 17 + 1)
    g.step(st, steps)
    prof = g.profile_end()
    torch.cuda.synchronize()
    obs = g.observables(st)
    return g, st, ms, wall, prof, obs


def roofline_for(prof, cfg, precision, steps):
    total = {k: v[0] for k, v in prof.items() if v[1] > 0}
    dom = max(total, key=total.get)
    ms_total, launches = prof[dom]
    avg_s = ms_total / launches / 1e3
    b = alg_bytes(dom, cfg, 8 if precision == 64 else 4)
    achieved = b / avg_s / 1e9
    kernels = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": v[1],
                   "share": round(v[0] / sum(total.values()), 4),
                   "alg_GBs": round(alg_bytes(k, cfg, 8 if precision == 64 else 4) / (v[0] / v[1] / 1e3) / 1e9, 1)}
               for k, v in prof.items() if v[1] > 0}
    traffic = traffic_entry(dom, precision, cfg.name)
    return {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": b, "avg_us": round(avg_s * 1e6, 2)}, kernels


def field_diff(a, b):
    """max |a - b| / max |b| and rms(a - b) / max |b| per field (tau: over its six
    components, when b has a non-zero stress)."""
    import numpy as np
    out = {}
    pairs = [(f, a[f][0], b[f][0]) for f in ("phi", "u", "v", "w", "p")]
    if any(float(np.max(np.abs(t))) > 0 for t in b["tau"][0]):
        pairs.append(("tau", np.stack(a["tau"][0]), np.stack(b["tau"][0])))
    for f, x, ref in pairs:
        den = float(np.max(np.abs(ref)))
        out[f] = float(np.max(np.abs(x - ref))) / (den if den > 0 else 1.0)
        out[f + "_rms"] = float(np.sqrt(np.mean((x - ref) ** 2))) / (den if den > 0 else 1.0)
    return {k: float(f"{v:.3e}") for k, v in out.items()}


def precision_error(drpf, W, name, nsteps):
    """Per-field difference of the FP32 form from the FP64 form (which matches the FP64 CPU
    reference to 1e-10) after nsteps steps of the named workload, and both masses."""
    import torch
    cfg = W.config(name)
    out = {}
    for prec in (32, 64):
        g = drpf.Grid(cfg, prec)
        st = g.state(W.droplet_state(cfg))
        g.step(st, nsteps)
        torch.cuda.synchronize()
        out[prec] = (st.to_host(), g.observables(st)["mass"])
        del g, st
        torch.cuda.empty_cache()
    d = field_diff(out[32][0], out[64][0])
    d.update({"after_steps": nsteps, "mass_fp32": out[32][1], "mass_fp64": out[64][1],
              "mass_rel": float(f"{abs(out[32][1] - out[64][1]) / abs(out[64][1]):.3e}")})
    return d


def copy_ceiling(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth on this GPU (read + write bytes / time)."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def time_adjoint(drpf, W, name, nsteps, every):
    """The gradient case: d(final wetted radius)/d(theta, Pe, Wi) through nsteps FP64 steps with
    checkpoints every `every` steps (torch.autograd.Function over drpf_step and
    drpf_adjoint_step). Times the plain forward run, the checkpointed forward and the
    backward pass with events on the stream the library launches on, and one reverse step
    (drpf_adjoint_step alone, which recomputes its forward step) against one forward step."""
    import torch
    import paper_2111_04577_amd.adjoint as ADJ
    cfg = W.config(name)
    nsteps = nsteps or cfg.steps
    init = W.droplet_state(cfg)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    g = drpf.Grid(cfg, 64)
    st = g.state(init)
    g.step(st, 10)
    st = g.state(init)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    g.step(st, nsteps)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    # one reverse step vs one forward step, on the state after nsteps: with the state after
    # the step handed in (as in the backward pass) and with the full forward recompute
    g.attach_adjoint()
    lam = g.adjoint(W.adjoint_seed(cfg, 1))
    g3 = torch.zeros(3, dtype=torch.float64, device=g.device)
    x0 = st.snapshot()
    g.step(st, 1)
    xs = type(st).struct_of(x0, bool(cfg.viscoelastic))
    reps = 50

    def per_call(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    adj_step_ms = per_call(lambda: g.adjoint_step(xs, lam, g3, next_state=st))
    adj_full_ms = per_call(lambda: g.adjoint_step(xs, lam, g3))
    del g, st, lam, x0
    th = torch.tensor(math.radians(cfg.theta_bottom_deg), dtype=torch.float64, requires_grad=True)
    pe = torch.tensor(cfg.pe, dtype=torch.float64, requires_grad=True)
    wi = torch.tensor(cfg.wi, dtype=torch.float64, requires_grad=True)
    t0, t1, t2 = ev(), ev(), ev()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t0.record()
    outs = ADJ.run(th, pe, wi, cfg, init, nsteps, every)
    t1.record()
    J = ADJ.wetted_radius(cfg, outs[0])
    J.backward()
    t2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ckpt_ms, bwd_ms = t0.elapsed_time(t1), t1.elapsed_time(t2)
    F, _ = grid_sizes(cfg)
    return {
        "workload": f"{cfg.name}: 2D Oldroyd-B drop, coarse {cfg.nx}x{cfg.nz}, fine {F['nx']}x{F['nz']}, "
                    f"{nsteps} steps, checkpoints every {every}, J = final wetted radius, "
                    f"theta {cfg.theta_bottom_deg:g} deg, Pe {cfg.pe:g}, Wi {cfg.wi:g}",
        "dtype": "f64",
        "fwd_ms_per_step": round(fwd_ms / nsteps, 5),
        "fwd_ckpt_ms_per_step": round(ckpt_ms / nsteps, 5),
        "bwd_ms_per_step": round(bwd_ms / nsteps, 5),
        "adj_fwd": round(bwd_ms / fwd_ms, 3),
        "adjoint_step_ms": round(adj_step_ms, 5),
        "adjoint_step_vs_fwd_step": round(adj_step_ms / (fwd_ms / nsteps), 3),
        "adjoint_step_full_recompute_ms": round(adj_full_ms, 5),
        "gradient_wall_s": round(wall, 3),
        "J": float(J.detach()),
        "grad": {"theta_per_rad": float(th.grad), "pe": float(pe.grad), "wi": float(wi.grad)},
    }


def host_info():
    """Host CPU model, logical CPU count and the NumPy / SciPy versions."""
    import numpy as np
    import scipy
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "numpy": np.__version__, "scipy": scipy.__version__}


def cpu_baseline(W, cfg, nsteps):
    """The FP64 oracle as it stands on the host, timed over the first nsteps steps of the
    workload, twice: with scipy.fft on every logical CPU (the transforms of its solves; its
    elementwise NumPy work is single-threaded either way) and on one. Returns the record and
    the oracle state after the steps."""
    import scipy.fft as sfft
    from oracle import model
    from oracle import step as S
    P = model.Params.from_config(cfg)
    F, _ = grid_sizes(cfg)
    legs = {}
    state = None
    ncpu = os.cpu_count() or 1
    for workers in (ncpu, 1):
        st = W.droplet_state(cfg)
        with sfft.set_workers(workers):
            t0 = time.perf_counter()
            for _ in range(nsteps):
                st = S.step(P, st)
            dt = time.perf_counter() - t0
        legs[workers] = (F["cells"] * nsteps / dt, dt)
        if state is None:
            state = st
        del st
    info = host_info()
    sample = (f"first {nsteps} steps of the same workload ({cfg.name}, full grid, {F['cells']} fine cells); "
              f"NumPy/SciPy FP64 oracle; scipy.fft workers = {ncpu} for its transforms, elementwise NumPy "
              f"single-threaded; {legs[ncpu][1]:.1f} s")
    rec = {"value": round(legs[ncpu][0], 1), "unit": "fine cell-updates/s", "cores": ncpu, "kind": "oracle",
           "sample": sample,
           "one_core": {"value": round(legs[1][0], 1), "cores": 1, "seconds": round(legs[1][1], 2),
                        "sample": f"the same {nsteps} steps with scipy.fft workers = 1"}}
    rec.update(info)
    return rec, state


# the oracle's rate on the other workloads: steps timed on every logical CPU (a few suffice)
ORACLE_RATE_STEPS = (("C1", 20), ("C2", 2), ("C3", 2))


def oracle_rates(W, plan=ORACLE_RATE_STEPS):
    """Fine cell-updates/s of the FP64 oracle on C1, C2 and C3 over their first steps, scipy.fft
    on every logical CPU (context beside the headline's own oracle timing)."""
    import scipy.fft as sfft
    from oracle import model
    from oracle import step as S
    ncpu = os.cpu_count() or 1
    out = {}
    for name, nsteps in plan:
        cfg = W.config(name)
        P = model.Params.from_config(cfg)
        F, _ = grid_sizes(cfg)
        st = W.droplet_state(cfg)
        with sfft.set_workers(ncpu):
            t0 = time.perf_counter()
            for _ in range(nsteps):
                st = S.step(P, st)
            dt = time.perf_counter() - t0
        out[name] = {"value": round(F["cells"] * nsteps / dt, 1), "steps": nsteps, "seconds": round(dt, 2),
                     "cores": ncpu}
        del st
    return out


def accuracy_vs_oracle(drpf, W, cfg, nsteps, oracle_state):
    """Per-field error of both GPU forms against the oracle after nsteps steps from the same
    initial state (max |x - x_ref| / max |x_ref| and rms / max |x_ref|)."""
    import torch
    out = {"after_steps": nsteps, "workload": cfg.name}
    for prec in (32, 64):
        g = drpf.Grid(cfg, prec)
        st = g.state(W.droplet_state(cfg))
        g.step(st, nsteps)
        torch.cuda.synchronize()
        out[f"fp{prec}"] = field_diff(st.to_host(), oracle_state)
        del g, st
        torch.cuda.empty_cache()
    return out


def ingest_pmc(fetch_csv, write_csv, out_json, workload):
    """rocprofv3 --pmc counter_collection.csv files (one run with FETCH_SIZE, one with
    WRITE_SIZE, each of `bench.py --copy-calibration` on one workload) -> HBM bytes per launch
    of every kernel on that workload, merged into out_json under kernel/precision/workload.
    Each counter (KiB per dispatch) is scaled by (copy bytes) / (the same counter read on the
    1 GiB device copy of that run). Kernels launched on both grids are told apart by their
    grid size (the larger is the fine grid)."""
    import csv
    import re
    from collections import defaultdict

    copy_bytes = 2 ** 30  # the largest copy dispatch of the run: 1 GiB (calibration, copy ceiling)

    def read(path, counter):
        per = defaultdict(list)
        copies = []
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name, val = row["Kernel_Name"], float(row["Counter_Value"])
                if "copyBuffer" in name or "copy" in name.lower() and "k_" not in name:
                    copies.append(val)
                    continue
                # template arguments: the element type, then (fft_y) the direction flag, then
                # launch-shape parameters that do not name a different operation
                m = re.search(r"(k_\w+)<(float|double)((?:, \w+)*)>", name)
                if not m:
                    continue
                # the run-time length forms of the transform passes (suffix _rt) are the same
                # operations
                kname = m.group(1)[:-3] if m.group(1).endswith("_rt") else m.group(1)
                flag = re.search(r"\b(true|false)\b", m.group(3)) if kname == "k_fft_y" else None
                per[(kname, m.group(2), flag.group(1) if flag else None,
                     int(row["Grid_Size"]))].append(val)
        scale = copy_bytes / (max(copies) * 1024) if copies else None
        return per, scale

    fetch, fs = read(fetch_csv, "FETCH_SIZE")
    write, ws = read(write_csv, "WRITE_SIZE")
    # the polymer divergence pass is timed with the momentum kernel (one profiling id): its bytes
    # are added to momentum_rhs's
    base = {"k_ch_rhs": "ch_rhs", "k_restrict_g": "restrict_g", "k_momentum_rhs": "momentum_rhs",
            "k_momentum_rhs_zm": "momentum_rhs", "k_polymer_div_zm": "momentum_rhs", "k_polymer_rk2_zm": "polymer_rk2",
            "k_zpass_ch": "zpass_ch", "k_zpass_ns": "zpass_ns",
            "k_fft_xy_fwd": "fft_xy_fwd_coarse", "k_fft_xy_inv": "fft_xy_inv_coarse"}
    sizes = defaultdict(set)
    for (k, t, inv, g) in fetch:
        sizes[(k, t, inv)].add(g)
    out = {}
    if os.path.exists(out_json):
        with open(out_json) as f:
            out = json.load(f)
    acc = {}
    for key, vals in fetch.items():
        k, t, inv, g = key
        if key not in write or fs is None or ws is None:
            continue
        if k in base:
            name = base[k]
        elif k in ("k_fft_x_fwd", "k_fft_x_inv", "k_fft_y"):
            grid = "fine" if g == max(sizes[(k, t, inv)]) else "coarse"
            kind = {"k_fft_x_fwd": "fft_x_fwd", "k_fft_x_inv": "fft_x_inv"}.get(k)
            if kind is None:
                kind = "fft_y_inv" if inv == "true" else "fft_y_fwd"
            name = f"{kind}_{grid}"
        else:
            continue
        prec = 32 if t == "float" else 64
        fb = sum(vals) / len(vals) * 1024 * fs
        wb = sum(write[key]) / len(write[key]) * 1024 * ws
        ent = acc.setdefault(f"{name}/fp{prec}/{workload}", {"fetch_bytes": 0.0, "write_bytes": 0.0,
                                                             "dispatches": len(vals), "name": name})
        ent["fetch_bytes"] += fb
        ent["write_bytes"] += wb
    for key, ent in acc.items():
        out[key] = {"bytes_per_launch": round(ent["fetch_bytes"] + ent["write_bytes"]),
                    "fetch_bytes": round(ent["fetch_bytes"]), "write_bytes": round(ent["write_bytes"]),
                    "dispatches": ent["dispatches"], "source_sha": source_sha(ent["name"])}
    out["_calibration"] = {"copy_bytes": copy_bytes, "fetch_scale": fs, "write_scale": ws}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out["_calibration"]))
    return out


def compulsory_bytes_per_cell(cfg, es):
    """Compulsory bytes per fine cell-update of the hot-path byte model (each stage reads its
    inputs and writes its outputs once, spectral intermediates not counted): 11 fine words plus
    60 coarse words per coarse cell (Newtonian) or 110 (viscoelastic), a coarse cell being 8
    fine cells in 3D and 4 in 2D (where the velocity has two components and the stress three:
    21.5 and 28.25 words)."""
    if cfg.ny == 1:
        words = 28.25 if cfg.viscoelastic else 21.5
    else:
        words = 24.75 if cfg.viscoelastic else 18.5
    return words * es


def describe(cfg):
    F, _ = grid_sizes(cfg)
    law = "Newtonian"
    if cfg.viscoelastic:
        law = f"Giesekus alpha {cfg.giesekus_alpha:g}" if cfg.giesekus_alpha else f"Oldroyd-B Wi {cfg.wi:g} beta {cfg.beta:g}"
        law += ", log-conformation" if cfg.constitutive == 1 else ", stress form"
    law += ", WENO-Z advection" if cfg.advection == 1 else ", central advection"
    if cfg.d_w > 0:
        law += f", relaxed walls D_w {cfg.d_w:g}"
    if cfg.refine == 1:
        law += ", single resolution"
    dim = "2D" if cfg.ny == 1 else "3D"
    return (f"{cfg.name}: {dim} drop on a wall, {law}, coarse {cfg.nx}x{cfg.ny}x{cfg.nz}, fine "
            f"{F['nx']}x{F['ny']}x{F['nz']} ({F['cells']} cells), rho ratio {cfg.rho_ratio:g}, mu ratio "
            f"{cfg.mu_ratio:g}, Re {cfg.re:g}, Cn {cfg.cn:g}, Pe {cfg.pe:g}, theta {cfg.theta_bottom_deg:g} deg, "
            f"dt {cfg.dt:g}")


def step_bandwidth(cfg, kernels, steps, ms_per_step, es, ceiling):
    """Whole-step bandwidth by two byte models: the sum of the kernels' algorithmic bytes
    (spectral intermediates included) and the compulsory bytes per fine cell of the hot-path
    model, each against the HBM peak and the measured copy ceiling."""
    F, _ = grid_sizes(cfg)
    kb = sum(alg_bytes(k, cfg, es) * v["launches"] / steps for k, v in kernels.items())
    sb = compulsory_bytes_per_cell(cfg, es) * F["cells"]
    out = {}
    for name, b in (("kernel_bytes", kb), ("compulsory_bytes", sb)):
        gbs = b / (ms_per_step / 1e3) / 1e9
        out[name] = {"bytes_per_step": int(b), "achieved": round(gbs, 1),
                     "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "frac_of_copy": round(gbs / ceiling, 4)}
    out["copy_ceiling"] = round(ceiling, 1)
    return out


def time_plain(drpf, W, cfg, precision, steps, warmup):
    """Step time without the per-kernel pass (the workload's own protocol)."""
    import torch
    g = drpf.Grid(cfg, precision)
    st = g.state(W.droplet_state(cfg))
    g.step(st, warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    g.step(st, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del g, st
    torch.cuda.empty_cache()
    return ms / steps


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {a.gpus}): the step is not decomposed across GPUs",
              file=sys.stderr)
        sys.exit(2)
    if a.ingest_pmc:
        ingest_pmc(*a.ingest_pmc)
        return
    import numpy as np
    import torch
    import workloads as W
    import paper_2111_04577_amd as drpf
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.only_adjoint:
        print(json.dumps(time_adjoint(drpf, W, a.adjoint_config, a.adjoint_steps, a.adjoint_every)), flush=True)
        return
    cfg = W.config(a.config)
    F, C = grid_sizes(cfg)
    forms = {"both": (32, 64), "32": (32,), "64": (64,)}[a.precision]
    res = {}
    for prec in forms:
        print(f"[bench] timing fp{prec} {cfg.name}: {a.warmup} warm-up + {a.steps} steps", file=sys.stderr, flush=True)
        g, st, ms, wall, prof, obs = time_form(drpf, W, cfg, prec, a.steps, a.warmup)
        roof, kernels = roofline_for(prof, cfg, prec, a.steps)
        res[prec] = {"ms_per_step": ms / a.steps, "value": F["cells"] * a.steps / (ms / 1e3),
                     "wall_s": wall, "roofline": roof, "kernels": kernels, "observables": obs}
        del g, st
        torch.cuda.empty_cache()
    if a.copy_calibration:
        x = torch.empty(2 ** 30 // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    head = 32 if 32 in res else 64
    out = {
        # the value is the FP32 form's rate; the FP64 form, the per-field errors of both forms
        # against the oracle and the adjoint's adj/fwd ratio are reported beside it
        "metric": "fine-grid cell-updates/s per dual-res step, FP32 vs FP64 at stated error; adj/fwd",
        "value": round(res[head]["value"], 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(res[head]["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": describe(cfg),
                   "fine_cells": F["cells"], "coarse_cells": C["cells"],
                   "precision_islands": "FP64 Poisson wall-normal solve, zero mode, mass sums"
                   if head == 32 else "all FP64"},
        "roofline": res[head]["roofline"],
        "kernels": res[head]["kernels"],
    }
    ceiling = copy_ceiling(torch)
    for prec in res:
        es = 4 if prec == 32 else 8
        res[prec]["step_bw"] = step_bandwidth(cfg, res[prec]["kernels"], a.steps, res[prec]["ms_per_step"], es, ceiling)
    out["step_bandwidth"] = res[head]["step_bw"]
    if 64 in res and head != 64:
        out["fp64"] = {"value": round(res[64]["value"], 1), "ms_per_step": round(res[64]["ms_per_step"], 4),
                       "roofline": res[64]["roofline"], "step_bandwidth": res[64]["step_bw"],
                       "kernels": res[64]["kernels"]}
        out["fp32_vs_fp64_speedup"] = round(res[32]["value"] / res[64]["value"], 3)
    # the workload's own protocol (10 warm-up, 200 timed steps), when K and W differ from it
    if (a.steps, a.warmup) != (200, 10) and not a.no_protocol:
        proto = {"warmup": 10, "steps": 200}
        for prec in forms:
            print(f"[bench] protocol fp{prec} {cfg.name}: 10 warm-up + 200 steps", file=sys.stderr, flush=True)
            msps = time_plain(drpf, W, cfg, prec, 200, 10)
            proto[f"fp{prec}"] = {"value": round(F["cells"] / (msps / 1e3), 1), "ms_per_step": round(msps, 4)}
        out["protocol_200_steps"] = proto
    if 64 in res and head != 64 and not a.no_error:
        print("[bench] FP32 vs FP64 error: C2 500 steps, C3, C3L and C3P 1000 steps", file=sys.stderr,
              flush=True)
        out["fp32_error_vs_fp64"] = {"C2": precision_error(drpf, W, "C2", 500),
                                     "C3": precision_error(drpf, W, "C3", 1000),
                                     "C3L": precision_error(drpf, W, "C3L", 1000),
                                     "C3P": precision_error(drpf, W, "C3P", 1000)}
    others = [x for x in a.others.split(",") if x and x != cfg.name]
    if others:
        out["other_workloads"] = {}
    for name in others:
        ocfg = W.config(name)
        OF, OC = grid_sizes(ocfg)
        ent = {"workload": describe(ocfg), "steps": a.other_steps}
        for prec in (32, 64):
            print(f"[bench] timing fp{prec} {name}: 5 warm-up + {a.other_steps} steps", file=sys.stderr, flush=True)
            g, st, ms, wall, prof, obs = time_form(drpf, W, ocfg, prec, a.other_steps, 5)
            roof, kern = roofline_for(prof, ocfg, prec, a.other_steps)
            es = 4 if prec == 32 else 8
            msps = ms / a.other_steps
            ent[f"fp{prec}"] = {"value": round(OF["cells"] * a.other_steps / (ms / 1e3), 1),
                                "ms_per_step": round(msps, 4),
                                "step_bandwidth": step_bandwidth(ocfg, kern, a.other_steps, msps, es, ceiling),
                                "roofline": roof}
            del g, st
            torch.cuda.empty_cache()
        ent["fp32_vs_fp64_speedup"] = round(ent["fp32"]["value"] / ent["fp64"]["value"], 3)
        out["other_workloads"][name] = ent
    # dual- vs single-resolution step time at the same phase-field grid (256x256x128):
    # C2 / C2S (Newtonian) and C3 / C3S (Oldroyd-B)
    ow = out.get("other_workloads", {})
    dvs = {}
    for kind, dname, sname in (("newtonian", "C2", "C2S"), ("viscoelastic", "C3", "C3S")):
        if dname not in ow or sname not in ow:
            continue
        dvs[kind] = {}
        for prec in (32, 64):
            t_dual = ow[dname][f"fp{prec}"]["ms_per_step"]
            t_single = ow[sname][f"fp{prec}"]["ms_per_step"]
            dvs[kind][f"fp{prec}"] = {"dual_ms": round(t_dual, 4), "single_ms": round(t_single, 4),
                                      "speedup": round(t_single / t_dual, 3)}
    if dvs:
        out["dual_vs_single_resolution"] = dvs
    if not a.no_adjoint:
        print(f"[bench] gradient case {a.adjoint_config}", file=sys.stderr, flush=True)
        out["adjoint"] = time_adjoint(drpf, W, a.adjoint_config, a.adjoint_steps, a.adjoint_every)
        out["adj_fwd"] = out["adjoint"]["adj_fwd"]
    else:
        out["adj_fwd"] = None
    if not a.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle, {a.cpu_steps} steps of {cfg.name}, all cores then one",
              file=sys.stderr, flush=True)
        out["cpu_baseline"], ostate = cpu_baseline(W, cfg, a.cpu_steps)
        print("[bench] oracle rates on C1, C2, C3", file=sys.stderr, flush=True)
        out["cpu_baseline"]["other_workloads"] = oracle_rates(W)
        print(f"[bench] both forms against the oracle after {a.cpu_steps} steps", file=sys.stderr, flush=True)
        out["error_vs_oracle"] = accuracy_vs_oracle(drpf, W, cfg, a.cpu_steps, ostate)
        del ostate
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
