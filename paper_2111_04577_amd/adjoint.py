"""Gradients through many coupled steps: a ``torch.autograd.Function`` over the library's
forward step and its discrete adjoint (drpf_adjoint_step), with checkpointed recomputation.

The forward pass runs the steps and keeps a device snapshot of the state every ``every``
steps. The backward pass walks the segments from the last to the first: it restores the
segment's snapshot, recomputes the segment's states, and applies the adjoint step to each in
reverse order, handing each reverse step the state after it, so that the library recomputes
only the two forward intermediates it needs (the restricted coarse set and the first polymer
stage). Memory: one snapshot per segment plus one segment of states (a snapshot is one
device copy); work: one extra forward step per step plus the reverse step.

Differentiable inputs: the bottom static contact angle theta (radians), Pe and Wi. Outputs:
phi, u, v, w, p at the final level (device tensors, FP64); any torch function of them can be
the objective, e.g. :func:`wetted_radius` or :func:`centroid_height` (the observables of the
adjoint case, Sec. 4 of the paper).
"""
from __future__ import annotations

import dataclasses
import math

from .binding import DeviceState, Grid


def _make_function():
    import torch

    class _Steps(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, pe, wi, cfg, init, nsteps, every):
            c = dataclasses.replace(cfg, theta_bottom_deg=math.degrees(float(theta)), pe=float(pe),
                                    wi=float(wi))
            grid = Grid(c, precision=64)
            grid.attach_adjoint()
            st = grid.state(init)
            ckpts = []
            for n in range(nsteps):
                if n % every == 0:
                    ckpts.append(st.snapshot())
                grid.step(st, 1)
            ctx.grid, ctx.state, ctx.ckpts = grid, st, ckpts
            ctx.nsteps, ctx.every = int(nsteps), int(every)
            ctx.like = (theta, pe, wi)
            return tuple(x.clone() for x in (st.phi[0], st.u[0], st.v[0], st.w[0], st.p[0]))

        @staticmethod
        def backward(ctx, gphi, gu, gv, gw, gp):
            grid, st = ctx.grid, ctx.state
            lam = grid.adjoint()
            for name, g in zip(("phi", "u", "v", "w", "p"), (gphi, gu, gv, gw, gp)):
                if g is not None:
                    getattr(lam, name)[0].copy_(g)
            grad3 = torch.zeros(3, dtype=torch.float64, device=grid.device)
            N, k = ctx.nsteps, ctx.every
            ve = bool(grid.params.viscoelastic)
            for s in reversed(range(len(ctx.ckpts))):
                start, end = s * k, min(N, s * k + k)
                st.restore(ctx.ckpts[s])
                seg = [ctx.ckpts[s]]
                for n in range(start, end):
                    grid.step(st, 1)
                    seg.append(st.snapshot())
                structs = [DeviceState.struct_of(x, ve) for x in seg]
                for n in reversed(range(start, end)):
                    i = n - start
                    grid.adjoint_step(structs[i], lam, grad3, next_state=structs[i + 1])
            ctx.lam0 = lam
            out = [grad3[a].to(dtype=x.dtype, device=x.device) if torch.is_tensor(x) else None
                   for a, x in enumerate(ctx.like)]
            return out[0], out[1], out[2], None, None, None, None

    return _Steps


_FN = None


def run(theta, pe, wi, cfg, init: dict, nsteps: int, every: int = 50):
    """Final (phi, u, v, w, p) after ``nsteps`` steps from the host state ``init`` with the
    set-up ``cfg`` whose theta_bottom_deg, pe and wi are replaced by the tensors ``theta``
    (radians), ``pe`` and ``wi``. Differentiable in those three; checkpoints every ``every``."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    if nsteps < 1 or every < 1:
        raise ValueError("need nsteps >= 1 and every >= 1")
    return _FN.apply(theta, pe, wi, cfg, init, int(nsteps), int(every))


def wetted_radius(cfg, phi):
    """2D: half the wetted length; 3D: sqrt(wetted area / pi); from (1 + phi)/2 on the
    wall-adjacent fine layer (as drpf_observables)."""
    import torch
    ry = 1 if cfg.ny == 1 else 2
    hx, hy = cfg.lx / (2 * cfg.nx), cfg.ly / (ry * cfg.ny)
    s = (0.5 * (1.0 + phi[0])).sum()
    return 0.5 * hx * s if cfg.ny == 1 else torch.sqrt(hx * hy * s / math.pi)


def centroid_height(cfg, phi):
    """sum(z (1 + phi)/2) / sum((1 + phi)/2) over the fine cells."""
    import torch
    hz = cfg.lz / (2 * cfg.nz)
    ind = 0.5 * (1.0 + phi)
    z = (torch.arange(phi.shape[0], dtype=phi.dtype, device=phi.device) + 0.5) * hz
    return (ind * z[:, None, None]).sum() / ind.sum()
