"""Differentiable FP64 form of the oracle step, for the discrete adjoint (test
infrastructure only).

The same discrete step as ``oracle.step`` (Sec. 3.2 of the paper; every formula and ghost
rule identical), written with plain PyTorch CPU float64 operations so that reverse-mode
differentiation gives the exact transpose of the step's Jacobian: the oracle's own adjoint.
The constant-coefficient solves use FFT in x and y and, across the walls, the orthonormal
eigenbasis of the wall-normal second difference (DCT-II / DST-II / DST-I vectors) applied as a
dense matrix -- the same exact direct solve as the NumPy oracle, in differentiable form.

Parameters that the gradient is taken with respect to -- the bottom static angle theta (in
radians), the Peclet number Pe and the Weissenberg number Wi -- enter as tensors.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .model import Params

TT = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=TT)


# ---- neighbour access (as in oracle.discrete) ----------------------------------------

def xp(a):
    return torch.roll(a, -1, 2)


def xm(a):
    return torch.roll(a, 1, 2)


def yp(a):
    return torch.roll(a, -1, 1)


def ym(a):
    return torch.roll(a, 1, 1)


def zp_neu(a):
    return torch.cat([a[1:], a[-1:]], 0)


def zm_neu(a):
    return torch.cat([a[:1], a[:-1]], 0)


def zp_wall(a, top):
    """a[k+1] with the no-slip ghost of eq. NS13 beyond the top wall: 2 u_w - adjacent."""
    return torch.cat([a[1:], 2.0 * top - a[-1:]], 0)


def zm_wall(a, bot):
    return torch.cat([2.0 * bot - a[:1], a[:-1]], 0)


def zp_dir(a):
    return torch.cat([a[1:], -a[-1:]], 0)


def zm_dir(a):
    return torch.cat([-a[:1], a[:-1]], 0)


def zm_face(w):
    return torch.cat([torch.zeros_like(w[:1]), w[:-1]], 0)


def zp_face(w):
    return torch.cat([w[1:], torch.zeros_like(w[:1])], 0)


def zero_top(a):
    return torch.cat([a[:-1], torch.zeros_like(a[-1:])], 0)


def _lap_xy(a, h):
    hx, hy, _ = h
    return (xp(a) - 2 * a + xm(a)) / hx ** 2 + (yp(a) - 2 * a + ym(a)) / hy ** 2


def lap_neumann(a, h):
    return _lap_xy(a, h) + (zp_neu(a) - 2 * a + zm_neu(a)) / h[2] ** 2


def lap_dirichlet(a, h):
    return _lap_xy(a, h) + (zp_dir(a) - 2 * a + zm_dir(a)) / h[2] ** 2


def lap_wface(w, h):
    return zero_top(_lap_xy(w, h) + (zp_face(w) - 2 * w + zm_face(w)) / h[2] ** 2)


# ---- exact constant-coefficient solves -----------------------------------------------

def _zbasis(kind, nz, hz):
    """Orthonormal eigenvectors (columns) and eigenvalues of the wall-normal second
    difference for each boundary kind (DCT-II / DST-II / DST-I vectors)."""
    k = np.arange(nz)
    if kind == "neumann":
        m = np.arange(nz)
        B = np.cos(np.pi * np.outer(k + 0.5, m) / nz)
    elif kind == "dirichlet":
        m = np.arange(1, nz + 1)
        B = np.sin(np.pi * np.outer(k + 0.5, m) / nz)
    else:
        k = np.arange(nz - 1)
        m = np.arange(1, nz)
        B = np.sin(np.pi * np.outer(k + 1, m) / nz)
    B = B / np.linalg.norm(B, axis=0)
    lam = -4.0 / hz ** 2 * np.sin(np.pi * m / (2 * nz)) ** 2
    return torch.as_tensor(B, dtype=TT), torch.as_tensor(lam, dtype=TT)


_ZB = {}


def helmholtz(rhs, coeff, shift, kind, h):
    """Solve coeff L x - shift x = rhs (coeff and shift may be tensors)."""
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    key = (kind, nz, hz)
    if key not in _ZB:
        _ZB[key] = _zbasis(kind, nz, hz)
    B, lz = _ZB[key]
    lx = -4.0 / hx ** 2 * torch.sin(math.pi * torch.arange(nx, dtype=TT) / nx) ** 2
    ly = -4.0 / hy ** 2 * torch.sin(math.pi * torch.arange(ny, dtype=TT) / ny) ** 2
    X = torch.fft.fft2(rhs.to(torch.complex128), dim=(1, 2))
    nb = B.shape[0]
    Bc = B.to(torch.complex128)
    Z = torch.einsum("km,kyx->myx", Bc, X[:nb])
    denom = coeff * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]) - shift
    if kind == "neumann" and isinstance(shift, float) and shift == 0.0:
        mask = torch.ones_like(denom)
        mask[0, 0, 0] = 0.0
        denom = torch.where(mask > 0, denom, torch.ones_like(denom))
        Z = Z / denom * mask
    else:
        Z = Z / denom
    Y = torch.einsum("km,myx->kyx", Bc, Z)
    if kind == "wface":
        Y = torch.cat([Y, torch.zeros_like(Y[:1])], 0)
    return torch.fft.ifft2(Y, dim=(1, 2)).real


def relaxed_ch_solve(rhs, s, c, d, h):
    """Solve [L_N (L_N + d W) - s L_N + c] x = rhs, W the indicator of the two wall-adjacent
    layers: eq. NS25 with the relaxed wall condition of eq. NS34 (s and c may be tensors).
    FFT in x and y; for every Fourier mode (x-y eigenvalue mu) the nz x nz matrix
    (T + mu)(T + mu + d W) - s (T + mu) + c, T the wall-normal second difference with Neumann
    ghosts, is formed densely and solved directly (real and imaginary parts alike)."""
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    T = torch.zeros((nz, nz), dtype=TT)
    for k in range(nz):
        T[k, k] = -2.0
        if k > 0:
            T[k, k - 1] = 1.0
        else:
            T[k, k] += 1.0
        if k < nz - 1:
            T[k, k + 1] = 1.0
        else:
            T[k, k] += 1.0
    T = T / hz ** 2
    Wd = torch.zeros((nz, nz), dtype=TT)
    Wd[0, 0] = 1.0
    Wd[nz - 1, nz - 1] += 1.0
    lx = -4.0 / hx ** 2 * torch.sin(math.pi * torch.arange(nx, dtype=TT) / nx) ** 2
    ly = -4.0 / hy ** 2 * torch.sin(math.pi * torch.arange(ny, dtype=TT) / ny) ** 2
    I = torch.eye(nz, dtype=TT)
    mu = (ly[:, None] + lx[None, :])[:, :, None, None]
    A = T + mu * I                                     # (ny, nx, nz, nz)
    M = A @ (A + d * Wd) - s * A + c * I
    X = torch.fft.fft2(rhs.to(torch.complex128), dim=(1, 2)).permute(1, 2, 0)  # (ny, nx, nz)
    Xr = torch.stack([X.real, X.imag], dim=-1)         # (ny, nx, nz, 2)
    Y = torch.linalg.solve(M, Xr)
    Yc = torch.complex(Y[..., 0], Y[..., 1]).permute(2, 0, 1)
    return torch.fft.ifft2(Yc, dim=(1, 2)).real


# ---- fifth-order WENO-Z advection (Sec. 3.2.3; oracle.weno in differentiable form) --------

_WENO_EPS = 1e-40


def _weno_face(vm2, vm1, v0, vp1, vp2):
    """WENO-Z value at the face between v0 and vp1 from the side of v0 (oracle.weno.reconstruct
    with torch operations; |beta_0 - beta_2| differentiates to sign(0) = 0 at a tie)."""
    q0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0
    q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0
    q2 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0
    b0 = 13.0 / 12.0 * (vm2 - 2.0 * vm1 + v0) ** 2 + 0.25 * (vm2 - 4.0 * vm1 + 3.0 * v0) ** 2
    b1 = 13.0 / 12.0 * (vm1 - 2.0 * v0 + vp1) ** 2 + 0.25 * (vm1 - vp1) ** 2
    b2 = 13.0 / 12.0 * (v0 - 2.0 * vp1 + vp2) ** 2 + 0.25 * (3.0 * v0 - 4.0 * vp1 + vp2) ** 2
    t5 = torch.abs(b0 - b2)
    a0 = 0.1 * (1.0 + t5 / (b0 + _WENO_EPS))
    a1 = 0.6 * (1.0 + t5 / (b1 + _WENO_EPS))
    a2 = 0.3 * (1.0 + t5 / (b2 + _WENO_EPS))
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def _weno_shift(q, s, axis, wall):
    """q at index i + s along `axis`: periodic, or mirrored beyond the walls."""
    if not wall:
        return torch.roll(q, -s, axis)
    n = q.shape[axis]
    idx = np.arange(n) + s
    idx = np.where(idx < 0, -idx - 1, idx)
    idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
    return torch.index_select(q, axis, torch.as_tensor(idx, dtype=torch.long))


def _weno_flux(q, u, axis, wall):
    v = {s: _weno_shift(q, s, axis, wall) for s in range(-2, 4)}
    pos = _weno_face(v[-2], v[-1], v[0], v[1], v[2])
    neg = _weno_face(v[3], v[2], v[1], v[0], v[-1])
    return u * torch.where(u > 0.0, pos, neg)


def weno_divergence(q, u, v, w, h):
    """div(u q) with WENO-Z face values, x and y periodic, no flux through the walls."""
    hx, hy, hz = h
    fx = _weno_flux(q, u, 2, False)
    fy = _weno_flux(q, v, 1, False)
    fz = zero_top(_weno_flux(q, w, 0, True))
    return (fx - xm(fx)) / hx + (fy - ym(fy)) / hy + (fz - zm_face(fz)) / hz


# ---- transfers ------------------------------------------------------------------------

def prolong(u, v, w, ry):
    nz, ny, nx = u.shape
    uf = torch.stack([0.5 * (xm(u) + u), u], dim=3).reshape(nz, ny, 2 * nx)
    if ry == 2:
        uf = uf.repeat_interleave(2, dim=1)
        vf = torch.stack([0.5 * (ym(v) + v), v], dim=2).reshape(nz, 2 * ny, nx)
    else:
        vf = v
    uf = uf.repeat_interleave(2, dim=0)
    vf = vf.repeat_interleave(2, dim=2).repeat_interleave(2, dim=0)
    wf = torch.stack([0.5 * (zm_face(w) + w), w], dim=1).reshape(2 * nz, ny, nx)
    wf = wf.repeat_interleave(2, dim=2)
    if ry == 2:
        wf = wf.repeat_interleave(2, dim=1)
    return uf, vf, wf


def _restrict_axis(f, axis, loc, r, wall):
    n = f.shape[axis]
    idx = lambda i: torch.index_select(f, axis, torch.as_tensor(i, dtype=torch.long))
    if loc == "c":
        if r == 1:
            return f
        return 0.5 * (idx(np.arange(0, n, 2)) + idx(np.arange(1, n, 2)))
    if wall:
        kf = np.arange(-1, n // 2)
        return 0.5 * (idx(np.clip(2 * kf + 1, 0, n - 1)) + idx(np.clip(2 * kf + 2, 0, n - 1)))
    if r == 1:
        return 0.5 * (f + torch.roll(f, -1, axis))
    nc = n // 2
    return 0.5 * (idx((2 * np.arange(nc) + 1) % n) + idx((2 * np.arange(nc) + 2) % n))


def restrict(f, loc, ry):
    lz, ly, lx = loc
    g = _restrict_axis(f, 2, lx, 2, False)
    g = _restrict_axis(g, 1, ly, ry, False)
    return _restrict_axis(g, 0, lz, 2, True)


def mixture(phi, a1, a2):
    return 0.5 * (1.0 + phi) * a1 + 0.5 * (1.0 - phi) * a2


def divergence(u, v, w, h):
    return (u - xm(u)) / h[0] + (v - ym(v)) / h[1] + (w - zm_face(w)) / h[2]


def gradient(p, h):
    return (xp(p) - p) / h[0], (yp(p) - p) / h[1], zero_top((zp_neu(p) - p) / h[2])


# ---- the step --------------------------------------------------------------------------

def _levels(a, first):
    if first:
        return a[0], a[0]
    return 2.0 * a[0] - a[1], 2.0 * a[0] - 0.5 * a[1]


def constants(P: Params, first, pe):
    g0 = 1.0 if first else 1.5
    cn2 = P.cn ** 2
    S = P.s_factor * P.cn * torch.sqrt(4.0 * g0 * pe / P.dt)
    disc = 1.0 - 1.0 / (P.s_factor * P.s_factor)
    alpha = -(S / (2.0 * cn2)) * (1.0 + math.sqrt(disc))
    c_psi = alpha + S / cn2
    rho1, rho2 = 1.0, 1.0 / P.rho_ratio
    mu1 = P.beta if P.viscoelastic else 1.0
    mu2 = 1.0 / P.mu_ratio
    rho0 = min(rho1, rho2)
    nu_m = max(mu1, mu2) / (P.re * rho0)
    k_sigma = 3.0 / (2.0 * math.sqrt(2.0) * P.re * P.ca * P.cn)
    c_j = 0.5 * (rho1 - rho2) / pe
    return dict(gamma0=g0, S=S, alpha=alpha, c_psi=c_psi, rho1=rho1, rho2=rho2, mu1=mu1, mu2=mu2,
                rho0=rho0, nu_m=nu_m, k_sigma=k_sigma, c_j=c_j)


def step(P: Params, st, theta, pe, wi):
    """One coupled step on tensors; st holds lists of tensors like the NumPy oracle state."""
    if P.constitutive != 0 or P.refine != 2 or (P.d_w > 0.0 and P.moving_walls):
        raise NotImplementedError("the differentiable step covers the dual-resolution step with "
                                  "the stress form (Oldroyd-B or Giesekus), relaxed walls at rest")
    first = st["step"] == 0
    C = constants(P, first, pe)
    hf, h = P.hf, P.h
    cn2 = P.cn ** 2
    # ---- Cahn-Hilliard
    phis, phih = _levels(st["phi"], first)
    us = _levels(st["u"], first)[0]
    vs = _levels(st["v"], first)[0]
    ws = _levels(st["w"], first)[0]
    uf, vf, wf = prolong(us, vs, ws, P.ry)
    if P.advection == 1:
        A = weno_divergence(phis, uf, vf, wf, hf)
    else:
        fx = uf * 0.5 * (phis + xp(phis))
        fy = vf * 0.5 * (phis + yp(phis))
        fz = zero_top(wf * 0.5 * (phis + zp_neu(phis)))
        A = (fx - xm(fx)) / hf[0] + (fy - ym(fy)) / hf[1] + (fz - zm_face(fz)) / hf[2]
    fstar = (phis ** 3 - phis) / cn2
    Q = (pe / cn2) * (phih / P.dt - A) + lap_neumann(fstar - (C["S"] / cn2) * phis, hf)
    nzf = phis.shape[0]
    kz = torch.arange(nzf)
    bot = (kz == 0).to(TT)[:, None, None]
    top = (kz == nzf - 1).to(TT)[:, None, None]
    g1 = (1.0 - phis * phis) / (math.sqrt(2.0) * P.cn) / hf[2]
    b = g1 * (torch.cos(theta) * bot + math.cos(math.radians(P.theta_top_deg)) * top)
    if P.d_w == 0.0:
        Psi = helmholtz(Q - C["c_psi"] * b, 1.0, C["c_psi"], "neumann", hf)
        phi_new = helmholtz(Psi - b, 1.0, -C["alpha"], "neumann", hf)
        G = -cn2 * (lap_neumann(phi_new, hf) + b) + C["S"] * (phi_new - phis) + phis ** 3 - phis
    else:
        # relaxed walls (eqs. NS15, NS33, NS34): with kappa = D_w gamma0 / dt the wall-adjacent
        # ghost of phi^{n+1} carries -kappa phi^{n+1} + kappa phi_hat / gamma0 besides g, so
        # L_w = L_N + dL + b_R with dL = -kappa / hz and b_R = b + (kappa / hz) phi_hat / gamma0
        # on the wall layers; NS25 becomes [L_N (L_N + dL) - (S/Cn^2) L_N + c] phi^{n+1} =
        # Q - L_N b_R, c = gamma0 Pe / (Cn^2 dt)
        kap = P.d_w * C["gamma0"] / P.dt
        wall = bot + top
        dwall = -kap / hf[2]
        bR = b + (kap / hf[2]) * phih / C["gamma0"] * wall
        c = C["gamma0"] * pe / (cn2 * P.dt)
        phi_new = relaxed_ch_solve(Q - lap_neumann(bR, hf), C["S"] / cn2, c, dwall, hf)
        lw = lap_neumann(phi_new, hf) + dwall * wall * phi_new + bR
        G = -cn2 * lw + C["S"] * (phi_new - phis) + phis ** 3 - phis
    # ---- restriction and properties
    ry = P.ry
    R = lambda f, loc: restrict(f, loc, ry)
    phic = R(phi_new, "ccc")
    Gc = R(G, "ccc")
    Gf, rinv = {}, {}
    for name, loc in (("x", "ccf"), ("y", "cfc"), ("z", "fcc")):
        Gf[name] = R(G, loc)
        rinv[name] = 1.0 / mixture(R(phi_new, loc), C["rho1"], C["rho2"])
    mu_c = mixture(phic, C["mu1"], C["mu2"])
    mu_xy = mixture(R(phi_new, "cff"), C["mu1"], C["mu2"])
    mu_xz = mixture(R(phi_new, "fcf"), C["mu1"], C["mu2"])
    mu_yz = mixture(R(phi_new, "ffc"), C["mu1"], C["mu2"])
    # ---- momentum right-hand side (oracle.step.momentum_rhs, term by term)
    hx, hy, hz = h
    us, uh = _levels(st["u"], first)
    vs, vh = _levels(st["v"], first)
    ws, wh = _levels(st["w"], first)
    ps = _levels(st["p"], first)[0]
    pn = st["p"][0]
    if P.viscoelastic:
        taus = [_levels([st["tau"][0][c], st["tau"][1][c]], first)[0] for c in range(6)]
        T = [0.5 * (1.0 + phic) * t for t in taus]
    zc = lambda a: torch.cat([torch.zeros_like(a[:1]), a], 0)           # w on faces -1..nz-1
    # tangential wall velocities (eq. NS13): (bottom, top) of u and of v; 0 for walls at rest
    uw, vw = P.walls(0), P.walls(1)
    gh = lambda a, wv: torch.cat([2.0 * wv[0] - a[:1], a, 2.0 * wv[1] - a[-1:]], 0)  # k = -1 .. nz
    ued = lambda a, wv: 0.5 * (gh(a, wv)[:-1] + gh(a, wv)[1:])        # z edges k = -1 .. nz-1
    jx = -C["c_j"] * (xp(Gc) - xm(Gc)) / (2 * hx)
    jy = -C["c_j"] * (yp(Gc) - ym(Gc)) / (2 * hy)
    jz = -C["c_j"] * (zp_neu(Gc) - zm_neu(Gc)) / (2 * hz)
    # advection
    uc, ucl = 0.5 * (us + xp(us)), 0.5 * (xm(us) + us)
    adv_u = (uc * uc - ucl * ucl) / hx
    f = 0.5 * (vs + xp(vs)) * 0.5 * (us + yp(us))
    adv_u = adv_u + (f - ym(f)) / hy
    f = 0.5 * (zc(ws) + xp(zc(ws))) * ued(us, uw)
    adv_u = adv_u + (f[1:] - f[:-1]) / hz
    vc, vcl = 0.5 * (vs + yp(vs)), 0.5 * (ym(vs) + vs)
    adv_v = (vc * vc - vcl * vcl) / hy
    f = 0.5 * (us + yp(us)) * 0.5 * (vs + xp(vs))
    adv_v = adv_v + (f - xm(f)) / hx
    f = 0.5 * (zc(ws) + yp(zc(ws))) * ued(vs, vw)
    adv_v = adv_v + (f[1:] - f[:-1]) / hz
    wcu, wcl = 0.5 * (ws + zp_face(ws)), 0.5 * (zm_face(ws) + ws)
    adv_w = (wcu * wcu - wcl * wcl) / hz
    f = 0.5 * (us + zp_wall(us, uw[1])) * 0.5 * (ws + xp(ws))
    adv_w = adv_w + (f - xm(f)) / hx
    f = 0.5 * (vs + zp_wall(vs, vw[1])) * 0.5 * (ws + yp(ws))
    adv_w = adv_w + (f - ym(f)) / hy
    # J . grad u*
    fax = lambda a: 0.5 * (a + xp(a))
    fay = lambda a: 0.5 * (a + yp(a))
    faz = lambda a: 0.5 * (a + zp_neu(a))
    jgu = fax(jx) * (xp(us) - xm(us)) / (2 * hx) + fax(jy) * (yp(us) - ym(us)) / (2 * hy) \
        + fax(jz) * (zp_wall(us, uw[1]) - zm_wall(us, uw[0])) / (2 * hz)
    jgv = fay(jx) * (xp(vs) - xm(vs)) / (2 * hx) + fay(jy) * (yp(vs) - ym(vs)) / (2 * hy) \
        + fay(jz) * (zp_wall(vs, vw[1]) - zm_wall(vs, vw[0])) / (2 * hz)
    jgw = faz(jx) * (xp(ws) - xm(ws)) / (2 * hx) + faz(jy) * (yp(ws) - ym(ws)) / (2 * hy) \
        + faz(jz) * (zp_face(ws) - zm_face(ws)) / (2 * hz)
    # viscous
    vis_u = (2 * xp(mu_c) * (xp(us) - us) / hx - 2 * mu_c * (us - xm(us)) / hx) / hx
    sxy = mu_xy * ((yp(us) - us) / hy + (xp(vs) - vs) / hx)
    vis_u = vis_u + (sxy - ym(sxy)) / hy
    ue = gh(us, uw)
    we = zc(ws)
    sxz = mu_xz * ((ue[1:] - ue[:-1]) / hz + (xp(we) - we) / hx)
    vis_u = vis_u + (sxz[1:] - sxz[:-1]) / hz
    vis_v = (2 * yp(mu_c) * (yp(vs) - vs) / hy - 2 * mu_c * (vs - ym(vs)) / hy) / hy
    vis_v = vis_v + (sxy - xm(sxy)) / hx
    ve_ = gh(vs, vw)
    syz = mu_yz * ((ve_[1:] - ve_[:-1]) / hz + (yp(we) - we) / hy)
    vis_v = vis_v + (syz[1:] - syz[:-1]) / hz
    vis_w = (2 * zp_neu(mu_c) * (zp_face(ws) - ws) / hz - 2 * mu_c * (ws - zm_face(ws)) / hz) / hz
    vis_w = vis_w + (sxz[1:] - xm(sxz[1:])) / hx + (syz[1:] - ym(syz[1:])) / hy
    # polymer
    if P.viscoelastic:
        def eax_z(a):
            ae = 0.5 * (a + xp(a))
            return 0.5 * (torch.cat([ae[:1], ae], 0) + torch.cat([ae, ae[-1:]], 0))

        def eay_z(a):
            ae = 0.5 * (a + yp(a))
            return 0.5 * (torch.cat([ae[:1], ae], 0) + torch.cat([ae, ae[-1:]], 0))

        txz, tyz = eax_z(T[4]), eay_z(T[5])
        ae = 0.5 * (T[3] + xp(T[3]))
        txy = 0.5 * (ae + yp(ae))
        pol_u = (xp(T[0]) - T[0]) / hx + (txy - ym(txy)) / hy + (txz[1:] - txz[:-1]) / hz
        pol_v = (txy - xm(txy)) / hx + (yp(T[1]) - T[1]) / hy + (tyz[1:] - tyz[:-1]) / hz
        pol_w = (txz[1:] - xm(txz[1:])) / hx + (tyz[1:] - ym(tyz[1:])) / hy + (zp_neu(T[2]) - T[2]) / hz
    else:
        pol_u = pol_v = pol_w = 0.0
    gpn, gps = gradient(pn, h), gradient(ps, h)
    cap = (Gf["x"] * (xp(phic) - phic) / hx, Gf["y"] * (yp(phic) - phic) / hy,
           Gf["z"][1:] * (zp_neu(phic) - phic) / hz)
    ri = (rinv["x"], rinv["y"], rinv["z"][1:])
    lap_w = lambda a, wv: _lap_xy(a, h) + (zp_wall(a, wv[1]) - 2 * a + zm_wall(a, wv[0])) / hz ** 2
    lap = (lap_w(us, uw), lap_w(vs, vw), lap_wface(ws, h))
    hats, advs, jgs = (uh, vh, wh), (adv_u, adv_v, adv_w), (jgu, jgv, jgw)
    viss, pols = (vis_u, vis_v, vis_w), (pol_u, pol_v, pol_w)
    r = []
    for a in range(3):
        ra = (-hats[a] / P.dt + advs[a] + ri[a] * jgs[a] + gpn[a] / C["rho0"]
              + (ri[a] - 1.0 / C["rho0"]) * gps[a] + C["nu_m"] * lap[a]
              - (1.0 / P.re) * ri[a] * pols[a] - (1.0 / P.re) * ri[a] * viss[a]
              - C["k_sigma"] * ri[a] * cap[a] - P.a_ext[a])
        r.append(ra)
    r[2] = zero_top(r[2])
    # ---- projection
    g = C["gamma0"] / P.dt
    # moving walls: the implicit Laplacian's ghosts carry 2 u_w / hz^2 on the wall layers, a
    # known term moved to the right-hand side
    nzc = r[0].shape[0]
    kz = torch.arange(nzc)
    wb_ = lambda wv: (2.0 / hz ** 2) * (wv[0] * (kz == 0).to(TT) + wv[1] * (kz == nzc - 1).to(TT))[:, None, None]
    ut = helmholtz(r[0] - C["nu_m"] * wb_(uw), C["nu_m"], g, "dirichlet", h)
    vt = helmholtz(r[1] - C["nu_m"] * wb_(vw), C["nu_m"], g, "dirichlet", h)
    wt = helmholtz(r[2], C["nu_m"], g, "wface", h)
    dp = helmholtz((C["gamma0"] * C["rho0"] / P.dt) * divergence(ut, vt, wt, h), 1.0, 0.0, "neumann", h)
    gx, gy, gz = gradient(dp, h)
    cc = P.dt / (C["gamma0"] * C["rho0"])
    u, v, w = ut - cc * gx, vt - cc * gy, zero_top(wt - cc * gz)
    p = st["p"][0] + dp
    # ---- polymer RK2-TVD
    if P.viscoelastic:
        tau = polymer(P, st["tau"][0], u, v, w, wi)
    else:
        tau = [torch.zeros_like(p) for _ in range(6)]
    return {"phi": [phi_new, st["phi"][0]], "u": [u, st["u"][0]], "v": [v, st["v"][0]],
            "w": [w, st["w"][0]], "p": [p, st["p"][0]], "tau": [tau, st["tau"][0]],
            "step": st["step"] + 1}


_PAIRS = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4,
          (1, 2): 5, (2, 1): 5}


def velocity_gradient(P, u, v, w):
    hx, hy, hz = P.h
    cen = (0.5 * (u + xm(u)), 0.5 * (v + ym(v)), 0.5 * (w + zm_face(w)))
    L = [[None] * 3 for _ in range(3)]
    L[0][0] = (u - xm(u)) / hx
    L[1][1] = (v - ym(v)) / hy
    L[2][2] = (w - zm_face(w)) / hz
    for b in range(3):
        f = cen[b]
        if b != 0:
            L[0][b] = (xp(f) - xm(f)) / (2 * hx)
        if b != 1:
            L[1][b] = (yp(f) - ym(f)) / (2 * hy)
        if b != 2:
            wv = P.walls(b)
            L[2][b] = (zp_wall(f, wv[1]) - zm_wall(f, wv[0])) / (2 * hz)
    return L


def polymer_rhs(P, tau, u, v, w, L, wi):
    hx, hy, hz = P.h
    out = []
    for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)):
        t = tau[_PAIRS[(a, b)]]
        if P.advection == 1:
            rh = -weno_divergence(t, u, v, w, P.h)
        else:
            fx = u * 0.5 * (t + xp(t))
            fy = v * 0.5 * (t + yp(t))
            fz = zero_top(w * 0.5 * (t + zp_neu(t)))
            rh = -((fx - xm(fx)) / hx + (fy - ym(fy)) / hy + (fz - zm_face(fz)) / hz)
        for c in range(3):
            rh = rh + L[c][a] * tau[_PAIRS[(c, b)]] + tau[_PAIRS[(a, c)]] * L[c][b]
        rh = rh + ((1.0 - P.beta) * (L[a][b] + L[b][a]) - t) / wi
        if P.giesekus_alpha != 0.0:
            # Giesekus (eq. NS4 with alpha > 0): -alpha / (1 - beta) tau.tau
            tt = sum(tau[_PAIRS[(a, c)]] * tau[_PAIRS[(c, b)]] for c in range(3))
            rh = rh - P.giesekus_alpha / (1.0 - P.beta) * tt
        out.append(rh)
    return out


def polymer(P, tau_n, u, v, w, wi):
    L = velocity_gradient(P, u, v, w)
    rh0 = polymer_rhs(P, tau_n, u, v, w, L, wi)
    t1 = [tau_n[c] + P.dt * rh0[c] for c in range(6)]
    rh1 = polymer_rhs(P, t1, u, v, w, L, wi)
    return [0.5 * tau_n[c] + 0.5 * (t1[c] + P.dt * rh1[c]) for c in range(6)]


# ---- observables ------------------------------------------------------------------------

def wetted_radius(P, phi):
    hx, hy, _ = P.hf
    ind0 = 0.5 * (1.0 + phi[0])
    if P.ny == 1:
        return 0.5 * hx * ind0.sum()
    return torch.sqrt(hx * hy * ind0.sum() / math.pi)


def centroid_height(P, phi):
    ind = 0.5 * (1.0 + phi)
    z = (torch.arange(phi.shape[0], dtype=TT) + 0.5) * P.hf[2]
    return (ind * z[:, None, None]).sum() / ind.sum()


# ---- helpers ------------------------------------------------------------------------------

FIELDS = ("phi", "u", "v", "w", "p")


def to_torch(st, requires_grad=False):
    out = {f: [_t(a).clone().requires_grad_(requires_grad) for a in st[f]] for f in FIELDS}
    out["tau"] = [[_t(a).clone().requires_grad_(requires_grad) for a in st["tau"][l]] for l in range(2)]
    out["step"] = st["step"]
    return out


def flat(st):
    """Ordered list of the state tensors (phi, u, v, w, p levels, then tau levels)."""
    xs = [a for f in FIELDS for a in st[f]]
    xs += [a for l in range(2) for a in st["tau"][l]]
    return xs


def _inner(a, b):
    return (a * b).sum()


def adjoint_step(P: Params, st, lam, theta_rad=None, pe=None, wi=None):
    """Transpose of one step's Jacobian, applied to ``lam`` (the adjoint of the state after the
    step, same structure as a state). Returns (adjoint of the state before the step,
    [dJ/dtheta_bottom (per radian), dJ/dPe, dJ/dWi]) where J = <lam, step(state)>.

    The wall-normal velocity on the top wall is identically zero in every state, so its
    adjoint carries no information; it is returned as zero.
    """
    theta_rad = math.radians(P.theta_bottom_deg) if theta_rad is None else theta_rad
    th = torch.tensor(theta_rad, dtype=TT, requires_grad=True)
    pe_t = torch.tensor(P.pe if pe is None else pe, dtype=TT, requires_grad=True)
    wi_t = torch.tensor(P.wi if wi is None else wi, dtype=TT, requires_grad=True)
    t = to_torch(st, requires_grad=True)
    new = step(P, t, th, pe_t, wi_t)
    lt = to_torch(lam)
    s = sum(_inner(a, b) for a, b in zip(flat(new), flat(lt)))
    ins = flat(t) + [th, pe_t, wi_t]
    gr = torch.autograd.grad(s, ins, allow_unused=True)
    gr = [torch.zeros_like(x) if g is None else g for x, g in zip(ins, gr)]
    it = iter(g.detach().numpy().copy() for g in gr[:-3])
    out = {f: [next(it), next(it)] for f in FIELDS}
    out["tau"] = [[next(it) for _ in range(6)] for _ in range(2)]
    out["step"] = st["step"]
    for l in range(2):
        out["w"][l][-1] = 0.0
    grad3 = np.array([float(g) for g in gr[-3:]])
    if not P.viscoelastic:
        grad3[2] = 0.0
    return out, grad3


def trajectory_gradient(P: Params, st0, nsteps, observable, theta_rad=None, pe=None, wi=None):
    """Gradient of observable(P, phi at the end) with respect to (theta_bottom [rad], Pe, Wi)
    by reverse differentiation through ``nsteps`` unrolled steps (small cases only)."""
    theta_rad = math.radians(P.theta_bottom_deg) if theta_rad is None else theta_rad
    th = torch.tensor(theta_rad, dtype=TT, requires_grad=True)
    pe_t = torch.tensor(P.pe if pe is None else pe, dtype=TT, requires_grad=True)
    wi_t = torch.tensor(P.wi if wi is None else wi, dtype=TT, requires_grad=True)
    s = to_torch(st0)
    for _ in range(nsteps):
        s = step(P, s, th, pe_t, wi_t)
    J = observable(P, s["phi"][0])
    gr = torch.autograd.grad(J, [th, pe_t, wi_t], allow_unused=True)
    g = np.array([0.0 if x is None else float(x) for x in gr])
    return float(J.detach()), g
