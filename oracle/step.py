"""One coupled dual-resolution time step (oracle; test infrastructure only).

Order of one step (Sec. 3.2): Cahn-Hilliard on the fine grid with the prolonged velocity,
restriction of phi and G to the coarse grid, Navier-Stokes projection, polymer stress.
Time levels: n (index 0) and n-1 (index 1). The first step (``step == 0``) is the
one-level start: gamma0 = 1 and g_hat = g_star = g^n; every later step uses the BDF2
weights and extrapolation of eqs. NS31-NS32.

State dictionary (FP64 numpy arrays): ``phi``, ``u``, ``v``, ``w``, ``p`` -- each a list
[level n, level n-1]; ``tau`` -- [level n, level n-1], each a list of the six components
(xx, yy, zz, xy, xz, yz); ``theta`` -- the six components of the log-conformation at level n
(advanced only by the log-conformation form, lcr.py); ``step`` -- int.
"""
from __future__ import annotations

import math

import numpy as np

from . import discrete as D
from . import lcr
from . import weno
from .model import Params, constants

XX, YY, ZZ, XY, XZ, YZ = range(6)


def _levels(a, first):
    """(g_star, g_hat): eq. NS32 and eq. NS31, or g^n twice on the first step."""
    if first:
        return a[0], a[0]
    return 2.0 * a[0] - a[1], 2.0 * a[0] - 0.5 * a[1]


# ---------------------------------------------------------------------------------------
# Cahn-Hilliard (Sec. 3.2.1)
# ---------------------------------------------------------------------------------------


def wall_data(P: Params, phis):
    """Wetting data b: the static-angle condition (eq. NS15 with D_w = 0, wall energy of
    eq. NS16) gives the outward normal derivative n.grad(phi) = cos(theta) (1 - phi_w^2) /
    (sqrt(2) Cn), with phi_w the extrapolated phase field of the wall-adjacent fine cell
    (eq. NS34 evaluated at phi*). A ghost equal to the adjacent value plus hz_f times that
    derivative adds b = g / hz_f to the Laplacian of the wall-adjacent cells."""
    hzf = P.hf[2]
    b = np.zeros_like(phis)
    for layer, th in ((0, P.theta_bottom_deg), (-1, P.theta_top_deg)):
        pw = phis[layer]
        g = math.cos(math.radians(th)) * (1.0 - pw * pw) / (math.sqrt(2.0) * P.cn)
        b[layer] += g / hzf
    return b


def advection_fine(phis, uf, vf, wf, hf, scheme=0):
    """div(u phi) in flux form with the mean of the two adjacent cells on each face (scheme 1:
    the WENO-Z face value, weno.py) and zero flux through the walls."""
    if scheme == 1:
        return weno.divergence(phis, uf, vf, wf, hf, D)
    hx, hy, hz = hf
    fx = uf * 0.5 * (phis + D.xp(phis))
    fy = vf * 0.5 * (phis + D.yp(phis))
    fz = wf * 0.5 * (phis + D.zp_neu(phis))
    fz[-1] = 0.0
    return (fx - D.xm(fx)) / hx + (fy - D.ym(fy)) / hy + (fz - D.zm_face(fz)) / hz


def cahn_hilliard(P: Params, st, C):
    """Eqs. NS25-NS34: returns (phi^{n+1}, G^{n+1}, phi_star, Psi)."""
    hf = P.hf
    first = st["step"] == 0
    cn2 = P.cn ** 2
    phis, phih = _levels(st["phi"], first)
    us = _levels(st["u"], first)[0]
    vs = _levels(st["v"], first)[0]
    ws = _levels(st["w"], first)[0]
    uf, vf, wf = D.prolong(us, vs, ws, P.ry, P.refine)              # eq. dual1
    A = advection_fine(phis, uf, vf, wf, hf, P.advection)
    fstar = (phis ** 3 - phis) / cn2                                  # eq. NS6, eta = Cn
    Q = (P.pe / cn2) * (phih / P.dt - A) + D.lap_neumann(fstar - (C.S / cn2) * phis, hf)  # NS28
    b = wall_data(P, phis)
    if P.d_w > 0.0:
        return _cahn_hilliard_relaxed(P, C, Q, b, phis, phih)
    # Eq. NS26 with the boundary condition of eq. NS33, and eq. NS27 with that of eq. NS34.
    # With L_N the Laplacian with homogeneous-Neumann ghosts and L_w = L_N + b the one with
    # the wetting ghosts, NS25 reads (L_N - c_psi)(L_N + alpha) phi = Q - L_N b; setting
    # Psi = L_w phi + alpha phi (eq. NS27) gives (L_N - c_psi) Psi = Q - c_psi b.
    Psi = D.helmholtz(Q - C.c_psi * b, 1.0, C.c_psi, "neumann", hf)
    phi_new = D.helmholtz(Psi - b, 1.0, -C.alpha, "neumann", hf)
    # Chemical potential at n+1: lambda times the bracket of eq. NS25, i.e.
    # Cn^2 [-L_w phi + (S/Cn^2)(phi - phi*) + f(phi*)].
    G = -cn2 * (D.lap_neumann(phi_new, hf) + b) + C.S * (phi_new - phis) + phis ** 3 - phis
    return phi_new, G, phis, Psi


def _cahn_hilliard_relaxed(P: Params, C, Q, b, phis, phih):
    """Eqs. NS25-NS34 with the wall relaxation D_w > 0 of eq. NS15.

    Eq. NS34 adds D_w (gamma0 phi^{n+1} - phi_hat) / dt to the wall derivative of phi^{n+1}
    and moves D_w u* . grad phi* to its right-hand side (the wall value is the wall-adjacent
    cell's, as for the static data b). On a wall u* is that wall's velocity (eq. NS13):
    tangential, so the term is D_w (u_w d/dx + v_w d/dy) phi* with central differences on the
    wall-adjacent layer, and zero at walls at rest. With kappa = D_w gamma0 / dt
    the ghost of the wall-adjacent cell becomes adjacent + hz (g - kappa phi^{n+1} +
    kappa phi_hat / gamma0): L_w phi = L_R phi + b_R, L_R = L_N + dL with dL = -kappa / hz
    on the wall-adjacent layers, b_R = b + (kappa / hz) phi_hat / gamma0 there.

    Eq. NS33 carries the wall derivative of phi^{n+1} itself, so the two Helmholtz problems
    are solved together: NS25 is [L_N L_R - (S/Cn^2) L_N + c] phi^{n+1} = Q - L_N b_R with
    c = gamma0 Pe / (Cn^2 dt), the outer Laplacian keeping the zero-flux walls of the chemical
    potential (mass is conserved exactly). Psi = (L_R + alpha) phi^{n+1} + b_R (eq. NS27).
    """
    hf = P.hf
    cn2 = P.cn ** 2
    kap = P.d_w * C.gamma0 / P.dt
    hz = hf[2]
    dL = np.zeros_like(phis)
    dL[0] = -kap / hz
    dL[-1] = -kap / hz
    bR = b.copy()
    bR[0] += (kap / hz) * phih[0] / C.gamma0
    bR[-1] += (kap / hz) * phih[-1] / C.gamma0
    if P.moving_walls:
        # the wall advection of eq. NS34, -D_w u_w . grad phi*, in the ghost: -(D_w / hz) u_w . grad phi*
        for layer, side in ((0, 0), (-1, 1)):
            pw = phis[layer]  # (ny, nx) on the wall-adjacent layer, periodic in x and y
            dx = (np.roll(pw, -1, axis=1) - np.roll(pw, 1, axis=1)) / (2.0 * hf[0])
            dy = (np.roll(pw, -1, axis=0) - np.roll(pw, 1, axis=0)) / (2.0 * hf[1])
            adv = P.walls(0)[side] * dx + P.walls(1)[side] * dy
            bR[layer] -= (P.d_w / hz) * adv
    c = C.gamma0 * P.pe / (cn2 * P.dt)
    phi_new = D.ch_relaxed_solve(Q - D.lap_neumann(bR, hf), C.S / cn2, c, -kap / hz, hf)
    lw = D.lap_neumann(phi_new, hf) + dL * phi_new + bR
    Psi = lw + C.alpha * phi_new
    G = -cn2 * lw + C.S * (phi_new - phis) + phis ** 3 - phis
    return phi_new, G, phis, Psi


def restricted_set(P: Params, phi, G, C):
    """Coarse quantities the momentum equation needs (eqs. dual2, dual3): phi and G at
    centres, G and 1/rho at the three face sets, solvent viscosity at centres and at the
    three edge sets. z-face and z-edge arrays carry nz + 1 layers (wall .. wall)."""
    ry = P.ry
    R = lambda f, loc: D.restrict(f, loc, ry, P.refine)
    out = {}
    out["phi_c"] = R(phi, "ccc")
    out["G_c"] = R(G, "ccc")
    for name, loc in (("x", "ccf"), ("y", "cfc"), ("z", "fcc")):
        ph = R(phi, loc)
        out["G_" + name] = R(G, loc)
        out["rinv_" + name] = 1.0 / D.mixture(ph, C.rho1, C.rho2)
    out["mu_c"] = D.mixture(out["phi_c"], C.mu1, C.mu2)
    for name, loc in (("xy", "cff"), ("xz", "fcf"), ("yz", "ffc")):
        out["mu_" + name] = D.mixture(R(phi, loc), C.mu1, C.mu2)
    return out


# ---------------------------------------------------------------------------------------
# Navier-Stokes (Sec. 3.2.2)
# ---------------------------------------------------------------------------------------


def _zc_dir(a, walls):
    """Cell-centred velocity with no-slip ghosts for the wall values (bottom, top):
    (a[k-1], a[k+1])."""
    return D.zm_dir(a, walls[0]), D.zp_dir(a, walls[1])


def momentum_rhs(P: Params, st, R, C):
    """Right-hand side r of eq. NS36 for each velocity component at its own faces
    (nu_m L u~ - gamma0/dt u~ = r), including the -u_hat/dt term of eq. NS35, the
    extrapolated velocity u* in every explicit term, p^n and p* in the pressure split,
    the polymer divergence of approach 2 (eq. NS12, drop = polymer phase) and the
    capillary force. Tangential velocities take the wall values of eq. NS13 (u = u_w) through
    their ghosts. Returns (r_u, r_v, r_w) with r_w[nz-1] = 0 (top wall)."""
    hx, hy, hz = P.h
    uw, vw = P.walls(0), P.walls(1)
    first = st["step"] == 0
    us, uh = _levels(st["u"], first)
    vs, vh = _levels(st["v"], first)
    ws, wh = _levels(st["w"], first)
    ps = _levels(st["p"], first)[0]
    pn = st["p"][0]
    if P.viscoelastic:
        taus = [(_levels([st["tau"][0][c], st["tau"][1][c]], first)[0]) for c in range(6)]
        wgt = 0.5 * (1.0 + R["phi_c"])
        T = [wgt * t for t in taus]
    else:
        T = None
    dt = P.dt
    inv_re = 1.0 / P.re
    mu_c = R["mu_c"]
    # edges: xy edge (i, j) at ((i+1) hx, (j+1) hy); xz edge layer m = k + 1 for
    # z = (k+1) hz, k = -1 .. nz-1; same for yz.
    mu_xy, mu_xz, mu_yz = R["mu_xy"], R["mu_xz"], R["mu_yz"]

    # ---- chemical-potential gradient at centres, J = -c_j grad G (text after eq. NS10)
    Gc = R["G_c"]
    jx = -C.c_j * (D.xp(Gc) - D.xm(Gc)) / (2 * hx)
    jy = -C.c_j * (D.yp(Gc) - D.ym(Gc)) / (2 * hy)
    jz = -C.c_j * (D.zp_neu(Gc) - D.zm_neu(Gc)) / (2 * hz)
    phic = R["phi_c"]

    # ---- u at x faces ---------------------------------------------------------------
    def edge_avg_xz(a):
        """Mean of a centred field over the 4 centres around each xz edge, layers
        k = -1 .. nz-1 (Neumann ghosts beyond the walls)."""
        ae = 0.5 * (a + D.xp(a))
        lo = np.concatenate([ae[:1], ae], axis=0)
        hi = np.concatenate([ae, ae[-1:]], axis=0)
        return 0.5 * (lo + hi)

    def edge_avg_yz(a):
        ae = 0.5 * (a + D.yp(a))
        lo = np.concatenate([ae[:1], ae], axis=0)
        hi = np.concatenate([ae, ae[-1:]], axis=0)
        return 0.5 * (lo + hi)

    def edge_avg_xy(a):
        ae = 0.5 * (a + D.xp(a))
        return 0.5 * (ae + D.yp(ae))

    # u at xz edges (z layers k = -1..nz-1) with no-slip ghosts, w at xz edges
    def with_ghosts(a, walls):
        return np.concatenate([2.0 * walls[0] - a[:1], a, 2.0 * walls[1] - a[-1:]], axis=0)  # k = -1 .. nz

    def u_on_zedges(a, walls):
        ext = with_ghosts(a, walls)
        return 0.5 * (ext[:-1] + ext[1:])                   # edges k = -1 .. nz-1

    def w_ext(a):
        """w on z faces k = -1 .. nz-1 (bottom wall 0 prepended)."""
        return np.concatenate([np.zeros_like(a[:1]), a], axis=0)

    # advection  div(u* u*)
    uc = 0.5 * (us + D.xp(us))                 # u at centre i+1 (right of face i)
    ucl = 0.5 * (D.xm(us) + us)                # u at centre i
    adv_u = (uc * uc - ucl * ucl) / hx
    fy = 0.5 * (vs + D.xp(vs)) * 0.5 * (us + D.yp(us))     # at xy edge (i, j)
    adv_u += (fy - D.ym(fy)) / hy
    fz = 0.5 * (w_ext(ws) + D.xp(w_ext(ws))) * u_on_zedges(us, uw)  # xz edges k=-1..nz-1
    adv_u += (fz[1:] - fz[:-1]) / hz

    # v at y faces
    vc = 0.5 * (vs + D.yp(vs))
    vcl = 0.5 * (D.ym(vs) + vs)
    adv_v = (vc * vc - vcl * vcl) / hy
    fx = 0.5 * (us + D.yp(us)) * 0.5 * (vs + D.xp(vs))     # at xy edge (i, j)
    adv_v += (fx - D.xm(fx)) / hx
    fz = 0.5 * (w_ext(ws) + D.yp(w_ext(ws))) * u_on_zedges(vs, vw)
    adv_v += (fz[1:] - fz[:-1]) / hz

    # w at z faces (k = 0..nz-2 meaningful)
    wcu = 0.5 * (ws + D.zp_face(ws))          # centre k+1
    wcl = 0.5 * (D.zm_face(ws) + ws)          # centre k
    adv_w = (wcu * wcu - wcl * wcl) / hz
    fx = 0.5 * (us + D.zp_dir(us, uw[1])) * 0.5 * (ws + D.xp(ws))   # xz edge (i, k), k = 0..nz-1
    adv_w += (fx - D.xm(fx)) / hx
    fy = 0.5 * (vs + D.zp_dir(vs, vw[1])) * 0.5 * (ws + D.yp(ws))
    adv_w += (fy - D.ym(fy)) / hy

    # ---- J . grad u* / rho
    def face_avg_x(a):
        return 0.5 * (a + D.xp(a))

    def face_avg_y(a):
        return 0.5 * (a + D.yp(a))

    def face_avg_z(a):
        return 0.5 * (a + D.zp_neu(a))

    dudx = (D.xp(us) - D.xm(us)) / (2 * hx)
    dudy = (D.yp(us) - D.ym(us)) / (2 * hy)
    zm, zp = _zc_dir(us, uw)
    dudz = (zp - zm) / (2 * hz)
    jgu = face_avg_x(jx) * dudx + face_avg_x(jy) * dudy + face_avg_x(jz) * dudz

    dvdx = (D.xp(vs) - D.xm(vs)) / (2 * hx)
    dvdy = (D.yp(vs) - D.ym(vs)) / (2 * hy)
    zm, zp = _zc_dir(vs, vw)
    dvdz = (zp - zm) / (2 * hz)
    jgv = face_avg_y(jx) * dvdx + face_avg_y(jy) * dvdy + face_avg_y(jz) * dvdz

    dwdx = (D.xp(ws) - D.xm(ws)) / (2 * hx)
    dwdy = (D.yp(ws) - D.ym(ws)) / (2 * hy)
    dwdz = (D.zp_face(ws) - D.zm_face(ws)) / (2 * hz)
    jgw = face_avg_z(jx) * dwdx + face_avg_z(jy) * dwdy + face_avg_z(jz) * dwdz

    # ---- viscous stress divergence div[mu (grad u* + grad u*^T)]
    # x-momentum
    sxx_r = 2 * D.xp(mu_c) * (D.xp(us) - us) / hx       # at centre i+1
    sxx_l = 2 * mu_c * (us - D.xm(us)) / hx             # at centre i
    vis_u = (sxx_r - sxx_l) / hx
    sxy = mu_xy * ((D.yp(us) - us) / hy + (D.xp(vs) - vs) / hx)    # xy edge (i, j)
    vis_u += (sxy - D.ym(sxy)) / hy
    ue = with_ghosts(us, uw)                                       # k = -1 .. nz
    we = w_ext(ws)                                                 # k = -1 .. nz-1
    sxz = mu_xz * ((ue[1:] - ue[:-1]) / hz + (D.xp(we) - we) / hx)  # xz edges k=-1..nz-1
    vis_u += (sxz[1:] - sxz[:-1]) / hz
    # y-momentum
    syy_r = 2 * D.yp(mu_c) * (D.yp(vs) - vs) / hy
    syy_l = 2 * mu_c * (vs - D.ym(vs)) / hy
    vis_v = (syy_r - syy_l) / hy
    vis_v += (sxy - D.xm(sxy)) / hx
    ve = with_ghosts(vs, vw)
    syz = mu_yz * ((ve[1:] - ve[:-1]) / hz + (D.yp(we) - we) / hy)
    vis_v += (syz[1:] - syz[:-1]) / hz
    # z-momentum (faces k = 0 .. nz-2): edges k = 0 .. nz-2 are layers 1 .. nz-1
    szz_u = 2 * D.zp_neu(mu_c) * (D.zp_face(ws) - ws) / hz   # centre k+1
    szz_l = 2 * mu_c * (ws - D.zm_face(ws)) / hz             # centre k
    vis_w = (szz_u - szz_l) / hz
    sxz_k = sxz[1:]                                          # xz edges at z face k
    vis_w += (sxz_k - D.xm(sxz_k)) / hx
    syz_k = syz[1:]
    vis_w += (syz_k - D.ym(syz_k)) / hy

    # ---- polymer divergence div[(1+phi)/2 tau*]
    if T is not None:
        txz_e = edge_avg_xz(T[XZ])   # layers k = -1 .. nz-1
        tyz_e = edge_avg_yz(T[YZ])
        txy_e = edge_avg_xy(T[XY])
        pol_u = (D.xp(T[XX]) - T[XX]) / hx + (txy_e - D.ym(txy_e)) / hy \
            + (txz_e[1:] - txz_e[:-1]) / hz
        pol_v = (txy_e - D.xm(txy_e)) / hx + (D.yp(T[YY]) - T[YY]) / hy \
            + (tyz_e[1:] - tyz_e[:-1]) / hz
        pol_w = (txz_e[1:] - D.xm(txz_e[1:])) / hx + (tyz_e[1:] - D.ym(tyz_e[1:])) / hy \
            + (D.zp_neu(T[ZZ]) - T[ZZ]) / hz
    else:
        pol_u = pol_v = pol_w = 0.0

    # ---- pressure
    gpn = D.gradient(pn, P.h)
    gps = D.gradient(ps, P.h)
    # ---- capillary force G grad(phi) at faces
    cap = (R["G_x"] * (D.xp(phic) - phic) / hx,
           R["G_y"] * (D.yp(phic) - phic) / hy,
           R["G_z"][1:] * (D.zp_neu(phic) - phic) / hz)

    rinv = (R["rinv_x"], R["rinv_y"], R["rinv_z"][1:])
    lap = (D.lap_dirichlet(us, P.h, uw), D.lap_dirichlet(vs, P.h, vw), D.lap_wface(ws, P.h))
    hats = (uh, vh, wh)
    advs = (adv_u, adv_v, adv_w)
    jgs = (jgu, jgv, jgw)
    viss = (vis_u, vis_v, vis_w)
    pols = (pol_u, pol_v, pol_w)
    out = []
    for a in range(3):
        ri = rinv[a]
        r = (-hats[a] / dt + advs[a] + ri * jgs[a]
             + gpn[a] / C.rho0 + (ri - 1.0 / C.rho0) * gps[a]
             + C.nu_m * lap[a]
             - inv_re * ri * pols[a]
             - inv_re * ri * viss[a]
             - C.k_sigma * ri * cap[a]
             - P.a_ext[a])
        out.append(np.ascontiguousarray(r))
    out[2][-1] = 0.0
    return out


def navier_stokes(P: Params, st, R, C):
    """Eqs. NS36-NS39: predictor, incremental pressure, correction.
    Returns (u, v, w, p) at n+1 and the pressure increment."""
    ru, rv, rw = momentum_rhs(P, st, R, C)
    g = C.gamma0 / P.dt
    # moving walls (eq. NS13): the no-slip ghosts of the implicit Laplacian carry u_w
    walls = (lambda c: P.walls(c)) if P.moving_walls else (lambda c: None)
    ut = D.helmholtz(ru, C.nu_m, g, "dirichlet", P.h, walls(0))
    vt = D.helmholtz(rv, C.nu_m, g, "dirichlet", P.h, walls(1))
    wt = D.helmholtz(rw, C.nu_m, g, "wface", P.h)
    # Eq. NS37 with the coefficient that makes eq. NS38 divergence free.
    div = D.divergence(ut, vt, wt, P.h)
    dp = D.helmholtz((C.gamma0 * C.rho0 / P.dt) * div, 1.0, 0.0, "neumann", P.h)
    gx, gy, gz = D.gradient(dp, P.h)
    c = P.dt / (C.gamma0 * C.rho0)
    u = ut - c * gx
    v = vt - c * gy
    w = wt - c * gz
    w[-1] = 0.0
    p = st["p"][0] + dp
    return u, v, w, p, dp


# ---------------------------------------------------------------------------------------
# polymer stress (Sec. 3.2.3, Giesekus / Oldroyd-B in stress form)
# ---------------------------------------------------------------------------------------


def velocity_gradient(P: Params, u, v, w):
    """grad u at cell centres, as L[a][b] = d u_b / d x_a. Diagonal entries from the compact
    face difference; off-diagonal entries from the 2h central difference of the
    cell-centred velocity, whose wall ghost is twice the wall velocity (eq. NS13) minus the
    adjacent value."""
    hx, hy, hz = P.h
    uc = 0.5 * (u + D.xm(u))
    vc = 0.5 * (v + D.ym(v))
    wc = 0.5 * (w + D.zm_face(w))
    L = [[None] * 3 for _ in range(3)]
    L[0][0] = (u - D.xm(u)) / hx
    L[1][1] = (v - D.ym(v)) / hy
    L[2][2] = (w - D.zm_face(w)) / hz
    cen = (uc, vc, wc)
    for b in range(3):
        f = cen[b]
        if b != 0:
            L[0][b] = (D.xp(f) - D.xm(f)) / (2 * hx)
        if b != 1:
            L[1][b] = (D.yp(f) - D.ym(f)) / (2 * hy)
        if b != 2:
            wb, wt = P.walls(b)
            L[2][b] = (D.zp_dir(f, wt) - D.zm_dir(f, wb)) / (2 * hz)
    return L


_PAIRS = {(0, 0): XX, (1, 1): YY, (2, 2): ZZ, (0, 1): XY, (1, 0): XY, (0, 2): XZ,
          (2, 0): XZ, (1, 2): YZ, (2, 1): YZ}


def polymer_rhs(P: Params, tau, u, v, w, L):
    """RH of eq. NS40-NS41 in stress form (Giesekus; Oldroyd-B at alpha = 0):
    -div(u tau) + (grad u)^T.tau + tau.(grad u) + [(1-beta)(grad u + grad u^T) - tau] / Wi
    - alpha/(1-beta) tau.tau,
    index form RH_ab = -div(u tau_ab) + L_ca tau_cb + tau_ac L_cb + ..., L_ab = du_b/dx_a.
    Advection: flux form with face-mean stress (or the WENO-Z face value) and zero wall flux."""
    hx, hy, hz = P.h
    out = []
    for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)):
        t = tau[_PAIRS[(a, b)]]
        if P.advection == 1:
            rh = -weno.divergence(t, u, v, w, P.h, D)
        else:
            fx = u * 0.5 * (t + D.xp(t))
            fy = v * 0.5 * (t + D.yp(t))
            fz = w * 0.5 * (t + D.zp_neu(t))
            fz[-1] = 0.0
            rh = -((fx - D.xm(fx)) / hx + (fy - D.ym(fy)) / hy + (fz - D.zm_face(fz)) / hz)
        for c in range(3):
            rh = rh + L[c][a] * tau[_PAIRS[(c, b)]] + tau[_PAIRS[(a, c)]] * L[c][b]
        rh = rh + ((1.0 - P.beta) * (L[a][b] + L[b][a]) - t) / P.wi
        if P.giesekus_alpha != 0.0:
            tt = sum(tau[_PAIRS[(a, c)]] * tau[_PAIRS[(c, b)]] for c in range(3))
            rh = rh - P.giesekus_alpha / (1.0 - P.beta) * tt
        out.append(rh)
    return out


def polymer(P: Params, tau_n, u, v, w):
    """Second-order TVD Runge-Kutta (eqs. NS42 and NS44) with u^{n+1} held fixed."""
    L = velocity_gradient(P, u, v, w)
    rh0 = polymer_rhs(P, tau_n, u, v, w, L)
    t1 = [tau_n[c] + P.dt * rh0[c] for c in range(6)]
    rh1 = polymer_rhs(P, t1, u, v, w, L)
    return [0.5 * tau_n[c] + 0.5 * (t1[c] + P.dt * rh1[c]) for c in range(6)]


# ---------------------------------------------------------------------------------------
# full step
# ---------------------------------------------------------------------------------------


def step(P: Params, st, return_parts=False):
    """Advance the state by one coupled step; returns the new state (inputs untouched)."""
    first = st["step"] == 0
    C = constants(P, first)
    phi_new, G, phis, Psi = cahn_hilliard(P, st, C)
    R = restricted_set(P, phi_new, G, C)
    u, v, w, p, dp = navier_stokes(P, st, R, C)
    theta = st.get("theta")
    if P.viscoelastic and P.constitutive == 1:
        theta, tau = lcr.polymer(P, st["theta"], u, v, w, velocity_gradient(P, u, v, w))
    elif P.viscoelastic:
        tau = polymer(P, st["tau"][0], u, v, w)
    else:
        tau = [np.zeros_like(st["p"][0]) for _ in range(6)]
    new = {
        "phi": [phi_new, st["phi"][0]],
        "u": [u, st["u"][0]], "v": [v, st["v"][0]], "w": [w, st["w"][0]],
        "p": [p, st["p"][0]],
        "tau": [tau, st["tau"][0]],
        "step": st["step"] + 1,
    }
    if theta is not None:
        new["theta"] = theta
    if return_parts:
        return new, {"G": G, "phi_star": phis, "Psi": Psi, "R": R, "dp": dp}
    return new


def run(P: Params, st, nsteps):
    for _ in range(nsteps):
        st = step(P, st)
    return st


# ---------------------------------------------------------------------------------------
# observables (FP64)
# ---------------------------------------------------------------------------------------


def observables(P: Params, st):
    """mass h_f^3 sum(phi); wetted radius (2D: half the wetted length, 3D: sqrt(A / pi),
    both from the indicator (1 + phi)/2 of the wall-adjacent fine layer); centroid height
    of the drop phase; kinetic energy; max |div u|."""
    phi = st["phi"][0]
    hx, hy, hz = P.hf
    mass = float(np.sum(phi)) * hx * hy * hz
    ind0 = 0.5 * (1.0 + phi[0])
    if P.ny == 1:
        rw = 0.5 * hx * float(np.sum(ind0))
    else:
        rw = math.sqrt(hx * hy * float(np.sum(ind0)) / math.pi)
    ind = 0.5 * (1.0 + phi)
    z = (np.arange(phi.shape[0]) + 0.5) * hz
    zc = float(np.sum(ind * z[:, None, None]) / np.sum(ind))
    Hx, Hy, Hz = P.h
    u, v, w = st["u"][0], st["v"][0], st["w"][0]
    ke = 0.5 * float(np.sum(u * u) + np.sum(v * v) + np.sum(w * w)) * Hx * Hy * Hz
    divmax = float(np.max(np.abs(D.divergence(u, v, w, P.h))))
    return {"mass": mass, "wetted_radius": rw, "centroid_height": zc, "kinetic_energy": ke,
            "max_div": divmax}
