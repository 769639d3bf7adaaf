"""Pins of the oracle's Navier-Stokes explicit terms and its velocity gradient.

The right-hand side r of eq. NS36 (with the -u_hat/dt of eq. NS35 and the polymer
divergence of approach 2, eq. NS12) is a sum of second-order stencils on the staggered
grid. Each stencil is pinned here against its continuous operator: smooth analytic fields
(periodic in x and y, compatible with the walls: velocities odd about both walls so that
the no-slip reflection ghost is exact, cell-centred scalars even so that the Neumann copy
ghost is exact), with density and viscosity varying in space, non-zero J, polymer stress
and phase field, are sampled at the points where the oracle stores them; the continuous
terms come from symbolic derivatives of the same fields. The discrete error must fall by
about 4 per halving of h (second order), which a wrong edge average, flux index, face
average or transposed operand does not do.

Every term is isolated from the one right-hand side the oracle computes:
* advection, the only term quadratic in the velocity, from three velocity scalings
  (r(2u) - 2 r(u) + r(0)) / 2;
* every other term as the difference of r with and without its coefficient or field.

The velocity gradient (L_ab = du_b/dx_a, the input of the polymer update, eqs. NS40-NS41)
must be exact on linear fields away from the periodic wrap and the walls, and converge at
second order on smooth fields; the polymer right-hand side likewise.
"""
from __future__ import annotations

import dataclasses
import functools
import importlib
import types
from pathlib import Path

import numpy as np
import pytest
import sympy as sp

from oracle import model
from oracle import step as S

X, Y, Z = sp.symbols("x y z", real=True)
LX, LY, LZ = 1.3, 0.9, 1.0
KX, KY, KZ = 2 * sp.pi / LX, 2 * sp.pi / LY, sp.pi / LZ
sin, cos = sp.sin, sp.cos

# --------------------------------------------------------------------------------------
# analytic fields
# --------------------------------------------------------------------------------------


UWB, UWT = (0.35, -0.2), (-0.5, 0.45)   # wall velocities (x, y) at z = 0 and z = lz


def _fields(two_d: bool, moving: bool = False):
    """Two time levels of every input. Velocities take the wall values on both walls and,
    less those values, are odd about them (a linear profile between the walls plus sin(m pi z)
    terms), so that the no-slip ghost 2 u_w - adjacent is exact; scalars are even about the
    walls (cos(m pi z)). In 2D nothing depends on y and v = 0."""
    cy = (lambda a: 1) if two_d else (lambda a: cos(KY * Y + a))
    sy = (lambda a: 0) if two_d else (lambda a: sin(KY * Y + a))
    F = {}
    F["uA"] = sin(KZ * Z) * (0.6 + 0.5 * sin(KX * X + 0.3) * cy(-0.7)) \
        + 0.2 * sin(2 * KZ * Z) * cos(KX * X - 0.4)
    F["uB"] = sin(KZ * Z) * (0.3 + 0.4 * cos(KX * X + 0.9) * cy(0.2))
    if two_d:
        F["vA"] = sp.Integer(0)
        F["vB"] = sp.Integer(0)
    else:
        F["vA"] = sin(KZ * Z) * (-0.4 + 0.7 * cos(KX * X + 1.1) * sy(0.4)) \
            + 0.15 * sin(2 * KZ * Z) * sy(0.0)
        F["vB"] = 0.5 * sin(KZ * Z) * sin(KX * X - 0.6) * cy(0.0)
    F["wA"] = sin(KZ * Z) * (0.3 * sin(KX * X - 0.5) + 0.45 * cy(0.2) + 0.1) \
        + 0.1 * sin(2 * KZ * Z) * cos(KX * X + 0.25) * cy(0.0)
    F["wB"] = 0.35 * sin(KZ * Z) * cos(KX * X) * cy(0.8)
    if moving:
        F["uA"] += UWB[0] + (UWT[0] - UWB[0]) * Z / LZ
        F["uB"] += UWB[0] + (UWT[0] - UWB[0]) * Z / LZ
        if not two_d:
            F["vA"] += UWB[1] + (UWT[1] - UWB[1]) * Z / LZ
            F["vB"] += UWB[1] + (UWT[1] - UWB[1]) * Z / LZ
    F["pA"] = cos(KZ * Z) * cos(KX * X + 0.2) * cy(-0.1) + 0.3 * cos(2 * KZ * Z)
    F["pB"] = 0.5 * sin(KX * X) * cos(KZ * Z) + 0.2 * cy(0.5)
    F["phi"] = 0.6 * cos(KZ * Z) * sin(KX * X + 0.5) * cy(0.3) + 0.2 * cos(2 * KZ * Z)
    F["G"] = 0.9 * cos(KZ * Z) * cos(KX * X - 0.2) * cy(0.6) + 0.4 * cos(2 * KZ * Z) * cy(1.0)
    F["rinv"] = 1 / (1.2 + 0.5 * cos(KZ * Z) * sin(KX * X + 0.7) * cy(0.0))
    F["mu"] = 0.8 + 0.3 * cos(KZ * Z) * cos(KX * X + 0.4) * cy(0.9) + 0.1 * cos(2 * KZ * Z)
    amps = [(0.7, 0.1), (-0.5, 0.6), (0.4, -0.3), (0.3, 1.2), (-0.6, 0.8), (0.25, -1.0)]
    for c, (a, ph) in enumerate(amps):
        F[f"tauA{c}"] = a * cos(KZ * Z) * cos(KX * X + ph) * cy(ph / 2) + 0.2 * (c + 1) * cos(2 * KZ * Z) / 6
        F[f"tauB{c}"] = 0.5 * a * cos(KX * X - ph) * cos(KZ * Z) + 0.1 * cy(ph)
    return F


def _mesh(n_shape, h, loc):
    """Coordinates of the points an array of location ``loc`` = (z, y, x) letters holds:
    'c' cell centres, 'f' right faces ((i+1) h), 'W' the nz + 1 z faces from wall to wall."""
    nz, ny, nx = n_shape
    hx, hy, hz = h
    lz, ly, lx = loc
    xs = (np.arange(nx) + (1.0 if lx == "f" else 0.5)) * hx
    ys = (np.arange(ny) + (1.0 if ly == "f" else 0.5)) * hy
    if lz == "W":
        zs = np.arange(nz + 1) * hz
    else:
        zs = (np.arange(nz) + (1.0 if lz == "f" else 0.5)) * hz
    return np.meshgrid(zs, ys, xs, indexing="ij")


def _sample(expr, n_shape, h, loc):
    zz, yy, xx = _mesh(n_shape, h, loc)
    f = sp.lambdify((X, Y, Z), expr, "numpy")
    return np.broadcast_to(np.asarray(f(xx, yy, zz), dtype=float), zz.shape).copy()


VLOC = ("ccf", "cfc", "fcc")     # u at x faces, v at y faces, w at z faces


def _params(n, two_d, moving=False):
    ny = 1 if two_d else n
    ub, ut = (UWB, UWT) if moving else ((0.0, 0.0), (0.0, 0.0))
    if two_d:
        ub, ut = (ub[0], 0.0), (ut[0], 0.0)
    return model.Params(nx=n, ny=ny, nz=n, lx=LX, ly=LY, lz=LZ, re=3.0, ca=1.0, cn=0.05,
                        pe=10.0, dt=0.25, viscoelastic=1, beta=0.4, wi=0.7,
                        a_ext=(0.3, -0.2, 0.5), u_wall_bottom=ub, u_wall_top=ut)


def _constants():
    # only rho0, nu_m, k_sigma and c_j enter the momentum right-hand side
    return model.Constants(gamma0=1.5, S=0.0, alpha=0.0, c_psi=0.0, rho1=1.0, rho2=1.0,
                           mu1=1.0, mu2=1.0, rho0=0.7, nu_m=0.9, k_sigma=1.7, c_j=0.45)


# --------------------------------------------------------------------------------------
# continuous right-hand side, term by term
# --------------------------------------------------------------------------------------


def _continuous_terms(F, P, C):
    """Each term of r (eq. NS36 with eq. NS35's -u_hat/dt) as it enters r, per component,
    as a sympy expression of the continuous fields at the component's own location."""
    co = (X, Y, Z)
    U = [2 * F[k + "A"] - F[k + "B"] for k in ("u", "v", "w")]          # u* (eq. NS32)
    Uh = [2 * F[k + "A"] - F[k + "B"] / 2 for k in ("u", "v", "w")]     # u_hat (eq. NS31)
    Ps = 2 * F["pA"] - F["pB"]
    tau = [[None] * 3 for _ in range(3)]
    pairs = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4,
             (1, 2): 5, (2, 1): 5}
    for (a, b), c in pairs.items():
        tau[a][b] = 2 * F[f"tauA{c}"] - F[f"tauB{c}"]
    Wt = (1 + F["phi"]) / 2
    J = [-C.c_j * sp.diff(F["G"], c) for c in co]
    ri, mu = F["rinv"], F["mu"]
    T = {}
    for a in range(3):
        d = lambda f, b: sp.diff(f, co[b])
        T[("hat", a)] = -Uh[a] / P.dt
        T[("adv", a)] = sum(d(U[b] * U[a], b) for b in range(3))
        T[("jgrad", a)] = ri * sum(J[b] * d(U[a], b) for b in range(3))
        T[("press", a)] = d(F["pA"], a) / C.rho0 + (ri - 1 / C.rho0) * d(Ps, a)
        T[("lap", a)] = C.nu_m * sum(d(d(U[a], b), b) for b in range(3))
        T[("pol", a)] = -(ri / P.re) * sum(d(Wt * tau[a][b], b) for b in range(3))
        T[("visc", a)] = -(ri / P.re) * sum(d(mu * (d(U[a], b) + d(U[b], a)), b)
                                            for b in range(3))
        T[("cap", a)] = -C.k_sigma * ri * F["G"] * d(F["phi"], a)
        T[("ext", a)] = -P.a_ext[a]
    return T


# --------------------------------------------------------------------------------------
# discrete right-hand side with selected inputs switched off
# --------------------------------------------------------------------------------------


def _discrete_inputs(F, P):
    sh, h = P.coarse_shape, P.h
    smp = lambda k, loc: _sample(F[k], sh, h, loc)
    st = {"step": 1}
    for k, loc in zip(("u", "v", "w"), VLOC):
        st[k] = [smp(k + "A", loc), smp(k + "B", loc)]
    st["p"] = [smp("pA", "ccc"), smp("pB", "ccc")]
    st["tau"] = [[smp(f"tauA{c}", "ccc") for c in range(6)],
                 [smp(f"tauB{c}", "ccc") for c in range(6)]]
    R = {"phi_c": smp("phi", "ccc"), "G_c": smp("G", "ccc"),
         "G_x": smp("G", "ccf"), "G_y": smp("G", "cfc"), "G_z": smp("G", "Wcc"),
         "rinv_x": smp("rinv", "ccf"), "rinv_y": smp("rinv", "cfc"),
         "rinv_z": smp("rinv", "Wcc"),
         "mu_c": smp("mu", "ccc"), "mu_xy": smp("mu", "cff"), "mu_xz": smp("mu", "Wcf"),
         "mu_yz": smp("mu", "Wfc")}
    return st, R


def _rhs(mod, P, st, R, C, *, vel=1.0, c_j=None, nu_m=None, k_sigma=None, p=True, tau=True,
         mu=True):
    st2 = dict(st)
    for k in ("u", "v", "w"):
        st2[k] = [vel * a for a in st[k]]
    if not p:
        st2["p"] = [np.zeros_like(a) for a in st["p"]]
    if not tau:
        st2["tau"] = [[np.zeros_like(a) for a in lev] for lev in st["tau"]]
    R2 = dict(R)
    if not mu:
        for k in ("mu_c", "mu_xy", "mu_xz", "mu_yz"):
            R2[k] = np.zeros_like(R[k])
    C2 = dataclasses.replace(C, **{k: v for k, v in (("c_j", c_j), ("nu_m", nu_m),
                                                      ("k_sigma", k_sigma)) if v is not None})
    return mod.momentum_rhs(P, st2, R2, C2)


def _discrete_terms(mod, P, st, R, C):
    r = lambda **kw: _rhs(mod, P, st, R, C, **kw)
    base = r()
    r2, r0 = r(vel=2.0), r(vel=0.0)
    out = {}
    for a in range(3):
        out[("adv", a)] = 0.5 * (r2[a] - 2 * base[a] + r0[a])
    off = {"jgrad": r(c_j=0.0), "press": r(p=False), "lap": r(nu_m=0.0), "pol": r(tau=False),
           "visc": r(mu=False), "cap": r(k_sigma=0.0)}
    for name, rr in off.items():
        for a in range(3):
            out[(name, a)] = base[a] - rr[a]
    for a in range(3):
        out[("total", a)] = base[a]
    return out


TERMS = ("adv", "jgrad", "press", "lap", "pol", "visc", "cap", "total")


@functools.lru_cache(maxsize=None)
def _problem(n, two_d, moving):
    """Discrete inputs and the continuous terms sampled at each component's points."""
    F = _fields(two_d, moving)
    P = _params(n, two_d, moving)
    C = _constants()
    st, R = _discrete_inputs(F, P)
    cont = _continuous_terms(F, P, C)
    comps = (0, 2) if two_d else (0, 1, 2)
    ref = {}
    for name in TERMS:
        for a in comps:
            if name == "total":
                expr = sum(cont[(t, a)] for t in ("hat", "adv", "jgrad", "press", "lap",
                                                  "pol", "visc", "cap", "ext"))
            else:
                expr = cont[(name, a)]
            ref[(name, a)] = _sample(expr, P.coarse_shape, P.h, VLOC[a])
    return P, C, st, R, comps, ref


def _term_errors(mod, n, two_d, moving=False):
    """Max error of each term over its component arrays, relative to the term's size."""
    P, C, st, R, comps, ref = _problem(n, two_d, moving)
    disc = _discrete_terms(mod, P, st, R, C)
    errs = {}
    for name in TERMS:
        num = den = 0.0
        for a in comps:
            r, got = ref[(name, a)], disc[(name, a)]
            if a == 2:                       # r_w on the top wall is not an unknown
                r, got = r[:-1], got[:-1]
            num = max(num, float(np.max(np.abs(got - r))))
            den = max(den, float(np.max(np.abs(r))))
        errs[name] = num / den
    return errs


NS = (12, 24, 48)


CASES = [(False, False), (True, False), (False, True), (True, True)]


@pytest.fixture(scope="module", params=CASES, ids=["3d", "2d", "3d-moving-walls", "2d-moving-walls"])
def momentum_errors(request):
    two_d, moving = request.param
    return two_d, [_term_errors(S, n, two_d, moving) for n in NS]


@pytest.mark.parametrize("term", TERMS)
def test_momentum_term_second_order(momentum_errors, term):
    """Each term of eq. NS36's right-hand side converges to its continuous operator at
    second order (ratio about 4 per halving) with variable density and viscosity, non-zero
    J, polymer stress and phase field."""
    two_d, errs = momentum_errors
    e = [d[term] for d in errs]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r2 < 4.7, (term, e)
    assert 3.0 < r1 < 5.0, (term, e)
    assert e[2] < 2e-2, (term, e)


# --------------------------------------------------------------------------------------
# velocity gradient (input of eqs. NS40-NS41)
# --------------------------------------------------------------------------------------


def test_velocity_gradient_exact_on_linear_fields():
    """L_ab = du_b/dx_a is exact for u_b = sum_a A_ab x_a + c_b at every centre whose
    stencil neither wraps around the periodic box nor touches a wall; A is not symmetric,
    so a transposed entry fails."""
    n = 10
    P = _params(n, False)
    A = np.array([[0.3, -1.1, 0.7], [2.3, 0.45, -0.6], [-0.9, 1.7, -0.25]])
    c = (0.2, -0.4, 0.1)
    arrs = []
    for b, loc in enumerate(VLOC):
        zz, yy, xx = _mesh(P.coarse_shape, P.h, loc)
        arrs.append(A[0, b] * xx + A[1, b] * yy + A[2, b] * zz + c[b])
    L = S.velocity_gradient(P, *arrs)
    inner = (slice(1, n - 1), slice(1, n - 1), slice(1, n - 1))
    for a in range(3):
        for b in range(3):
            got = L[a][b][inner]
            assert np.max(np.abs(got - A[a, b])) <= 1e-12, (a, b)


def _grad_errors(mod, n, moving=False):
    F = _fields(False, moving)
    P = _params(n, False, moving)
    co = (X, Y, Z)
    U = [F["uA"], F["vA"], F["wA"]]
    arrs = [_sample(U[b], P.coarse_shape, P.h, VLOC[b]) for b in range(3)]
    L = mod.velocity_gradient(P, *arrs)
    errs = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            ref = _sample(sp.diff(U[b], co[a]), P.coarse_shape, P.h, "ccc")
            errs[a, b] = np.max(np.abs(L[a][b] - ref)) / np.max(np.abs(ref))
    return errs


@pytest.mark.parametrize("moving", [False, True], ids=["walls-at-rest", "moving-walls"])
def test_velocity_gradient_second_order(moving):
    """All nine entries converge at second order on smooth no-slip fields, walls included."""
    e = [_grad_errors(S, n, moving) for n in NS]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert np.all(r2 > 3.3) and np.all(r2 < 4.7), (r2, e[2])
    assert np.all(r1 > 3.0), r1


# --------------------------------------------------------------------------------------
# polymer right-hand side (eqs. NS40-NS41, stress form)
# --------------------------------------------------------------------------------------


def _polymer_errors(mod, n, alpha, moving=False):
    """RH_ab = -div(u tau_ab) + L_ca tau_cb + tau_ac L_cb + [(1-beta)(L_ab + L_ba) - tau_ab]
    / Wi - alpha / (1 - beta) (tau.tau)_ab against the discrete one (the advection in the flux
    form the oracle uses; equal to u.grad(tau) for a divergence-free velocity)."""
    F = _fields(False, moving)
    P = dataclasses.replace(_params(n, False, moving), giesekus_alpha=alpha)
    co = (X, Y, Z)
    U = [F["uA"], F["vA"], F["wA"]]
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    idx = {p: c for c, p in enumerate(pairs)}
    idx.update({(b, a): c for (a, b), c in list(idx.items())})
    tau_s = [F[f"tauA{c}"] for c in range(6)]
    Ls = [[sp.diff(U[b], co[a]) for b in range(3)] for a in range(3)]
    arrs = [_sample(U[b], P.coarse_shape, P.h, VLOC[b]) for b in range(3)]
    tau = [_sample(t, P.coarse_shape, P.h, "ccc") for t in tau_s]
    L = mod.velocity_gradient(P, *arrs)
    rh = mod.polymer_rhs(P, tau, *arrs, L)
    errs = []
    for c, (a, b) in enumerate(pairs):
        t = tau_s[c]
        e = -sum(sp.diff(U[k] * t, co[k]) for k in range(3))
        e += sum(Ls[k][a] * tau_s[idx[(k, b)]] + tau_s[idx[(a, k)]] * Ls[k][b] for k in range(3))
        e += ((1 - P.beta) * (Ls[a][b] + Ls[b][a]) - t) / P.wi
        e -= alpha / (1 - P.beta) * sum(tau_s[idx[(a, k)]] * tau_s[idx[(k, b)]] for k in range(3))
        ref = _sample(e, P.coarse_shape, P.h, "ccc")
        errs.append(np.max(np.abs(rh[c] - ref)) / np.max(np.abs(ref)))
    return np.array(errs)


@pytest.mark.parametrize("alpha,moving", [(0.0, False), (0.3, False), (0.3, True)])
def test_polymer_rhs_second_order(alpha, moving):
    e = [_polymer_errors(S, n, alpha, moving) for n in NS]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert np.all(r2 > 3.3) and np.all(r2 < 4.7), (r2, e[2])
    assert np.all(r1 > 3.0), r1


# --------------------------------------------------------------------------------------
# the pins see plausible mistakes (planted in a copy of the oracle, on the CPU)
# --------------------------------------------------------------------------------------

MISTAKES = {
    "advection edge average of v": (
        "fy = 0.5 * (vs + D.xp(vs)) * 0.5 * (us + D.yp(us))",
        "fy = 0.5 * (vs + D.xm(vs)) * 0.5 * (us + D.yp(us))"),
    "advection flux index of w": (
        "adv_w += (fx - D.xm(fx)) / hx",
        "adv_w += (D.xp(fx) - fx) / hx"),
    "advection w at xz edges": (
        "fz = 0.5 * (w_ext(ws) + D.xp(w_ext(ws))) * u_on_zedges(us, uw)",
        "fz = w_ext(ws) * u_on_zedges(us, uw)"),
    "wall ghost without twice the wall value": (
        "return np.concatenate([2.0 * walls[0] - a[:1], a, 2.0 * walls[1] - a[-1:]], axis=0)",
        "return np.concatenate([walls[0] - a[:1], a, walls[1] - a[-1:]], axis=0)"),
    "wall velocity of the gradient swapped": (
        "L[2][b] = (D.zp_dir(f, wt) - D.zm_dir(f, wb)) / (2 * hz)",
        "L[2][b] = (D.zp_dir(f, wb) - D.zm_dir(f, wt)) / (2 * hz)"),
    "J without face average": (
        "face_avg_x(jz) * dudz", "jz * dudz"),
    "J z difference sign": (
        "jz = -C.c_j * (D.zp_neu(Gc) - D.zm_neu(Gc)) / (2 * hz)",
        "jz = -C.c_j * (D.zm_neu(Gc) - D.zp_neu(Gc)) / (2 * hz)"),
    "grad u* one-sided": (
        "dvdx = (D.xp(vs) - D.xm(vs)) / (2 * hx)",
        "dvdx = (D.xp(vs) - vs) / hx"),
    "viscous transposed part dropped": (
        "sxy = mu_xy * ((D.yp(us) - us) / hy + (D.xp(vs) - vs) / hx)",
        "sxy = mu_xy * ((D.yp(us) - us) / hy)"),
    "viscous cross term index": (
        "sxz = mu_xz * ((ue[1:] - ue[:-1]) / hz + (D.xp(we) - we) / hx)",
        "sxz = mu_xz * ((ue[1:] - ue[:-1]) / hz + (we - D.xm(we)) / hx)"),
    "viscosity at the wrong point": (
        "sxx_r = 2 * D.xp(mu_c) * (D.xp(us) - us) / hx",
        "sxx_r = 2 * mu_c * (D.xp(us) - us) / hx"),
    "polymer normal stress index": (
        "pol_u = (D.xp(T[XX]) - T[XX]) / hx",
        "pol_u = (T[XX] - D.xm(T[XX])) / hx"),
    "polymer edge difference index": (
        "pol_v = (txy_e - D.xm(txy_e)) / hx",
        "pol_v = (D.xp(txy_e) - txy_e) / hx"),
    "polymer phase weight": (
        "wgt = 0.5 * (1.0 + R[\"phi_c\"])", "wgt = 0.5 * (1.0 - R[\"phi_c\"])"),
    "capillary G layer": (
        "R[\"G_z\"][1:] * (D.zp_neu(phic) - phic) / hz",
        "R[\"G_z\"][:-1] * (D.zp_neu(phic) - phic) / hz"),
    "pressure split": (
        "(ri - 1.0 / C.rho0) * gps[a]", "(ri - 1.0 / C.rho0) * gpn[a]"),
    "gradient centre average": (
        "vc = 0.5 * (v + D.ym(v))", "vc = 0.5 * (v + D.yp(v))"),
    "gradient components swapped": (
        "cen = (uc, vc, wc)", "cen = (uc, wc, vc)"),
    "gradient spacing": (
        "L[1][b] = (D.yp(f) - D.ym(f)) / (2 * hy)",
        "L[1][b] = (D.yp(f) - D.ym(f)) / (2 * hx)"),
    "upper-convected operand transposed": (
        "rh = rh + L[c][a] * tau[_PAIRS[(c, b)]]",
        "rh = rh + L[a][c] * tau[_PAIRS[(c, b)]]"),
    "polymer flux face mean": (
        "fy = v * 0.5 * (t + D.yp(t))", "fy = v * 0.5 * (t + D.ym(t))"),
}


def _mutant(old, new):
    src = Path(S.__file__).read_text()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle._step_mutant")
    mod.__package__ = "oracle"
    mod.__file__ = S.__file__
    exec(compile(src.replace(old, new), S.__file__ + "<mutant>", "exec"), mod.__dict__)
    return mod


def _second_order(e0, e1):
    ratio = np.asarray(e0) / np.asarray(e1)
    return bool(np.all(ratio > 3.0) and np.all(ratio < 5.0))


def _pins_hold(mod):
    """The convergence pins above on the two coarser grids (the first failure ends it)."""
    for two_d, moving in CASES:
        e = [_term_errors(mod, n, two_d, moving) for n in NS[:2]]
        if not all(_second_order(e[0][t], e[1][t]) for t in TERMS):
            return False
    for moving in (False, True):
        if not _second_order(*[_grad_errors(mod, n, moving) for n in NS[:2]]):
            return False
        if not _second_order(*[_polymer_errors(mod, n, 0.0, moving) for n in NS[:2]]):
            return False
    return True


def test_pins_hold_on_the_oracle_itself():
    assert _pins_hold(importlib.import_module("oracle.step"))


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_pins_catch_planted_mistake(name):
    old, new = MISTAKES[name]
    assert not _pins_hold(_mutant(old, new)), name
