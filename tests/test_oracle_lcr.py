"""Pins of the oracle's log-conformation update (oracle/lcr.py) and of the Giesekus term of the
stress form, against things other than themselves:

* homogeneous start-up of simple shear and of planar extension (Oldroyd-B): closed-form c(t);
  the two-stage scheme of eqs. NS42-NS44 must converge to it at second order;
* Giesekus start-up shear: the conformation ODE integrated by scipy (an independent
  formulation, in c rather than Theta), again at second order;
* c = I: the source reduces to 2 sym(grad u) exactly (the paper's rule for tau_p = 0);
* frame covariance: rotating Theta and grad u rotates the source;
* equal eigenvalues: the source is continuous through them;
* the stress form with the Giesekus term and the log-conformation form approximate the same
  homogeneous trajectory to O(dt^2);
* one full coupled step of a small viscoelastic drop: both forms agree to the scheme's order.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp

import workloads as W
from oracle import lcr, model
from oracle import step as S


def _rk2_source(theta, K, wi, alpha, dt, nsteps):
    """The two stages of eqs. NS42-NS44 on the source alone (homogeneous field)."""
    for _ in range(nsteps):
        t1 = theta + dt * lcr.source(theta, K, wi, alpha)
        theta = 0.5 * theta + 0.5 * (t1 + dt * lcr.source(t1, K, wi, alpha))
    return theta


def _shear_K(rate):
    K = np.zeros((1, 3, 3))
    K[0, 0, 1] = rate  # u_x = rate * y: K_xy = du_x/dy
    return K


def _errors(exact, wi, alpha, K, T, dts):
    out = []
    for dt in dts:
        n = int(round(T / dt))
        th = _rk2_source(np.zeros((1, 3, 3)), K, wi, alpha, dt, n)
        c = lcr.conformation(th)[0]
        out.append(np.max(np.abs(c - exact)))
    return out


def test_oldroyd_b_shear_startup_closed_form():
    wi, rate, T = 1.0, 2.0, 3.0
    a = wi * rate
    e = math.exp(-T / wi)
    exact = np.eye(3)
    exact[0, 1] = exact[1, 0] = a * (1.0 - e)
    exact[0, 0] = 1.0 + 2.0 * a * a * (1.0 - e * (1.0 + T / wi))
    e1, e2 = _errors(exact, wi, 0.0, _shear_K(rate), T, (0.01, 0.005))
    assert e2 < 2e-4, (e1, e2)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_oldroyd_b_planar_extension_closed_form():
    wi, rate, T = 1.0, 0.2, 2.0
    K = np.zeros((1, 3, 3))
    K[0, 0, 0], K[0, 1, 1] = rate, -rate
    exact = np.eye(3)
    for i, r in ((0, rate), (1, -rate)):
        k = 1.0 / wi - 2.0 * r
        cinf = (1.0 / wi) / k
        exact[i, i] = cinf + (1.0 - cinf) * math.exp(-k * T)
    e1, e2 = _errors(exact, wi, 0.0, K, T, (0.02, 0.01))
    assert e2 < 1e-5, (e1, e2)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def _c_ode(K, wi, alpha):
    I = np.eye(3)

    def f(_, y):
        c = y.reshape(3, 3)
        d = K @ c + c @ K.T - (I + alpha * (c - I)) @ (c - I) / wi
        return d.ravel()
    return f


def test_giesekus_shear_startup_vs_conformation_ode():
    wi, rate, alpha, T = 0.8, 3.0, 0.3, 2.0
    K = _shear_K(rate)
    sol = solve_ivp(_c_ode(K[0], wi, alpha), (0.0, T), np.eye(3).ravel(), rtol=1e-12, atol=1e-14,
                    method="DOP853")
    exact = sol.y[:, -1].reshape(3, 3)
    e1, e2 = _errors(exact, wi, alpha, K, T, (0.01, 0.005))
    assert e2 < 1e-4, (e1, e2)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)
    # shear thinning: the Giesekus shear stress stays below the Oldroyd-B one
    ob = _rk2_source(np.zeros((1, 3, 3)), K, wi, 0.0, 0.005, int(T / 0.005))
    assert lcr.conformation(ob)[0, 0, 1] > exact[0, 1]


def test_identity_conformation_gives_symmetric_gradient():
    rng = np.random.default_rng(5)
    K = rng.standard_normal((4, 3, 3))
    K -= np.trace(K, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3.0
    s = lcr.source(np.zeros((4, 3, 3)), K, 0.7, 0.2)
    assert np.max(np.abs(s - (K + np.swapaxes(K, 1, 2)))) < 1e-14


def _random_theta(rng, n):
    A = rng.standard_normal((n, 3, 3))
    return 0.5 * (A + np.swapaxes(A, 1, 2))


def test_frame_covariance():
    rng = np.random.default_rng(6)
    th = _random_theta(rng, 8)
    K = rng.standard_normal((8, 3, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    s = lcr.source(th, K, 0.9, 0.25)
    sq = lcr.source(Q @ th @ Q.T, Q @ K @ Q.T, 0.9, 0.25)
    assert np.max(np.abs(sq - Q @ s @ Q.T)) < 1e-12 * np.max(np.abs(s))


def test_continuous_through_equal_eigenvalues():
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    K = rng.standard_normal((1, 3, 3))
    base = np.diag([0.3, 0.3, -0.5])
    s0 = lcr.source((Q @ base @ Q.T)[None], K, 1.0, 0.1)
    for eps in (1e-4, 1e-7):
        th = Q @ np.diag([0.3, 0.3 + eps, -0.5]) @ Q.T
        s = lcr.source(th[None], K, 1.0, 0.1)
        assert np.max(np.abs(s - s0)) < 10 * eps * np.max(np.abs(s0)), eps


def test_stress_form_and_log_conformation_agree_homogeneous():
    """Uniform fields, zero velocity arrays, a prescribed uniform gradient: both polymer
    updates see only their source terms and approximate the same c(t)."""
    cfg = W.config("C3", nx=4, ny=4, nz=4, wi=0.8, beta=0.4, giesekus_alpha=0.3)
    errs = []
    for dt in (0.01, 0.005):
        P = model.Params.from_config(cfg.replace(dt=dt))
        cs = P.coarse_shape
        z = np.zeros(cs)
        L = [[np.zeros(cs) for _ in range(3)] for _ in range(3)]
        L[1][0] = np.full(cs, 2.5)  # du_x/dy
        L[0][0], L[1][1] = np.full(cs, 0.4), np.full(cs, -0.4)
        tau = [np.zeros(cs) for _ in range(6)]
        theta = [np.zeros(cs) for _ in range(6)]
        n = int(round(1.5 / dt))
        for _ in range(n):
            rh0 = S.polymer_rhs(P, tau, z, z, z, L)
            t1 = [tau[c] + dt * rh0[c] for c in range(6)]
            rh1 = S.polymer_rhs(P, t1, z, z, z, L)
            tau = [0.5 * tau[c] + 0.5 * (t1[c] + dt * rh1[c]) for c in range(6)]
            theta, tau_l = lcr.polymer(P, theta, z, z, z, L)
        errs.append(max(float(np.max(np.abs(tau[c] - tau_l[c]))) for c in range(6)))
    assert errs[1] < 1e-3 and 3.0 < errs[0] / errs[1] < 5.0, errs


def test_full_step_forms_agree_small_drop():
    cfg = W.config("C3", nx=16, ny=8, nz=8, noise=1e-2, dt=2e-4, wi=0.5, giesekus_alpha=0.2)
    st_s = W.droplet_state(cfg)
    st_l = W.droplet_state(cfg)
    Ps = model.Params.from_config(cfg)
    Pl = model.Params.from_config(cfg.replace(constitutive=1))
    for _ in range(4):
        st_s = S.step(Ps, st_s)
        st_l = S.step(Pl, st_l)
    scale = max(float(np.max(np.abs(t))) for t in st_s["tau"][0])
    assert scale > 0
    diff = max(float(np.max(np.abs(a - b))) for a, b in zip(st_s["tau"][0], st_l["tau"][0]))
    assert diff < 2e-2 * scale, (diff, scale)
    # Theta and tau of the log-conformation state describe the same c
    tau_from_theta = lcr.stress(Pl, st_l["theta"])
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(tau_from_theta, st_l["tau"][0])) < 1e-14 * scale
