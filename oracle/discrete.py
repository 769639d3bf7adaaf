"""Discrete operators of the dual staggered grid (oracle; test infrastructure only).

Array layout ``[z][y][x]``: axis 0 is the wall-normal z, axes 1 and 2 are the periodic y
and x. Coarse grid (Sec. 3.1): pressure and polymer stress at cell centres, velocity
components at the right faces of their own direction (u[k][j][i] at x = (i+1) hx,
v at y = (j+1) hy, w[k] at z = (k+1) hz with w[nz-1] the top wall, always 0; the bottom
wall w is implicit and 0). Fine grid: every coarse cell halved in x and z (and in y when
ny > 1), phase field at fine cell centres.

Wall ghost rules (second-order central differences, Sec. 3.2):
* homogeneous Neumann (phase field, chemical potential, pressure increment, polymer stress,
  eqs. NS14, NS37 and the closing paragraph of Sec. 3.2.3): ghost = adjacent cell;
* no-slip (eq. NS13, u = u_w) for cell-centred-in-z velocity: ghost = 2 u_w - adjacent
  (-adjacent for a wall at rest);
* w lives on z faces: its wall values are 0.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

# ---------------------------------------------------------------------------------------
# neighbour access
# ---------------------------------------------------------------------------------------


def xp(a):
    return np.roll(a, -1, axis=2)


def xm(a):
    return np.roll(a, 1, axis=2)


def yp(a):
    return np.roll(a, -1, axis=1)


def ym(a):
    return np.roll(a, 1, axis=1)


def zp_neu(a):
    return np.concatenate([a[1:], a[-1:]], axis=0)


def zm_neu(a):
    return np.concatenate([a[:1], a[:-1]], axis=0)


def zp_dir(a, wall=0.0):
    """a[k+1] of a cell-centred field with the no-slip ghost above the top wall: the wall value
    is the mean of the ghost and the adjacent cell, ghost = 2 wall - adjacent (eq. NS13,
    u = u_w; 0 for a wall at rest)."""
    return np.concatenate([a[1:], 2.0 * wall - a[-1:]], axis=0)


def zm_dir(a, wall=0.0):
    """a[k-1] with the no-slip ghost below the bottom wall (ghost = 2 wall - adjacent)."""
    return np.concatenate([2.0 * wall - a[:1], a[:-1]], axis=0)


def zm_face(w):
    """w[k-1] on z faces with the bottom-wall value w[-1] = 0."""
    return np.concatenate([np.zeros_like(w[:1]), w[:-1]], axis=0)


def zp_face(w):
    """w[k+1] on z faces; the layer above the top wall is never used, set to 0."""
    return np.concatenate([w[1:], np.zeros_like(w[:1])], axis=0)


# ---------------------------------------------------------------------------------------
# Laplacians (7-point; 5-point when ny == 1 since the single periodic y cell adds 0)
# ---------------------------------------------------------------------------------------


def _lap_xy(a, h):
    hx, hy, _ = h
    return (xp(a) - 2 * a + xm(a)) / hx ** 2 + (yp(a) - 2 * a + ym(a)) / hy ** 2


def lap_neumann(a, h):
    return _lap_xy(a, h) + (zp_neu(a) - 2 * a + zm_neu(a)) / h[2] ** 2


def lap_dirichlet(a, h, walls=(0.0, 0.0)):
    """Laplacian of a cell-centred field with no-slip ghosts for the wall values
    walls = (bottom, top)."""
    return _lap_xy(a, h) + (zp_dir(a, walls[1]) - 2 * a + zm_dir(a, walls[0])) / h[2] ** 2


def lap_wface(w, h):
    r = _lap_xy(w, h) + (zp_face(w) - 2 * w + zm_face(w)) / h[2] ** 2
    r[-1] = 0.0
    return r


# ---------------------------------------------------------------------------------------
# constant-coefficient Helmholtz / Poisson solves (the "FFT solver", Sec. 3.2.1-3.2.2)
# ---------------------------------------------------------------------------------------


def _eig_periodic(n, h):
    return -4.0 / h ** 2 * np.sin(np.pi * np.arange(n) / n) ** 2


def wall_vector(shape, kind, h, walls):
    """The part of ``L x`` that the wall data carry, as a field b with ``L x = L_0 x + b``
    (L_0 the operator with homogeneous wall data): on the wall-adjacent layers,
    'neumann' -- walls = outward normal derivatives (g_bottom, g_top); the ghost is the
      adjacent value plus hz g, so b = g / hz;
    'dirichlet' -- walls = wall values; ghost = 2 wall - adjacent, so b = 2 wall / hz^2;
    'wface' -- walls = wall values of the face field at z = 0 and z = lz, next to the
      unknowns k = 0 and k = nz - 2: b = wall / hz^2 there.
    Each wall entry is a scalar or an (ny, nx) array."""
    nz = shape[0]
    hz = h[2]
    b = np.zeros(shape)
    if kind == "neumann":
        b[0] += walls[0] / hz
        b[-1] += walls[1] / hz
    elif kind == "dirichlet":
        b[0] += 2.0 * walls[0] / hz ** 2
        b[-1] += 2.0 * walls[1] / hz ** 2
    elif kind == "wface":
        b[0] += walls[0] / hz ** 2
        b[nz - 2] += walls[1] / hz ** 2
    else:
        raise ValueError(kind)
    return b


def helmholtz(rhs, coeff, shift, kind, h, walls=None):
    """Solve ``coeff * L x - shift * x = rhs`` exactly.

    ``kind``: 'neumann' (cell-centred in z, homogeneous Neumann walls), 'dirichlet'
    (cell-centred in z, zero-value walls, ghost = -adjacent) or 'wface' (z-face located,
    unknowns k = 0..nz-2, wall values 0; layer nz-1 of the result is 0).
    FFT in x and y; in z the transform whose basis vectors are the exact eigenvectors of
    the wall-normal second difference: DCT-II (Neumann), DST-II (Dirichlet, centred),
    DST-I of length nz-1 (Dirichlet, faces). A singular Neumann Poisson problem
    (shift == 0) returns the zero-mean solution.
    ``walls`` (bottom, top): inhomogeneous wall data for L (``wall_vector``); the known part
    moves to the right-hand side, coeff L_0 x - shift x = rhs - coeff b. For 'wface' layer
    nz-1 of the result is then the top-wall value.
    """
    if walls is not None:
        x = helmholtz(rhs - coeff * wall_vector(rhs.shape, kind, h, walls), coeff, shift, kind, h)
        if kind == "wface":
            x[-1] = walls[1]
        return x
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    X = sfft.fft2(rhs, axes=(1, 2))
    lam_xy = _eig_periodic(ny, hy)[:, None] + _eig_periodic(nx, hx)[None, :]
    if kind == "neumann":
        Z = sfft.dct(X, type=2, axis=0, norm="ortho")
        m = np.arange(nz)
    elif kind == "dirichlet":
        Z = sfft.dst(X, type=2, axis=0, norm="ortho")
        m = np.arange(1, nz + 1)
    elif kind == "wface":
        Z = sfft.dst(X[: nz - 1], type=1, axis=0, norm="ortho")
        m = np.arange(1, nz)
    else:
        raise ValueError(kind)
    lam_z = -4.0 / hz ** 2 * np.sin(np.pi * m / (2 * nz)) ** 2
    denom = coeff * (lam_z[:, None, None] + lam_xy[None, :, :]) - shift
    singular = denom == 0.0
    denom = np.where(singular, 1.0, denom)
    Z = np.where(singular, 0.0, Z / denom)
    if kind == "neumann":
        Y = sfft.idct(Z, type=2, axis=0, norm="ortho")
    elif kind == "dirichlet":
        Y = sfft.idst(Z, type=2, axis=0, norm="ortho")
    else:
        Y = np.zeros((nz,) + Z.shape[1:], dtype=complex)
        Y[: nz - 1] = sfft.idst(Z, type=1, axis=0, norm="ortho")
    return np.ascontiguousarray(sfft.ifft2(Y, axes=(1, 2)).real)


def helmholtz_robin(rhs, coeff, shift, d, h):
    """Solve ``coeff * (L_N + d W) x - shift * x = rhs`` exactly, W the indicator of the two
    wall-adjacent layers: the cell-centred Laplacian whose wall ghost carries a term linear in
    the wall-adjacent value (a Robin condition), d = -kappa / hz.

    FFT in x and y; in z the eigenvectors of the symmetric wall-normal matrix (second
    difference with Neumann ghosts plus d on the two corner entries), from numpy.linalg.eigh.
    """
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    _, TR = _wall_normal_matrices(nz, hz, d)
    lam_z, V = np.linalg.eigh(TR)
    X = sfft.fft2(rhs, axes=(1, 2))
    lam_xy = _eig_periodic(ny, hy)[:, None] + _eig_periodic(nx, hx)[None, :]
    Z = np.tensordot(V.T, X, axes=(1, 0))
    Z = Z / (coeff * (lam_z[:, None, None] + lam_xy[None, :, :]) - shift)
    Y = np.tensordot(V, Z, axes=(1, 0))
    return np.ascontiguousarray(sfft.ifft2(Y, axes=(1, 2)).real)


def _wall_normal_matrices(nz, hz, d):
    """Dense z second differences: Neumann ghosts, and the same plus d on the two corners."""
    T = np.zeros((nz, nz))
    for k in range(nz):
        T[k, k] = -2.0 / hz ** 2
        if k > 0:
            T[k, k - 1] = 1.0 / hz ** 2
        else:
            T[k, k] += 1.0 / hz ** 2
        if k < nz - 1:
            T[k, k + 1] = 1.0 / hz ** 2
        else:
            T[k, k] += 1.0 / hz ** 2
    TR = T.copy()
    TR[0, 0] += d
    TR[nz - 1, nz - 1] += d
    return T, TR


def ch_relaxed_solve(rhs, s, c, d, h):
    """Solve [L_N (L_N + d W) - s L_N + c] x = rhs exactly (W the indicator of the two
    wall-adjacent layers): eq. NS25 with the relaxed wall condition of eq. NS34.

    FFT in x and y; for every Fourier mode (wavenumber shift mu of the x-y Laplacian) the
    nz x nz matrix (T + mu)(T_R + mu) - s (T + mu) + c is built densely and solved with
    numpy.linalg.solve.
    """
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    T, TR = _wall_normal_matrices(nz, hz, d)
    X = sfft.fft2(rhs, axes=(1, 2))
    lam_xy = _eig_periodic(ny, hy)[:, None] + _eig_periodic(nx, hx)[None, :]
    Y = np.empty_like(X)
    I = np.eye(nz)
    for j in range(ny):
        mus = lam_xy[j]
        M = np.stack([(T + mu * I) @ (TR + mu * I) - s * (T + mu * I) + c * I for mu in mus])
        Y[:, j, :] = np.linalg.solve(M, X[:, j, :].T[:, :, None])[:, :, 0].T
    return np.ascontiguousarray(sfft.ifft2(Y, axes=(1, 2)).real)


# ---------------------------------------------------------------------------------------
# dual-grid transfer (Sec. 3.1)
# ---------------------------------------------------------------------------------------


def prolong(u, v, w, ry, r=2):
    """Coarse face velocities -> fine face velocities (eq. dual1, Rudman's interpolation);
    with refinement r = 1 (single resolution) the phase field lives on the flow grid and the
    face velocities are used as they are.

    Along the component's own axis, a fine face that coincides with a coarse face takes
    its value and the fine face through a coarse cell centre takes the mean of the two
    coarse faces; across the other axes the value is constant over the two fine cells.
    The bottom-wall w is 0. The result keeps the discrete divergence of every fine cell
    equal to that of its coarse parent cell.
    """
    if r == 1:
        return u.copy(), v.copy(), w.copy()
    nz, ny, nx = u.shape

    def rep(a, axes):
        for ax, r in axes:
            if r > 1:
                a = np.repeat(a, r, axis=ax)
        return a

    uf = np.empty((nz, ny, 2 * nx))
    uf[:, :, 1::2] = u
    uf[:, :, 0::2] = 0.5 * (xm(u) + u)
    uf = rep(uf, [(1, ry), (0, 2)])

    if ry == 2:
        vf = np.empty((nz, 2 * ny, nx))
        vf[:, 1::2, :] = v
        vf[:, 0::2, :] = 0.5 * (ym(v) + v)
    else:
        vf = v.copy()
    vf = rep(vf, [(2, 2), (0, 2)])

    wf = np.empty((2 * nz, ny, nx))
    wf[1::2] = w
    wf[0::2] = 0.5 * (zm_face(w) + w)
    wf = rep(wf, [(2, 2), (1, ry)])
    return uf, vf, wf


def _restrict_axis(f, axis, loc, r, wall):
    """1D rule of eq. dual2 along one axis (refinement r = 2, or r = 1 when the axis is not
    refined). 'c': coarse centre i averages fine (r i .. r i + r - 1); 'f': coarse face i (at
    (i+1) h) averages the two fine cells on either side of it. Periodic axes wrap; on the
    wall axis the faces run from the bottom wall (index -1) to the top wall (nz - 1), and a
    fine neighbour beyond a wall is replaced by the wall-adjacent fine cell (Neumann ghost),
    giving nz + 1 face layers."""
    n = f.shape[axis]
    take = lambda idx: np.take(f, idx, axis=axis)
    if loc == "c":
        if r == 1:
            return f.copy()
        return 0.5 * (take(np.arange(0, n, 2)) + take(np.arange(1, n, 2)))
    if wall:
        kf = np.arange(-1, n // r)
        a = np.clip(r * kf + r - 1, 0, n - 1)
        b = np.clip(r * kf + r, 0, n - 1)
        return 0.5 * (take(a) + take(b))
    if r == 1:
        return 0.5 * (f + np.roll(f, -1, axis=axis))
    nc = n // 2
    a = (2 * np.arange(nc) + 1) % n
    b = (2 * np.arange(nc) + 2) % n
    return 0.5 * (take(a) + take(b))


def restrict(f, loc, ry, r=2):
    """Fine cell-centred field -> coarse location ``loc`` = (z, y, x) letters in {'c','f'}
    (eq. dual2, extended to 3D as a tensor product of the 1D rules; refinement r in x and z,
    ry in y). A z face location returns nz + 1 layers (bottom wall .. top wall). With r = ry
    = 1 (single resolution) a centre is the cell itself, a face the mean of its two cells and
    an edge the mean of its four."""
    lz, ly, lx = loc
    g = _restrict_axis(f, 2, lx, r, False)
    g = _restrict_axis(g, 1, ly, ry, False)
    g = _restrict_axis(g, 0, lz, r, True)
    return g


def mixture(phi, a1, a2):
    """Property linear in phi (eqs. NS8, NS9, dual3): phase 1 at phi = +1."""
    return 0.5 * (1.0 + phi) * a1 + 0.5 * (1.0 - phi) * a2


# ---------------------------------------------------------------------------------------
# divergence / gradient on the staggered coarse grid
# ---------------------------------------------------------------------------------------


def divergence(u, v, w, h):
    hx, hy, hz = h
    return (u - xm(u)) / hx + (v - ym(v)) / hy + (w - zm_face(w)) / hz


def gradient(p, h):
    """Face gradient of a centred field with zero normal gradient at the walls."""
    hx, hy, hz = h
    gz = (zp_neu(p) - p) / hz
    gz[-1] = 0.0
    return (xp(p) - p) / hx, (yp(p) - p) / hy, gz
