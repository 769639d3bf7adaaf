"""Loop-by-loop reference stencils for tiny grids, written independently of ``oracle/``.

Each function states a discrete equation cell by cell with explicit ghost rules, so that a
test can check the oracle's vectorised / spectral code against the plain definition.
Arrays are indexed [k][j][i] (z, y, x); x and y periodic, z bounded by walls.
"""
from __future__ import annotations

import numpy as np


def idx(shape):
    nz, ny, nx = shape
    return lambda k, j, i: (k * ny + j) * nx + i


def dense_operator(shape, h, coeff, shift, kind, kappa=0.0):
    """Dense matrix of coeff * Laplacian - shift * I on a z-bounded box.
    kind 'neumann': ghost = adjacent cell; 'dirichlet': ghost = -adjacent;
    'wface': unknowns are the interior z faces k = 0..nz-2, wall faces are 0;
    'robin': ghost = adjacent - hz kappa adjacent (a wall derivative -kappa times the value)."""
    nz, ny, nx = shape
    hx, hy, hz = h
    nzu = nz - 1 if kind == "wface" else nz
    n = nzu * ny * nx
    I = lambda k, j, i: (k * ny + j) * nx + i
    A = np.zeros((n, n))
    for k in range(nzu):
        for j in range(ny):
            for i in range(nx):
                r = I(k, j, i)
                A[r, r] -= shift
                for (dj, di, hh) in ((0, 1, hx), (0, -1, hx), (1, 0, hy), (-1, 0, hy)):
                    c = I(k, (j + dj) % ny, (i + di) % nx)
                    A[r, c] += coeff / hh ** 2
                    A[r, r] -= coeff / hh ** 2
                for dk in (1, -1):
                    kk = k + dk
                    A[r, r] -= coeff / hz ** 2
                    if 0 <= kk < nzu:
                        A[r, I(kk, j, i)] += coeff / hz ** 2
                    elif kind == "neumann":
                        A[r, r] += coeff / hz ** 2
                    elif kind == "dirichlet":
                        A[r, r] -= coeff / hz ** 2
                    elif kind == "robin":
                        A[r, r] += coeff / hz ** 2 * (1.0 - hz * kappa)
                    # 'wface': wall value 0 contributes nothing
    return A


def lap(a, h, zghost):
    """Loop Laplacian of a cell-centred field; zghost(k_ghost, a, j, i) gives ghost values."""
    nz, ny, nx = a.shape
    hx, hy, hz = h
    out = np.zeros_like(a)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = a[k, j, i]
                s = (a[k, j, (i + 1) % nx] - 2 * c + a[k, j, (i - 1) % nx]) / hx ** 2
                s += (a[k, (j + 1) % ny, i] - 2 * c + a[k, (j - 1) % ny, i]) / hy ** 2
                up = a[k + 1, j, i] if k + 1 < nz else zghost(nz, a, j, i)
                dn = a[k - 1, j, i] if k - 1 >= 0 else zghost(-1, a, j, i)
                s += (up - 2 * c + dn) / hz ** 2
                out[k, j, i] = s
    return out


def neumann_ghost(kg, a, j, i):
    return a[0, j, i] if kg < 0 else a[-1, j, i]
