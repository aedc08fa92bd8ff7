"""Brute-force finite-volume solve of the steady heat equation -- pin for the oracle (test only).

Discretises Eq. fourier (Sec. II-A) at steady state, div(k grad T) = 0, on the die box
[0, Lx] x [0, Ly] x [0, t] with cell-centred finite volumes: a prescribed heat flux q(x, y)
into the top face, zero flux through the four side walls, T = T_amb on the bottom face.  Power
is piecewise constant on the coarse N x N cells; the fine lateral grid refines each coarse cell
r x r times (r odd, so every coarse cell centre is a fine cell centre).

Two solvers of the *same* linear system:
  * ``solve_sparse``  -- scipy sparse LU of the full 3-D system (small grids);
  * ``solve_modes``   -- the zero-flux second difference on a uniform lateral grid is
    diagonalised exactly by cosine vectors, so the 3-D system splits into one tridiagonal
    system in depth per lateral cosine mode (large grids).
Richardson extrapolation in the refinement removes the leading O(h^2) error.

Parity: pinned (``solve_modes`` against ``solve_sparse`` to rounding; convergence order checked).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _fine_flux(q_coarse: np.ndarray, r: int) -> np.ndarray:
    return np.kron(q_coarse, np.ones((r, r)))


def _surface_from_top_cells(t_top: np.ndarray, q_fine: np.ndarray, dz: float, k: float) -> np.ndarray:
    # T(0) = T(dz/2) + q (dz/2) / k to second order (flux through the upper half cell)
    return t_top + q_fine * 0.5 * dz / k


def _coarse_centres(fine: np.ndarray, r: int) -> np.ndarray:
    c = r // 2
    return fine[c::r, c::r]


def solve_modes(q_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, r: int, nz: int) -> np.ndarray:
    """Top-surface rise at the coarse cell centres [K] (cosine-mode split + tridiagonal solves)."""
    if r % 2 == 0:
        raise ValueError("refinement must be odd")
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy, dz = lx / mfx, ly / mfy, t / nz
    q_fine = _fine_flux(q_coarse, r)
    # eigenvalues of the zero-flux second difference (per unit k)
    lam_x = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfx) / mfx)) / (hx * hx)
    lam_y = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfy) / mfy)) / (hy * hy)
    lam = lam_y[:, None] + lam_x[None, :]
    qh = sfft.dctn(q_fine, type=2, norm="ortho")
    # tridiagonal in depth per mode, unknowns T_z at cell centres z = 0 (top) .. nz-1 (bottom)
    # rows scaled by dz^2 / k:  -T_{z-1} + (2 + lam dz^2) T_z - T_{z+1} = rhs
    a = -np.ones(nz)  # sub-diagonal (z-1)
    c = -np.ones(nz)  # super-diagonal (z+1)
    diag = [np.full(lam.shape, 2.0) + lam * dz * dz for _ in range(nz)]
    diag[0] = diag[0] - 1.0  # top: zero-flux face to the outside, flux enters as source
    diag[-1] = diag[-1] + 1.0  # bottom: T = 0 on the face half a cell below
    rhs = [np.zeros(lam.shape) for _ in range(nz)]
    rhs[0] = qh * dz / k
    # Thomas algorithm, vectorised over modes
    cp = [None] * nz
    dp = [None] * nz
    cp[0] = c[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for z in range(1, nz):
        den = diag[z] - a[z] * cp[z - 1]
        cp[z] = c[z] / den
        dp[z] = (rhs[z] - a[z] * dp[z - 1]) / den
    x_top = dp[-1]
    for z in range(nz - 2, -1, -1):
        x_top = dp[z] - cp[z] * x_top
    t_top = sfft.idctn(x_top, type=2, norm="ortho")
    return _coarse_centres(_surface_from_top_cells(t_top, q_fine, dz, k), r)


def solve_sparse(q_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, r: int, nz: int) -> np.ndarray:
    """Same discretisation as ``solve_modes``, assembled as one sparse 3-D system (small grids)."""
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy, dz = lx / mfx, ly / mfy, t / nz
    q_fine = _fine_flux(q_coarse, r)
    n = mfx * mfy * nz

    def idx(z, y, x):
        return (z * mfy + y) * mfx + x

    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    gx, gy, gz = k / (hx * hx), k / (hy * hy), k / (dz * dz)
    for z in range(nz):
        for y in range(mfy):
            for x in range(mfx):
                i = idx(z, y, x)
                dsum = 0.0
                for (zz, yy, xx, g) in ((z, y, x - 1, gx), (z, y, x + 1, gx), (z, y - 1, x, gy),
                                        (z, y + 1, x, gy), (z - 1, y, x, gz), (z + 1, y, x, gz)):
                    if 0 <= xx < mfx and 0 <= yy < mfy and 0 <= zz < nz:
                        rows.append(i)
                        cols.append(idx(zz, yy, xx))
                        vals.append(-g)
                        dsum += g
                    elif zz == nz:  # bottom face held at ambient, half a cell away
                        dsum += 2.0 * g
                rows.append(i)
                cols.append(i)
                vals.append(dsum)
                if z == 0:
                    rhs[i] = q_fine[y, x] / dz
    a = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    sol = spla.spsolve(a, rhs)
    t_top = sol[:mfx * mfy].reshape(mfy, mfx)
    return _coarse_centres(_surface_from_top_cells(t_top, q_fine, dz, k), r)


def richardson(q_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, r0: int = 9,
               nz0: int = 18, levels: int = 2) -> np.ndarray:
    """Refine laterally and in depth by 3 per level and extrapolate away the O(h^2) term."""
    sols = []
    r, nz = r0, nz0
    for _ in range(levels + 1):
        sols.append(solve_modes(q_coarse, lx, ly, t, k, r, nz))
        r *= 3
        nz *= 3
    cur = sols
    order = 2
    for _ in range(levels):
        f = 3.0 ** order
        cur = [(f * cur[i + 1] - cur[i]) / (f - 1.0) for i in range(len(cur) - 1)]
        order += 2
    return cur[-1]
