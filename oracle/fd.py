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

A spatially varying conductivity k(x, y) = k m(x, y) (the conductivity-variation map of
Sec. II-E, constant through the depth, piecewise constant on the coarse cells) couples the
cosine modes; ``solve_lateral_k`` then solves the same finite-volume system (harmonic-mean face
conductances) by conjugate gradients preconditioned with the exact constant-conductivity
solve, and ``solve_sparse`` takes the same map for a direct check on tiny grids.

A layered box (``solve_modes_stack``: the package stack of Table param, constant conductivity per
layer, isothermal or convective bottom face) keeps the cosine-mode split, with the vertical
conductance between cell centres the series resistance of their half cells.

``transient_modes`` adds the heat capacity (the transient form of Eq. fourier) to the same box
and solves each lateral mode's depth system exactly in time through its eigenvectors.

Parity: pinned (``solve_modes`` and ``solve_lateral_k`` against ``solve_sparse`` to rounding;
``transient_modes`` at long times against ``solve_modes``;
``solve_modes_stack`` of one layer against ``solve_modes``; convergence order checked).
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


def solve_modes_stack(q_coarse: np.ndarray, lx: float, ly: float, layers, h_bottom: float | None, r: int,
                      nz_per_layer) -> np.ndarray:
    """Top-surface rise at the coarse cell centres [K] of a layered box (layers = [(t, k), ...]
    top first, each split into nz_per_layer[i] cells in depth), bottom face isothermal
    (h_bottom None) or convective with coefficient h_bottom: the same cosine-mode split and one
    tridiagonal system in depth per mode, the vertical conductance between two cell centres the
    series resistance of their half cells."""
    if r % 2 == 0:
        raise ValueError("refinement must be odd")
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy = lx / mfx, ly / mfy
    q_fine = _fine_flux(q_coarse, r)
    lam_x = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfx) / mfx)) / (hx * hx)
    lam_y = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfy) / mfy)) / (hy * hy)
    lam = lam_y[:, None] + lam_x[None, :]
    dz, kz = [], []
    for (t, k), nz in zip(layers, nz_per_layer):
        dz += [t / nz] * nz
        kz += [k] * nz
    nzt = len(dz)
    # conductance per unit area between centres z and z + 1, and from the last centre to the
    # bottom boundary (through the half cell, plus 1 / h for a convective face)
    g = [1.0 / (0.5 * dz[z] / kz[z] + 0.5 * dz[z + 1] / kz[z + 1]) for z in range(nzt - 1)]
    rb = 0.5 * dz[-1] / kz[-1] + (0.0 if h_bottom is None else 1.0 / h_bottom)
    gb = 1.0 / rb
    qh = sfft.dctn(q_fine, type=2, norm="ortho")
    diag, sub, sup = [], [], []
    for z in range(nzt):
        d = kz[z] * lam * dz[z]
        if z > 0:
            d = d + g[z - 1]
        if z < nzt - 1:
            d = d + g[z]
        else:
            d = d + gb
        diag.append(d)
        sub.append(-g[z - 1] if z > 0 else 0.0)
        sup.append(-g[z] if z < nzt - 1 else 0.0)
    rhs = [np.zeros(lam.shape) for _ in range(nzt)]
    rhs[0] = qh
    cp, dp = [None] * nzt, [None] * nzt
    cp[0] = sup[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for z in range(1, nzt):
        den = diag[z] - sub[z] * cp[z - 1]
        cp[z] = sup[z] / den
        dp[z] = (rhs[z] - sub[z] * dp[z - 1]) / den
    x_top = dp[-1]
    for z in range(nzt - 2, -1, -1):
        x_top = dp[z] - cp[z] * x_top
    t_top = sfft.idctn(x_top, type=2, norm="ortho")
    return _coarse_centres(t_top + q_fine * 0.5 * dz[0] / kz[0], r)


def richardson_stack(q_coarse: np.ndarray, lx: float, ly: float, layers, h_bottom: float | None, r0: int = 3,
                     nz0=(4, 2, 4), levels: int = 2) -> np.ndarray:
    """``richardson`` for a layered box: refine laterally and in depth by 3 per level."""
    sols = []
    r, nz = r0, list(nz0)
    for _ in range(levels + 1):
        sols.append(solve_modes_stack(q_coarse, lx, ly, layers, h_bottom, r, nz))
        r *= 3
        nz = [3 * v for v in nz]
    cur = sols
    order = 2
    for _ in range(levels):
        f = 3.0 ** order
        cur = [(f * cur[i + 1] - cur[i]) / (f - 1.0) for i in range(len(cur) - 1)]
        order += 2
    return cur[-1]


def transient_modes(q_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, rho_c: float, r: int, nz: int,
                    times) -> np.ndarray:
    """Top-surface rise at the coarse cell centres [K] at each of ``times`` after the flux q is
    switched on at t = 0 (Eq. fourier with its heat-capacity term), for the same finite-volume
    box as ``solve_modes``: per lateral cosine mode the depth system rho_c dz dT/dt = -A T + b
    is solved exactly in time through the eigenvectors of the symmetric tridiagonal A."""
    from scipy.linalg import eigh_tridiagonal

    if r % 2 == 0:
        raise ValueError("refinement must be odd")
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy, dz = lx / mfx, ly / mfy, t / nz
    q_fine = _fine_flux(q_coarse, r)
    lam_x = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfx) / mfx)) / (hx * hx)
    lam_y = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfy) / mfy)) / (hy * hy)
    lam = (lam_y[:, None] + lam_x[None, :]).ravel()
    qh = sfft.dctn(q_fine, type=2, norm="ortho").ravel()
    g = k / dz  # conductance per unit area between neighbouring centres
    cap = rho_c * dz
    times = np.atleast_1d(np.asarray(times, dtype=np.float64))
    top = np.empty((len(times), lam.size))
    off = np.full(nz - 1, -g / cap)
    for i, lm in enumerate(lam):
        d = np.full(nz, 2.0 * g + k * lm * dz)
        d[0] -= g  # adiabatic top face (the flux enters as a source)
        d[-1] += g  # isothermal bottom face half a cell below (conductance 2 k / dz in total)
        mu, v = eigh_tridiagonal(d / cap, off)
        proj = v[0, :] * (qh[i] / cap)  # b has the flux in the top cell only
        # T_top(t) = sum_j v[0, j] proj_j (1 - exp(-mu_j t)) / mu_j
        top[:, i] = (-np.expm1(-np.outer(times, mu)) / mu) @ (v[0, :] * proj)
    out = []
    for it in range(len(times)):
        t_top = sfft.idctn(top[it].reshape(mfy, mfx), type=2, norm="ortho")
        out.append(_coarse_centres(t_top + q_fine * 0.5 * dz / k, r))
    return np.array(out)


def solve_sparse(q_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, r: int, nz: int,
                 m_coarse: np.ndarray | None = None) -> np.ndarray:
    """Same discretisation as ``solve_modes`` (or ``solve_lateral_k`` when a conductivity map
    ``m_coarse`` is given), assembled as one sparse 3-D system with explicit loops (small grids)."""
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy, dz = lx / mfx, ly / mfy, t / nz
    q_fine = _fine_flux(q_coarse, r)
    kc = k * (_fine_flux(m_coarse, r) if m_coarse is not None else np.ones((mfy, mfx)))
    n = mfx * mfy * nz

    def idx(z, y, x):
        return (z * mfy + y) * mfx + x

    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    for z in range(nz):
        for y in range(mfy):
            for x in range(mfx):
                i = idx(z, y, x)
                dsum = 0.0
                for (zz, yy, xx, h2) in ((z, y, x - 1, hx * hx), (z, y, x + 1, hx * hx), (z, y - 1, x, hy * hy),
                                         (z, y + 1, x, hy * hy), (z - 1, y, x, dz * dz), (z + 1, y, x, dz * dz)):
                    if 0 <= xx < mfx and 0 <= yy < mfy and 0 <= zz < nz:
                        a_, b_ = kc[y, x], kc[yy, xx]
                        g = 2.0 * a_ * b_ / (a_ + b_) / h2  # harmonic mean of the two cells
                        rows.append(i)
                        cols.append(idx(zz, yy, xx))
                        vals.append(-g)
                        dsum += g
                    elif zz == nz:  # bottom face held at ambient, half a cell away
                        dsum += 2.0 * kc[y, x] / h2
                rows.append(i)
                cols.append(i)
                vals.append(dsum)
                if z == 0:
                    rhs[i] = q_fine[y, x] / dz
    a = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    sol = spla.spsolve(a, rhs)
    t_top = sol[:mfx * mfy].reshape(mfy, mfx)
    return _coarse_centres(t_top + q_fine * 0.5 * dz / kc, r)


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


# ----------------------------------------------------------------------------- lateral k(x, y)
def _apply_operator(temp: np.ndarray, kc: np.ndarray, hx: float, hy: float, dz: float) -> np.ndarray:
    """A T for the finite-volume system of ``solve_sparse`` with column conductivities kc[y][x]
    (temp: [nz][ny][nx], top layer first)."""
    out = np.zeros_like(temp)
    gx = 2.0 * kc[:, :-1] * kc[:, 1:] / (kc[:, :-1] + kc[:, 1:]) / (hx * hx)
    flux = gx * (temp[:, :, 1:] - temp[:, :, :-1])
    out[:, :, :-1] -= flux
    out[:, :, 1:] += flux
    gy = 2.0 * kc[:-1, :] * kc[1:, :] / (kc[:-1, :] + kc[1:, :]) / (hy * hy)
    flux = gy * (temp[:, 1:, :] - temp[:, :-1, :])
    out[:, :-1, :] -= flux
    out[:, 1:, :] += flux
    gz = kc / (dz * dz)
    flux = gz * (temp[1:] - temp[:-1])
    out[:-1] -= flux
    out[1:] += flux
    out[-1] += 2.0 * gz * temp[-1]
    return out


def _constant_k_solve(rhs: np.ndarray, k: float, hx: float, hy: float, dz: float) -> np.ndarray:
    """Exact inverse of the operator with a uniform conductivity k (cosine modes laterally, one
    tridiagonal system in depth per mode), for a right-hand side in every layer."""
    nz, mfy, mfx = rhs.shape
    lam_x = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfx) / mfx)) / (hx * hx)
    lam_y = (2.0 - 2.0 * np.cos(np.pi * np.arange(mfy) / mfy)) / (hy * hy)
    lam = lam_y[:, None] + lam_x[None, :]
    b = sfft.dctn(rhs, type=2, norm="ortho", axes=(1, 2)) * (dz * dz / k)
    off = -1.0
    diag = [np.full(lam.shape, 2.0) + lam * dz * dz for _ in range(nz)]
    diag[0] = diag[0] - 1.0
    diag[-1] = diag[-1] + 1.0
    cp = [None] * nz
    dp = [None] * nz
    cp[0] = off / diag[0]
    dp[0] = b[0] / diag[0]
    for z in range(1, nz):
        den = diag[z] - off * cp[z - 1]
        cp[z] = off / den
        dp[z] = (b[z] - off * dp[z - 1]) / den
    x = np.empty_like(b)
    x[-1] = dp[-1]
    for z in range(nz - 2, -1, -1):
        x[z] = dp[z] - cp[z] * x[z + 1]
    return sfft.idctn(x, type=2, norm="ortho", axes=(1, 2))


def solve_lateral_k(q_coarse: np.ndarray, m_coarse: np.ndarray, lx: float, ly: float, t: float, k: float, r: int,
                    nz: int, rtol: float = 1e-14, max_iter: int = 500) -> np.ndarray:
    """Top-surface rise at the coarse cell centres [K] with conductivity k m(x, y) (m piecewise
    constant on the coarse cells, constant through the depth): preconditioned conjugate
    gradients on the finite-volume system, the preconditioner the exact solve at the mean
    conductivity."""
    if r % 2 == 0:
        raise ValueError("refinement must be odd")
    ny, nx = q_coarse.shape
    mfx, mfy = nx * r, ny * r
    hx, hy, dz = lx / mfx, ly / mfy, t / nz
    q_fine = _fine_flux(q_coarse, r)
    kc = k * _fine_flux(np.asarray(m_coarse, dtype=np.float64), r)
    kbar = float(np.mean(kc))
    rhs = np.zeros((nz, mfy, mfx))
    rhs[0] = q_fine / dz
    x = _constant_k_solve(rhs, kbar, hx, hy, dz)
    res = rhs - _apply_operator(x, kc, hx, hy, dz)
    zv = _constant_k_solve(res, kbar, hx, hy, dz)
    p = zv.copy()
    rz = float(np.vdot(res, zv))
    bnorm = float(np.linalg.norm(rhs))
    for _ in range(max_iter):
        if float(np.linalg.norm(res)) <= rtol * bnorm:
            break
        ap = _apply_operator(p, kc, hx, hy, dz)
        alpha = rz / float(np.vdot(p, ap))
        x += alpha * p
        res -= alpha * ap
        zv = _constant_k_solve(res, kbar, hx, hy, dz)
        rz_new = float(np.vdot(res, zv))
        p = zv + (rz_new / rz) * p
        rz = rz_new
    else:
        raise RuntimeError("conjugate gradients did not converge")
    return _coarse_centres(x[0] + q_fine * 0.5 * dz / kc, r)


def richardson_lateral_k(q_coarse: np.ndarray, m_coarse: np.ndarray, lx: float, ly: float, t: float, k: float,
                         r0: int = 3, nz0: int = 6, levels: int = 2) -> np.ndarray:
    """``richardson`` for a conductivity map: refine by 3 per level, extrapolate the h^2, h^4 terms."""
    sols = []
    r, nz = r0, nz0
    for _ in range(levels + 1):
        sols.append(solve_lateral_k(q_coarse, m_coarse, lx, ly, t, k, r, nz))
        r *= 3
        nz *= 3
    cur = sols
    order = 2
    for _ in range(levels):
        f = 3.0 ** order
        cur = [(f * cur[i + 1] - cur[i]) / (f - 1.0) for i in range(len(cur) - 1)]
        order += 2
    return cur[-1]
