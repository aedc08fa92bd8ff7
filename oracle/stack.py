"""Green's function of a layered package (Table param's Si / TIM / spreader stack) with an
isothermal or convective bottom -- oracle (test infrastructure only).

The paper models the package below the silicon as a constant added to the die's Green's
function (Sec. II-B: f_sp = f_silic + const) and lists the stack in Table param.  The exact
symbol of a stack follows from Eq. fourier layer by layer: in the 2-D Fourier domain a layer
of conductivity k and thickness t relates temperature and downward flux at its two faces, so
the thermal impedance Z = T / q seen from the top of the layer is

    Z_top = (Z_below + tanh(s t) / (k s)) / (1 + k s tanh(s t) Z_below),

starting from Z = 0 under an isothermal bottom (T = T_amb) or Z = 1 / h under a convective one
(-k dT/dz = h (T - T_amb)).  The stack's point response F(s) = Z at the top of the first layer;
F(0) = sum t_i / k_i (+ 1 / h), the one-dimensional series resistance.

The cell kernel of the stack is the single-slab kernel of the first layer (``oracle.kernel``,
exact image series, isothermal bottom) plus the difference dF = F_stack - F_slab, which decays
like exp(-2 s t_1) and so is summed as the plain cosine series of the side-wall images (Poisson
summation of the periodised, cell-averaged response):

    dK_per(a, b) = (1 / (Lx Ly)) sum_{m, n >= 0} w_m w_n dF(kappa_mn) S(kappa_mn)
                   cos(pi m a / nx) cos(pi n b / ny),
    kappa_mn = (pi m / Lx, pi n / Ly),  S = sinc(kappa_x hx / 2) sinc(kappa_y hy / 2) (the
    source cell average),  w_0 = 1/2, w_{m > 0} = 1,

truncated where exp(-2 |kappa| t_1) < 1e-22.

Parity: pinned -- two layers of equal conductivity equal one slab of their total thickness
(against the image series of ``oracle.kernel``); uniform power gives q (sum t_i / k_i + 1 / h);
h -> infinity gives the isothermal stack; the whole operator against a finite-volume solve of
the layered box with the same bottom (``oracle.fd.solve_modes_stack``).
"""
from __future__ import annotations

import math

import numpy as np

from . import kernel as _kernel


def stack_symbol(s: np.ndarray, layers, h_bottom: float | None) -> np.ndarray:
    """F(s) = T / q at the top of the stack; layers = [(t, k), ...] top first; h_bottom None for
    an isothermal bottom.  s > 0 (the s -> 0 limit is F(0) = sum t / k + 1 / h)."""
    s = np.asarray(s, dtype=np.float64)
    z = np.zeros_like(s) if h_bottom is None else np.full(s.shape, 1.0 / h_bottom)
    for t, k in reversed(layers):
        th = np.tanh(s * t)
        z = (z + th / (k * s)) / (1.0 + k * s * th * z)
    return z


def stack_symbol_at_zero(layers, h_bottom: float | None) -> float:
    return sum(t / k for t, k in layers) + (0.0 if h_bottom is None else 1.0 / h_bottom)


def delta_symbol(s: np.ndarray, layers, h_bottom: float | None) -> np.ndarray:
    """F_stack(s) - F_slab(s) with F_slab = tanh(s t1) / (k1 s) the first layer alone over an
    isothermal bottom (finite at s = 0)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    zero = s == 0.0
    t1, k1 = layers[0]
    out[zero] = stack_symbol_at_zero(layers, h_bottom) - t1 / k1
    sp = s[~zero]
    out[~zero] = stack_symbol(sp, layers, h_bottom) - np.tanh(sp * t1) / (k1 * sp)
    return out


def delta_table(nx: int, ny: int, lx: float, ly: float, layers, h_bottom: float | None) -> np.ndarray:
    """dK_per(a, b) for a in [0, nx], b in [0, ny] (array [ny + 1][nx + 1]), K/W."""
    t1 = layers[0][0]
    smax = 25.0 / t1  # exp(-2 s t1) < 2e-22 beyond
    mmax = int(math.ceil(smax * lx / math.pi)) + 1
    nmax = int(math.ceil(smax * ly / math.pi)) + 1
    m = np.arange(mmax + 1)
    n = np.arange(nmax + 1)
    kx = math.pi * m / lx
    ky = math.pi * n / ly
    hx, hy = lx / nx, ly / ny
    s = np.hypot(ky[:, None], kx[None, :])
    sinc = lambda u: np.sinc(u / math.pi)  # sin(u) / u
    g = delta_symbol(s, layers, h_bottom) * sinc(ky * hy / 2.0)[:, None] * sinc(kx * hx / 2.0)[None, :]
    wm = np.where(m == 0, 0.5, 1.0)
    wn = np.where(n == 0, 0.5, 1.0)
    g = g * wn[:, None] * wm[None, :] / (lx * ly)
    cx = np.cos(math.pi * np.outer(np.arange(nx + 1), m) / nx)  # [a][m]
    cy = np.cos(math.pi * np.outer(np.arange(ny + 1), n) / ny)  # [b][n]
    return cy @ g @ cx.T


def periodized_stack_table(nx: int, ny: int, lx: float, ly: float, layers, h_bottom: float | None) -> np.ndarray:
    """K_per of the stack: the first layer's image-series table plus the cosine series of dF."""
    t1, k1 = layers[0]
    base = _kernel.periodized_table(nx, ny, lx, ly, t1, k1)
    if len(layers) == 1 and h_bottom is None:
        return base
    return base + delta_table(nx, ny, lx, ly, layers, h_bottom)
