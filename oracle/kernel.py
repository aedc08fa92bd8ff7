"""Cell-averaged Green's function of a single-layer die -- oracle (test infrastructure only).

What is computed
----------------
The Green's function f_sp of Sec. II-B (Eq. Green) is the temperature rise on the top face
of the die due to a unit power source on that face.  For one silicon layer of thickness t and
conductivity k, adiabatic on top (apart from the injected power) and held at ambient on the
bottom, it follows from the heat equation (Eq. fourier) by the method of images in depth:

    f(r) = 1/(2 pi k) * sum_{n in Z} (-1)^n / sqrt(r^2 + (2 n t)^2)                  (1)

Its 2-D Fourier transform is tanh(rho t) / (k rho): by Theorem I (Appendix) that is 2 pi times
the order-0 Hankel transform of f, so (1) is the inverse Hankel transform of that closed form.
Split off the n = 0 term:

    2 pi k f(r) = 1/r + R(r),  R(r) = sum_{n != 0} (-1)^n / sqrt(r^2 + (2 n t)^2),   R(0) = -ln 2 / t

R is smooth.  Closing the Hankel integral on the poles of tanh gives the modal form

    2 pi k f(r) = (2/t) sum_{m >= 0} K0((m + 1/2) pi r / t)                           (2)

which converges fast for r >~ t.  The grid only sets output resolution (Sec. II-B): power is
piecewise constant over cells, so the table entry K(a, b) is the rise at the centre of cell
(a, b) per watt spread uniformly over the cell at the origin, i.e. the cell average of f.

The die edges are adiabatic; Sec. IV-F mirrors the power map about each edge.  Mirroring about
both edges of an axis repeats with period 2N, so the table the direct sum needs is the
periodised kernel  K_per(a, b) = sum_{m, n} K(a + 2 N_x m, b + 2 N_y n).

Evaluation routes (each cell picks one; tests pin them against one another):
  near cells   : closed-form cell integral of 1/r (corner antiderivative) for the cells around
                 the origin, Gauss-Legendre elsewhere; Gauss-Legendre of R, with R summed from
                 the image series (1) accelerated by repeated averaging of partial sums
                 (Euler / van Wijngaarden transform of an alternating series);
  far cells    : Gauss-Legendre of the modal form (2) with scipy's K0;
  pins only    : the Hankel integral 1/r - 2 int_0^inf J0(s r) / (exp(2 s t) + 1) ds by
                 scipy quadrature (``point_kernel_hankel``).

Parity: pinned (closed forms R(0), the origin cell, the sum rule sum K = t/(k hx hy), the
three representations against each other, and a finite-volume solve in ``fd``).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy import integrate, special


# ----------------------------------------------------------------------------- 1/r cell integral
def _corner(x: np.ndarray, y: np.ndarray, d: float) -> np.ndarray:
    """Antiderivative F with d2F/dxdy = (x^2 + y^2 + d^2)^(-1/2)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(np.broadcast(x, y).shape)
    rxd = np.sqrt(x * x + d * d)
    ryd = np.sqrt(y * y + d * d)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(rxd > 0, x * np.arcsinh(y / np.where(rxd > 0, rxd, 1.0)), 0.0)
        t2 = np.where(ryd > 0, y * np.arcsinh(x / np.where(ryd > 0, ryd, 1.0)), 0.0)
    out = t1 + t2
    if d > 0.0:
        r = np.sqrt(x * x + y * y + d * d)
        out = out - d * np.arctan(x * y / (d * r))
    return out


def cell_integral_inv_r(x0, y0, hx: float, hy: float, d: float = 0.0) -> np.ndarray:
    """Integral over the cell centred at (x0, y0) of (x^2 + y^2 + d^2)^(-1/2) dx dy (closed form)."""
    x0 = np.asarray(x0, dtype=np.float64)
    y0 = np.asarray(y0, dtype=np.float64)
    x1, x2 = x0 - 0.5 * hx, x0 + 0.5 * hx
    y1, y2 = y0 - 0.5 * hy, y0 + 0.5 * hy
    return _corner(x2, y2, d) - _corner(x1, y2, d) - _corner(x2, y1, d) + _corner(x1, y1, d)


# ----------------------------------------------------------------------------- point kernels
def image_remainder(r, t: float, n_direct: int = 24, n_avg: int = 40) -> np.ndarray:
    """R(r) = sum_{n != 0} (-1)^n / sqrt(r^2 + (2 n t)^2) from the image series.

    The alternating tail is accelerated by averaging consecutive partial sums ``n_avg`` times
    (Euler transform); the first ``n_direct`` terms are summed as they are.
    """
    r = np.asarray(r, dtype=np.float64)
    n = np.arange(1, n_direct + n_avg + 1, dtype=np.float64)
    sign = np.where(n % 2 == 1, -1.0, 1.0)
    terms = sign / np.sqrt(r[..., None] ** 2 + (2.0 * n * t) ** 2)
    s = np.cumsum(terms, axis=-1)[..., n_direct - 1:]
    for _ in range(n_avg):
        s = 0.5 * (s[..., 1:] + s[..., :-1])
    return 2.0 * s[..., 0]


def modal_sum(r, t: float, rel: float = 1e-19, m_max: int = 4000) -> np.ndarray:
    """(2/t) sum_m K0((m + 1/2) pi r / t) = 2 pi k f(r), the modal form of the image series."""
    r = np.asarray(r, dtype=np.float64)
    total = np.zeros_like(r)
    first = None
    for m in range(m_max):
        term = special.k0((m + 0.5) * math.pi * r / t)
        if first is None:
            first = term
        total += term
        if np.all(term <= rel * first):
            break
    return (2.0 / t) * total


def point_kernel_hankel(r: float, t: float) -> float:
    """2 pi k f(r) from the inverse Hankel transform of tanh(s t)/(k s) (scipy quadrature)."""
    if r <= 0.0:
        raise ValueError("r must be positive")

    def integrand(s):
        return special.j0(s * r) / (math.exp(min(2.0 * s * t, 700.0)) + 1.0)

    upper = 40.0 / t
    val, _ = integrate.quad(integrand, 0.0, upper, limit=2000, epsabs=1e-16 / t, epsrel=1e-13)
    return 1.0 / r - 2.0 * val


# ----------------------------------------------------------------------------- cell kernel
@lru_cache(maxsize=None)
def _gauss_legendre(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return x, w


def _cell_average(func, x0, y0, hx, hy, q):
    """Tensor Gauss-Legendre average over cells centred at (x0, y0) of func(x, y)."""
    xi, wi = _gauss_legendre(q)
    xs = x0[:, None, None] + 0.5 * hx * xi[None, :, None]
    ys = y0[:, None, None] + 0.5 * hy * xi[None, None, :]
    w2 = 0.25 * wi[:, None] * wi[None, :]
    vals = func(xs, ys)
    return np.sum(vals * w2[None], axis=(1, 2))


def cell_kernel(a, b, hx: float, hy: float, t: float, k: float) -> np.ndarray:
    """K(a, b): rise at the centre of cell (a, b) per watt spread over the cell at the origin [K/W].

    ``a`` indexes x (columns), ``b`` indexes y (rows); both are integer cell offsets.
    """
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    b = np.atleast_1d(np.asarray(b, dtype=np.float64))
    a, b = np.broadcast_arrays(a, b)
    shape = a.shape
    a = np.abs(a.ravel())
    b = np.abs(b.ravel())
    x0 = a * hx
    y0 = b * hy
    hmax = max(hx, hy)
    rho = np.hypot(x0, y0)
    out = np.empty(a.shape)

    near = rho < 2.0 * t + hmax
    if np.any(near):
        xn, yn, an, bn = x0[near], y0[near], a[near], b[near]
        # 1/r part: corner formula next to the origin, Gauss-Legendre further out
        inv_r = np.empty(xn.shape)
        closed = np.maximum(an, bn) <= 3
        if np.any(closed):
            inv_r[closed] = cell_integral_inv_r(xn[closed], yn[closed], hx, hy) / (hx * hy)
        if np.any(~closed):
            inv_r[~closed] = _cell_average(lambda x, y: 1.0 / np.hypot(x, y), xn[~closed], yn[~closed], hx, hy, 16)
        rem = _cell_average(lambda x, y: image_remainder(np.hypot(x, y), t), xn, yn, hx, hy, 16)
        out[near] = inv_r + rem

    far = ~near
    if np.any(far):
        xf, yf = x0[far], y0[far]
        dist = rho[far] / min(hx, hy)
        vals = np.empty(xf.shape)
        for lo, hi, q in ((0.0, 8.0, 16), (8.0, 64.0, 8), (64.0, 512.0, 4), (512.0, np.inf, 2)):
            sel = (dist >= lo) & (dist < hi)
            if np.any(sel):
                vals[sel] = _cell_average(lambda x, y: modal_sum(np.hypot(x, y), t), xf[sel], yf[sel], hx, hy, q)
        out[far] = vals

    return (out / (2.0 * math.pi * k)).reshape(shape)


def periods_needed(lx: float, ly: float, t: float, rel: float = 1e-30) -> int:
    """Number of 2L periods per side beyond which the kernel is below rel of its peak."""
    # f decays like exp(-pi r / (2 t)); the nearest image of period m sits at (2m - 1) L.
    lmin = min(lx, ly)
    m = 1
    while math.exp(-math.pi * (2 * m + 1) * lmin / (2.0 * t)) > rel and m < 64:
        m += 1
    return m


def periodized_table(nx: int, ny: int, lx: float, ly: float, t: float, k: float) -> np.ndarray:
    """K_per(a, b) for a in [0, nx] (x offset), b in [0, ny] (y offset); array [ny + 1][nx + 1].

    K_per(a, b) = sum_{m, n} K(a + 2 nx m, b + 2 ny n): the images of Sec. IV-F repeated over
    both edges of each axis.
    """
    hx, hy = lx / nx, ly / ny
    mp = periods_needed(lx, ly, t)
    aa = np.arange(nx + 1)
    bb = np.arange(ny + 1)
    table = np.zeros((ny + 1, nx + 1))
    for m in range(-mp, mp + 1):
        for n in range(-mp, mp + 1):
            A = aa[None, :] + 2 * nx * m
            B = bb[:, None] + 2 * ny * n
            table += cell_kernel(A, B, hx, hy, t, k)
    return table
