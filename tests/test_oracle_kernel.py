"""Pins of the oracle's cell-averaged Green's function (Sec. II-B, Appendix Theorem I, Sec. IV-F).

Each check compares the oracle against something other than itself: closed forms, library
quadrature, independent series representations, or the sum rule that Poisson summation fixes.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import kernel as K

T = 0.5e-3
KC = 150.0


def test_cell_integral_inv_r_closed_forms():
    # square cell centred on the singularity: int int 1/r over [-h/2, h/2]^2 = 4 h ln(1 + sqrt 2)
    for h in (1e-4, 3.7e-5):
        got = K.cell_integral_inv_r(0.0, 0.0, h, h)
        assert got == pytest.approx(4.0 * h * math.log(1.0 + math.sqrt(2.0)), rel=1e-14)


@pytest.mark.parametrize("x0,y0,hx,hy,d", [(0.0, 0.0, 1.0, 2.0, 0.0), (1.3, -0.4, 0.7, 0.5, 0.0),
                                            (2.0, 1.0, 1.0, 1.0, 0.6), (0.0, 0.0, 1.0, 1.5, 2.0)])
def test_cell_integral_inv_r_vs_quadrature(x0, y0, hx, hy, d):
    f = lambda y, x: 1.0 / math.sqrt(x * x + y * y + d * d)
    # split at the axes so that a singular point only ever sits on a sub-rectangle corner
    xs = sorted({x0 - hx / 2, x0 + hx / 2} | ({0.0} if abs(x0) < hx / 2 else set()))
    ys = sorted({y0 - hy / 2, y0 + hy / 2} | ({0.0} if abs(y0) < hy / 2 else set()))
    ref = 0.0
    for xa, xb in zip(xs[:-1], xs[1:]):
        for ya, yb in zip(ys[:-1], ys[1:]):
            ref += integrate.dblquad(f, xa, xb, ya, yb, epsabs=1e-14, epsrel=1e-13)[0]
    got = float(K.cell_integral_inv_r(x0, y0, hx, hy, d))
    assert got == pytest.approx(ref, rel=1e-11)


def test_image_remainder_at_origin():
    # R(0) = sum_{n != 0} (-1)^n / (2 |n| t) = -ln 2 / t
    assert float(K.image_remainder(0.0, T)) == pytest.approx(-math.log(2.0) / T, rel=1e-14)


def test_image_remainder_taylor_series():
    # R(r) = (1/t) sum_j binom(-1/2, j) (r / 2t)^(2j) * (-eta(2j + 1)), eta the Dirichlet eta
    # function = (1 - 2^(-2j)) zeta(2j + 1); valid for r < 2t.
    for r in (0.1 * T, 0.5 * T, 1.0 * T, 1.4 * T):
        acc = 0.0
        for j in range(0, 200):
            eta = math.log(2.0) if j == 0 else (1.0 - 2.0 ** (-2 * j)) * special.zeta(2 * j + 1)
            acc += special.binom(-0.5, j) * (r / (2 * T)) ** (2 * j) * (-eta)
        assert float(K.image_remainder(r, T)) == pytest.approx(acc / T, rel=1e-12, abs=1e-12 / T)


@pytest.mark.parametrize("rt", [0.4, 0.8, 1.0, 1.5, 2.0, 2.5])
def test_three_representations_agree(rt):
    r = rt * T
    images = 1.0 / r + float(K.image_remainder(r, T))
    modes = float(K.modal_sum(r, T))
    hankel = K.point_kernel_hankel(r, T)
    assert modes == pytest.approx(images, rel=1e-13)
    assert hankel == pytest.approx(images, rel=1e-12)


def _r_taylor(r, terms=120):
    # R(r) = (1/t) sum_j binom(-1/2, j) (r / 2t)^(2j) (-eta(2j + 1)), r < 2t
    acc = 0.0
    for j in range(terms):
        eta = math.log(2.0) if j == 0 else (1.0 - 2.0 ** (-2 * j)) * special.zeta(2 * j + 1)
        acc += special.binom(-0.5, j) * (r / (2 * T)) ** (2 * j) * (-eta)
    return acc / T


@pytest.mark.parametrize("n,a,b", [(64, 0, 0), (64, 1, 0), (32, 1, 1), (256, 3, 2)])
def test_near_cells_vs_independent_quadrature(n, a, b):
    # K(a,b) 2 pi k h^2 = closed-form integral of 1/r over the cell + adaptive quadrature of
    # the Taylor series of R (independent of the oracle's Gauss-Legendre / image-series route)
    h = 10e-3 / n
    got = float(K.cell_kernel(a, b, h, h, T, KC)[0]) * 2 * math.pi * KC * h * h
    sing = float(K.cell_integral_inv_r(a * h, b * h, h, h))
    rem, _ = integrate.dblquad(lambda y, x: _r_taylor(math.hypot(x, y)), a * h - h / 2, a * h + h / 2,
                               b * h - h / 2, b * h + h / 2, epsabs=1e-16, epsrel=1e-13)
    assert got == pytest.approx(sing + rem, rel=1e-11)


def test_origin_cell_split():
    # K(0,0) 2 pi k = cell average of 1/r, 2 ln(1 + sqrt 2) * 4 / (4 h) ... plus R(0) + O(h^2)
    n = 64
    h = 10e-3 / n
    k00 = float(K.cell_kernel(0, 0, h, h, T, KC)[0])
    singular = 2.0 * math.log(1.0 + math.sqrt(2.0)) / (math.pi * KC * h)
    rem = (k00 - singular) * 2 * math.pi * KC
    c1 = 0.75 * special.zeta(3) / (8.0 * T ** 3)  # R(r) = R(0) + c1 r^2 + O(r^4)
    assert rem == pytest.approx(-math.log(2.0) / T + c1 * h * h / 6.0, rel=5e-5)


def test_near_and_far_routes_agree_on_the_boundary():
    # the near route (images) and far route (modes) must agree where both are valid
    n = 64
    h = 10e-3 / n
    a = np.arange(4, 12)
    near_like = []
    for ai in a:
        x0 = ai * h
        xi, wi = np.polynomial.legendre.leggauss(16)
        xs = x0 + 0.5 * h * xi[:, None]
        ys = 0.5 * h * xi[None, :]
        r = np.hypot(xs, ys)
        w2 = 0.25 * wi[:, None] * wi[None, :]
        near_like.append((np.sum(w2 * (1.0 / r + K.image_remainder(r, T))),
                          np.sum(w2 * K.modal_sum(r, T))))
    for im, md in near_like:
        assert md == pytest.approx(im, rel=1e-12)


@pytest.mark.parametrize("nx,ny,lx,ly", [(16, 16, 10e-3, 10e-3), (64, 64, 10e-3, 10e-3),
                                         (8, 16, 2e-3, 3e-3), (32, 8, 1e-3, 1e-3)])
def test_sum_rule(nx, ny, lx, ly):
    # Poisson summation: the cell average kills every non-zero reciprocal-lattice term, so
    # sum over Z^2 of K = f_hat(0) / (hx hy) = t / (k hx hy)  (uniform power gives q t / k)
    tab = K.periodized_table(nx, ny, lx, ly, T, KC)
    wx = np.full(nx + 1, 2.0); wx[0] = wx[-1] = 1.0
    wy = np.full(ny + 1, 2.0); wy[0] = wy[-1] = 1.0
    total = float(np.sum(wy[:, None] * wx[None, :] * tab))
    hx, hy = lx / nx, ly / ny
    assert total == pytest.approx(T / (KC * hx * hy), rel=1e-12)


def test_symmetry_positivity_decay():
    n = 64
    h = 10e-3 / n
    tab = K.periodized_table(n, n, 10e-3, 10e-3, T, KC)
    assert np.allclose(tab, tab.T, rtol=1e-13, atol=0)
    assert np.all(tab > 0)
    assert np.all(np.diff(tab[0, :n // 2]) < 0)
    # nearly radial: K(5,0) and K(3,4) sit at the same distance; the cell average differs at O((h/r)^2)
    k50 = float(K.cell_kernel(5, 0, h, h, T, KC)[0])
    k34 = float(K.cell_kernel(3, 4, h, h, T, KC)[0])
    assert abs(k50 / k34 - 1.0) < 5e-4
    # scaling: K k h depends only on (a, b, t/h)
    k_a = K.cell_kernel(np.arange(6), 2, h, h, T, KC)
    k_b = K.cell_kernel(np.arange(6), 2, 2 * h, 2 * h, 2 * T, 2 * KC)
    assert np.allclose(k_a * KC * h, k_b * 2 * KC * 2 * h, rtol=1e-12)


def test_half_space_limit():
    # a very thick die: R -> -ln 2 / t -> 0, K -> cell average of 1/(2 pi k r)
    h = 1e-4
    t_big = 1e3
    a = np.arange(0, 6)
    got = K.cell_kernel(a, 1, h, h, t_big, KC)
    inv_r = np.array([float(K.cell_integral_inv_r(ai * h, h, h, h)) for ai in a]) / (h * h)
    # what is left over is the image remainder, R = -ln 2 / t + O(r^2 / t^3)
    assert np.allclose(got * 2 * math.pi * KC - inv_r, -math.log(2.0) / t_big, rtol=1e-6)
    assert np.allclose(got * 2 * math.pi * KC, inv_r, rtol=1e-6)
    # far field of the cell average of 1/r: 1/r + (hx^2 + hy^2) ... = 1/r + h^2 / (24 r^3) + O(h^4 / r^5)
    for big in (20, 40, 80):
        avg = float(K.cell_integral_inv_r(big * h, 0.0, h, h)) / (h * h)
        r = big * h
        assert abs(avg - (1.0 / r + h * h / (24 * r ** 3))) < (h / r) ** 4 / r
