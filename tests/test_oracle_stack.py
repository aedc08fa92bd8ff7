"""Pins of the oracle's layered-package Green's function (Table param's stack; Sec. II-B's
f_sp = f_silic + const) with an isothermal or convective bottom."""
import numpy as np
import pytest

from oracle import fd
from oracle import kernel as K
from oracle import stack as ST
from oracle import steady as S

PKG = [(0.15e-3, 130.0), (0.02e-3, 4.0), (3.5e-3, 400.0)]  # Si, TIM, spreader (Table param)


def _powers(n, seed):
    return np.random.default_rng(seed).uniform(0.1e6, 2e6, (n, n))


def test_two_equal_layers_are_one_slab():
    # the impedance recursion and the cosine series against the image series of one slab
    for nx, ny, lx, ly in ((8, 8, 4e-3, 4e-3), (16, 8, 10e-3, 5e-3)):
        t = ST.periodized_stack_table(nx, ny, lx, ly, [(0.2e-3, 150.0), (0.3e-3, 150.0)], None)
        ref = K.periodized_table(nx, ny, lx, ly, 0.5e-3, 150.0)
        assert np.max(np.abs(t - ref)) <= 1e-13 * np.max(ref)


@pytest.mark.parametrize("h", [None, 2e4, 5e3])
def test_uniform_power_is_the_series_resistance(h):
    n, lx = 8, 4e-3
    g = S.Geometry(lx, lx, n, n, PKG[0][0], PKG[0][1], 0.0, 318.0)
    op = S.DirectSum(g, table=ST.periodized_stack_table(n, n, lx, lx, PKG, h))
    theta = op.apply(np.full((n, n), g.hx * g.hy * 1e6))
    want = 1e6 * (sum(t / k for t, k in PKG) + (0.0 if h is None else 1.0 / h))
    assert np.max(np.abs(theta - want)) <= 1e-12 * want


def test_infinite_convection_is_the_isothermal_stack():
    a = ST.periodized_stack_table(8, 8, 4e-3, 4e-3, PKG, 1e15)
    b = ST.periodized_stack_table(8, 8, 4e-3, 4e-3, PKG, None)
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(b)


def test_one_layer_stack_solver_is_the_slab_solver():
    q = _powers(6, 1)
    a = fd.solve_modes_stack(q, 3e-3, 3e-3, [(0.5e-3, 150.0)], None, 3, [6])
    b = fd.solve_modes(q, 3e-3, 3e-3, 0.5e-3, 150.0, 3, 6)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(b)


@pytest.mark.parametrize("h", [None, 2e4])
def test_stack_operator_against_finite_volume(h):
    # the whole layered operator against a finite-volume solve of the layered box (Richardson,
    # two levels): agreement to the finite-volume solve's own error
    n, lx = 8, 4e-3
    q = _powers(n, 5)
    g = S.Geometry(lx, lx, n, n, PKG[0][0], PKG[0][1], 0.0, 318.0)
    op = S.DirectSum(g, table=ST.periodized_stack_table(n, n, lx, lx, PKG, h))
    theta = op.apply(g.hx * g.hy * q)
    ref = fd.richardson_stack(q, lx, lx, PKG, h, r0=3, nz0=(4, 2, 4), levels=2)
    assert np.max(np.abs(theta - ref)) <= 2e-5 * np.max(ref)
