"""Pins of the oracle's Anderson(1)-accelerated fixed point: the exact secant landing on the
uniform closed form, and the same fixed point as the Picard loop."""
import numpy as np
import pytest

import workloads as W
from oracle import anderson as A
from oracle import steady as S

MM2 = 1.0e6


@pytest.mark.parametrize("eta", [0.0])
def test_uniform_linear_problem_lands_on_closed_form_at_second_mixing(eta):
    # every iterate is uniform and G is affine on that line: x_2 is the fixed point, and the
    # third application of G finds a zero residual
    n, qd, ql, beta = 16, 1.0 * MM2, 0.4 * MM2, 0.0275
    g = S.Geometry(10e-3, 10e-3, n, n, 0.5e-3, 150.0, eta, 318.0)
    prob = S.SteadyProblem(g, np.full((n, n), qd), np.full((n, n), ql))
    opts = S.Options(leak="linear", beta=beta, max_iter=20, tol=1e-9)
    dT, st = A.solve_steady_anderson(prob, opts)
    R = 0.5e-3 / 150.0
    exact = R * (qd + ql) / (1.0 - beta * R * ql)
    assert st.status == S.Status.OK and st.iterations == 3
    assert np.max(np.abs(dT - exact)) <= 1e-12 * exact
    # Picard needs many more applications for the same tolerance
    _, sp = S.solve_steady(prob, opts, residual=False)
    assert sp.iterations > st.iterations


@pytest.mark.parametrize("sample", [0, 3])
def test_same_fixed_point_as_picard(sample):
    inp = W.config2(sample=sample, n=32)
    prob, opts = S.problem_from_inputs(inp)
    opts.tol, opts.max_iter = 1e-11, 100
    ref, sp = S.solve_steady(prob, opts, residual=False)
    dT, sa = A.solve_steady_anderson(prob, opts)
    assert sp.status == sa.status == S.Status.OK
    assert np.max(np.abs(dT - ref)) <= 1e-9
    assert sa.iterations < sp.iterations
