"""Pins of the oracle's one-shot modified Green's functions (Sec. IV-C: Eqs. detsol, randsol,
detrandsol) against closed forms, the converged fixed point of the steady oracle, the error
order of the random part, and a dense linear solve."""
import numpy as np
import pytest

import workloads as W
from oracle import oneshot as O
from oracle import steady as S

T = 0.5e-3
KC = 150.0
MM2 = 1.0e6


def _prob(q_dyn, q_leak, m=None, eta=0.0, n=None, lx=10e-3):
    ny, nx = q_dyn.shape
    g = S.Geometry(lx, lx * ny / nx, nx, ny, T, KC, eta, 318.0)
    return S.SteadyProblem(g, q_dyn, q_leak, None, m)


def _loop(prob, beta, leak="linear", tol=1e-14):
    opts = S.Options(leak=leak, beta=beta, max_iter=200, tol=tol)
    dT, st = S.solve_steady(prob, opts, residual=False)
    assert st.status == S.Status.OK
    return dT


@pytest.mark.parametrize("eta", [0.0, 1.3])
@pytest.mark.parametrize("random_part", [False, True])
def test_uniform_leakage_closed_form(eta, random_part):
    # uniform q_d and q_l, linear leakage: theta = R (q_d + q_l) / (1 - beta R q_l), R = t / k_ref
    n, qd, ql, beta = 16, 1.0 * MM2, 0.2 * MM2, 0.0275
    prob = _prob(np.full((n, n), qd), np.full((n, n), ql), eta=eta)
    dT, th_det, th_rand = O.oneshot(prob, beta, mu=ql, random_part=random_part)
    R = T / prob.geom.k_ref
    theta = R * (qd + ql) / (1.0 - beta * R * ql)
    assert np.max(np.abs(th_det - theta)) <= 1e-12 * theta
    assert np.max(np.abs(th_rand)) <= 1e-13 * theta  # no variation: no random part
    if eta == 0.0:
        ref = theta
    else:  # Phi^-1 of k = k_ref (T / T_amb)^-eta, by quadrature-free closed form of the integral
        a = 1.0 - eta
        ref = 318.0 * ((1.0 + a * theta / 318.0) ** (1.0 / a) - 1.0)
    assert np.max(np.abs(dT - ref)) <= 1e-12 * ref


@pytest.mark.parametrize("m_const", [None, 1.04])
def test_detsol_is_the_fixed_point_for_uniform_leakage(m_const):
    # Eq. detsol at alpha = 0: with a uniform leakage density (per unit conductivity) the
    # deterministic Green's function alone reaches the converged loop, for any dynamic map
    inp = W.steady_problem(2, 16, 8, floorplan=1, variation=False)
    n = inp.n
    ql = np.full((n, n), 0.3 * MM2)
    m = None if m_const is None else np.full((n, n), m_const)
    prob = _prob(inp.q_dyn, ql, m=m)
    mu = 0.3 * MM2 / (1.0 if m_const is None else m_const)
    beta = 0.0275
    dT, _, th_rand = O.oneshot(prob, beta, mu=mu)
    ref = _loop(prob, beta)
    assert np.max(np.abs(dT - ref)) <= 1e-11 * np.max(ref)
    assert np.max(np.abs(th_rand)) <= 1e-13 * np.max(ref)


def _varied(eps, n=16):
    """Block floorplan with leakage q_l = mu0 (1 + eps w), w a fixed zero-mean smooth pattern."""
    inp = W.steady_problem(2, n, 8, floorplan=2, variation=False)
    rng = np.random.default_rng(11)
    w = W.gaussian_field(n, 10e-3 / n, 2e-3, rng)
    w = (w - w.mean()) / np.max(np.abs(w - w.mean()))
    mu0 = 0.5 * MM2
    return _prob(inp.q_dyn, mu0 * (1.0 + eps * w)), mu0


def test_random_part_makes_the_error_second_order():
    beta = 0.05
    err_det, err_full = [], []
    for eps in (0.4, 0.2, 0.1):
        prob, mu = _varied(eps)
        ref = _loop(prob, beta)
        d_det, _, _ = O.oneshot(prob, beta, mu, random_part=False)
        d_full, _, _ = O.oneshot(prob, beta, mu, random_part=True)
        err_det.append(np.max(np.abs(d_det - ref)))
        err_full.append(np.max(np.abs(d_full - ref)))
    # deterministic part only (the paper's "ignoring f_rand"): first order in the variation
    for a, b in zip(err_det, err_det[1:]):
        assert 1.8 < a / b < 2.3, err_det
    # with the random part: second order
    for a, b in zip(err_full, err_full[1:]):
        assert 3.5 < a / b < 4.6, err_full
    assert all(f < 0.2 * d for f, d in zip(err_full, err_det))


@pytest.mark.parametrize("nx,ny", [(6, 6), (6, 4)])
def test_neumann_solve_equals_dense_lu(nx, ny):
    rng = np.random.default_rng(nx * 7 + ny)
    qd = rng.uniform(0.1, 2.0, (ny, nx)) * MM2
    ql = rng.uniform(0.1, 0.6, (ny, nx)) * MM2
    m = rng.uniform(0.95, 1.05, (ny, nx))
    prob = _prob(qd, ql, m=m, lx=2e-3)
    beta, mu = 0.04, float(np.mean(ql / m))
    _, th_det, _ = O.oneshot(prob, beta, mu, random_part=False)
    ref = O.dense_det_solve(prob, beta, mu)
    assert np.max(np.abs(th_det - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_ignoring_the_random_part_costs_accuracy_on_high_variance_maps():
    # the paper's high-variance ablation: the workload's exp leakage, Vth variation of twice the
    # usual spread, conductivity map and k(T); one-shot against the converged loop
    n = 32
    inp = W.steady_problem(2, n, 64, floorplan=3, sample=0, variation=True)
    inp.leak_var = inp.leak_var ** 2.0  # twice the log-spread
    prob, opts = S.problem_from_inputs(inp)
    opts.tol, opts.max_iter = 1e-12, 100
    ref, st = S.solve_steady(prob, opts, residual=False)
    assert st.status == S.Status.OK
    mu = float(np.mean(prob.q_leak / prob.m))
    d_det, _, _ = O.oneshot(prob, inp.beta, mu, random_part=False)
    d_full, _, _ = O.oneshot(prob, inp.beta, mu, random_part=True)
    e_det, e_full = np.max(np.abs(d_det - ref)), np.max(np.abs(d_full - ref))
    assert e_full < 0.5 * e_det, (e_full, e_det)
