"""Pins of the transient oracle (Eqs. Ttran, tranGreen, tranapprox)."""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import workloads as W
from oracle import fd
from oracle import steady as S
from oracle import transient as T

TD, KC, RHOC = 0.5e-3, 150.0, 1.66e6


def _geom(n=16, l=10e-3, eta=0.0):
    return S.Geometry(l, l, n, n, TD, KC, eta, 318.0, RHOC)


@pytest.mark.parametrize("s", [0.0, 10.0, 1e3, 3e3, 1e4, 1e5])
def test_tau_is_first_moment_of_slab_modes(s):
    # slab modes cos(mu_m z), mu_m = (m + 1/2) pi / t: steady gain per mode (2/t) / (k (mu^2 + s^2)),
    # decay time 1 / (alpha (mu^2 + s^2)); the response's first moment is sum A tau / sum A
    alpha = KC / RHOC
    m = np.arange(200000)
    mu2 = ((m + 0.5) * math.pi / TD) ** 2 + s * s
    a = (2.0 / TD) / (KC * mu2)
    tau_m = 1.0 / (alpha * mu2)
    gain = a.sum()
    steady = TD / KC if s == 0 else math.tanh(s * TD) / (KC * s)
    assert gain == pytest.approx(steady, rel=1e-4)  # truncated sum, tail ~ 2 t s / (pi^2 M)
    # numerator terms fall off like m^-4 (truncation ~1e-16); divide by the exact steady gain
    moment = (a * tau_m).sum() / steady
    assert float(T.tau_moment(np.array([s]), TD, alpha)[0]) == pytest.approx(moment, rel=1e-9)


def test_long_time_kernel_is_steady_kernel():
    model = T.TransientModel(_geom(16), RHOC)
    k_inf = model.step_kernel(1.0)  # 1 s >> every tau
    assert np.allclose(k_inf, model.op.table, rtol=1e-12, atol=1e-15 * np.max(model.op.table))


def test_uniform_power_single_pole():
    g = _geom(16)
    model = T.TransientModel(g, RHOC)
    q = 1.0e6
    dt = 50e-6
    steps = np.full((12, 16, 16), q)
    rec, _ = T.solve_transient(model, steps, dt, leak="none")
    tau0 = TD * TD * RHOC / (3.0 * KC)
    for n in range(12):
        expect = q * TD / KC * (1.0 - math.exp(-(n + 1) * dt / tau0))
        assert np.allclose(rec[n], expect, rtol=1e-11)


def test_lumped_tau_matches_moment_at_dc():
    g = _geom(16)
    a = T.TransientModel(g, RHOC, "moment")
    b = T.TransientModel(g, RHOC, "lumped")
    assert b.tau[0, 0] == pytest.approx(a.tau[0, 0], rel=1e-12)
    assert np.all(b.tau[1:, 1:] < a.tau[1:, 1:] * 10)


@pytest.mark.parametrize("cond", ["source", "target"])
def test_superposition_equals_single_pole_recursion(cond):
    """Eq. tranapprox (full history, real-space step kernels, direct sums) against an independent
    per-mode recursion theta_hat_n = a theta_hat_{n-1} + b P_hat_n, with the lagged leakage, the
    conductivity map (either placement) and k(T)."""
    n, steps, dt = 16, 25, 20e-6
    g = _geom(n, eta=1.3)
    model = T.TransientModel(g, RHOC)
    tr = W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=6, hold_s=5 * dt)
    qd = np.stack([W.raster_trace_step(tr.block_rects, tr.trace[i], n) for i in range(steps)])
    ql = tr.q_leak0 * tr.leak_var
    rec, last = T.solve_transient(model, qd, dt, q_leak=ql, cond_map=tr.cond_map, cond=cond)
    lam = model.lam_full[:n, :n]
    tau = model.tau[:n, :n]
    a = np.exp(-dt / tau)
    b = -np.expm1(-dt / tau) * lam
    th_hat = np.zeros((n, n))
    dT = np.zeros((n, n))
    for i in range(steps):
        p = g.hx * g.hy * (qd[i] + ql * np.exp(0.017 * dT))
        if cond == "source":
            p = p / tr.cond_map
        th_hat = a * th_hat + b * sfft.dctn(p, type=2)
        theta = sfft.idctn(th_hat, type=2)
        if cond == "target":
            theta = theta / tr.cond_map
        dT, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
        assert np.allclose(rec[i], dT, rtol=1e-11, atol=1e-12 * np.max(np.abs(dT)))
    assert np.max(last) > 0.5


@pytest.mark.parametrize("cond", ["source", "target"])
def test_long_time_limit_with_conductivity_map_is_steady(cond):
    """Constant power held far longer than every tau reaches the steady fixed point of the same
    conductivity placement (no leakage, eta = 0: the steady map is linear)."""
    n, steps, dt = 8, 3, 0.05
    g = _geom(n)
    model = T.TransientModel(g, RHOC)
    rng = np.random.default_rng(4)
    q = rng.uniform(0.1e6, 2e6, (n, n))
    m = rng.uniform(0.95, 1.05, (n, n))
    _, last = T.solve_transient(model, np.stack([q] * steps), dt, cond_map=m, leak="none", cond=cond)
    steady, st = S.solve_steady(S.SteadyProblem(g, q, cond_map=m, operator=model.op),
                                S.Options(leak="none", cond=cond, tol=1e-14))
    assert st.status == S.Status.OK
    assert np.allclose(last, steady, rtol=1e-12)


# ----------------------------------------------------------------------------- multi-pole model
def test_modal_model_one_pole_is_the_moment_model():
    g = S.Geometry(4e-3, 4e-3, 8, 8, 0.5e-3, 150.0, 0.0, 318.0)
    a = T.TransientModel(g, 1.66e6, "moment")
    b = T.TransientModel(g, 1.66e6, "modal", n_poles=1)
    for tt in (1e-5, 1e-4, 1e-3):
        assert np.allclose(a.step_kernel(tt), b.step_kernel(tt), rtol=1e-14, atol=0)


@pytest.mark.parametrize("n_poles", [2, 4, 8])
def test_modal_weights_sum_to_one_and_keep_the_first_moment(n_poles):
    s = np.array([0.0, 1.0, 3e2, 1e3, 1e4, 1e5])
    t, alpha = 0.5e-3, 150.0 / 1.66e6
    w, tau = T.slab_poles(s, t, alpha, n_poles)
    assert np.allclose(w.sum(axis=0), 1.0, rtol=0, atol=1e-13)
    assert np.all(w > 0) and np.all(tau > 0)
    assert np.allclose((w * tau).sum(axis=0), T.tau_moment(s, t, alpha), rtol=1e-12)
    # the explicit poles are the slab's depth modes: tau_m = t^2 / (alpha ((s t)^2 + ((m + 1/2) pi)^2))
    for m in range(n_poles - 1):
        want = t * t / (alpha * ((s * t) ** 2 + ((m + 0.5) * math.pi) ** 2))
        assert np.allclose(tau[m], want, rtol=1e-14)


def test_transient_finite_volume_reaches_the_steady_solve():
    q = np.random.default_rng(2).uniform(0, 2e6, (6, 6))
    late = fd.transient_modes(q, 3e-3, 3e-3, 0.5e-3, 150.0, 1.66e6, 3, 12, [10.0])[0]
    steady = fd.solve_modes(q, 3e-3, 3e-3, 0.5e-3, 150.0, 3, 12)
    assert np.max(np.abs(late - steady)) <= 1e-10 * np.max(steady)


def test_pole_models_against_finite_volume_transient():
    # characterisation of the paper's single-pole reading (Eq. tranGreen) against the heat
    # equation: a 1 mm block on a 4 mm die, surface rise at 0.05 - 5 ms after switch-on, against
    # the finite-volume transient (exact in time, Richardson in space).  One pole per mode (the
    # moment model) misses the early sqrt(t) rise by ~14 % of the final max rise; the modal model
    # with 4 poles is within 2 %.
    n, lx, t, k, rc = 8, 4e-3, 0.5e-3, 150.0, 1.66e6
    q = np.zeros((n, n))
    q[3:5, 3:5] = 2e6
    times = np.array([0.05e-3, 0.2e-3, 1e-3, 5e-3])
    f3 = fd.transient_modes(q, lx, lx, t, k, rc, 3, 20, times)
    f9 = fd.transient_modes(q, lx, lx, t, k, rc, 9, 60, times)
    ref = f9 + (f9 - f3) / 8.0
    g = S.Geometry(lx, lx, n, n, t, k, 0.0, 318.0)
    err = {}
    for name, kw in (("moment", {"tau_model": "moment"}), ("modal4", {"tau_model": "modal", "n_poles": 4})):
        m = T.TransientModel(g, rc, **kw)
        out = np.array([S.DirectSum(g, table=m.step_kernel(tt)).apply(g.hx * g.hy * q) for tt in times])
        err[name] = float(np.max(np.abs(out - ref)) / np.max(ref[-1]))
    assert 0.10 < err["moment"] < 0.20, err
    assert err["modal4"] < 0.025, err


# ----------------------------------------------------------------------------- truncated history
def test_truncated_history_longer_than_the_run_is_the_full_history():
    n, steps, dt = 8, 9, 30e-6
    g = _geom(n)
    model = T.TransientModel(g, RHOC)
    q = np.random.default_rng(5).uniform(0.0, 2e6, (steps, n, n))
    full, _ = T.solve_transient(model, q, dt, leak="none")
    trunc, _ = T.solve_transient(model, q, dt, leak="none", horizon=steps + 1)
    assert np.array_equal(full, trunc)
    with pytest.raises(ValueError):
        T.solve_transient(model, q, dt, leak="none", horizon=1)


@pytest.mark.parametrize("horizon", [2, 3, 6])
def test_truncated_history_uniform_pulse_closed_form(horizon):
    """Uniform power on for m steps, then off: only the uniform mode responds, with step response
    R (1 - exp(-t / tau0)), saturated to R from the horizon on.  The rise at step n is
    q R (s(n) - s(n - m)) with s(j) = 1 - exp(-j dt / tau0) for 0 < j < h, 1 for j >= h, 0 for
    j <= 0 -- exactly zero once the switch-off is h steps old."""
    n, dt, on, steps = 8, 40e-6, 4, 14
    g = _geom(n)
    model = T.TransientModel(g, RHOC)
    q = 1.5e6
    trace = np.zeros((steps, n, n))
    trace[:on] = q
    rec, _ = T.solve_transient(model, trace, dt, leak="none", horizon=horizon)
    tau0 = TD * TD * RHOC / (3.0 * KC)

    def s(j):
        return 0.0 if j <= 0 else (1.0 if j >= horizon else 1.0 - math.exp(-j * dt / tau0))

    for i in range(steps):
        step = i + 1
        expect = q * TD / KC * (s(step) - s(step - on))
        assert np.allclose(rec[i], expect, rtol=1e-11, atol=1e-12 * q * TD / KC)
    assert np.all(rec[on + horizon - 1:] == pytest.approx(0.0, abs=1e-12 * q * TD / KC))


@pytest.mark.parametrize("n_poles,tau_model", [(1, "moment"), (3, "modal")])
def test_truncated_history_equals_its_recursive_form(n_poles, tau_model):
    """The truncated superposition (real-space step kernels, direct sums) against an independent
    per-mode recursion: with pole weights c_j = lambda w_j and a_j = exp(-dt / tau_j), the history
    cut at h obeys y_j,n = a_j y_j,n-1 + c_j (1 - a_j) (P_n - a_j^(h-1) P_(n-h+1)) and
    theta_n = sum_j (y_j,n + c_j a_j^(h-1) P_(n-h+1)) (the transform of P is zero before step 1),
    with the lagged leakage and a conductivity map."""
    n, steps, dt, h = 16, 20, 20e-6, 7
    g = _geom(n, eta=1.3)
    model = T.TransientModel(g, RHOC, tau_model, n_poles=n_poles)
    tr = W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=6, hold_s=3 * dt)
    qd = np.stack([W.raster_trace_step(tr.block_rects, tr.trace[i], n) for i in range(steps)])
    ql = tr.q_leak0 * tr.leak_var
    rec, _ = T.solve_transient(model, qd, dt, q_leak=ql, cond_map=tr.cond_map, horizon=h)
    c = model.lam_full[None, :n, :n] * model.weights[:, :n, :n]
    a = np.exp(-dt / model.taus[:, :n, :n])
    ah = a ** (h - 1)
    y = np.zeros((n_poles, n, n))
    hist = []
    dT = np.zeros((n, n))
    for i in range(steps):
        p = g.hx * g.hy * (qd[i] + ql * np.exp(0.017 * dT)) / tr.cond_map
        hist.append(sfft.dctn(p, type=2))
        old = hist[i - h + 1] if i - h + 1 >= 0 else 0.0
        y = a * y + c * (1.0 - a) * (hist[i] - ah * old)
        theta = sfft.idctn(np.sum(y + c * ah * old, axis=0), type=2)
        dT, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
        assert np.allclose(rec[i], dT, rtol=1e-10, atol=1e-11 * np.max(np.abs(dT)))


def test_truncated_history_against_full_history_and_finite_volume():
    # characterisation of the paper's 5 ms horizon (Sec. IV-E): a 2 ms power pulse on a 1 mm block
    # of a 4 mm die, 0.1 ms steps, against the finite-volume transient (switch-on response,
    # Richardson in space, superposed for the switch-off).  Cutting the history at 5 ms changes
    # the rise by under 0.2 % of its maximum, for one pole per mode and for four; a 1 ms cut
    # misses the cool-down by over 10 %.
    n, lx, t, k, rc = 8, 4e-3, 0.5e-3, 150.0, 1.66e6
    q = np.zeros((n, n))
    q[3:5, 3:5] = 2e6
    dt, steps, on = 0.1e-3, 60, 20
    trace = np.zeros((steps, n, n))
    trace[:on] = q
    samples = np.array([5, 10, 20, 30, 40, 60])
    times = samples * dt
    switch = np.unique(np.concatenate([times, times - on * dt]))
    switch = switch[switch > 0]
    f3 = fd.transient_modes(q, lx, lx, t, k, rc, 3, 20, switch)
    f9 = fd.transient_modes(q, lx, lx, t, k, rc, 9, 60, switch)
    rise = f9 + (f9 - f3) / 8.0

    def at(tt):
        return np.zeros((n, n)) if tt <= 1e-12 else rise[int(np.argmin(np.abs(switch - tt)))]

    ref = np.array([at(tt) - at(tt - on * dt) for tt in times])
    g = S.Geometry(lx, lx, n, n, t, k, 0.0, 318.0)
    for kw, model_err in (({"tau_model": "moment"}, 0.06), ({"tau_model": "modal", "n_poles": 4}, 0.02)):
        m = T.TransientModel(g, rc, **kw)
        full = T.solve_transient(m, trace, dt, leak="none")[0][samples - 1]
        cut5 = T.solve_transient(m, trace, dt, leak="none", horizon=50)[0][samples - 1]
        cut1 = T.solve_transient(m, trace, dt, leak="none", horizon=10)[0][samples - 1]
        peak = np.max(ref)
        assert np.max(np.abs(cut5 - full)) <= 2e-3 * peak, kw
        assert np.max(np.abs(full - ref)) <= model_err * peak, kw
        assert np.max(np.abs(cut1 - ref)) >= 0.10 * peak, kw
