"""Transient temperature solve -- oracle (test infrastructure only).

Definition followed:
  * Eq. Ttran: T = f_sp (*) P - C f_sp (*) dT/dt makes every spatial Fourier (here: cosine)
    mode of the die a single pole: with P constant from t = 0 the mode's rise is
    F(T_ss) (1 - exp(-t / tau))  (Eq. tranGreen with the alpha C g term dropped as the paper
    does).  In the discrete, mirrored setting the steady response of mode (p, q) is the
    eigenvalue lambda[p, q] of the Green's operator, so the step response of that mode is
        S_hat[p, q](t) = lambda[p, q] (1 - exp(-t / tau[p, q])).
  * tau: the paper leaves C undetermined.  Default ("moment"): tau(s) is the exact first moment
    of the slab's multi-exponential response to a heat-flux step at lateral wavenumber s,
        tau(s) = (1 - x / sinh x) / (2 alpha s^2),  x = 2 s t_d,  alpha = k_ref / (rho c),
    with tau(0) = t_d^2 / (3 alpha).  Option "lumped": the paper's tau = C F(f_sp0) with
    C = rho c t_d / 3 per unit area, i.e. tau = (rho c t_d / 3) hx hy lambda[p, q] (it equals the
    moment value for the uniform mode).  s for mode (p, q) is pi sqrt((p/Lx)^2 + (q/Ly)^2).
  * Eq. tranapprox: a power map held over (t_{n-1}, t_n] enters through the step kernels,
        theta_n = sum_{j=1..n} S_j (*) (P_{n-j+1} - P_{n-j}),   P_0 = 0,
    with S_j the real-space kernel whose cosine eigenvalues are S_hat(j dt) and (*) the same
    mirror-image direct sum as the steady oracle.  By default the whole history is kept.
  * Truncated history (Sec. IV-E, the paper's 5 ms horizon): with horizon h the step kernels
    are taken as saturated from the h-th on (S_j = S_inf, the steady kernel, for j >= h), so the
    differences older than h - 1 steps telescope into one term,
        theta_n = sum_{j=1..min(n, h-1)} S_j (*) (P_{n-j+1} - P_{n-j}) + [n >= h] S_inf (*) P_{n-h+1}.
    The paper's printed collapse pairs S_inf with P(t_{n-5}) for its five kernels; the pattern of
    the sum (S_j multiplies the difference that ends at t_{n-j+1}) puts the saturated kernel on
    P_{n-h+1}, which is the reading taken here.
  * Leakage and k(T) (Sec. IV-E: "substitute the leakage-aware Green's function"): step n uses
    the previous step's rise, P_n = hx hy [q_dyn(t_n) + q_leak0 v L(dT_{n-1})], and
    dT_n = Phi^-1(theta_n) pointwise; the conductivity map enters as in the steady oracle, on the
    source side (P_n / m enters the superposition, the default) or on the target side
    (theta_n / m).

Multi-pole ("modal") option: each cosine mode responds with the slab's slowest depth modes
exactly and the rest lumped into one pole that keeps the first moment (``slab_poles``); one pole
is the moment model.

The step kernels come from lambda (an (N+1)-point cosine transform of the periodised steady
kernel) by the inverse transform; the superposition itself is a plain direct sum.

Parity: pinned -- the superposition against an independent single-pole recursion, the long-time
limit against the steady operator, uniform power against q t / k (1 - exp(-t / tau(0))), and
tau(s) against a numerically summed modal first moment.  The single-pole model itself (how well
one pole per mode approximates the slab) is the paper's reading: parity unpinned against the
full heat equation.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from . import steady as S


def slab_poles(s: np.ndarray, t: float, alpha: float, n_poles: int):
    """Weights w_j and time constants tau_j of the multi-pole ("modal") transient model.

    The slab's surface response to a flux step at lateral wavenumber s is exactly the sum over
    its depth modes cos(beta_m z), beta_m = (m + 1/2) pi / t (adiabatic top, isothermal bottom),
    of c_m (1 - exp(-t / tau_m)) with tau_m = 1 / (alpha (s^2 + beta_m^2)) and
    c_m = 2 / (k t (s^2 + beta_m^2)); the c_m sum to the steady symbol tanh(s t) / (k s).  The
    model keeps the slowest n_poles - 1 depth modes as they are (normalised weights
    w_m = c_m k s / tanh(s t)) and lumps the rest into one pole with the remaining weight and
    the time constant that keeps the total first moment equal to tau_moment(s): the steady
    value and the first moment are exact, and n_poles = 1 is the moment model.
    Returns (w, tau), arrays of shape (n_poles,) + s.shape."""
    s = np.asarray(s, dtype=np.float64)
    x = s * t
    with np.errstate(invalid="ignore", divide="ignore"):
        x_over_tanh = np.where(x < 1e-8, 1.0, x / np.tanh(np.where(x < 1e-8, 1.0, x)))
    w, tau = [], []
    for m in range(n_poles - 1):
        bt = (m + 0.5) * math.pi  # beta_m t
        w.append(2.0 * x_over_tanh / (x * x + bt * bt))
        tau.append(t * t / (alpha * (x * x + bt * bt)))
    w_rest = 1.0 - sum(w) if w else np.ones_like(s)
    first = tau_moment(s, t, alpha) - sum(wi * ti for wi, ti in zip(w, tau)) if w else tau_moment(s, t, alpha)
    w.append(w_rest)
    tau.append(first / w_rest)
    return np.array(w), np.array(tau)


def tau_moment(s: np.ndarray, t: float, alpha: float) -> np.ndarray:
    """First moment of the slab's step response at lateral wavenumber s (closed form)."""
    s = np.asarray(s, dtype=np.float64)
    x = 2.0 * s * t
    out = np.empty_like(s)
    small = x < 1e-3
    xs = x[small]
    # 1 - x / sinh x = x^2/6 - 7 x^4/360 + 31 x^6/15120 - ...
    out[small] = t * t / (3.0 * alpha) * (1.0 - 7.0 * xs * xs / 60.0 + 31.0 * xs ** 4 / 2520.0)
    xl = x[~small]
    sl = s[~small]
    out[~small] = (1.0 - xl / np.sinh(xl)) / (2.0 * alpha * sl * sl)
    return out


class TransientModel:
    """Transient model of one die: one pole per cosine mode (Eqs. Ttran, tranGreen; "moment" or
    "lumped" time constants), or the slab's slowest depth modes plus one lumped pole per cosine
    mode ("modal", n_poles poles; see ``slab_poles``)."""

    def __init__(self, geom: S.Geometry, rho_c: float, tau_model: str = "moment",
                 operator: S.DirectSum | None = None, n_poles: int = 1):
        self.geom = geom
        self.op = operator or S.DirectSum(geom)
        g = geom
        # lambda over p, q in [0, N] from the periodised kernel (cosine transform, type I)
        self.lam_full = sfft.dct(sfft.dct(self.op.table, type=1, axis=0), type=1, axis=1)
        self.alpha = g.k_ref / rho_c
        pp = np.arange(g.ny + 1)[:, None]
        qq = np.arange(g.nx + 1)[None, :]
        s = math.pi * np.sqrt((pp / g.ly) ** 2 + (qq / g.lx) ** 2)
        if tau_model == "moment":
            self.tau = tau_moment(s, g.t, self.alpha)
        elif tau_model == "lumped":
            self.tau = rho_c * g.t / 3.0 * g.hx * g.hy * self.lam_full
        elif tau_model == "modal":
            self.tau = tau_moment(s, g.t, self.alpha)  # the first moment of every mode's response
        else:
            raise ValueError(tau_model)
        # poles of every mode: weights [n_poles][N+1][N+1] and time constants
        if tau_model == "modal":
            self.weights, self.taus = slab_poles(s, g.t, self.alpha, n_poles)
        else:
            self.weights, self.taus = np.ones((1,) + s.shape), self.tau[None]
        self.rho_c = rho_c

    def step_kernel(self, time: float) -> np.ndarray:
        """Real-space periodised kernel whose cosine eigenvalues are
        lambda sum_j w_j (1 - exp(-time / tau_j))."""
        shat = self.lam_full * np.sum(self.weights * -np.expm1(-time / self.taus), axis=0)
        return sfft.idct(sfft.idct(shat, type=1, axis=0), type=1, axis=1)


def solve_transient(model: TransientModel, q_dyn_steps: np.ndarray, dt: float, q_leak: np.ndarray | None = None,
                    cond_map: np.ndarray | None = None, leak: str = "exp", beta: float = 0.017,
                    record_every: int = 1, cond: str = "source", horizon: int | None = None):
    """Superposition of step responses (Eq. tranapprox) with the one-step-lagged leakage loop.

    q_dyn_steps: [n_steps][ny][nx] dynamic power density held over each step.  horizon None keeps
    the whole history; horizon h >= 2 saturates the step kernels from the h-th on (the paper's
    truncated history).  Returns the rises dT_n for n = record_every, 2 record_every, ... (array
    [n_rec][ny][nx]) and the final rise.
    """
    g = model.geom
    n_steps = q_dyn_steps.shape[0]
    if horizon is not None and horizon < 2:
        raise ValueError("horizon must be at least 2")
    n_kern = n_steps if horizon is None else min(n_steps, horizon - 1)
    kernels = [S.DirectSum(g, table=model.step_kernel((j + 1) * dt)) for j in range(n_kern)]
    dT = np.zeros((g.ny, g.nx))
    p_hist = []  # P_1 .. P_n in W per cell
    out = []
    for n in range(1, n_steps + 1):
        q = q_dyn_steps[n - 1]
        if q_leak is not None and leak != "none":
            lf = np.exp(beta * dT) if leak == "exp" else 1.0 + beta * dT
            q = q + q_leak * lf
        if cond not in ("source", "target"):
            raise ValueError(cond)
        p_new = g.hx * g.hy * q
        if cond_map is not None and cond == "source":
            p_new = p_new / cond_map
        p_hist.append(p_new)
        theta = np.zeros((g.ny, g.nx))
        last = n if horizon is None else min(n, horizon - 1)
        for j in range(1, last + 1):  # S_j applied to P_{n-j+1} - P_{n-j}
            newer = p_hist[n - j]
            older = p_hist[n - j - 1] if n - j - 1 >= 0 else 0.0
            theta += kernels[j - 1].apply(newer - older)
        if horizon is not None and n >= horizon:  # the saturated kernel on P_{n-h+1}
            theta += model.op.apply(p_hist[n - horizon])
        if cond_map is not None and cond == "target":
            theta = theta / cond_map
        dT, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
        if n % record_every == 0:
            out.append(dT.copy())
    return np.array(out), dT
