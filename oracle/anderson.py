"""Anderson-accelerated fixed point (depth 1) of the steady map G -- oracle (test infrastructure only).

Not from the paper: a classical acceleration of the same fixed point dT = G(dT) (the steady
oracle's map, Sec. V-C's iterate-to-convergence ground truth), used as a non-learned baseline
for the learned warm start.  Anderson mixing with one stored difference (Anderson 1965; the
"type II" form of Walker and Ni 2011):

    g_k = G(x_k),  f_k = g_k - x_k                    (residual of iterate k)
    x_1 = g_0                                         (a plain Picard step)
    gamma_k = <f_k - f_{k-1}, f_k> / <f_k - f_{k-1}, f_k - f_{k-1}>   (k >= 1; 0 if the
              denominator vanishes)
    x_{k+1} = g_k - gamma_k (g_k - g_{k-1})

with <., .> the plain sum over all cells.  Stopping rule as in the Picard oracle: after the k-th
application of G, stop when max |g - x| <= tol and return g = G(x) (so "iterations" counts
applications of G, as for Picard).

Parity: pinned -- on a uniform problem with linear leakage and constant k every iterate is
uniform and G is affine on that line, so the secant step lands on the closed-form fixed point
R (q_d + q_l) / (1 - beta R q_l) exactly at the second mixing; on variation maps it converges to
the Picard fixed point.
"""
from __future__ import annotations

import math

import numpy as np

from . import steady as S


def solve_steady_anderson(prob: S.SteadyProblem, opts: S.Options, init: np.ndarray | None = None):
    """Anderson(1) iteration of G to the first max |G(x) - x| <= tol; returns (dT, Stats)."""
    g = prob.geom
    x = np.zeros((g.ny, g.nx)) if init is None else np.array(init, dtype=np.float64)
    g_prev = f_prev = None
    incs = []
    for it in range(1, opts.max_iter + 1):
        gk, ok = prob.map(x, opts)
        if (not np.all(ok)) or (not np.all(np.isfinite(gk))) or float(np.max(gk)) > opts.dT_cap:
            return gk, S.Stats(S.Status.RUNAWAY, it, math.inf, math.inf, math.nan, math.nan, -1, incs)
        fk = gk - x
        inc = float(np.max(np.abs(fk)))
        incs.append(inc)
        if inc <= opts.tol:
            return gk, S.Stats(S.Status.OK, it, inc, math.nan, float(np.max(gk)), float(np.mean(gk)),
                               int(np.argmax(gk)), incs)
        if f_prev is None:
            x_new = gk
        else:
            df = fk - f_prev
            den = float(np.sum(df * df))
            gamma = float(np.sum(df * fk)) / den if den > 0.0 else 0.0
            x_new = gk - gamma * (gk - g_prev)
        g_prev, f_prev, x = gk, fk, x_new
    return gk, S.Stats(S.Status.NOT_CONVERGED, opts.max_iter, incs[-1], math.nan, float(np.max(gk)),
                       float(np.mean(gk)), int(np.argmax(gk)), incs)
