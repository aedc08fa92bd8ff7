"""One-shot leakage-aware modified Green's functions (Sec. IV-C) -- oracle (test infrastructure only).

The paper avoids iterating: it linearises leakage (Eq. Pt, P = P_dyn + P_leak0 (1 + beta dT)),
splits the baseline leakage into its mean mu and a varying part P_var (Eq. expanded2), solves
the mean part exactly in the spectral domain (Eqs. expanded3 and detsol, the deterministic
Green's function F(f_det) = F(f) / (1 - mu beta F(f)) when the conductivity term alpha is
zero) and adds a random part driven by P_var (Eqs. randTsplit, randsol), combined in
Eq. detrandsol.  Its derivation mixes spatial and spectral quantities (Lemma I; Q_rand of
Eq. randTsplit), so it is read here in the one form that is well posed on the discrete,
mirrored grid:

  linearised problem (source-side conductivity map m, Kirchhoff variable theta):
      theta = K (*) [ g + beta hx hy (q_leak / m) theta ],   g = hx hy (q_dyn + q_leak) / m,
  with q_leak = q_leak0 v and K (*) the images-folded direct sum of the steady oracle.  Write
  q_leak / m = mu + r with a scalar mu (the leakage density the deterministic part treats as
  uniform) and the remainder r (the variation map, Eq. expanded2's P_var, per unit power).

  deterministic part (Eq. detsol, alpha = 0):
      (I - beta hx hy mu K) theta_det = K (*) g
  -- in the cosine basis the paper's division lambda / (1 - beta hx hy mu lambda);
  random part (Eq. randsol at first order in r: the feedback of the variation through the
  deterministic operator, evaluated on theta_det):
      (I - beta hx hy mu K) theta_rand = K (*) (beta hx hy r theta_det)
  total (Eq. detrandsol): theta = theta_det + theta_rand (theta_rand omitted: the paper's
  "ignoring f_rand" ablation of Sec. V-C), and dT = Phi^-1(theta), the Kirchhoff inverse of k(T)
  in place of the paper's empirical alpha (Eqs. fspvsk, fspvsT).

Both linear equations are solved by their own Neumann iteration to machine precision (the
contraction factor is beta mu t / k_ref, about 1e-2 for the workloads); ``dense_det_solve``
solves the first one with a dense matrix on tiny grids as a cross-check.

Parity: pinned -- for a uniform leakage map, linear leakage and constant k the deterministic
part alone is the exact fixed point (Eq. detsol at alpha = 0), checked against the linear
uniform closed form R (q_d + q_l) / (1 - beta R q_l) and against the steady oracle's converged
loop; the random part makes the one-shot error second order in the variation amplitude
(halving the variation quarters the error; without it the error halves), checked against the
converged loop; the Neumann solve equals a dense LU solve on an 8 x 8 grid.
"""
from __future__ import annotations

import numpy as np

from . import steady as S


def _neumann(op: S.DirectSum, rhs_conv: np.ndarray, c: float, rel_tol: float = 1e-16, max_terms: int = 200):
    """Solve (I - c K) theta = rhs_conv (rhs_conv = K (*) source, already applied) by theta_{j+1} =
    rhs_conv + c K (*) theta_j from theta_0 = rhs_conv, to a relative increment below rel_tol."""
    theta = rhs_conv.copy()
    scale = float(np.max(np.abs(rhs_conv))) or 1.0
    for _ in range(max_terms):
        new = rhs_conv + c * op.apply(theta)
        inc = float(np.max(np.abs(new - theta)))
        theta = new
        if inc <= rel_tol * scale:
            return theta
    raise RuntimeError("Neumann series did not converge: beta mu t / k >= 1 (no linearised fixed point)")


def _split(prob: S.SteadyProblem, mu: float):
    """(g, r): the source map hx hy (q_dyn + q_leak) / m and the remainder q_leak / m - mu."""
    hxhy = prob.geom.hx * prob.geom.hy
    q_leak = prob.q_leak if prob.q_leak is not None else np.zeros_like(prob.q_dyn)
    minv = 1.0 / prob.m if prob.m is not None else np.ones_like(prob.q_dyn)
    g = hxhy * (prob.q_dyn + q_leak) * minv
    r = q_leak * minv - mu
    return g, r


def oneshot(prob: S.SteadyProblem, beta: float, mu: float, random_part: bool = True):
    """One-shot rise dT = Phi^-1(theta_det [+ theta_rand]); returns (dT, theta_det, theta_rand).

    beta: the leakage coefficient of the linearised law (0 for no leakage); mu: leakage density
    (W/m^2) treated as uniform by the deterministic part."""
    geom = prob.geom
    c = beta * geom.hx * geom.hy * mu
    g, r = _split(prob, mu)
    theta_det = _neumann(prob.op, prob.op.apply(g), c)
    theta_rand = np.zeros_like(theta_det)
    if random_part and beta != 0.0:
        src = beta * geom.hx * geom.hy * r * theta_det
        theta_rand = _neumann(prob.op, prob.op.apply(src), c)
    dT, ok = S.kirchhoff_inverse(theta_det + theta_rand, geom.t_amb, geom.eta)
    if not np.all(ok):
        raise FloatingPointError("Kirchhoff base non-positive: the one-shot rise is outside k(T)'s domain")
    return dT, theta_det, theta_rand


def dense_det_solve(prob: S.SteadyProblem, beta: float, mu: float) -> np.ndarray:
    """theta_det by a dense LU solve of (I - c K) theta = K g, K assembled column by column from
    the literal quadruple-loop direct sum (tiny grids only)."""
    geom = prob.geom
    ny, nx = geom.ny, geom.nx
    n = nx * ny
    kmat = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        kmat[:, j] = S.direct_sum_literal(prob.op.table, e.reshape(ny, nx)).ravel()
    g, _ = _split(prob, mu)
    c = beta * geom.hx * geom.hy * mu
    return np.linalg.solve(np.eye(n) - c * kmat, kmat @ g.ravel()).reshape(ny, nx)
