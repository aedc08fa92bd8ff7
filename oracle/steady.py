"""Steady leakage- and conductivity-coupled temperature solve -- oracle (test infrastructure only).

Definition followed (one map G of the fixed point; the paper's ground truth of Sec. V-C
iterates exactly this: "update the leakage power and conductivity ... keep iterating until the
temperature values converge"):

  1. total power per cell (Eqs. Pt and Pleak, with the variation-scaled leakage of Eq. Ileakmod):
         P = hx hy [ q_dyn + q_leak0 * v * L(dT) ],   L = exp(beta dT)  or  1 + beta dT
  2. shift-invariant rise by the Green's function convolution (Eq. Green) with the die edges
     handled by mirror-image sources (Sec. IV-F), evaluated as a plain direct sum over all
     source cells and their images:
         theta_SI(i, j) = sum_{k, l} P(k, l) [K(i-k, j-l) + K(i+k+1, j-l) + K(i-k, j+l+1) + K(i+k+1, j+l+1)]
     with K the periodised cell kernel of ``oracle.kernel`` at k_ref = k(T_amb);
  3. conductivity variation map m (Sec. II-E): the Green's function scales as 1/k (Eq. fspvsk
     with c' = 1/k0'), applied as a Hadamard factor.  The paper does not say at which end of
     the source -> target path the local conductivity acts; two placements are offered:
         source (default):  theta = K (*) (P / m)    (each source's spreading uses its own k)
         target:            theta = (K (*) P) / m    (the target cell's k scales its rise)
     Both are exact for a uniform m.  Against a finite-volume solve of Eq. fourier with the
     conductivity k m(x, y) (``oracle.fd.solve_lateral_k``), the source placement's error is
     about a quarter of the target placement's (0.47 % vs 2.0 % of the max rise for a +-5 %
     map), so it is the default;
  4. temperature-dependent conductivity k = k0 (T/300)^-eta (Eq. condsi): theta is the Kirchhoff
     transform  Phi(dT) = int_{T_amb}^{T_amb + dT} k(T)/k_ref dT,  inverted in closed form
         dT' = T_amb [ (1 + (1 - eta) theta / T_amb)^(1/(1 - eta)) - 1 ]   (dT' = theta if eta = 0,
     T_amb (exp(theta / T_amb) - 1) if eta = 1).

Picard iteration from dT = 0 (or a given start): dT_{k+1} = G(dT_k), stop at the first k with
max |dT_{k+1} - dT_k| <= tol.  Status: NOT_CONVERGED after max_iter maps, RUNAWAY on a
non-finite iterate, dT above the cap, or a non-positive Kirchhoff base.

Parity: pinned -- the blocked direct sum against a literal quadruple loop, uniform power
against q t / k, linear and exponential leakage against their closed forms (Lambert W), the
leakage-aware spectral form of Eq. detsol at alpha = 0, Phi(Phi^-1) against quadrature of k(T)
(eta = 1.3 and eta = 1), and the whole operator against a finite-volume solve of Eq. fourier.
A non-uniform m is pinned only to the accuracy of the Hadamard model itself: the finite-volume
solve with k m(x, y) bounds the source placement's error and separates it from the target
placement's; the model error (linear in the amplitude of m) is the paper's approximation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from enum import IntEnum

import numpy as np

from . import kernel as _kernel


class Status(IntEnum):
    OK = 0
    INVALID = 1
    UNSUPPORTED = 2
    NOT_CONVERGED = 3
    RUNAWAY = 4


@dataclass
class Geometry:
    lx: float
    ly: float
    nx: int
    ny: int
    t: float
    k0: float
    eta: float
    t_amb: float
    rho_c: float = 1.66e6

    @property
    def hx(self) -> float:
        return self.lx / self.nx

    @property
    def hy(self) -> float:
        return self.ly / self.ny

    @property
    def k_ref(self) -> float:
        """k(T_amb) = k0 (T_amb / 300)^-eta."""
        return self.k0 * (self.t_amb / 300.0) ** (-self.eta)


@dataclass
class Options:
    leak: str = "exp"  # "exp", "linear", "none"
    beta: float = 0.017
    max_iter: int = 50
    tol: float = 1e-6
    dT_cap: float = 1000.0
    cond: str = "source"  # placement of the conductivity factor 1/m: "source" or "target"


@dataclass
class Stats:
    status: Status
    iterations: int
    last_increment: float
    residual: float
    dT_max: float
    dT_mean: float
    hotspot_index: int
    increments: list = field(default_factory=list)


def geometry_from_die(die, n: int, ny: int | None = None) -> Geometry:
    """Geometry of an n x n grid (n columns by ny rows when ny is given) of a die."""
    return Geometry(die.lx_m, die.ly_m, n, ny or n, die.t_m, die.k0, die.eta, die.t_amb, die.rho_c)


# ----------------------------------------------------------------------------- direct sum
def _fold(idx: np.ndarray, n: int) -> np.ndarray:
    """Map any integer cell offset onto [0, n] using evenness and 2n-periodicity of K_per."""
    a = np.abs(idx) % (2 * n)
    return np.where(a > n, 2 * n - a, a)


class DirectSum:
    """theta_SI = images-folded direct sum of the periodised cell kernel with a power map [W/cell]."""

    def __init__(self, geom: Geometry, table: np.ndarray | None = None):
        self.geom = geom
        if table is None:
            table = _kernel.periodized_table(geom.nx, geom.ny, geom.lx, geom.ly, geom.t, geom.k_ref)
        self.table = np.ascontiguousarray(table)  # [ny + 1][nx + 1]
        nx = geom.nx
        j = np.arange(nx)
        self._col_minus = _fold(j[:, None] - j[None, :], nx)  # fold(j - l)
        self._col_plus = _fold(j[:, None] + j[None, :] + 1, nx)  # fold(j + l + 1)

    def apply(self, p: np.ndarray) -> np.ndarray:
        """Direct sum over every source cell and its mirror images (O(N^4), BLAS-3 by row offset)."""
        ny, nx = self.geom.ny, self.geom.nx
        assert p.shape == (ny, nx)
        theta = np.zeros((ny, nx))
        for d in range(ny + 1):
            row = self.table[d]
            a_d = row[self._col_minus] + row[self._col_plus]  # [j, l]
            q = p @ a_d.T  # q[k, j] = sum_l p[k, l] a_d[j, l]
            if d < ny:  # |i - k| = d
                theta[d:, :] += q[:ny - d, :]
                if d > 0:
                    theta[:ny - d, :] += q[d:, :]
            if d >= 1:  # i + k + 1 = d
                theta[:d, :] += q[:d][::-1]
            if 1 <= d <= ny - 1:  # i + k + 1 = 2 ny - d
                theta[ny - d:, :] += q[ny - d:][::-1]
        return theta

    def apply_at(self, p: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """theta_SI at selected cells only (O(N^2) per cell), for sampled checks at large N."""
        ny, nx = self.geom.ny, self.geom.nx
        k = np.arange(ny)
        l = np.arange(nx)
        out = np.empty(len(rows))
        for s, (i, j) in enumerate(zip(rows, cols)):
            r1, r2 = _fold(i - k, ny), _fold(i + k + 1, ny)
            c1, c2 = _fold(j - l, nx), _fold(j + l + 1, nx)
            w = (self.table[r1[:, None], c1[None, :]] + self.table[r2[:, None], c1[None, :]]
                 + self.table[r1[:, None], c2[None, :]] + self.table[r2[:, None], c2[None, :]])
            out[s] = float(np.sum(w * p))
        return out


def direct_sum_literal(table: np.ndarray, p: np.ndarray) -> np.ndarray:
    """The same sum as four nested loops (tiny grids only; pins ``DirectSum.apply``)."""
    ny, nx = p.shape
    theta = np.zeros((ny, nx))
    for i in range(ny):
        for j in range(nx):
            acc = 0.0
            for k in range(ny):
                for l in range(nx):
                    for a in (i - k, i + k + 1):
                        for b in (j - l, j + l + 1):
                            acc += p[k, l] * table[int(_fold(np.array(a), ny)), int(_fold(np.array(b), nx))]
            theta[i, j] = acc
    return theta


# ----------------------------------------------------------------------------- fixed point pieces
def kirchhoff_inverse(theta: np.ndarray, t_amb: float, eta: float):
    """dT = Phi^-1(theta) for k = k_ref (T / T_amb)^-eta; returns (dT, domain_ok)."""
    if eta == 0.0:
        return theta.copy(), np.ones(theta.shape, dtype=bool)
    if eta == 1.0:
        return t_amb * np.expm1(theta / t_amb), np.ones(theta.shape, dtype=bool)
    base = 1.0 + (1.0 - eta) * theta / t_amb
    ok = base > 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        dT = t_amb * (np.power(np.where(ok, base, 1.0), 1.0 / (1.0 - eta)) - 1.0)
    return dT, ok


def kirchhoff(dT: np.ndarray, t_amb: float, eta: float) -> np.ndarray:
    """theta = Phi(dT) = int_{T_amb}^{T_amb + dT} (T / T_amb)^-eta dT."""
    if eta == 0.0:
        return dT.copy()
    if eta == 1.0:
        return t_amb * np.log1p(dT / t_amb)
    return t_amb / (1.0 - eta) * (np.power(1.0 + dT / t_amb, 1.0 - eta) - 1.0)


class SteadyProblem:
    """Inputs of one steady solve in SI units (maps [ny][nx] float64; None means absent / 1)."""

    def __init__(self, geom: Geometry, q_dyn, q_leak0=None, leak_var=None, cond_map=None,
                 operator: DirectSum | None = None):
        self.geom = geom
        self.q_dyn = np.asarray(q_dyn, dtype=np.float64)
        self.q_leak = None
        if q_leak0 is not None:
            self.q_leak = np.asarray(q_leak0, dtype=np.float64)
            if leak_var is not None:
                self.q_leak = self.q_leak * np.asarray(leak_var, dtype=np.float64)
        self.m = None if cond_map is None else np.asarray(cond_map, dtype=np.float64)
        self.op = operator or DirectSum(geom)

    def power(self, dT: np.ndarray, opts: Options) -> np.ndarray:
        """P = hx hy [q_dyn + q_leak0 v L(dT)] in W per cell (Eqs. Pt, Pleak)."""
        q = self.q_dyn
        if self.q_leak is not None and opts.leak != "none":
            if opts.leak == "exp":
                lf = np.exp(opts.beta * dT)
            elif opts.leak == "linear":
                lf = 1.0 + opts.beta * dT
            else:
                raise ValueError(opts.leak)
            q = q + self.q_leak * lf
        return self.geom.hx * self.geom.hy * q

    def map(self, dT: np.ndarray, opts: Options):
        """One application of G; returns (dT', domain_ok)."""
        p = self.power(dT, opts)
        if self.m is None:
            theta = self.op.apply(p)
        elif opts.cond == "source":
            theta = self.op.apply(p / self.m)
        elif opts.cond == "target":
            theta = self.op.apply(p) / self.m
        else:
            raise ValueError(opts.cond)
        return kirchhoff_inverse(theta, self.geom.t_amb, self.geom.eta)


def solve_steady(prob: SteadyProblem, opts: Options, init: np.ndarray | None = None,
                 residual: bool = True):
    """Picard iteration of G to the first increment <= tol; returns (dT, Stats)."""
    g = prob.geom
    dT = np.zeros((g.ny, g.nx)) if init is None else np.array(init, dtype=np.float64)
    incs = []
    status = Status.NOT_CONVERGED
    it = 0
    for it in range(1, opts.max_iter + 1):
        new, ok = prob.map(dT, opts)
        if (not np.all(ok)) or (not np.all(np.isfinite(new))) or float(np.max(new)) > opts.dT_cap:
            return new, Stats(Status.RUNAWAY, it, math.inf, math.inf, math.nan, math.nan, -1, incs)
        inc = float(np.max(np.abs(new - dT)))
        incs.append(inc)
        dT = new
        if inc <= opts.tol:
            status = Status.OK
            break
    res = math.nan
    if residual:
        again, _ = prob.map(dT, opts)
        res = float(np.max(np.abs(again - dT)))
    return dT, Stats(status, it, incs[-1] if incs else math.nan, res, float(np.max(dT)),
                     float(np.mean(dT)), int(np.argmax(dT)), incs)


def problem_from_inputs(inp, operator: DirectSum | None = None) -> tuple[SteadyProblem, Options]:
    """Build the oracle problem from a ``workloads.SteadyInputs``."""
    geom = geometry_from_die(inp.die, inp.n, getattr(inp, "ny", None))
    prob = SteadyProblem(geom, inp.q_dyn, inp.q_leak0, inp.leak_var, inp.cond_map, operator)
    opts = Options(leak=inp.leak, beta=inp.beta)
    return prob, opts
