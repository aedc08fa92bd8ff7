"""Seeded synthetic inputs for the steady and transient thermal solves.

Everything here is input preparation: block floorplans, rasterised power-density maps,
Gaussian random fields for the threshold-voltage and conductivity variation, and per-block
power traces.  The thermal method itself (Green's function, convolution, leakage and
conductivity feedback) lives elsewhere; this module computes none of it.

Recipe (the paper's own floorplans and Varius maps are not available, so these stand in for
them with the shapes the paper describes):

* die: 10 mm x 10 mm, one silicon layer 0.5 mm thick, T_amb = 318 K, k0 = 150 W/mK
  (conductivity law of Sec. II-E), rho*c = 1.66e6 J/(m^3 K);
* floorplan: ``n_blocks`` axis-aligned rectangles snapped to a 1024 x 1024 unit lattice,
  side lengths uniform integers in [0.5 s, 1.5 s] with s = 1024 / sqrt(2 n_blocks), lower-left
  corner uniform with the block inside the die, painter's order (later blocks overwrite);
  dynamic power density per block U[0.1, 2] W/mm^2; a grid of N cells per edge takes the area
  average over (1024/N)^2 lattice units;
* systematic variation (Sec. II-C): a zero-mean unit-variance Gaussian random field with
  Gaussian covariance exp(-r^2 / 2 l^2), l = 1 mm, drawn on a periodic 2N x 2N lattice and
  cropped to N x N; threshold-voltage shift dVth = 0.1 * 0.30 V * z scales leakage through the
  subthreshold exponent (Eq. bsim) as v = exp(-dVth / (n v_T)), n = 1.5, v_T = k_B T_amb / q;
* conductivity variation (Sec. II-E): an independent field of the same recipe mapped to a
  uniform +-5 % multiplier m = 1 + 0.05 (2 Phi(z_k) - 1);
* transient traces: per block, power density held for 1 ms, drawn U[0, 3] W/mm^2 and then a
  reflected random walk with N(0, 0.5^2) W/mm^2 steps at each hold boundary.

All densities are SI (W/m^2).  Seeds come from ``SeedSequence([230712119, *key])`` with PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from functools import lru_cache

import numpy as np
import scipy.fft as sfft
from scipy.special import ndtr

SEED_ROOT = 230712119
LATTICE = 1024
W_PER_MM2 = 1.0e6  # W/m^2 in one W/mm^2

FFT_WORKERS = -1  # scipy.fft worker threads for the random fields (-1: all cores)

K_BOLTZMANN = 1.380649e-23
Q_ELECTRON = 1.602176634e-19


def make_rng(*key: int) -> np.random.Generator:
    """PCG64 generator seeded from ``SeedSequence([230712119, *key])``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, *key])))


@dataclass(frozen=True)
class Die:
    """Single-layer die: lateral size, silicon thickness and material constants (SI)."""

    lx_m: float = 10e-3
    ly_m: float = 10e-3
    t_m: float = 0.5e-3
    k0: float = 150.0  # W/mK at 300 K
    eta: float = 0.0  # exponent of k = k0 (T/300)^-eta
    rho_c: float = 1.66e6  # J/(m^3 K)
    t_amb: float = 318.0  # K


@dataclass
class Blocks:
    """Axis-aligned rectangles on a square lattice of ``lattice`` units per die edge."""

    x0: np.ndarray
    y0: np.ndarray
    w: np.ndarray
    h: np.ndarray
    lattice: int = LATTICE

    def __len__(self) -> int:
        return len(self.x0)


@dataclass
class SteadyInputs:
    """One steady problem: maps are float64 [ny][nx] row-major, densities in W/m^2."""

    die: Die
    n: int
    q_dyn: np.ndarray
    q_leak0: np.ndarray | None
    leak_var: np.ndarray | None
    cond_map: np.ndarray | None
    beta: float = 0.017
    leak: str = "exp"  # "exp", "linear" or "none"
    meta: dict = field(default_factory=dict)
    ny: int | None = None  # rows when the grid is not square (then n is the column count nx)

    @property
    def shape(self) -> tuple[int, int]:
        return (self.ny or self.n, self.n)


@dataclass
class TransientInputs:
    """One transient problem: block id map, per-step block power densities and static maps."""

    die: Die
    n: int
    dt_s: float
    n_steps: int
    block_rects: np.ndarray  # int32 [n_blocks][4] = x0, y0, w, h in cell units
    trace: np.ndarray  # float64 [n_steps][n_blocks], W/m^2 held over (t_{n-1}, t_n]
    q_leak0: np.ndarray | None
    leak_var: np.ndarray | None
    cond_map: np.ndarray | None
    beta: float = 0.017
    leak: str = "exp"


# ----------------------------------------------------------------------------- floorplans
def random_blocks(n_blocks: int, rng: np.random.Generator, lattice: int = LATTICE) -> Blocks:
    """Random rectangles with sides uniform in [0.5 s, 1.5 s], s = lattice / sqrt(2 n_blocks)."""
    sbar = lattice / math.sqrt(2.0 * n_blocks)
    lo = max(1, math.ceil(0.5 * sbar))
    hi = max(lo, min(lattice, math.floor(1.5 * sbar)))
    w = rng.integers(lo, hi + 1, size=n_blocks)
    h = rng.integers(lo, hi + 1, size=n_blocks)
    x0 = rng.integers(0, lattice - w + 1)
    y0 = rng.integers(0, lattice - h + 1)
    return Blocks(x0.astype(np.int64), y0.astype(np.int64), w.astype(np.int64), h.astype(np.int64), lattice)


def paint(blocks: Blocks, values: np.ndarray) -> np.ndarray:
    """Lattice map with each block's value, later blocks painted over earlier ones."""
    lat = np.zeros((blocks.lattice, blocks.lattice), dtype=np.float64)
    for b in range(len(blocks)):
        lat[blocks.y0[b]:blocks.y0[b] + blocks.h[b], blocks.x0[b]:blocks.x0[b] + blocks.w[b]] = values[b]
    return lat


def block_id_map(blocks: Blocks, n: int) -> np.ndarray:
    """int32 [n][n] map of the block that owns each cell (-1: none); blocks must snap to cells."""
    if blocks.lattice % n:
        raise ValueError("grid must divide the lattice")
    s = blocks.lattice // n
    for arr in (blocks.x0, blocks.y0, blocks.w, blocks.h):
        if np.any(arr % s):
            raise ValueError("blocks do not snap to the cell grid")
    ids = np.full((n, n), -1, dtype=np.int32)
    for b in range(len(blocks)):
        y0, x0 = blocks.y0[b] // s, blocks.x0[b] // s
        ids[y0:y0 + blocks.h[b] // s, x0:x0 + blocks.w[b] // s] = b
    return ids


def area_average(lat: np.ndarray, n: int) -> np.ndarray:
    """Average a lattice map over (L/n)^2 blocks of units, giving an n x n cell map."""
    s = lat.shape[0] // n
    if s * n != lat.shape[0]:
        raise ValueError("grid must divide the lattice")
    return lat.reshape(n, s, n, s).mean(axis=(1, 3))


# ----------------------------------------------------------------------------- random fields
def gaussian_field(n: int, cell_m: float, ell_m: float, rng: np.random.Generator) -> np.ndarray:
    """Zero-mean unit-variance field with covariance exp(-r^2 / 2 l^2) on an n x n grid.

    White noise on a periodic 2n x 2n lattice is filtered in Fourier space with the square
    root of the Gaussian spectral density, normalised so that every cell has unit variance,
    and the n x n corner is kept.
    """
    m = 2 * n
    noise = rng.standard_normal((m, m))
    k = 2.0 * np.pi * np.fft.fftfreq(m, d=cell_m)
    kk = k[:, None] ** 2 + k[None, :] ** 2
    amp = np.exp(-0.25 * ell_m * ell_m * kk)
    amp /= math.sqrt(float(np.mean(amp * amp)))
    z = sfft.ifft2(sfft.fft2(noise, workers=FFT_WORKERS) * amp, workers=FFT_WORKERS).real
    return np.ascontiguousarray(z[:n, :n])


def vth_leak_scale(t_amb: float, vth0: float = 0.30, rel_sigma: float = 0.1, n_sub: float = 1.5) -> float:
    """Log-sigma s of v = exp(-s z) for dVth = rel_sigma * vth0 * z through the subthreshold slope."""
    v_t = K_BOLTZMANN * t_amb / Q_ELECTRON
    return rel_sigma * vth0 / (n_sub * v_t)


# ----------------------------------------------------------------------------- workloads
@lru_cache(maxsize=64)
def _floorplan_density(config: int, floorplan: int, n_blocks: int, n: int) -> np.ndarray:
    frng = make_rng(config, floorplan, 0, 0)
    blocks = random_blocks(n_blocks, frng)
    q = frng.uniform(0.1, 2.0, size=n_blocks) * W_PER_MM2
    out = area_average(paint(blocks, q), n)
    out.setflags(write=False)
    return out


def floorplan_density(config: int, floorplan: int, n_blocks: int, n: int) -> np.ndarray:
    """Dynamic power density of a seeded block floorplan rasterised on an n x n grid [W/m^2]."""
    return _floorplan_density(config, floorplan, n_blocks, n).copy()


def steady_problem(config: int, n: int, n_blocks: int, floorplan: int = 0, sample: int = 0,
                   variation: bool = True, eta: float = 1.3, die: Die | None = None,
                   beta: float = 0.017, leak_fraction: float = 0.2) -> SteadyInputs:
    """A steady problem of the block-floorplan family.

    The floorplan depends on (config, floorplan); the variation maps on (config, floorplan,
    sample).  ``variation=False`` gives v = m = 1 and k independent of T (eta = 0).
    """
    die = die or Die()
    die = replace(die, eta=eta if variation else 0.0)
    q_dyn = floorplan_density(config, floorplan, n_blocks, n)
    q_leak0 = leak_fraction * q_dyn
    if variation:
        cell = die.lx_m / n
        z_v = gaussian_field(n, cell, 1.0e-3, make_rng(config, floorplan, sample, 1))
        z_k = gaussian_field(n, cell, 1.0e-3, make_rng(config, floorplan, sample, 2))
        leak_var = np.exp(-vth_leak_scale(die.t_amb) * z_v)
        cond_map = 1.0 + 0.05 * (2.0 * ndtr(z_k) - 1.0)
    else:
        leak_var = None
        cond_map = None
    return SteadyInputs(die, n, q_dyn, q_leak0, leak_var, cond_map, beta, "exp",
                        {"config": config, "floorplan": floorplan, "sample": sample, "n_blocks": n_blocks})


def config1(seed: int = 0, n: int = 64) -> SteadyInputs:
    """64 x 64, 16 blocks, no variation, eta = 0, exp leakage with beta = 0.017 / K."""
    return steady_problem(1, n, 16, floorplan=seed, variation=False)


def config2(sample: int = 0, n: int = 512, floorplan: int = 0) -> SteadyInputs:
    """512 x 512, 64 blocks, Vth and conductivity variation, k(T) with eta = 1.3."""
    return steady_problem(2, n, 64, floorplan=floorplan, sample=sample, variation=True)


def config3(size_class: int, sample: int) -> SteadyInputs:
    """Mixed-size Monte Carlo batch: floorplan f is rasterised at N = 128 * 2^f."""
    n = 128 << size_class
    return steady_problem(3, n, 64, floorplan=size_class, sample=sample, variation=True)


def rect_problem(nx: int, ny: int, lx_m: float = 10e-3, ly_m: float = 10e-3, seed: int = 0, n_blocks: int = 16,
                 variation: bool = True, eta: float = 1.3, beta: float = 0.017) -> SteadyInputs:
    """A block-floorplan problem on an nx x ny grid of an lx x ly die (rectangular grids; cells
    may be anisotropic).  Blocks, the Vth field and the conductivity field live on a square
    lattice of the finer cell size, are cropped to the die and area-averaged to the grid."""
    die = replace(Die(lx_m=lx_m, ly_m=ly_m), eta=eta if variation else 0.0)
    fine = min(lx_m / nx, ly_m / ny)
    fx, fy = round(lx_m / fine), round(ly_m / fine)
    if abs(fx * fine - lx_m) > 1e-9 * lx_m or abs(fy * fine - ly_m) > 1e-9 * ly_m or fx % nx or fy % ny:
        raise ValueError("die and grid must share a fine lattice")
    side = max(fx, fy)
    rng = make_rng(7, seed, nx, ny)
    # blocks drawn on the square lattice and stretched onto the fy x fx die lattice
    blocks = random_blocks(n_blocks, rng, lattice=side)
    lat = np.zeros((fy, fx))
    q = rng.uniform(0.1, 2.0, size=n_blocks) * W_PER_MM2
    for b in range(n_blocks):
        x0, x1 = blocks.x0[b] * fx // side, (blocks.x0[b] + blocks.w[b]) * fx // side
        y0, y1 = blocks.y0[b] * fy // side, (blocks.y0[b] + blocks.h[b]) * fy // side
        lat[y0:max(y1, y0 + 1), x0:max(x1, x0 + 1)] = q[b]

    def to_grid(a):
        return a.reshape(ny, fy // ny, nx, fx // nx).mean(axis=(1, 3))

    q_dyn = to_grid(lat)
    leak_var = cond_map = None
    if variation:
        z_v = gaussian_field(side, fine, 1.0e-3, make_rng(7, seed, nx, ny, 1))[:fy, :fx]
        z_k = gaussian_field(side, fine, 1.0e-3, make_rng(7, seed, nx, ny, 2))[:fy, :fx]
        leak_var = to_grid(np.exp(-vth_leak_scale(die.t_amb) * z_v))
        cond_map = to_grid(1.0 + 0.05 * (2.0 * ndtr(z_k) - 1.0))
    return SteadyInputs(die, nx, q_dyn, 0.2 * q_dyn, leak_var, cond_map, beta, "exp",
                        {"seed": seed, "n_blocks": n_blocks}, ny=ny)


def uniform_problem(n: int, q_w_mm2: float, leak_w_mm2: float = 0.0, die: Die | None = None,
                    beta: float = 0.017, leak: str = "exp") -> SteadyInputs:
    """Uniform power over the whole die (the shape of the paper's uniform-power test case)."""
    die = die or Die()
    q_dyn = np.full((n, n), q_w_mm2 * W_PER_MM2)
    q_leak0 = np.full((n, n), leak_w_mm2 * W_PER_MM2) if leak_w_mm2 else None
    return SteadyInputs(die, n, q_dyn, q_leak0, None, None, beta, leak if leak_w_mm2 else "none")


def alternate_points_problem(n: int = 64, watts: float = 0.05, die: Die | None = None,
                             offset: tuple[int, int] = (0, 0)) -> SteadyInputs:
    """Sources of ``watts`` at every other grid point in both axes (alternate-points test case)."""
    die = die or Die()
    cell_area = (die.lx_m / n) * (die.ly_m / n)
    q = np.zeros((n, n))
    q[offset[0]::2, offset[1]::2] = watts / cell_area
    return SteadyInputs(die, n, q, None, None, None, 0.0, "none")


def dense_sources_problem(n: int, seed: int = 0, die: Die | None = None) -> SteadyInputs:
    """A few small, very dense sources (the shape of the paper's stress test case)."""
    die = die or Die()
    rng = make_rng(9, seed, 0, 0)
    side = max(1, round(0.3e-3 / (die.lx_m / n)))
    q = np.zeros((n, n))
    for _ in range(4):
        x0, y0 = rng.integers(0, n - side + 1, size=2)
        q[y0:y0 + side, x0:x0 + side] = rng.uniform(8.0, 20.0) * W_PER_MM2
    return SteadyInputs(die, n, q, 0.2 * q, None, None, 0.017, "exp")


def power_traces(n_blocks: int, n_steps: int, hold_steps: int, rng: np.random.Generator,
                 hi_w_mm2: float = 3.0, step_sigma: float = 0.5) -> np.ndarray:
    """Piecewise-constant reflected random walks in [0, hi]; float64 [n_steps][n_blocks], W/m^2."""
    n_holds = -(-n_steps // hold_steps)
    q = rng.uniform(0.0, hi_w_mm2, size=n_blocks)
    levels = np.empty((n_holds, n_blocks))
    for j in range(n_holds):
        if j:
            q = q + rng.normal(0.0, step_sigma, size=n_blocks)
            q = np.abs(q)
            q = hi_w_mm2 - np.abs(hi_w_mm2 - q)
            q = np.clip(q, 0.0, hi_w_mm2)
        levels[j] = q
    return np.repeat(levels, hold_steps, axis=0)[:n_steps] * W_PER_MM2


def transient_problem(n: int = 1024, n_steps: int = 1000, dt_s: float = 10e-6, n_blocks: int = 64,
                      hold_s: float = 1e-3, seed: int = 0, variation: bool = True,
                      eta: float = 1.3, leak_w_mm2: float = 0.3) -> TransientInputs:
    """Block floorplan on the cell grid with per-block power traces (transient configuration)."""
    die = replace(Die(), eta=eta if variation else 0.0)
    frng = make_rng(4, seed, 0, 0)
    blocks = random_blocks(n_blocks, frng, lattice=n)
    rects = np.stack([blocks.x0, blocks.y0, blocks.w, blocks.h], axis=1).astype(np.int32)
    hold = max(1, round(hold_s / dt_s))
    trace = power_traces(n_blocks, n_steps, hold, make_rng(4, seed, 0, 3))
    ids = block_id_map(blocks, n)
    q_leak0 = np.where(ids >= 0, leak_w_mm2 * W_PER_MM2, 0.0)
    if variation:
        cell = die.lx_m / n
        leak_var = np.exp(-vth_leak_scale(die.t_amb) * gaussian_field(n, cell, 1e-3, make_rng(4, seed, 0, 1)))
        cond_map = 1.0 + 0.05 * (2.0 * ndtr(gaussian_field(n, cell, 1e-3, make_rng(4, seed, 0, 2))) - 1.0)
    else:
        leak_var = cond_map = None
    return TransientInputs(die, n, dt_s, n_steps, rects, trace, q_leak0, leak_var, cond_map)


def raster_trace_step(rects: np.ndarray, trace_row: np.ndarray, n: int) -> np.ndarray:
    """Dynamic power density map for one step: each cell takes its last covering block's value."""
    q = np.zeros((n, n))
    for b in range(rects.shape[0]):
        x0, y0, w, h = (int(v) for v in rects[b])
        q[y0:y0 + h, x0:x0 + w] = trace_row[b]
    return q
