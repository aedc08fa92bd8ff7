"""ctypes binding of libvarsim.so (argument marshalling only).

Every step of the solve runs in the HIP library; this module only builds the C structs of
``include/varsim.h`` from torch tensors (device memory) and plain numbers, passes device
pointers and the current HIP stream, and turns status codes into exceptions.  It fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvarsim.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_NOT_CONVERGED, ERR_RUNAWAY, ERR_DEVICE, ERR_NO_MEMORY = range(7)
LEAK_NONE, LEAK_EXP, LEAK_LINEAR = 0, 1, 2
F32, F64 = 0, 1
TAU_MOMENT, TAU_LUMPED, TAU_MODAL = 0, 1, 2
COND_SOURCE, COND_TARGET = 0, 1


class VarsimError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"varsim status {status}: {message}")
        self.status = status


class Layer(Structure):
    _fields_ = [("thickness_m", c_double), ("k0_W_mK", c_double), ("eta", c_double), ("rho_c_J_m3K", c_double)]


class Geometry(Structure):
    _fields_ = [("lx_m", c_double), ("ly_m", c_double), ("nx", c_int32), ("ny", c_int32), ("n_layers", c_int32),
                ("layers", POINTER(Layer)), ("bottom_bc", c_int32), ("h_bottom_W_m2K", c_double),
                ("t_amb_K", c_double)]


class Options(Structure):
    _fields_ = [("leak", c_int32), ("beta_per_K", c_double), ("sv_radius", c_int32), ("precision", c_int32),
                ("max_iter", c_int32), ("tol_K", c_double), ("dT_cap_K", c_double), ("final_f64_residual", c_int32),
                ("cond_model", c_int32), ("compensated_twiddles", c_int32), ("anderson", c_int32)]


class Problem(Structure):
    _fields_ = [("geom", POINTER(Geometry)), ("q_dyn", c_void_p), ("q_leak0", c_void_p), ("leak_var", c_void_p),
                ("cond_map", c_void_p), ("dT_init", c_void_p), ("dT_out", c_void_p)]


class Stats(Structure):
    _fields_ = [("status", c_int32), ("iterations", c_int32), ("last_increment_K", c_double),
                ("residual_f64_K", c_double), ("dT_max_K", c_double), ("dT_mean_K", c_double),
                ("hotspot_index", c_int64), ("warm_start_rejected", c_int32), ("reserved", c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Transient(Structure):
    _fields_ = [("dt_s", c_double), ("n_steps", c_int32), ("out_every", c_int32), ("n_blocks", c_int32),
                ("block_rects", c_void_p), ("trace", c_void_p), ("tau_model", c_int32), ("n_poles", c_int32),
                ("history_steps", c_int32)]


class OneShot(Structure):
    _fields_ = [("mu_W_m2", c_double), ("random_part", c_int32)]


class NetConfig(Structure):
    _fields_ = [("n", c_int32), ("width", c_int32 * 5), ("shift", ctypes.c_float * 3), ("scale", ctypes.c_float * 3),
                ("out_scale", ctypes.c_float), ("k0_W_mK", ctypes.c_float)]


NN_FWD, NN_DGRAD, NN_WGRAD = 0, 1, 2

EXPORTS = {
    "varsim_create": (c_int, [c_int, POINTER(c_void_p)]),
    "varsim_destroy": (None, [c_void_p]),
    "varsim_status_string": (c_char_p, [c_int]),
    "varsim_last_error": (c_char_p, [c_void_p]),
    "varsim_green_table": (c_int, [c_void_p, POINTER(Geometry), c_void_p, c_void_p, c_void_p]),
    "varsim_conv": (c_int, [c_void_p, POINTER(Geometry), c_int32, c_void_p, c_void_p, c_int32, c_void_p]),
    "varsim_workspace_size": (c_int, [c_void_p, POINTER(Problem), c_int32, POINTER(Options), POINTER(c_size_t)]),
    "varsim_solve_steady": (c_int, [c_void_p, POINTER(Problem), POINTER(Options), c_void_p, c_size_t,
                                    POINTER(Stats), c_void_p]),
    "varsim_solve_batch": (c_int, [c_void_p, POINTER(Problem), c_int32, POINTER(Options), c_void_p, c_size_t,
                                   POINTER(Stats), c_void_p]),
    "varsim_solve_batch_noalloc": (c_int, [c_void_p, POINTER(Problem), c_int32, POINTER(Options), POINTER(Stats),
                                           c_void_p]),
    "varsim_noalloc_scratch_bytes": (c_int, [POINTER(c_size_t)]),
    "varsim_solve_oneshot": (c_int, [c_void_p, POINTER(Problem), c_int32, POINTER(Options), POINTER(OneShot),
                                     c_void_p, c_size_t, POINTER(Stats), c_void_p]),
    "varsim_solve_transient": (c_int, [c_void_p, POINTER(Problem), POINTER(Transient), POINTER(Options), c_void_p,
                                       c_void_p, c_size_t, POINTER(Stats), c_void_p]),
    "varsim_transient_workspace_size": (c_int, [c_void_p, POINTER(Problem), POINTER(Transient), POINTER(Options),
                                                POINTER(c_size_t)]),
    "varsim_net_create": (c_int, [c_void_p, POINTER(NetConfig), POINTER(c_void_p)]),
    "varsim_net_destroy": (None, [c_void_p]),
    "varsim_net_param_count": (c_int, [c_void_p, POINTER(c_int64)]),
    "varsim_net_set_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "varsim_net_get_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "varsim_net_workspace_size": (c_int, [c_void_p, c_int32, c_int32, POINTER(c_size_t)]),
    "varsim_net_forward": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]),
    "varsim_net_gradient": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "varsim_net_adam": (c_int, [c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                c_void_p]),
    "varsim_nn_conv_workspace": (c_int, [c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                                         POINTER(c_size_t)]),
    "varsim_nn_conv": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, c_void_p,
                               c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "varsim_set_autotune": (c_int, [c_void_p, c_int32]),
    "varsim_autotune_report": (c_int, [c_void_p, c_char_p, c_size_t]),
    "varsim_autotune_export": (c_int, [c_void_p, c_char_p, c_size_t, POINTER(c_size_t)]),
    "varsim_autotune_import": (c_int, [c_void_p, c_char_p]),
    "varsim_force_col_variant": (c_int, [c_void_p, c_int32]),
    "varsim_force_transient_variant": (c_int, [c_void_p, c_int32, c_int32]),
    "varsim_set_small_path": (c_int, [c_void_p, c_int32]),
    "varsim_set_graph_iterations": (c_int, [c_void_p, c_int32]),
    "varsim_set_timing": (c_int, [c_void_p, c_int32]),
    "varsim_kernel_times": (c_int, [c_void_p, POINTER(c_char_p), POINTER(c_int64), POINTER(c_double),
                                    POINTER(c_int32)]),
    "varsim_reset_timing": (c_int, [c_void_p]),
    "varsim_set_timing_only": (c_int, [c_void_p, c_char_p]),
}


class Library:
    """The loaded shared library with typed entry points."""

    _instance = None

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is not built; run paper_2307_12119_amd.build.build() first")
        self.path = path
        self.cdll = ctypes.CDLL(path)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(self.cdll, name)
            fn.restype = res
            fn.argtypes = args
            setattr(self, name, fn)

    @classmethod
    def load(cls) -> "Library":
        if cls._instance is None:
            cls._instance = cls()
        return cls._instance


# ----------------------------------------------------------------------------------------- helpers
def _ptr(t) -> int | None:
    """Device address of a contiguous torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to varsim must be contiguous")
    return t.data_ptr()


def _stream() -> int:
    import torch

    return torch.cuda.current_stream().cuda_stream


@dataclass
class Die:
    """Geometry and material of a die (SI units): the silicon layer, optionally the package
    layers below it (``stack``: (thickness, k0, eta) per layer, top first) and a convective
    bottom (``h_bottom`` in W/m^2K; None: isothermal at t_amb)."""

    lx_m: float
    ly_m: float
    t_m: float
    k0: float
    eta: float
    t_amb: float
    rho_c: float = 1.66e6
    stack: tuple = ()
    h_bottom: float | None = None


def make_geometry(die: Die, n: int, ny: int | None = None):
    """Geometry of an n x n grid (n columns by ny rows when ny is given) and its layer array
    (keep both alive while the geometry is used); geom.layers already points at the array."""
    layers = [Layer(die.t_m, die.k0, die.eta, die.rho_c)] + [Layer(t, k, e, die.rho_c) for t, k, e in die.stack]
    arr = (Layer * len(layers))(*layers)
    bc = 0 if die.h_bottom is None else 1
    geom = Geometry(die.lx_m, die.ly_m, n, ny or n, len(layers), ctypes.cast(arr, POINTER(Layer)), bc,
                    0.0 if die.h_bottom is None else float(die.h_bottom), die.t_amb)
    return geom, arr


def make_options(precision: int = F32, leak: int = LEAK_EXP, beta: float = 0.017, max_iter: int = 50,
                 tol: float = 1e-3, cap: float = 1000.0, f64_residual: bool = False,
                 cond: int = COND_SOURCE, compensated_twiddles: bool = False, anderson: bool = False) -> Options:
    return Options(leak, beta, 0, precision, max_iter, tol, cap, 1 if f64_residual else 0, cond,
                   1 if compensated_twiddles else 0, 1 if anderson else 0)


class Context:
    """A library context on one device (owns the Green's-function and twiddle caches)."""

    def __init__(self, device: int = 0, lib: Library | None = None):
        self.lib = lib or Library.load()
        h = c_void_p()
        st = self.lib.varsim_create(device, ctypes.byref(h))
        if st != OK:
            raise VarsimError(st, "varsim_create failed")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self.lib.varsim_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow=(OK,)):
        if st not in allow:
            msg = self.lib.varsim_last_error(self.handle)
            raise VarsimError(st, msg.decode() if msg else "")
        return st

    # -------------------------------------------------------------------------------- table
    def green_table(self, die: Die, n: int, ny: int | None = None):
        """(K_per [ny+1][n+1], lambda [ny][n]) as FP64 device tensors (ny = n by default); K_per is
        None for a package stack (only its eigenvalues are tabulated)."""
        import torch

        ny = ny or n
        geom, layer = make_geometry(die, n, ny)
        dev = torch.device("cuda", self.device)
        slab = not die.stack and die.h_bottom is None
        kper = torch.empty((ny + 1, n + 1), dtype=torch.float64, device=dev) if slab else None
        lam = torch.empty((ny, n), dtype=torch.float64, device=dev)
        self._check(self.lib.varsim_green_table(self.handle, ctypes.byref(geom), _ptr(kper), _ptr(lam), _stream()))
        return kper, lam

    def conv(self, die: Die, power, out=None):
        """theta = mirrored Green's convolution of power maps [..., ny, nx] (W per cell)."""
        import torch

        ny, n = power.shape[-2], power.shape[-1]
        geom, layer = make_geometry(die, n, ny)
        prec = F64 if power.dtype == torch.float64 else F32
        out = torch.empty_like(power) if out is None else out
        n_maps = power.numel() // (n * ny)
        self._check(self.lib.varsim_conv(self.handle, ctypes.byref(geom), prec, _ptr(power), _ptr(out), n_maps,
                                         _stream()))
        return out

    # -------------------------------------------------------------------------------- solves
    def _problems(self, items: list[dict]):
        geoms, layers, probs = [], [], (Problem * len(items))()
        for i, it in enumerate(items):
            geom, layer = make_geometry(it["die"], it["dT_out"].shape[-1], it["dT_out"].shape[-2])
            layers.append(layer)
            geoms.append(geom)
            probs[i] = Problem(ctypes.pointer(geom), _ptr(it.get("q_dyn")), _ptr(it.get("q_leak0")),
                               _ptr(it.get("leak_var")), _ptr(it.get("cond_map")), _ptr(it.get("dT_init")),
                               _ptr(it["dT_out"]))
        return probs, (geoms, layers)

    def prepare(self, items: list[dict]) -> "PreparedBatch":
        """Descriptors of a batch built once, for repeated solves of the same tensors."""
        return PreparedBatch(self, items)

    def _ws_query(self, probs, n: int, opts: Options) -> int:
        nbytes = c_size_t()
        self._check(self.lib.varsim_workspace_size(self.handle, probs, n, ctypes.byref(opts), ctypes.byref(nbytes)))
        return nbytes.value

    def workspace_bytes(self, items, opts: Options) -> int:
        if isinstance(items, PreparedBatch):
            return items.workspace_bytes(opts)
        probs, keep = self._problems(items)
        return self._ws_query(probs, len(items), opts)

    def solve_batch(self, items, opts: Options, workspace=None, raise_on=(ERR_INVALID,
                    ERR_UNSUPPORTED, ERR_DEVICE, ERR_NO_MEMORY), stats_out=None):
        """Solve every problem (dicts of device tensors: die, q_dyn, dT_out, optional q_leak0,
        leak_var, cond_map, dT_init); returns per-problem stats dicts.  Given a PreparedBatch,
        returns the stats as a numpy structured array (one record per problem).  With stats_out
        (a device tensor of at least n * sizeof(Stats) bytes) the statistics are written there on
        the current stream and the call returns without synchronising (None); read them with
        stats_from_bytes."""
        import numpy as np
        import torch

        if isinstance(items, PreparedBatch):
            prep = items
            probs, n, stats, need = prep.probs, prep.n, prep.stats, prep.workspace_bytes(opts)
        else:
            prep = None
            probs, keep = self._problems(items)
            n = len(items)
            stats = (Stats * n)()
            need = self._ws_query(probs, n, opts)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))
        if stats_out is not None:
            if not stats_out.is_cuda or stats_out.numel() * stats_out.element_size() < n * ctypes.sizeof(Stats):
                raise ValueError("stats_out must be a device tensor of n * sizeof(Stats) bytes")
            st = self.lib.varsim_solve_batch(self.handle, probs, n, ctypes.byref(opts), _ptr(workspace),
                                             workspace.numel(), ctypes.cast(_ptr(stats_out), POINTER(Stats)),
                                             _stream())
            self._check(st)
            return None
        arr = np.ctypeslib.as_array(stats)
        arr["status"] = -1
        st = self.lib.varsim_solve_batch(self.handle, probs, n, ctypes.byref(opts), _ptr(workspace),
                                         workspace.numel(), stats, _stream())
        filled = bool((arr["status"] >= 0).all())
        # argument / device errors leave the stats unfilled; per-problem statuses are returned
        if st in raise_on and not (filled and st == ERR_INVALID):
            self._check(st, allow=())
        if prep is not None:
            return arr.copy()
        return [stats[i].as_dict() for i in range(n)]

    def solve_batch_noalloc(self, items: list[dict], opts: Options) -> list[dict]:
        """varsim_solve_batch_noalloc: the same solve with the library's static workspace (no
        device allocation by the library or here); every geometry's table must be cached
        (green_table).  Returns per-problem stats dicts; raises on argument / device errors."""
        probs, keep = self._problems(items)
        n = len(items)
        stats = (Stats * n)()
        for i in range(n):
            stats[i].status = -1
        st = self.lib.varsim_solve_batch_noalloc(self.handle, probs, n, ctypes.byref(opts), stats, _stream())
        if st in (ERR_INVALID, ERR_UNSUPPORTED, ERR_DEVICE, ERR_NO_MEMORY) and not all(
                stats[i].status >= 0 for i in range(n)):
            self._check(st, allow=())
        return [stats[i].as_dict() for i in range(n)]

    def noalloc_scratch_bytes(self) -> int:
        nbytes = c_size_t()
        self._check(self.lib.varsim_noalloc_scratch_bytes(ctypes.byref(nbytes)))
        return nbytes.value

    def solve_oneshot(self, items, opts: Options, mu_W_m2: float, random_part: bool = True, workspace=None,
                      stats_out=None):
        """varsim_solve_oneshot: the one-shot modified-Green's-function rise of every problem (same
        items as solve_batch; dT_init is ignored).  Returns per-problem stats dicts (a numpy
        structured array for a PreparedBatch); with stats_out, as solve_batch."""
        import numpy as np
        import torch

        if isinstance(items, PreparedBatch):
            probs, n, stats, need = items.probs, items.n, items.stats, items.workspace_bytes(opts)
        else:
            probs, keep = self._problems(items)
            n = len(items)
            stats = (Stats * n)()
            need = self._ws_query(probs, n, opts)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))
        os_ = OneShot(float(mu_W_m2), 1 if random_part else 0)
        if stats_out is not None:
            st = self.lib.varsim_solve_oneshot(self.handle, probs, n, ctypes.byref(opts), ctypes.byref(os_),
                                               _ptr(workspace), workspace.numel(),
                                               ctypes.cast(_ptr(stats_out), POINTER(Stats)), _stream())
            self._check(st)
            return None
        arr = np.ctypeslib.as_array(stats)
        arr["status"] = -1
        st = self.lib.varsim_solve_oneshot(self.handle, probs, n, ctypes.byref(opts), ctypes.byref(os_),
                                           _ptr(workspace), workspace.numel(), stats, _stream())
        if st in (ERR_INVALID, ERR_UNSUPPORTED, ERR_DEVICE, ERR_NO_MEMORY) or not bool((arr["status"] >= 0).all()):
            self._check(st, allow=(OK, ERR_RUNAWAY) if bool((arr["status"] >= 0).all()) else (OK,))
        if isinstance(items, PreparedBatch):
            return arr.copy()
        return [stats[i].as_dict() for i in range(n)]

    def solve_steady(self, item: dict, opts: Options, workspace=None) -> dict:
        return self.solve_batch([item], opts, workspace)[0]

    # ----------------------------------------------------------------------------- transient
    def _transient(self, block_rects, trace, dt_s: float, out_every: int, tau_model: int,
                   n_poles: int = 1, history_steps: int = 0) -> Transient:
        return Transient(dt_s, trace.shape[0], out_every, trace.shape[1], _ptr(block_rects), _ptr(trace), tau_model,
                         n_poles, history_steps)

    def transient_workspace_bytes(self, item: dict, block_rects, trace, dt_s: float, opts: Options,
                                  out_every: int = 1, tau_model: int = TAU_MOMENT, n_poles: int = 1,
                                  history_steps: int = 0) -> int:
        probs, keep = self._problems([item])
        tr = self._transient(block_rects, trace, dt_s, out_every, tau_model, n_poles, history_steps)
        n = ctypes.c_size_t(0)
        self._check(self.lib.varsim_transient_workspace_size(self.handle, probs, ctypes.byref(tr),
                                                             ctypes.byref(opts), ctypes.byref(n)))
        return n.value

    def solve_transient(self, item: dict, block_rects, trace, dt_s: float, opts: Options, snapshots=None,
                        out_every: int = 1, tau_model: int = TAU_MOMENT, workspace=None,
                        raise_on=(ERR_INVALID, ERR_UNSUPPORTED, ERR_DEVICE, ERR_NO_MEMORY), n_poles: int = 1,
                        history_steps: int = 0) -> dict:
        """Transient solve from dT = 0 (item: die, dT_out, optional q_leak0, leak_var, cond_map as
        device tensors).  block_rects: int32 [n_blocks][4] device tensor; trace: [n_steps][n_blocks]
        device tensor of the map dtype; snapshots: optional [n_steps // out_every][n][n] output;
        history_steps: 0 for the whole history, h >= 2 for the history truncated after h steps."""
        import torch

        probs, keep = self._problems([item])
        tr = self._transient(block_rects, trace, dt_s, out_every, tau_model, n_poles, history_steps)
        need = self.transient_workspace_bytes(item, block_rects, trace, dt_s, opts, out_every, tau_model, n_poles,
                                              history_steps)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))
        stats = Stats()
        stats.status = -1
        st = self.lib.varsim_solve_transient(self.handle, probs, ctypes.byref(tr), ctypes.byref(opts),
                                             _ptr(snapshots), _ptr(workspace), workspace.numel(),
                                             ctypes.byref(stats), _stream())
        if st in raise_on and not (stats.status >= 0 and st == ERR_INVALID):
            self._check(st, allow=())
        return stats.as_dict()

    # ------------------------------------------------------------------------------ autotune
    def set_autotune(self, enable: int):
        """1: time launch-shape candidates at first use; 0: stop; -1: stop and forget choices."""
        self._check(self.lib.varsim_set_autotune(self.handle, int(enable)))

    def set_small_path(self, max_n: int):
        """Largest N solved by one LDS-resident workgroup per map (-1 default, 0 off)."""
        self._check(self.lib.varsim_set_small_path(self.handle, int(max_n)))

    def set_graph_iterations(self, iterations: int):
        """Fixed-point iterations per captured HIP graph (0: direct launches)."""
        self._check(self.lib.varsim_set_graph_iterations(self.handle, int(iterations)))

    def force_col_variant(self, variant: int):
        self._check(self.lib.varsim_force_col_variant(self.handle, int(variant)))

    def force_transient_variant(self, row: int, col: int):
        """Pin the transient row / column pass candidates (0..2: two sequences per DFT, 3..5: one
        sequence per half-length DFT); -1 returns to the tuned or default choice."""
        self._check(self.lib.varsim_force_transient_variant(self.handle, int(row), int(col)))

    def autotune_report(self) -> str:
        buf = ctypes.create_string_buffer(8192)
        self._check(self.lib.varsim_autotune_report(self.handle, buf, len(buf)))
        return buf.value.decode()

    def autotune_export(self) -> str:
        """The kept launch-shape choices as text (varsim_autotune_export)."""
        need = ctypes.c_size_t(0)
        self._check(self.lib.varsim_autotune_export(self.handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        self._check(self.lib.varsim_autotune_export(self.handle, buf, len(buf), None))
        return buf.value.decode()

    def autotune_import(self, text: str):
        """Add the choices of autotune_export text to this context (varsim_autotune_import)."""
        self._check(self.lib.varsim_autotune_import(self.handle, text.encode()))

    # -------------------------------------------------------------------------------- timing
    def set_timing(self, enable: bool):
        self._check(self.lib.varsim_set_timing(self.handle, 1 if enable else 0))

    def reset_timing(self):
        self._check(self.lib.varsim_reset_timing(self.handle))

    def set_timing_only(self, kernel_class: str | None):
        """Time only `kernel_class` (None: every class)."""
        self._check(self.lib.varsim_set_timing_only(self.handle, kernel_class.encode() if kernel_class else None))

    def kernel_times(self) -> dict:
        cap = 256
        names = (c_char_p * cap)()
        counts = (c_int64 * cap)()
        tot = (c_double * cap)()
        n = c_int32(cap)
        self._check(self.lib.varsim_kernel_times(self.handle, names, counts, tot, ctypes.byref(n)))
        return {names[i].decode(): {"count": counts[i], "total_ms": tot[i]} for i in range(n.value)}


def stats_from_bytes(buf, n: int):
    """Per-problem statistics written by solve_batch(stats_out=...) (a tensor or bytes) as a
    numpy structured array."""
    import numpy as np

    raw = bytes(buf.cpu().numpy().tobytes()) if hasattr(buf, "cpu") else bytes(buf)
    arr = (Stats * n).from_buffer_copy(raw[:n * ctypes.sizeof(Stats)])
    return np.ctypeslib.as_array(arr).copy()


class PreparedBatch:
    """ctypes descriptors of a batch of problems, built once (the tensors must stay alive)."""

    def __init__(self, ctx: "Context", items: list[dict]):
        self.ctx = ctx
        self.probs, self._keep = ctx._problems(items)
        self._items = items
        self.n = len(items)
        self.stats = (Stats * self.n)()
        self._ws = {}

    def workspace_bytes(self, opts: Options) -> int:
        key = bytes(opts)
        if key not in self._ws:
            self._ws[key] = self.ctx._ws_query(self.probs, self.n, opts)
        return self._ws[key]


# ------------------------------------------------------------------------------- surrogate
@dataclass
class NetSpec:
    """Configuration of the learned warm start (fields of varsim_net_config)."""
    n: int = 512
    width: tuple = (32, 48, 64, 96, 128)
    shift: tuple = (1.0, 0.0, 1.0)
    scale: tuple = (1.0, 1.0 / 0.73, 20.0)
    out_scale: float = 10.0
    k0: float = 150.0

    def param_shapes(self) -> list:
        """(name, shape) of every parameter tensor in the flat order of varsim.h."""
        w = self.width
        out = [("stem.w", (w[0], 48)), ("stem.b", (w[0],))]
        for l in range(5):
            cin = w[0] if l == 0 else w[l - 1]
            out += [(f"enc{l}a.w", (w[l], 3, 3, cin)), (f"enc{l}a.b", (w[l],)),
                    (f"enc{l}b.w", (w[l], 3, 3, w[l])), (f"enc{l}b.b", (w[l],))]
        for l in range(3, -1, -1):
            out += [(f"dec{l}.w", (w[l], 3, 3, w[l + 1] + w[l])), (f"dec{l}.b", (w[l],))]
        return out + [("head.w", (16, w[0])), ("head.b", (16,))]

    def he_init(self, seed: int = 0):
        """He-normal weights (fan-in; gain 1 for the linear head), zero biases: float32 flat vector."""
        import numpy as np

        rng = np.random.default_rng(seed)
        parts = []
        for name, shp in self.param_shapes():
            if name.endswith(".b"):
                parts.append(np.zeros(shp))
            else:
                fan_in = int(np.prod(shp[1:]))
                parts.append(rng.standard_normal(shp) * np.sqrt((1.0 if name.startswith("head") else 2.0) / fan_in))
        return np.concatenate([p.ravel() for p in parts]).astype(np.float32)

    def c_config(self) -> NetConfig:
        c = NetConfig()
        c.n = self.n
        for i in range(5):
            c.width[i] = self.width[i]
        for i in range(3):
            c.shift[i] = self.shift[i]
            c.scale[i] = self.scale[i]
        c.out_scale = self.out_scale
        c.k0_W_mK = self.k0
        return c


class Net:
    """The learned warm start on one context (parameters live on the device)."""

    def __init__(self, ctx: "Context", spec: NetSpec):
        self.ctx, self.spec = ctx, spec
        self.lib = ctx.lib
        h = c_void_p()
        ctx._check(self.lib.varsim_net_create(ctx.handle, ctypes.byref(spec.c_config()), ctypes.byref(h)))
        self.handle = h
        n = c_int64()
        ctx._check(self.lib.varsim_net_param_count(self.handle, ctypes.byref(n)))
        self.param_count = n.value

    def close(self):
        if self.handle:
            self.lib.varsim_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        """params: float32 device tensor [param_count] (the header's order)."""
        assert params.numel() == self.param_count and params.is_contiguous()
        self.ctx._check(self.lib.varsim_net_set_params(self.handle, _ptr(params), _stream()))

    def get_params(self):
        import torch

        out = torch.empty(self.param_count, dtype=torch.float32, device=torch.device("cuda", self.ctx.device))
        self.ctx._check(self.lib.varsim_net_get_params(self.handle, _ptr(out), _stream()))
        return out

    def workspace_bytes(self, batch: int, training: bool) -> int:
        n = c_size_t(0)
        self.ctx._check(self.lib.varsim_net_workspace_size(self.handle, batch, int(training), ctypes.byref(n)))
        return n.value

    def _ws(self, workspace, batch, training):
        import torch

        need = self.workspace_bytes(batch, training)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=torch.device("cuda", self.ctx.device))
        return workspace

    def forward(self, q, v, m, out, batch=None, sample_idx=None, workspace=None):
        """Predicted rise into out [batch][n][n] (float32 device tensors; v, m may be None)."""
        batch = batch or out.shape[0]
        workspace = self._ws(workspace, batch, False)
        self.ctx._check(self.lib.varsim_net_forward(self.handle, batch, _ptr(q), _ptr(v), _ptr(m), _ptr(sample_idx),
                                                    _ptr(out), _ptr(workspace), workspace.numel(), _stream()))
        return out

    def gradient(self, q, v, m, target, grad, loss, batch, sample_idx=None, workspace=None):
        workspace = self._ws(workspace, batch, True)
        self.ctx._check(self.lib.varsim_net_gradient(self.handle, batch, _ptr(q), _ptr(v), _ptr(m), _ptr(sample_idx),
                                                     _ptr(target), _ptr(grad), _ptr(loss), _ptr(workspace),
                                                     workspace.numel(), _stream()))

    def adam(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.ctx._check(self.lib.varsim_net_adam(self.handle, _ptr(grad), lr, beta1, beta2, eps, _stream()))


def nn_conv(ctx: "Context", op: int, k: int, a, b, out, bias=None, relu: bool = False, workspace=None):
    """One convolution layer op (varsim_nn_conv) on BF16 tensors stored as int16 / uint16 bits."""
    import torch

    if op == NN_WGRAD:
        batch, h, w, cin = a.shape
        cout = b.shape[-1]
    else:
        batch, h, w, c = a.shape
        cout, cin = b.shape[0], b.shape[-1]
    need = c_size_t(0)
    ctx._check(ctx.lib.varsim_nn_conv_workspace(op, k, batch, h, w, cin, cout, ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=a.device)
    ctx._check(ctx.lib.varsim_nn_conv(ctx.handle, op, k, batch, h, w, cin, cout, _ptr(a), _ptr(b), _ptr(bias),
                                      int(relu), _ptr(out), _ptr(workspace), workspace.numel(), _stream()))
    return out
