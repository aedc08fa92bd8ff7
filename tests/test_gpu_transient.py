"""GPU parity of the transient solve against the FP64 CPU oracle (through the C ABI).

Tolerances: FP64 max |dT_gpu - dT_oracle| <= 1e-9 * max dT_oracle over every recorded step;
FP32 max |dT_gpu - dT_oracle| <= 0.05 K.  At the full 1024 x 1024 size: the uniform-power
closed form, and the oracle's superposition evaluated at sampled cells with the power history
rebuilt from the recorded rises.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import steady as S
from oracle import transient as T
from tests._util import die_of, to_dev

pytestmark = pytest.mark.gpu

FP32_GATE_K = 0.05
FP64_GATE_REL = 1e-9


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2307_12119_amd import varsim as V

    c = V.Context(0, gpu_lib)
    yield c
    c.close()


def _tau_code(name):
    from paper_2307_12119_amd import varsim as V

    return {"moment": V.TAU_MOMENT, "lumped": V.TAU_LUMPED}[name]


def _leak_code(name):
    from paper_2307_12119_amd import varsim as V

    return {"exp": V.LEAK_EXP, "linear": V.LEAK_LINEAR, "none": V.LEAK_NONE}[name]


def _run_gpu(ctx, inp, dtype, out_every=1, tau="moment", leak="exp", cap=1000.0, snapshots=True, cond="source",
             history_steps=0):
    import torch
    from paper_2307_12119_amd import varsim as V

    n = inp.n
    prec = V.F64 if dtype == torch.float64 else V.F32
    item = {
        "die": die_of(inp),
        "q_leak0": to_dev(inp.q_leak0, dtype) if leak != "none" else None,
        "leak_var": to_dev(inp.leak_var, dtype),
        "cond_map": to_dev(inp.cond_map, dtype),
        "dT_out": torch.full((n, n), float("nan"), dtype=dtype, device="cuda"),
    }
    rects = to_dev(inp.block_rects, torch.int32)
    trace = to_dev(inp.trace, dtype)
    snaps = None
    if snapshots and inp.n_steps // out_every > 0:
        snaps = torch.full((inp.n_steps // out_every, n, n), float("nan"), dtype=dtype, device="cuda")
    opts = V.make_options(prec, _leak_code(leak), inp.beta, 1, 1e-3, cap=cap,
                          cond={"source": V.COND_SOURCE, "target": V.COND_TARGET}[cond])
    st = ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snapshots=snaps, out_every=out_every,
                             tau_model=_tau_code(tau), raise_on=(V.ERR_INVALID, V.ERR_UNSUPPORTED, V.ERR_DEVICE,
                                                                  V.ERR_NO_MEMORY), history_steps=history_steps)
    torch.cuda.synchronize()
    rec = None if snaps is None else snaps.cpu().numpy().astype(np.float64)
    return st, rec, item["dT_out"].cpu().numpy().astype(np.float64)


class _variants:
    """Pin the transient row / column pass candidates for the duration of a block (None: the
    library's own choice)."""

    def __init__(self, ctx, rv_cv):
        self.ctx, self.rv_cv = ctx, rv_cv

    def __enter__(self):
        if self.rv_cv is not None:
            self.ctx.force_transient_variant(*self.rv_cv)

    def __exit__(self, *exc):
        self.ctx.force_transient_variant(-1, -1)


def _oracle(inp, out_every=1, tau="moment", leak="exp", cond="source"):
    g = S.geometry_from_die(inp.die, inp.n)
    model = T.TransientModel(g, inp.die.rho_c, tau)
    steps = np.stack([W.raster_trace_step(inp.block_rects, inp.trace[k], inp.n) for k in range(inp.n_steps)])
    q_leak = None
    if leak != "none" and inp.q_leak0 is not None:
        q_leak = inp.q_leak0 * (inp.leak_var if inp.leak_var is not None else 1.0)
    return T.solve_transient(model, steps, inp.dt_s, q_leak=q_leak, cond_map=inp.cond_map, leak=leak,
                             beta=inp.beta, record_every=out_every, cond=cond)


CASES = [
    # n, steps, dt, variation, leak, tau, out_every
    (16, 30, 50e-6, False, "exp", "moment", 1),
    (16, 24, 100e-6, True, "exp", "lumped", 1),
    (32, 20, 50e-6, True, "exp", "moment", 3),
    (32, 16, 200e-6, True, "linear", "moment", 4),
    (64, 12, 100e-6, True, "exp", "moment", 1),
    (64, 10, 100e-6, False, "none", "lumped", 5),
    (128, 6, 100e-6, True, "exp", "moment", 2),
]


def _case_input(n, steps, dt, variation, seed=0):
    return W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=8 if n <= 32 else 24, hold_s=3 * dt,
                               seed=seed, variation=variation)


@pytest.mark.parametrize("n,steps,dt,variation,leak,tau,every", CASES)
def test_transient_fp64_matches_oracle(ctx, n, steps, dt, variation, leak, tau, every):
    import torch

    inp = _case_input(n, steps, dt, variation)
    ref, ref_last = _oracle(inp, every, tau, leak)
    st, rec, last = _run_gpu(ctx, inp, torch.float64, every, tau, leak)
    assert st["status"] == 0 and st["iterations"] == steps
    scale = max(np.max(np.abs(ref)), np.max(np.abs(ref_last)))
    assert scale > 0.1  # a meaningful rise
    assert rec.shape == ref.shape
    assert np.max(np.abs(rec - ref)) <= FP64_GATE_REL * scale
    assert np.max(np.abs(last - ref_last)) <= FP64_GATE_REL * scale
    assert st["dT_max_K"] == pytest.approx(float(np.max(ref_last)), rel=1e-9)
    assert st["hotspot_index"] == int(np.argmax(ref_last))
    assert st["dT_mean_K"] == pytest.approx(float(np.mean(ref_last)), rel=1e-9)


@pytest.mark.parametrize("rv_cv", [(0, 0), (3, 3)], ids=["pair", "one-row"])
@pytest.mark.parametrize("n,eta,cond", [(32, 1.3, "target"), (64, 1.3, "target"), (32, 1.0, "source"),
                                        (64, 1.0, "target")])
def test_transient_fp64_placement_and_eta_one(ctx, n, eta, cond, rv_cv):
    """The target-side conductivity factor and the eta = 1 Kirchhoff branch in both transient
    pass families, against the full-history oracle."""
    import torch

    inp = W.transient_problem(n=n, n_steps=12, dt_s=100e-6, n_blocks=8 if n <= 32 else 24, hold_s=3e-4, seed=5,
                              variation=True, eta=eta)
    ref, ref_last = _oracle(inp, 2, cond=cond)
    with _variants(ctx, rv_cv):
        st, rec, last = _run_gpu(ctx, inp, torch.float64, 2, cond=cond)
    assert st["status"] == 0
    scale = max(np.max(np.abs(ref)), np.max(np.abs(ref_last)))
    assert np.max(np.abs(rec - ref)) <= FP64_GATE_REL * scale
    assert np.max(np.abs(last - ref_last)) <= FP64_GATE_REL * scale


@pytest.mark.parametrize("n,steps,dt,variation,leak,tau,every", [CASES[0], CASES[2], CASES[4], CASES[6]])
def test_transient_fp32_matches_oracle(ctx, n, steps, dt, variation, leak, tau, every):
    import torch

    inp = _case_input(n, steps, dt, variation, seed=1)
    ref, ref_last = _oracle(inp, every, tau, leak)
    st, rec, last = _run_gpu(ctx, inp, torch.float32, every, tau, leak)
    assert st["status"] == 0
    assert np.max(np.abs(rec - ref)) <= FP32_GATE_K
    assert np.max(np.abs(last - ref_last)) <= FP32_GATE_K


# (row, column) pass candidates: two sequences per DFT (0) and one per half-length DFT (3..5)
ONE_ROW = [(3, 3), (4, 4), (5, 5), (3, 0), (0, 3)]


@pytest.mark.parametrize("rv_cv", ONE_ROW, ids=lambda v: f"row{v[0]}-col{v[1]}")
@pytest.mark.parametrize("case", [CASES[4], CASES[5], CASES[6]], ids=["64", "64-noleak-lumped", "128"])
def test_transient_one_row_passes_fp64_match_oracle(ctx, rv_cv, case):
    import torch

    n, steps, dt, variation, leak, tau, every = case
    inp = _case_input(n, steps, dt, variation)
    ref, ref_last = _oracle(inp, every, tau, leak)
    with _variants(ctx, rv_cv):
        st, rec, last = _run_gpu(ctx, inp, torch.float64, every, tau, leak)
    assert st["status"] == 0 and st["iterations"] == steps
    scale = max(np.max(np.abs(ref)), np.max(np.abs(ref_last)))
    assert np.max(np.abs(rec - ref)) <= FP64_GATE_REL * scale
    assert np.max(np.abs(last - ref_last)) <= FP64_GATE_REL * scale
    assert st["hotspot_index"] == int(np.argmax(ref_last))


def test_transient_one_row_passes_fp32_match_oracle(ctx):
    import torch

    n, steps, dt, variation, leak, tau, every = CASES[6]
    inp = _case_input(n, steps, dt, variation, seed=1)
    ref, ref_last = _oracle(inp, every, tau, leak)
    with _variants(ctx, (3, 3)):
        st, rec, last = _run_gpu(ctx, inp, torch.float32, every, tau, leak)
    assert st["status"] == 0
    assert np.max(np.abs(rec - ref)) <= FP32_GATE_K
    assert np.max(np.abs(last - ref_last)) <= FP32_GATE_K


@pytest.mark.parametrize("rv_cv", [(0, 0), (3, 3), (6, 6), (7, 7)], ids=["pair", "one-row", "split", "split-2"])
@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
@pytest.mark.parametrize("eta", [0.0, 1.3])
def test_transient_uniform_power_closed_form_1024(ctx, dtype_name, eta, rv_cv):
    """Uniform power excites only the uniform mode: theta_n = q t / k_ref (1 - exp(-n dt / tau(0))),
    tau(0) = t^2 rho c / (3 k_ref), and dT_n = Phi^-1(theta_n) in every cell."""
    import torch

    dtype = getattr(torch, dtype_name)
    n, steps, dt, q = 1024, 40, 100e-6, 2.0e6
    die = W.Die(eta=eta)
    inp = W.TransientInputs(die, n, dt, steps, np.array([[0, 0, n, n]], np.int32), np.full((steps, 1), q), None,
                            None, None)
    with _variants(ctx, rv_cv):
        st, rec, last = _run_gpu(ctx, inp, dtype, out_every=1, leak="none")
    assert st["status"] == 0
    k_ref = die.k0 * (die.t_amb / 300.0) ** (-eta)
    tau0 = die.t_m ** 2 * die.rho_c / (3.0 * k_ref)
    theta = q * die.t_m / k_ref * -np.expm1(-(np.arange(steps) + 1) * dt / tau0)
    expect, ok = S.kirchhoff_inverse(theta, die.t_amb, eta)
    assert np.all(ok)
    tol = 1e-9 * expect[-1] if dtype == torch.float64 else 2e-3
    assert np.max(np.abs(rec - expect[:, None, None])) <= tol
    assert np.max(np.abs(last - expect[-1])) <= tol


def test_transient_long_time_reaches_steady_fixed_point(ctx):
    """Constant block powers held for many time constants: the lagged-leakage transient settles on
    the steady leakage + variation fixed point."""
    import torch

    n, steps, dt = 64, 150, 2e-3
    inp = W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=16, hold_s=1.0, seed=3)
    inp.trace[:] = inp.trace[0]
    _, _, last = _run_gpu(ctx, inp, torch.float64, out_every=steps, snapshots=False)
    g = S.geometry_from_die(inp.die, n)
    q_dyn = W.raster_trace_step(inp.block_rects, inp.trace[0], n)
    prob = S.SteadyProblem(g, q_dyn, inp.q_leak0, inp.leak_var, inp.cond_map)
    opts = S.Options(leak="exp", beta=inp.beta, max_iter=200, tol=1e-12)
    ref, stat = S.solve_steady(prob, opts)
    assert stat.status == S.Status.OK
    assert np.max(np.abs(last - ref)) <= 1e-9 * np.max(ref)


@pytest.mark.parametrize("rv_cv", [(0, 0), (3, 3), (4, 5), (6, 6), (7, 7), (6, 4)],
                         ids=["pair", "one-row", "one-row-narrow", "split", "split-2", "split-row-one-row-col"])
def test_transient_full_size_sampled(ctx, rv_cv):
    """1024 x 1024, FP32, leakage + variation: at sampled cells the recorded rise of the last step
    equals the oracle's superposition of the power history rebuilt from the recorded rises."""
    import torch

    n, steps, dt = 1024, 10, 50e-6
    inp = W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=64, hold_s=2 * dt, seed=2)
    with _variants(ctx, rv_cv):
        st, rec, last = _run_gpu(ctx, inp, torch.float32, out_every=1)
    assert st["status"] == 0
    assert np.array_equal(rec[-1], last)
    g = S.geometry_from_die(inp.die, n)
    model = T.TransientModel(g, inp.die.rho_c)
    ql = inp.q_leak0 * inp.leak_var
    hist = [np.zeros((n, n))]
    prev = np.zeros((n, n))
    for k in range(steps):
        q = W.raster_trace_step(inp.block_rects, inp.trace[k], n) + ql * np.exp(inp.beta * prev)
        hist.append(g.hx * g.hy * q / inp.cond_map)  # conductivity factor on the source side
        prev = rec[k]
    rng = np.random.default_rng(11)
    hot = np.unravel_index(int(np.argmax(last)), last.shape)
    rows = np.concatenate([[0, n - 1, hot[0]], rng.integers(0, n, 12)])
    cols = np.concatenate([[0, n - 1, hot[1]], rng.integers(0, n, 12)])
    theta = np.zeros(len(rows))
    for j in range(1, steps + 1):
        op = S.DirectSum(g, table=model.step_kernel(j * dt))
        theta += op.apply_at(hist[steps - j + 1] - hist[steps - j], rows, cols)
    expect, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
    assert np.all(ok)
    assert np.max(np.abs(last[rows, cols] - expect)) <= FP32_GATE_K
    assert np.max(expect) > 1.0


def test_transient_split_passes_fp64_1024(ctx):
    """1024 x 1024, FP64, leakage + variation: the passes that spread each row (column) over two
    wavefronts (candidates 6, 7, alone and mixed with the one-wavefront passes) agree with the
    one-wavefront passes to rounding, also with two poles per mode and with a truncated history,
    and the last step equals the oracle's superposition at sampled cells to 1e-9 of the max rise."""
    import torch
    from paper_2307_12119_amd import varsim as V

    n, steps, dt = 1024, 8, 50e-6
    inp = W.transient_problem(n=n, n_steps=steps, dt_s=dt, n_blocks=64, hold_s=2 * dt, seed=5)

    def run(rv_cv, **kw):
        with _variants(ctx, rv_cv):
            st, rec, last = _run_gpu(ctx, inp, torch.float64, out_every=1, **kw)
        assert st["status"] == 0
        return rec, last

    base_rec, base = run((3, 3))
    scale = np.max(np.abs(base))
    for rv_cv in ((6, 6), (7, 7), (6, 3), (3, 7)):
        rec, last = run(rv_cv)
        assert np.max(np.abs(rec - base_rec)) <= 1e-12 * scale, rv_cv
    for kw in ({"history_steps": 4}, {"tau": "lumped"}):
        ref_rec, _ = run((3, 3), **kw)
        rec, _ = run((6, 6), **kw)
        assert np.max(np.abs(rec - ref_rec)) <= 1e-12 * np.max(np.abs(ref_rec)), kw
    # two poles per mode (the multi-pole model) through the binding's modal option
    item_kw = dict(n_poles=2)
    outs = []
    for rv_cv in ((3, 3), (6, 6)):
        dtype = torch.float64
        item = {"die": die_of(inp), "q_leak0": to_dev(inp.q_leak0, dtype), "leak_var": to_dev(inp.leak_var, dtype),
                "cond_map": to_dev(inp.cond_map, dtype), "dT_out": torch.zeros((n, n), dtype=dtype, device="cuda")}
        snaps = torch.zeros((steps, n, n), dtype=dtype, device="cuda")
        opts = V.make_options(V.F64, V.LEAK_EXP, inp.beta, 1, 1e-3)
        with _variants(ctx, rv_cv):
            st = ctx.solve_transient(item, to_dev(inp.block_rects, torch.int32), to_dev(inp.trace, dtype), dt, opts,
                                     snaps, 1, tau_model=V.TAU_MODAL, **item_kw)
        assert st["status"] == 0
        outs.append(snaps.cpu().numpy())
    assert np.max(np.abs(outs[1] - outs[0])) <= 1e-12 * np.max(np.abs(outs[0]))
    # the oracle's superposition at sampled cells, power history rebuilt from the split run
    rec, last = run((6, 6))
    g = S.geometry_from_die(inp.die, n)
    model = T.TransientModel(g, inp.die.rho_c)
    ql = inp.q_leak0 * inp.leak_var
    hist = [np.zeros((n, n))]
    prev = np.zeros((n, n))
    for k in range(steps):
        q = W.raster_trace_step(inp.block_rects, inp.trace[k], n) + ql * np.exp(inp.beta * prev)
        hist.append(g.hx * g.hy * q / inp.cond_map)
        prev = rec[k]
    rng = np.random.default_rng(12)
    hot = np.unravel_index(int(np.argmax(last)), last.shape)
    rows = np.concatenate([[0, n - 1, hot[0], 511, 512], rng.integers(0, n, 10)])
    cols = np.concatenate([[0, n - 1, hot[1], 512, 511], rng.integers(0, n, 10)])
    theta = np.zeros(len(rows))
    for j in range(1, steps + 1):
        op = S.DirectSum(g, table=model.step_kernel(j * dt))
        theta += op.apply_at(hist[steps - j + 1] - hist[steps - j], rows, cols)
    expect, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
    assert np.all(ok)
    assert np.max(np.abs(last[rows, cols] - expect)) <= FP64_GATE_REL * np.max(last)


def test_transient_statuses_and_edges(ctx):
    import torch
    from paper_2307_12119_amd import varsim as V

    # one step, no snapshots (out_every > n_steps)
    inp = _case_input(16, 1, 50e-6, True)
    ref, ref_last = _oracle(inp, 1)
    st, rec, last = _run_gpu(ctx, inp, torch.float64, out_every=5)
    assert st["status"] == V.OK and rec is None
    assert np.max(np.abs(last - ref_last)) <= FP64_GATE_REL * np.max(ref_last)
    # non-positive conductivity: INVALID
    bad = _case_input(16, 3, 50e-6, True)
    bad.cond_map[3, 4] = 0.0
    st, _, _ = _run_gpu(ctx, bad, torch.float64)
    assert st["status"] == V.ERR_INVALID
    # runaway: enormous leakage with a steep exponential law
    hot = _case_input(16, 40, 1e-3, True)
    hot.q_leak0 = hot.q_leak0 * 400.0
    st, _, _ = _run_gpu(ctx, hot, torch.float32, cap=500.0)
    assert st["status"] == V.ERR_RUNAWAY
    assert st["hotspot_index"] == -1
    # argument errors raise
    good = _case_input(16, 3, 50e-6, False)
    with pytest.raises(V.VarsimError):
        bad_dt = W.TransientInputs(good.die, 16, -1.0, 3, good.block_rects, good.trace, None, None, None)
        _run_gpu(ctx, bad_dt, torch.float64)
    with pytest.raises(V.VarsimError):
        _run_gpu(ctx, _case_input(24, 3, 50e-6, False), torch.float64)  # not a power of two


@pytest.mark.parametrize("n", [32, 256])
def test_transient_launch_shapes_give_identical_results(ctx, n):
    """Launch shapes of one transform family compute the same arithmetic (identical FP32 bits);
    the two families (two sequences per DFT, one per half-length DFT) agree to FP64 rounding and
    may be mixed between the row and column passes."""
    import torch

    inp = _case_input(n, 6, 100e-6, True)

    def run(rv_cv, dtype):
        with _variants(ctx, rv_cv):
            st, rec, last = _run_gpu(ctx, inp, dtype, out_every=2)
        assert st["status"] == 0
        return rec, last

    pair = [run((v, v), torch.float32) for v in range(3)]
    for rec, last in pair[1:]:
        assert np.array_equal(rec, pair[0][0]) and np.array_equal(last, pair[0][1])
    # the force_col_variant switch also pins the transient candidates 0..2
    try:
        ctx.force_col_variant(2)
        st, rec, last = _run_gpu(ctx, inp, torch.float32, out_every=2)
    finally:
        ctx.force_col_variant(-1)
    assert np.array_equal(last, pair[0][1])
    one = [run((v, w), torch.float32) for v, w in ((3, 3), (4, 4), (5, 5), (3, 5))]
    for rec, last in one[1:]:
        assert np.array_equal(rec, one[0][0]) and np.array_equal(last, one[0][1])
    if n < 64:  # no one-row passes below 64: the request falls back to candidate 0
        assert np.array_equal(one[0][1], pair[0][1])
    f64 = [run(v, torch.float64)[1] for v in ((0, 0), (3, 3), (3, 0), (0, 3))]
    scale = np.max(np.abs(f64[0]))
    for last in f64[1:]:
        assert np.max(np.abs(last - f64[0])) <= 1e-12 * scale
    assert np.max(np.abs(one[0][1] - pair[0][1])) <= 1e-4 * scale


# ----------------------------------------------------------------------------- multi-pole model
@pytest.mark.parametrize("n,poles,rv_cv", [(32, 3, None), (64, 4, (3, 3)), (64, 4, (0, 0)), (64, 2, (4, 5))])
def test_transient_modal_fp64_matches_oracle(ctx, n, poles, rv_cv):
    """The multi-pole ("modal") model: each cosine mode's slowest depth modes as separate poles
    with their own spectral states, through both pass families, against the oracle's
    full-history superposition of the same model."""
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.transient_problem(n=n, n_steps=12, dt_s=50e-6, n_blocks=8, hold_s=200e-6, seed=n + poles)
    g = S.geometry_from_die(inp.die, inp.n)
    model = T.TransientModel(g, inp.die.rho_c, "modal", n_poles=poles)
    steps = np.stack([W.raster_trace_step(inp.block_rects, inp.trace[k], inp.n) for k in range(inp.n_steps)])
    rec, _ = T.solve_transient(model, steps, inp.dt_s, q_leak=inp.q_leak0 * inp.leak_var, cond_map=inp.cond_map,
                               leak="exp", beta=inp.beta, record_every=2)
    item = {"die": die_of(inp), "q_leak0": to_dev(inp.q_leak0, torch.float64),
            "leak_var": to_dev(inp.leak_var, torch.float64), "cond_map": to_dev(inp.cond_map, torch.float64),
            "dT_out": torch.zeros((n, n), dtype=torch.float64, device="cuda")}
    snaps = torch.zeros((inp.n_steps // 2, n, n), dtype=torch.float64, device="cuda")
    opts = V.make_options(V.F64, V.LEAK_EXP, inp.beta, 1, 1e-3)
    with _variants(ctx, rv_cv):
        st = ctx.solve_transient(item, to_dev(inp.block_rects, torch.int32), to_dev(inp.trace, torch.float64),
                                 inp.dt_s, opts, snapshots=snaps, out_every=2, tau_model=V.TAU_MODAL, n_poles=poles)
    got = snaps.cpu().numpy()
    print(f"modal transient {n}^2, {poles} poles, variants {rv_cv}: max rel err "
          f"{np.max(np.abs(got - rec)) / np.max(rec):.2e}", flush=True)
    assert st["status"] == V.OK
    assert np.max(np.abs(got - rec)) <= FP64_GATE_REL * np.max(rec)


def test_transient_modal_one_pole_is_the_moment_model(ctx):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.transient_problem(n=64, n_steps=10, dt_s=50e-6, n_blocks=8, hold_s=200e-6, seed=3)
    outs = []
    for tau, poles in ((V.TAU_MOMENT, 1), (V.TAU_MODAL, 1)):
        item = {"die": die_of(inp), "q_leak0": to_dev(inp.q_leak0, torch.float32),
                "leak_var": to_dev(inp.leak_var, torch.float32), "cond_map": to_dev(inp.cond_map, torch.float32),
                "dT_out": torch.zeros((64, 64), dtype=torch.float32, device="cuda")}
        ctx.solve_transient(item, to_dev(inp.block_rects, torch.int32), to_dev(inp.trace, torch.float32), inp.dt_s,
                            V.make_options(V.F32, V.LEAK_EXP, inp.beta, 1, 1e-3), tau_model=tau, n_poles=poles)
        outs.append(item["dT_out"].cpu())
    assert torch.equal(outs[0], outs[1])


# ----------------------------------------------------------------------------- truncated history
@pytest.mark.parametrize("n,h,tau,poles,rv_cv", [(32, 4, "moment", 1, None), (64, 5, "moment", 1, (3, 3)),
                                                 (64, 3, "modal", 3, (0, 0)), (64, 7, "lumped", 1, (4, 5)),
                                                 (16, 2, "moment", 1, None)])
def test_transient_truncated_history_fp64_matches_oracle(ctx, n, h, tau, poles, rv_cv):
    """The paper's truncated history (step responses saturated from the h-th step on), kept on the
    GPU as a ring of the last h - 1 spectra, against the oracle's direct superposition."""
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.transient_problem(n=n, n_steps=14, dt_s=50e-6, n_blocks=8, hold_s=150e-6, seed=n + h)
    g = S.geometry_from_die(inp.die, inp.n)
    model = T.TransientModel(g, inp.die.rho_c, tau, n_poles=poles)
    steps = np.stack([W.raster_trace_step(inp.block_rects, inp.trace[k], inp.n) for k in range(inp.n_steps)])
    rec, _ = T.solve_transient(model, steps, inp.dt_s, q_leak=inp.q_leak0 * inp.leak_var, cond_map=inp.cond_map,
                               leak="exp", beta=inp.beta, horizon=h)
    item = {"die": die_of(inp), "q_leak0": to_dev(inp.q_leak0, torch.float64),
            "leak_var": to_dev(inp.leak_var, torch.float64), "cond_map": to_dev(inp.cond_map, torch.float64),
            "dT_out": torch.zeros((n, n), dtype=torch.float64, device="cuda")}
    snaps = torch.zeros((inp.n_steps, n, n), dtype=torch.float64, device="cuda")
    opts = V.make_options(V.F64, V.LEAK_EXP, inp.beta, 1, 1e-3)
    code = {"moment": V.TAU_MOMENT, "lumped": V.TAU_LUMPED, "modal": V.TAU_MODAL}[tau]
    with _variants(ctx, rv_cv):
        st = ctx.solve_transient(item, to_dev(inp.block_rects, torch.int32), to_dev(inp.trace, torch.float64),
                                 inp.dt_s, opts, snapshots=snaps, tau_model=code, n_poles=poles, history_steps=h)
    got = snaps.cpu().numpy()
    print(f"truncated history {n}^2, h {h}, {tau} ({poles} poles), variants {rv_cv}: max rel err "
          f"{np.max(np.abs(got - rec)) / np.max(rec):.2e}", flush=True)
    assert st["status"] == V.OK
    assert np.max(np.abs(got - rec)) <= FP64_GATE_REL * np.max(rec)


@pytest.mark.parametrize("rv_cv", [(0, 0), (3, 3), (6, 6)], ids=["pair", "one-row", "split"])
@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_transient_truncated_history_uniform_pulse_1024(ctx, dtype_name, rv_cv):
    """Uniform power on for 6 steps, then off, history cut at h = 9: the rise at step n is
    q R (s(n) - s(n - 6)), s(j) = 1 - exp(-j dt / tau(0)) below h, 1 from h on (0 for j <= 0), so
    it is exactly zero from step 6 + h on (eta = 0: dT = theta)."""
    import torch

    dtype = getattr(torch, dtype_name)
    n, steps, dt, q, on, h = 1024, 20, 100e-6, 2.0e6, 6, 9
    die = W.Die(eta=0.0)
    trace = np.zeros((steps, 1))
    trace[:on] = q
    inp = W.TransientInputs(die, n, dt, steps, np.array([[0, 0, n, n]], np.int32), trace, None, None, None)
    with _variants(ctx, rv_cv):
        st, rec, _ = _run_gpu(ctx, inp, dtype, out_every=1, leak="none", history_steps=h)
    assert st["status"] == 0
    tau0 = die.t_m ** 2 * die.rho_c / (3.0 * die.k0)
    R = die.t_m / die.k0

    def sat(j):
        return 0.0 if j <= 0 else (1.0 if j >= h else -math.expm1(-j * dt / tau0))

    expect = np.array([q * R * (sat(k + 1) - sat(k + 1 - on)) for k in range(steps)])
    tol = 1e-9 * q * R if dtype == torch.float64 else 2e-3
    assert np.max(np.abs(rec - expect[:, None, None])) <= tol
    assert np.max(np.abs(rec[on + h - 1:])) <= tol and np.max(np.abs(rec[on + h - 2])) > 0.01


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_transient_history_longer_than_the_run_is_the_full_history(ctx, dtype_name):
    """A history longer than the run never drops a term: the ring path returns the bits of the
    full-history recursion (every leaving spectrum is zero)."""
    import torch

    dtype = getattr(torch, dtype_name)
    inp = _case_input(64, 8, 50e-6, True, seed=4)
    _, full, _ = _run_gpu(ctx, inp, dtype)
    _, cut, _ = _run_gpu(ctx, inp, dtype, history_steps=9)
    assert np.array_equal(full, cut)


def test_transient_history_argument_errors(ctx):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = _case_input(16, 3, 50e-6, False)
    for h in (1, -2, (1 << 20) + 1):
        with pytest.raises(V.VarsimError) as e:
            _run_gpu(ctx, inp, torch.float64, history_steps=h)
        assert e.value.status == V.ERR_INVALID


def test_transient_autotune_picks_a_pair_and_matches_it(ctx):
    """With autotuning on, the first transient solve of a size times every (row, column) pass pair
    and keeps the fastest; the solve then equals the same pair forced, bit for bit."""
    import torch

    inp = _case_input(128, 6, 50e-6, True, seed=6)
    ctx.set_autotune(1)
    try:
        st, tuned, _ = _run_gpu(ctx, inp, torch.float32)
        line = [l for l in ctx.autotune_report().splitlines() if l.startswith("transient n=128 f32")]
    finally:
        ctx.set_autotune(-1)
    assert st["status"] == 0 and len(line) == 1
    rows = line[0].split(":", 1)[1].split(";")
    assert len(rows) == 6 and all(len(r.split(":")[1].split()) == 6 for r in rows)
    cells = [[v for v in r.split(":")[1].split()] for r in rows]
    # at n >= 64 the one-sequence pairs (candidates 3..5) are the ones timed
    assert all((v != "-") == (i >= 3 and j >= 3) for i, r in enumerate(cells) for j, v in enumerate(r))
    pick = [(i, j) for i, r in enumerate(cells) for j, v in enumerate(r) if v.endswith("*")]
    assert len(pick) == 1 and pick[0][0] >= 3 and pick[0][1] >= 3
    with _variants(ctx, pick[0]):
        _, forced, _ = _run_gpu(ctx, inp, torch.float32)
    assert np.array_equal(tuned, forced)
