"""GPU parity of the layered package (Table param's Si / TIM / spreader stack) with an isothermal
or convective bottom against the oracle's stack kernel (through the C ABI).

Tolerances: eigenvalues and convolution 1e-12 of their maxima; FP64 solves 1e-9 of the max
rise with equal iteration counts; FP32 0.05 K (achieved level 1e-4 K)."""
import numpy as np
import pytest
import scipy.fft as sfft

import workloads as W
from oracle import stack as ST
from oracle import steady as S
from tests._util import gpu_item, leak_code

pytestmark = pytest.mark.gpu

PKG = [(0.02e-3, 4.0, 0.0), (3.5e-3, 400.0, 0.0)]  # TIM, spreader under the silicon (Table param)
T_SI, K_SI = 0.15e-3, 130.0


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2307_12119_amd import varsim as V

    c = V.Context(0, gpu_lib)
    yield c
    c.close()


def _die(h, eta=0.0, lx=10e-3, ly=10e-3):
    from paper_2307_12119_amd import varsim as V

    return V.Die(lx, ly, T_SI, K_SI, eta, 318.0, 1.66e6, tuple(PKG), h)


def _layers(eta=0.0):
    kref = K_SI * (318.0 / 300.0) ** -eta
    return [(T_SI, kref)] + [(t, k) for t, k, _ in PKG]


def _oracle_problem(inp, h, eta):
    g = S.Geometry(inp.die.lx_m, inp.die.ly_m, inp.q_dyn.shape[1], inp.q_dyn.shape[0], T_SI, K_SI, eta, 318.0)
    table = ST.periodized_stack_table(g.nx, g.ny, g.lx, g.ly, _layers(eta), h)
    return S.SteadyProblem(g, inp.q_dyn, inp.q_leak0, inp.leak_var, inp.cond_map, S.DirectSum(g, table=table))


def _item(inp, die, dtype):
    it = gpu_item(inp, dtype)
    it["die"] = die
    return it


@pytest.mark.parametrize("h", [None, 2e4])
@pytest.mark.parametrize("nx,ny", [(64, 64), (32, 64)])
def test_stack_eigenvalues_and_conv_match_oracle(ctx, h, nx, ny):
    import torch

    die = _die(h, lx=10e-3, ly=10e-3 * ny / nx)
    kper, lam = ctx.green_table(die, nx, ny)
    assert kper is None
    table = ST.periodized_stack_table(nx, ny, die.lx_m, die.ly_m, _layers(), h)
    lam_ref = sfft.dct(sfft.dct(table, type=1, axis=0), type=1, axis=1)[:ny, :nx]
    assert np.max(np.abs(lam.cpu().numpy() - lam_ref)) <= 1e-12 * np.max(np.abs(lam_ref))
    g = S.Geometry(die.lx_m, die.ly_m, nx, ny, T_SI, K_SI, 0.0, 318.0)
    p = np.random.default_rng(nx + ny).uniform(0.0, 1e-2, (ny, nx))
    theta = ctx.conv(die, torch.from_numpy(p).cuda()).cpu().numpy()
    want = S.DirectSum(g, table=table).apply(p)
    assert np.max(np.abs(theta - want)) <= 1e-12 * np.max(want)


@pytest.mark.parametrize("h", [None, 2e4])
def test_stack_fp64_solve_matches_oracle(ctx, h):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=4, n=64)
    eta = inp.die.eta
    prob = _oracle_problem(inp, h, eta)
    opts = S.Options(leak="exp", beta=inp.beta, tol=1e-9, max_iter=50)
    ref, rst = S.solve_steady(prob, opts, residual=False)
    item = _item(inp, _die(h, eta), torch.float64)
    st = ctx.solve_steady(item, V.make_options(V.F64, leak_code(inp), inp.beta, 50, 1e-9, f64_residual=True))
    got = item["dT_out"].cpu().numpy()
    print(f"stack FP64 64^2 h={h}: iterations {st['iterations']} (oracle {rst.iterations}), max rise "
          f"{np.max(ref):.3f} K, max rel err {np.max(np.abs(got - ref)) / np.max(ref):.2e}", flush=True)
    assert st["status"] == rst.status == V.OK and st["iterations"] == rst.iterations
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(ref)


def test_stack_uniform_power_series_resistance(ctx):
    import torch

    n, h = 128, 5e3
    die = _die(h)
    g = S.Geometry(die.lx_m, die.ly_m, n, n, T_SI, K_SI, 0.0, 318.0)
    p = torch.full((n, n), 1e6 * g.hx * g.hy, dtype=torch.float64, device="cuda")
    theta = ctx.conv(die, p).cpu().numpy()
    want = 1e6 * (sum(t / k for t, k in _layers()) + 1.0 / h)
    assert np.max(np.abs(theta - want)) <= 1e-12 * want


def test_stack_fp32_256_matches_oracle(ctx):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=6, n=256)
    h = 2e4
    prob = _oracle_problem(inp, h, inp.die.eta)
    ref, rst = S.solve_steady(prob, S.Options(leak="exp", beta=inp.beta, tol=1e-3, max_iter=50), residual=False)
    item = _item(inp, _die(h, inp.die.eta), torch.float32)
    st = ctx.solve_steady(item, V.make_options(V.F32, leak_code(inp), inp.beta, 50, 1e-3))
    err = float(np.max(np.abs(item["dT_out"].cpu().numpy().astype(np.float64) - ref)))
    print(f"stack FP32 256^2: iterations {st['iterations']} (oracle {rst.iterations}), max err {err:.2e} K",
          flush=True)
    assert st["status"] == V.OK and st["iterations"] == rst.iterations
    assert err <= 0.05 and err <= 1e-4


def test_stack_unsupported_and_invalid(ctx):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=0, n=64)
    item = _item(inp, _die(2e4), torch.float64)
    rects = torch.tensor([[0, 0, 8, 8]], dtype=torch.int32, device="cuda")
    trace = torch.ones((4, 1), dtype=torch.float64, device="cuda") * 1e6
    with pytest.raises(V.VarsimError) as e:
        ctx.solve_transient(item, rects, trace, 1e-5, V.make_options(V.F64, V.LEAK_EXP, 0.017, 1, 1e-3))
    assert e.value.status == V.ERR_UNSUPPORTED
    with pytest.raises(V.VarsimError) as e:  # a convective bottom needs h > 0
        ctx.solve_steady(_item(inp, _die(-1.0), torch.float64), V.make_options(V.F64, V.LEAK_EXP, 0.017, 5, 1e-3))
    assert e.value.status == V.ERR_INVALID
