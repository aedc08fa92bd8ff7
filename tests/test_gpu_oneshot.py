"""GPU parity of the one-shot modified-Green's-function solve (Sec. IV-C: Eqs. detsol, randsol,
detrandsol) against the oracle's one-shot functions (through the C ABI).

Tolerances: FP64 max |dT_gpu - dT_oracle| <= 1e-9 * max dT_oracle; FP32 <= 0.05 K (and the
achieved level, 1e-4 K, as a regression bound)."""
import numpy as np
import pytest

import workloads as W
from oracle import oneshot as O
from oracle import steady as S
from tests._util import gpu_item, leak_code

pytestmark = pytest.mark.gpu

FP64_GATE_REL = 1e-9
FP32_GATE_K = 0.05
FP32_ACHIEVED_K = 1e-4


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2307_12119_amd import varsim as V

    c = V.Context(0, gpu_lib)
    yield c
    c.close()


def _opts(prec, inp, res=False, cond=None):
    from paper_2307_12119_amd import varsim as V

    return V.make_options(prec, leak_code(inp), inp.beta, 50, 1e-3, f64_residual=res,
                          cond=V.COND_SOURCE if cond is None else cond)


def _mu(inp):
    ql = inp.q_leak0 * (inp.leak_var if inp.leak_var is not None else 1.0)
    return float(np.mean(ql / (inp.cond_map if inp.cond_map is not None else 1.0)))


def _oracle(inp, mu, random_part):
    prob, _ = S.problem_from_inputs(inp)
    beta = 0.0 if inp.leak == "none" else inp.beta
    dT, _, _ = O.oneshot(prob, beta, mu, random_part)
    return dT, prob


@pytest.mark.parametrize("n", [16, 64, 128, 256])
@pytest.mark.parametrize("random_part", [False, True])
def test_oneshot_fp64_matches_oracle(ctx, n, random_part):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=3, n=n)
    mu = _mu(inp)
    ref, _ = _oracle(inp, mu, random_part)
    item = gpu_item(inp, torch.float64)
    st = ctx.solve_oneshot([item], _opts(V.F64, inp), mu, random_part)[0]
    got = item["dT_out"].cpu().numpy()
    print(f"oneshot FP64 {n}^2 random={random_part}: max rel err "
          f"{np.max(np.abs(got - ref)) / np.max(ref):.2e}", flush=True)
    assert st["status"] == V.OK and st["iterations"] == 0
    assert np.max(np.abs(got - ref)) <= FP64_GATE_REL * np.max(ref)
    assert st["dT_max_K"] == pytest.approx(float(np.max(ref)), rel=1e-9)
    assert st["hotspot_index"] == int(np.argmax(ref))
    assert st["dT_mean_K"] == pytest.approx(float(np.mean(ref)), rel=1e-9)


@pytest.mark.parametrize("random_part", [False, True])
def test_oneshot_fp32_matches_oracle(ctx, random_part):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=5, n=256)
    mu = _mu(inp)
    ref, _ = _oracle(inp, mu, random_part)
    item = gpu_item(inp, torch.float32)
    st = ctx.solve_oneshot([item], _opts(V.F32, inp), mu, random_part)[0]
    err = float(np.max(np.abs(item["dT_out"].cpu().numpy().astype(np.float64) - ref)))
    print(f"oneshot FP32 256^2 random={random_part}: max err {err:.2e} K", flush=True)
    assert st["status"] == V.OK
    assert err <= FP32_GATE_K
    assert err <= FP32_ACHIEVED_K


def test_oneshot_is_the_fixed_point_for_uniform_leakage(ctx):
    # Eq. detsol at alpha = 0: linear leakage of uniform density, constant k -- the one-shot rise
    # equals the converged loop (the GPU's own iterative solve, FP64)
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.steady_problem(2, 128, 64, floorplan=2, variation=False)
    inp.q_leak0 = np.full_like(inp.q_dyn, 0.4e6)
    inp.leak = "linear"
    inp.beta = 0.0275
    one, it = gpu_item(inp, torch.float64), gpu_item(inp, torch.float64)
    ctx.solve_oneshot([one], _opts(V.F64, inp), 0.4e6, True)
    st = ctx.solve_steady(it, V.make_options(V.F64, V.LEAK_LINEAR, 0.0275, 100, 1e-13))
    assert st["status"] == V.OK
    a, b = one["dT_out"].cpu().numpy(), it["dT_out"].cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(b)


def test_oneshot_residual_batch_and_warm_start(ctx):
    # a batch mixing sizes; the reported FP64 residual is the oracle's max |G(dT) - dT| at the
    # one-shot rise; as a warm start it converges to the cold-start fixed point in fewer steps
    import torch

    from paper_2307_12119_amd import varsim as V

    inps = [W.config2(sample=s, n=n) for s, n in ((0, 64), (1, 32), (2, 64))]
    mu = _mu(inps[0])
    items = [gpu_item(i, torch.float64) for i in inps]
    stats = ctx.solve_oneshot(items, _opts(V.F64, inps[0], res=True), mu, True)
    for inp, item, st in zip(inps, items, stats):
        ref, prob = _oracle(inp, mu, True)
        got = item["dT_out"].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= FP64_GATE_REL * np.max(ref)
        opts = S.Options(leak="exp", beta=inp.beta)
        again, _ = prob.map(got, opts)
        res = float(np.max(np.abs(again - got)))
        assert st["residual_f64_K"] == pytest.approx(res, rel=1e-6)
        # warm start from the one-shot rise
        cold = gpu_item(inp, torch.float64)
        warm = gpu_item(inp, torch.float64, dT_init=got)
        o = V.make_options(V.F64, V.LEAK_EXP, inp.beta, 50, 1e-9)
        sc, sw = ctx.solve_steady(cold, o), ctx.solve_steady(warm, o)
        assert sc["status"] == sw["status"] == V.OK
        assert sw["iterations"] < sc["iterations"]
        assert np.max(np.abs(cold["dT_out"].cpu().numpy() - warm["dT_out"].cpu().numpy())) <= 1e-8


def test_oneshot_argument_errors(ctx):
    import torch

    from paper_2307_12119_amd import varsim as V

    inp = W.config2(sample=0, n=32)
    item = gpu_item(inp, torch.float64)
    with pytest.raises(V.VarsimError) as e:
        ctx.solve_oneshot([item], _opts(V.F64, inp, cond=V.COND_TARGET), _mu(inp), True)
    assert e.value.status == V.ERR_UNSUPPORTED
    with pytest.raises(V.VarsimError) as e:
        ctx.solve_oneshot([item], _opts(V.F64, inp), -1.0, True)
    assert e.value.status == V.ERR_INVALID
    # beta mu t / k >= 1: no linearised fixed point
    with pytest.raises(V.VarsimError) as e:
        ctx.solve_oneshot([item], _opts(V.F64, inp), 1.0e9, True)
    assert e.value.status == V.ERR_RUNAWAY
