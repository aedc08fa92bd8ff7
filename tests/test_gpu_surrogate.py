"""GPU parity of the learned warm start's kernels against the FP64 oracle (through the C ABI).

Layer ops take BF16 operands (exactly representable, so the oracle sees the same numbers) and
accumulate in FP32: |gpu - oracle| <= 2^-8 |oracle| (BF16 output rounding, forward only) +
1e-5 sum |w| |x| (FP32 accumulation).  The whole network rounds every activation to BF16, so
its output and gradient are compared in relative norm (3 % / 5 %) and direction.
"""
import numpy as np
import pytest

from oracle import surrogate as NN
from oracle import steady as S
import workloads as W
from tests._util import gpu_item, leak_code

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2307_12119_amd import varsim as V

    c = V.Context(0, gpu_lib)
    yield c
    c.close()


def _bf16(a):
    """Round to BF16 (nearest even) and back, as float64."""
    import torch

    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _dev_bf16(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(torch.bfloat16).contiguous()


def _conv1x1(x, w, b=None):
    z = x @ w[:, 0, 0, :].T
    return z + b if b is not None else z


CONV_CASES = [  # k, batch, h, w, cin, cout
    # W % 64 == 0 and H % 4 == 0 take the LDS-staged 3x3 path (input channels staged in phases of
    # at most 64: cin 80 and 112 take two; cin 16 pads the K chunk with staged zeros)
    (3, 2, 8, 64, 32, 32),
    (3, 1, 4, 128, 48, 48),
    (3, 2, 8, 64, 80, 64),
    (3, 1, 4, 64, 112, 48),
    (3, 1, 4, 64, 16, 16),
    (3, 2, 6, 64, 32, 32),
    (3, 2, 12, 12, 32, 32),
    # weight gradient: widths 8..128 (powers of two) whose rows fill 128-pixel steps take the
    # nine-tap kernel (here W = 32 with 16 outputs: one output block, four input blocks); H = 6
    # does not fill the steps and takes the per-tap kernel
    (3, 1, 8, 32, 64, 16),
    (3, 1, 6, 32, 32, 32),
    (3, 1, 8, 8, 48, 48),
    (3, 2, 16, 16, 64, 96),
    (3, 3, 5, 7, 16, 128),
    (3, 2, 8, 8, 224, 96),
    (3, 4, 2, 2, 96, 80),
    (1, 2, 16, 16, 64, 32),
    (1, 2, 16, 16, 32, 16),
]


@pytest.mark.parametrize("k,batch,h,w,cin,cout", CONV_CASES)
def test_nn_conv_forward(ctx, k, batch, h, w, cin, cout):
    import torch
    from paper_2307_12119_amd import varsim as V

    rng = np.random.default_rng(cin * 7 + cout)
    x = _bf16(rng.standard_normal((batch, h, w, cin)))
    wt = _bf16(rng.standard_normal((cout, k, k, cin)) / np.sqrt(k * k * cin))
    bias = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    out = torch.empty((batch, h, w, cout), dtype=torch.bfloat16, device="cuda")
    V.nn_conv(ctx, V.NN_FWD, k, _dev_bf16(x), _dev_bf16(wt), out,
              bias=torch.from_numpy(bias.astype(np.float32)).cuda(), relu=True)
    got = out.to(torch.float64).cpu().numpy()
    z = (NN.conv3x3(x, wt, bias) if k == 3 else _conv1x1(x, wt, bias))
    ref = NN.relu(z)
    scale = NN.conv3x3(np.abs(x), np.abs(wt)) if k == 3 else _conv1x1(np.abs(x), np.abs(wt))
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * (scale + np.abs(bias)))


@pytest.mark.parametrize("k,batch,h,w,cin,cout", CONV_CASES)
def test_nn_conv_dgrad_and_wgrad(ctx, k, batch, h, w, cin, cout):
    import torch
    from paper_2307_12119_amd import varsim as V

    rng = np.random.default_rng(cin * 11 + cout)
    x = _bf16(rng.standard_normal((batch, h, w, cin)))
    wt = _bf16(rng.standard_normal((cout, k, k, cin)) / np.sqrt(k * k * cin))
    dz = _bf16(rng.standard_normal((batch, h, w, cout)))
    dx = torch.empty((batch, h, w, cin), dtype=torch.float32, device="cuda")
    V.nn_conv(ctx, V.NN_DGRAD, k, _dev_bf16(dz), _dev_bf16(wt), dx)
    dw = torch.empty((cout, k, k, cin), dtype=torch.float32, device="cuda")
    V.nn_conv(ctx, V.NN_WGRAD, k, _dev_bf16(x), _dev_bf16(dz), dw)
    if k == 3:
        ref_dx, ref_dw = NN.conv3x3_dgrad(dz, wt), NN.conv3x3_wgrad(x, dz)
        sx, sw = NN.conv3x3_dgrad(np.abs(dz), np.abs(wt)), NN.conv3x3_wgrad(np.abs(x), np.abs(dz))
    else:
        ref_dx = dz @ wt[:, 0, 0, :]
        ref_dw = (dz.reshape(-1, cout).T @ x.reshape(-1, cin))[:, None, None, :]
        sx = np.abs(dz) @ np.abs(wt[:, 0, 0, :])
        sw = (np.abs(dz).reshape(-1, cout).T @ np.abs(x).reshape(-1, cin))[:, None, None, :]
    assert np.all(np.abs(dx.cpu().numpy() - ref_dx) <= 1e-5 * sx + 1e-30)
    assert np.all(np.abs(dw.cpu().numpy() - ref_dw) <= 1e-5 * sw + 1e-30)


# ----------------------------------------------------------------------------- network
def _net(ctx, spec_kw=None, seed=0):
    import torch
    from paper_2307_12119_amd import varsim as V

    spec = NN.NetSpec(**(spec_kw or {}))
    net = V.Net(ctx, V.NetSpec(spec.n, spec.width, spec.shift, spec.scale, spec.out_scale, spec.k0))
    assert net.param_count == spec.param_count()
    p = spec.init(seed)
    rng = np.random.default_rng(seed + 100)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    flat = spec.flatten(p).astype(np.float32)
    net.set_params(torch.from_numpy(flat).cuda())
    return net, spec, spec.unflatten(flat.astype(np.float64))


def _inputs(n, batch, seed=0):
    rng = np.random.default_rng(seed)
    q = (rng.uniform(0.1, 2.0, (batch, n, n)) * 1e6).astype(np.float32)
    v = np.exp(0.7 * rng.standard_normal((batch, n, n))).astype(np.float32)
    m = (1.0 + 0.05 * rng.uniform(-1, 1, (batch, n, n))).astype(np.float32)
    t = (5.0 + 3.0 * rng.standard_normal((batch, n, n))).astype(np.float32)
    return q, v, m, t


def _bf16_weights(spec, p):
    return {k: (_bf16(v) if k.endswith(".w") else v) for k, v in p.items()}


@pytest.mark.parametrize("n", [64, 256])
def test_net_forward_matches_oracle(ctx, n):
    """n = 256 puts level 0 (64 x 64) on the LDS-staged convolutions, the decoder's fused
    upsample + concatenation gather and the fused head included."""
    import torch

    net, spec, p = _net(ctx, {"n": n})
    q, v, m, _ = _inputs(n, 3)
    out = torch.empty((3, n, n), dtype=torch.float32, device="cuda")
    net.forward(*(torch.from_numpy(a).cuda() for a in (q, v, m)), out)
    got = out.cpu().numpy().astype(np.float64)
    ref, _ = NN.forward(spec, _bf16_weights(spec, p), q.astype(np.float64), v.astype(np.float64),
                        m.astype(np.float64))
    # every element within 2^-6 of the prediction's largest magnitude (measured: 6.9e-3 at n = 64,
    # 6.5e-3 at n = 256).  The kernels store each layer's activations in BF16; the FP32
    # accumulation of the matrix cores differs from FP64 by enough to flip the BF16 rounding of
    # activations wherever a pre-activation cancels, so even an oracle that rounds its own
    # activations to BF16 agrees no better (5.0e-3 and 7.1e-3) and agreement to FP32 is out of reach.
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"network forward n={n}: max |gpu - oracle| {err:.2e} of the largest magnitude")
    assert err <= 2.0 ** -6
    assert np.corrcoef(got.ravel(), ref.ravel())[0, 1] > 0.999


@pytest.mark.parametrize("n", [64, 256])
def test_net_gradient_matches_oracle(ctx, n):
    """Per parameter tensor: relative L2 distance <= 5 % and cosine >= 0.998 against the FP64
    oracle.  The bound is on whole tensors: with BF16 activations and output-side gradients, an
    element of a deep layer's weight gradient sums over few pixels (2 x 2 at level 3 of a 64 x 64
    map) whose ReLU masks and BF16 roundings can differ from FP64's, so single elements move by up
    to 15 % of their tensor's largest (measured; an oracle rounding its own activations and
    gradients to BF16 agrees no better elementwise)."""
    import torch

    net, spec, p = _net(ctx, {"n": n}, seed=1)
    q, v, m, t = _inputs(n, 2, seed=1)
    grad = torch.empty(net.param_count, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    dq, dv, dm, dt = (torch.from_numpy(a).cuda() for a in (q, v, m, t))
    net.gradient(dq, dv, dm, dt, grad, loss, batch=2)
    g_gpu = spec.unflatten(grad.cpu().numpy().astype(np.float64))
    L, g_ref, _ = NN.loss_and_grads(spec, _bf16_weights(spec, p), q.astype(np.float64), v.astype(np.float64),
                                    m.astype(np.float64), t.astype(np.float64))
    assert float(loss.item()) == pytest.approx(L, rel=0.02)
    for k in spec.shapes():
        a, b = g_gpu[k].ravel(), g_ref[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        assert rel <= 0.05 and cos >= 0.998, (k, rel, cos)
    # the sample index selects maps: reversed order, same gradient
    idx = torch.tensor([1, 0], dtype=torch.int32, device="cuda")
    grad2 = torch.empty_like(grad)
    net.gradient(dq, dv, dm, dt, grad2, loss, batch=2, sample_idx=idx)
    assert float(torch.linalg.norm(grad - grad2) / torch.linalg.norm(grad)) <= 1e-4


def test_net_adam_matches_oracle(ctx):
    import torch

    net, spec, p = _net(ctx, {"n": 64}, seed=2)
    rng = np.random.default_rng(3)
    opt = NN.Adam(lr=1e-3)
    ref = {k: v.copy() for k, v in p.items()}
    for _ in range(3):
        g = rng.standard_normal(net.param_count).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), 1e-3)
        opt.step(ref, spec.unflatten(g.astype(np.float64)))
    got = net.get_params().cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - spec.flatten(ref))) <= 1e-6


def test_training_reduces_loss(ctx):
    """A few Adam steps on one batch of method-generated maps lower the MSE."""
    import torch
    from paper_2307_12119_amd import varsim as V

    n, batch = 64, 4
    net, spec, _ = _net(ctx, {"n": n}, seed=4)
    inps = [W.config2(sample=i, n=n) for i in range(batch)]
    q = torch.from_numpy(np.stack([i.q_dyn for i in inps]).astype(np.float32)).cuda()
    v = torch.from_numpy(np.stack([i.leak_var for i in inps]).astype(np.float32)).cuda()
    m = torch.from_numpy(np.stack([i.cond_map for i in inps]).astype(np.float32)).cuda()
    items = [gpu_item(i, torch.float32) for i in inps]
    opts = V.make_options(V.F32, leak_code(inps[0]), inps[0].beta, 50, 1e-4)
    ctx.solve_batch(items, opts)
    t = torch.stack([it["dT_out"] for it in items])
    grad = torch.empty(net.param_count, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(net.workspace_bytes(batch, True), dtype=torch.uint8, device="cuda")
    losses = []
    for _ in range(40):
        net.gradient(q, v, m, t, grad, loss, batch, workspace=ws)
        losses.append(float(loss.item()))
        net.adam(grad, 3e-3)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]


def test_warm_start_reaches_cold_fixed_point(ctx):
    """Warm-started and cold-started solves converge to the same rise within the tolerance."""
    import torch
    from paper_2307_12119_amd import varsim as V

    n = 128
    net, spec, _ = _net(ctx, {"n": n}, seed=5)
    inp = W.config2(sample=3, n=n)
    cold = gpu_item(inp, torch.float32)
    opts = V.make_options(V.F32, leak_code(inp), inp.beta, 100, 1e-5)
    st_cold = ctx.solve_steady(cold, opts)
    init = torch.empty((1, n, n), dtype=torch.float32, device="cuda")
    net.forward(cold["q_dyn"], cold["leak_var"], cold["cond_map"], init)
    warm = gpu_item(inp, torch.float32)
    warm["dT_init"] = init[0]
    st_warm = ctx.solve_steady(warm, opts)
    assert st_cold["status"] == V.OK and st_warm["status"] == V.OK
    assert torch.max(torch.abs(warm["dT_out"] - cold["dT_out"])).item() <= 2e-4


def test_trained_network_gains_over_cold_start(ctx):
    """The committed trained weights, on held-out maps (floorplan 0, samples 0-15, never trained
    on): the prediction is within a fraction of a kelvin, the warm-started solve needs fewer
    iterations than the cold start, and both reach the same rise within the tolerance."""
    import os

    import torch
    from paper_2307_12119_amd import varsim as V

    path = os.path.join(os.path.dirname(V.__file__), "weights", "surrogate_512.npy")
    n, batch = 512, 16
    net = V.Net(ctx, V.NetSpec(n=n))
    net.set_params(torch.from_numpy(np.load(path)).cuda())
    inps = [W.config2(sample=i, n=n) for i in range(batch)]
    cold = [gpu_item(i, torch.float32) for i in inps]
    opts = V.make_options(V.F32, leak_code(inps[0]), inps[0].beta, 50, 1e-3)
    st_cold = ctx.solve_batch(cold, opts)
    q = torch.stack([c["q_dyn"] for c in cold])
    v = torch.stack([c["leak_var"] for c in cold])
    m = torch.stack([c["cond_map"] for c in cold])
    init = torch.empty_like(q)
    net.forward(q, v, m, init)
    warm = [dict(gpu_item(inp, torch.float32), dT_init=init[i]) for i, inp in enumerate(inps)]
    st_warm = ctx.solve_batch(warm, opts)
    ref = torch.stack([c["dT_out"] for c in cold])
    got = torch.stack([w["dT_out"] for w in warm])
    assert all(s["status"] == V.OK for s in st_cold + st_warm)
    it_cold = np.mean([s["iterations"] for s in st_cold])
    it_warm = np.mean([s["iterations"] for s in st_warm])
    assert it_warm < it_cold - 1.0
    assert float((init - ref).abs().mean()) < 0.1
    assert float((got - ref).abs().max()) <= 5e-3
