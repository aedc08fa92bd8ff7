"""Fixed-point iterations launched as captured HIP graphs (varsim_set_graph_iterations) give the
same bits as direct launches: maps, statistics and statuses, over several calls that reuse and
rewrite the context's executable graphs, with direct-launch work between the calls."""
import ctypes
import math

import pytest

import workloads as W
from tests._util import gpu_item, leak_code

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    from paper_2307_12119_amd import varsim as V

    c = V.Context(0, gpu_lib)
    yield c
    c.close()


def _opts(prec, inp, max_iter, tol, res=False):
    from paper_2307_12119_amd import varsim as V

    return V.make_options(prec, leak_code(inp), inp.beta, max_iter, tol, f64_residual=res)


def _same_stats(a, b):
    """Bitwise equal statistics (the mean adds its per-workgroup partial sums in a fixed order)."""
    for k, v in a.items():
        assert b[k] == v or (v != v and b[k] != b[k]), (k, v, b[k])


def _solve(ctx, inps, opts, dtype):
    items = [gpu_item(i, dtype) for i in inps]
    return items, ctx.solve_batch(items, opts)


@pytest.mark.parametrize("chunk", [1, 2, 3])
def test_graph_chunks_equal_direct_launches(ctx, chunk):
    import torch
    from paper_2307_12119_amd import varsim as V

    inps = [W.steady_problem(3, n, 16, floorplan=i, sample=i) for i, n in enumerate([256, 512, 16, 256])]
    other = [W.steady_problem(3, n, 16, floorplan=9 + i, sample=9 + i) for i, n in enumerate([512, 256])]
    opts = _opts(V.F32, inps[0], 50, 1e-3, res=True)
    ctx.set_graph_iterations(0)
    ref_items, ref = _solve(ctx, inps, opts, torch.float32)
    assert all(s["status"] == V.OK for s in ref)
    for rep in range(3):
        ctx.set_graph_iterations(chunk)
        items, got = _solve(ctx, inps, opts, torch.float32)
        torch.cuda.synchronize()
        for r, g, a, b in zip(ref, got, ref_items, items):
            _same_stats(r, g)
            assert torch.equal(a["dT_out"], b["dT_out"]), (chunk, rep)
        # direct launches of another batch between the graph calls
        ctx.set_graph_iterations(0)
        _solve(ctx, other, opts, torch.float32)
    ctx.set_graph_iterations(0)


def test_graph_last_chunk_shorter_and_not_converged(ctx):
    """max_iter = 4 with 3 iterations per graph: the second chunk holds the last iteration
    alone; a tolerance no map reaches leaves every map NOT_CONVERGED after 4 iterations."""
    import torch
    from paper_2307_12119_amd import varsim as V

    inps = [W.steady_problem(3, 256, 16, floorplan=i, sample=i) for i in range(3)]
    for tol, status in ((1e-12, V.ERR_NOT_CONVERGED), (1e-3, None)):
        opts = _opts(V.F32, inps[0], 4, tol)
        ctx.set_graph_iterations(0)
        ref_items, ref = _solve(ctx, inps, opts, torch.float32)
        ctx.set_graph_iterations(3)
        items, got = _solve(ctx, inps, opts, torch.float32)
        ctx.set_graph_iterations(0)
        for r, g, a, b in zip(ref, got, ref_items, items):
            if status is not None:
                assert r["status"] == status and r["iterations"] == 4
            _same_stats(r, g)
            assert torch.equal(a["dT_out"], b["dT_out"])


def test_graph_fp64_two_pass(ctx):
    import torch
    from paper_2307_12119_amd import varsim as V

    inps = [W.config1(s, n=128) for s in range(2)]
    opts = _opts(V.F64, inps[0], 20, 1e-9)
    ctx.set_graph_iterations(0)
    ref_items, ref = _solve(ctx, inps, opts, torch.float64)
    ctx.set_graph_iterations(2)
    items, got = _solve(ctx, inps, opts, torch.float64)
    ctx.set_graph_iterations(0)
    for r, g, a, b in zip(ref, got, ref_items, items):
        assert r["status"] == V.OK
        _same_stats(r, g)
        assert torch.equal(a["dT_out"], b["dT_out"])


def test_graph_device_stats_back_to_back(ctx):
    """Calls with device-side statistics return after enqueue, so the second call rewrites
    executable graphs whose previous launch may still be queued: its results must still equal
    direct launches."""
    import torch
    from paper_2307_12119_amd import varsim as V

    sets = [[W.steady_problem(3, n, 16, floorplan=i + k, sample=i + k) for i, n in enumerate([256, 512, 256])]
            for k in (0, 5, 11)]
    opts = _opts(V.F32, sets[0][0], 50, 1e-3, res=True)
    ctx.set_graph_iterations(0)
    host = [_solve(ctx, inps, opts, torch.float32) for inps in sets]
    ctx.set_graph_iterations(2)
    dev_items = [[gpu_item(i, torch.float32) for i in inps] for inps in sets]
    bufs = [torch.zeros((len(inps) * ctypes.sizeof(V.Stats),), dtype=torch.uint8, device="cuda") for inps in sets]
    for items, buf in zip(dev_items, bufs):
        assert ctx.solve_batch(items, opts, stats_out=buf) is None
    torch.cuda.synchronize()
    ctx.set_graph_iterations(0)
    for (h_items, h), items, buf, inps in zip(host, dev_items, bufs, sets):
        got = V.stats_from_bytes(buf, len(inps))
        for hs, g, a, b in zip(h, got, h_items, items):
            assert hs["status"] == V.OK
            _same_stats(hs, g)
            assert torch.equal(a["dT_out"], b["dT_out"])


def test_graph_iterations_out_of_range(ctx):
    from paper_2307_12119_amd import varsim as V

    for bad in (-1, 17):
        with pytest.raises(V.VarsimError):
            ctx.set_graph_iterations(bad)
    ctx.set_graph_iterations(16)
    ctx.set_graph_iterations(0)


def test_two_streams_back_to_back(ctx):
    """Batches alternating between two streams with device-side statistics: each call returns
    once its iterations are read, so its residual passes overlap the next call on the other
    stream, which reuses the context's convergence words.  Every result equals the
    single-stream one."""
    import torch
    from paper_2307_12119_amd import varsim as V

    sets = [[W.steady_problem(3, n, 16, floorplan=i + k, sample=i + k) for i, n in enumerate([512, 256, 512])]
            for k in (0, 4, 8, 12)]
    opts = _opts(V.F32, sets[0][0], 50, 1e-3, res=True)
    host = [_solve(ctx, inps, opts, torch.float32) for inps in sets]
    streams = (torch.cuda.current_stream(), torch.cuda.Stream())
    dev_items = [[gpu_item(i, torch.float32) for i in inps] for inps in sets]
    bufs = [torch.zeros((len(inps) * ctypes.sizeof(V.Stats),), dtype=torch.uint8, device="cuda") for inps in sets]
    torch.cuda.synchronize()
    for k, (items, buf) in enumerate(zip(dev_items, bufs)):
        with torch.cuda.stream(streams[k & 1]):
            assert ctx.solve_batch(items, opts, stats_out=buf) is None
    torch.cuda.synchronize()
    for (h_items, h), items, buf, inps in zip(host, dev_items, bufs, sets):
        got = V.stats_from_bytes(buf, len(inps))
        for hs, g, a, b in zip(h, got, h_items, items):
            assert hs["status"] == V.OK
            _same_stats(hs, g)
            assert torch.equal(a["dT_out"], b["dT_out"])


def test_two_streams_with_graphs(ctx):
    """Graph-launched calls alternating between two streams: executable graph j is rewritten by
    each call after the previous call's launch of it (on the other stream) has finished."""
    import torch
    from paper_2307_12119_amd import varsim as V

    sets = [[W.steady_problem(3, n, 16, floorplan=i + k, sample=i + k) for i, n in enumerate([256, 512, 256])]
            for k in (1, 6, 10, 15)]
    opts = _opts(V.F32, sets[0][0], 50, 1e-3, res=True)
    ctx.set_graph_iterations(0)
    host = [_solve(ctx, inps, opts, torch.float32) for inps in sets]
    streams = (torch.cuda.current_stream(), torch.cuda.Stream())
    dev_items = [[gpu_item(i, torch.float32) for i in inps] for inps in sets]
    bufs = [torch.zeros((len(inps) * ctypes.sizeof(V.Stats),), dtype=torch.uint8, device="cuda") for inps in sets]
    torch.cuda.synchronize()
    ctx.set_graph_iterations(2)
    for k, (items, buf) in enumerate(zip(dev_items, bufs)):
        with torch.cuda.stream(streams[k & 1]):
            assert ctx.solve_batch(items, opts, stats_out=buf) is None
    torch.cuda.synchronize()
    ctx.set_graph_iterations(0)
    for (h_items, h), items, buf, inps in zip(host, dev_items, bufs, sets):
        got = V.stats_from_bytes(buf, len(inps))
        for hs, g, a, b in zip(h, got, h_items, items):
            assert hs["status"] == V.OK
            _same_stats(hs, g)
            assert torch.equal(a["dT_out"], b["dT_out"])
