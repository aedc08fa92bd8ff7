"""The batched steady solve that allocates nothing (varsim_solve_batch_noalloc): its workspace is
the library's static device array, and its results must equal varsim_solve_batch's bitwise
(the same kernels and arithmetic), call after call, with a smaller batch following a larger one
in the same array."""
import numpy as np
import pytest

import workloads as W
from tests._util import die_of, gpu_item, leak_code

pytestmark = pytest.mark.gpu


def _opts(prec, inp, res):
    from paper_2307_12119_amd import varsim as V

    return V.make_options(prec, leak_code(inp), inp.beta, 50, 1e-3, f64_residual=res)


def _items(inps, dtype):
    return [gpu_item(inp, dtype) for inp in inps]


def _same(a, b):
    return [x["dT_out"].cpu().numpy() for x in a], [x["dT_out"].cpu().numpy() for x in b]


def test_noalloc_equals_batch_on_consecutive_calls(gpu_lib):
    import torch

    from paper_2307_12119_amd import varsim as V

    ctx = V.Context(0, gpu_lib)
    try:
        assert ctx.noalloc_scratch_bytes() == 32 << 20
        calls = [
            # two 256^2 FP32 maps with both variation maps, k(T) and the FP64 residual ...
            ([W.config2(sample=s, n=256) for s in (0, 1)], torch.float32, True),
            # ... then a smaller batch in the same array: one 128^2 FP32 map (LDS-resident path)
            ([W.config2(sample=2, n=128)], torch.float32, True),
            # ... and one 64^2 FP64 map of the small-die family
            ([W.config1(3, n=64)], torch.float64, False),
        ]
        for inps, dtype, res in calls:
            prec = V.F64 if dtype == torch.float64 else V.F32
            opts = _opts(prec, inps[0], res)
            for inp in inps:  # the no-allocation call needs the geometry's cached table
                ctx.green_table(die_of(inp), inp.n)
            ref_items, got_items = _items(inps, dtype), _items(inps, dtype)
            # fill the outputs with garbage first: the solve must not read them
            for it in got_items:
                it["dT_out"].fill_(float("nan"))
            ref_stats = ctx.solve_batch(ref_items, opts)
            got_stats = ctx.solve_batch_noalloc(got_items, opts)
            torch.cuda.synchronize()
            print(f"noalloc: {len(inps)} x {inps[0].n}^2 {dtype}: iterations "
                  f"{[s['iterations'] for s in got_stats]}", flush=True)
            for r, g in zip(*_same(ref_items, got_items)):
                assert np.array_equal(r, g)
            for rs, gs in zip(ref_stats, got_stats):
                assert gs["status"] == V.OK
                for key in ("status", "iterations", "last_increment_K", "dT_max_K", "dT_mean_K", "hotspot_index"):
                    assert rs[key] == gs[key], key
                if res:
                    assert rs["residual_f64_K"] == gs["residual_f64_K"]
    finally:
        ctx.close()


def test_noalloc_rejects_uncached_geometry_and_oversized_batch(gpu_lib):
    import torch

    from paper_2307_12119_amd import varsim as V

    ctx = V.Context(0, gpu_lib)
    try:
        inp = W.config2(sample=0, n=256)
        opts = _opts(V.F32, inp, True)
        # no table for this geometry in a fresh context: refused before any launch
        with pytest.raises(V.VarsimError) as e:
            ctx.solve_batch_noalloc([gpu_item(inp, torch.float32)], opts)
        assert e.value.status == V.ERR_INVALID and "varsim_green_table" in str(e.value)
        # five 1024^2 FP64 maps with both variation maps need more than the static array
        big = W.config2(sample=0, n=1024)
        ctx.green_table(die_of(big), 1024)
        item = gpu_item(big, torch.float64)
        items = [dict(item, dT_out=torch.zeros_like(item["dT_out"])) for _ in range(5)]
        with pytest.raises(V.VarsimError) as e:
            ctx.solve_batch_noalloc(items, _opts(V.F64, big, False))
        assert e.value.status == V.ERR_NO_MEMORY and "static scratch" in str(e.value)
        for it in items:
            assert float(it["dT_out"].abs().max()) == 0.0  # nothing ran
    finally:
        ctx.close()
