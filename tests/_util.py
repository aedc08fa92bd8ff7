"""Helpers shared by the GPU tests: move seeded inputs to the device and run oracle solves."""
import numpy as np


def die_of(inp):
    from paper_2307_12119_amd import varsim as V

    d = inp.die
    return V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)


def to_dev(a, dtype):
    import torch

    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def gpu_item(inp, dtype, dT_init=None):
    """Dict of device tensors for Context.solve_* from a workloads.SteadyInputs."""
    import torch

    shape = inp.q_dyn.shape
    return {
        "die": die_of(inp),
        "q_dyn": to_dev(inp.q_dyn, dtype),
        "q_leak0": to_dev(inp.q_leak0, dtype) if inp.leak != "none" else None,
        "leak_var": to_dev(inp.leak_var, dtype),
        "cond_map": to_dev(inp.cond_map, dtype),
        "dT_init": to_dev(dT_init, dtype) if dT_init is not None else None,
        "dT_out": torch.zeros(shape, dtype=dtype, device="cuda"),
    }


def leak_code(inp):
    from paper_2307_12119_amd import varsim as V

    return {"exp": V.LEAK_EXP, "linear": V.LEAK_LINEAR, "none": V.LEAK_NONE}[inp.leak]


def oracle_solve(inp, tol, max_iter, init=None, operator=None, cond="source"):
    from oracle import steady as S

    prob, opts = S.problem_from_inputs(inp, operator)
    opts.tol, opts.max_iter, opts.cond = tol, max_iter, cond
    return S.solve_steady(prob, opts, init=init), prob
