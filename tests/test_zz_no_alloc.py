"""The allocation-free step VJP (nsc_step_vjp_noalloc, through the C ABI)
against nsc_step_vjp: two calls in a row on two contexts, the second on a
smaller grid (the shared static scratch then holds the first call's data),
each checked element by element; and a grid past the scratch size refused
before any device work."""
import math
import sys

import pytest
import torch

import oracle as O
from synthetic import direction

pytestmark = pytest.mark.gpu

LARGER = (0.71, 200.0, 0.0, 0.0, 1.0, 64, 32, 63, 2 * math.pi)   # 4 states: 24.8 MB
SMALLER = (0.71, 100.0, 0.0, 1.0e4, 0.7, 16, 8, 15, 2 * math.pi)  # heated, 0.5 MB
TOO_BIG = (0.71, 100.0, 0.0, 1.0e4, 0.7, 128, 64, 127, 2 * math.pi)  # 4 states: 266 MB


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(args, seed):
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd._lib import check
    from paper_1908_00587_amd.adjoint import step_stages_fused, step_vjp_fused
    p = O.Params(*args)
    ctx = nsc.Context(*args)
    ctx.set_timestep(dt=5e-4)
    sh = (p.F, p.N_r, p.M_theta, p.M_z)
    u = (O.base_state(p) + 1e-2 * direction(*sh, seed=seed)).cuda()
    ub_next = direction(*sh, seed=seed + 1).cuda()
    stages, _ = step_stages_fused(ctx, u)
    ref = step_vjp_fused(ctx, u, stages, ub_next)
    got = torch.full_like(u, float("nan"))
    ctx._sync_stream()
    check(ctx._L.nsc_step_vjp_noalloc(ctx._h, u.data_ptr(), stages.data_ptr(),
                                      ub_next.data_ptr(), got.data_ptr()),
          "nsc_step_vjp_noalloc")
    torch.cuda.synchronize()
    ctx.close()
    return ref.cpu(), got.cpu()


def test_noalloc_step_vjp_matches_two_calls_second_smaller():
    for name, args, seed in (("larger", LARGER, 61), ("smaller", SMALLER, 71)):
        _say("noalloc step vjp", name, args[5:8])
        ref, got = _pair(args, seed)
        assert torch.isfinite(got).all()
        # same kernels, same order, same inputs: the same bits
        err = float((got - ref).abs().max())
        _say("  max |noalloc - step_vjp| =", err)
        assert torch.equal(got, ref), err


def test_noalloc_step_vjp_rejects_states_past_the_scratch():
    import paper_1908_00587_amd as nsc
    from paper_1908_00587_amd._lib import NSC_ERR_ARG
    _say("noalloc step vjp size limit", TOO_BIG[5:8])
    ctx = nsc.Context(*TOO_BIG)
    u = ctx.empty()
    stages = torch.zeros((1,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    ub = torch.zeros_like(u)
    out = torch.zeros_like(u)
    rc = ctx._L.nsc_step_vjp_noalloc(ctx._h, u.data_ptr(), stages.data_ptr(), ub.data_ptr(),
                                     out.data_ptr())
    assert rc == NSC_ERR_ARG
    ctx.close()
