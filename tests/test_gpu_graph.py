"""The whole VMC step (E_loc, energy statistics, O_k, SR solve) captured once
in a HIP graph and replayed: every replay must reproduce the eagerly computed
outputs bit for bit (all kernels are deterministic), with the program's own
eager work and synchronizations between replays."""
import numpy as np
import pytest
import torch

from paper_2204_07816_amd import inputs
from gpu_helpers import make_ctx, say, to_dev

pytestmark = pytest.mark.gpu

GRAPH_CASES = [
    # unwrapped-window incremental kernel (BF16), stress weights so that the
    # outputs are far from trivial
    ("16x16 K6 C32 bf16 incremental", 16, 0.5, 6, 32, 48, "bf16", "incremental"),
    # wrapped-window incremental kernel
    ("10x10 K4 C16 bf16 incremental", 10, 0.5, 4, 16, 64, "bf16", "incremental"),
    # plain FP64 form (full recompute, FP64 matrix cores)
    ("8x8 K3 C16 fp64 full", 8, 0.5, 3, 16, 40, "fp64", "full"),
]


@pytest.mark.parametrize("name,L,J2,K,C,B,dtype,mode", GRAPH_CASES,
                         ids=[c[0] for c in GRAPH_CASES])
def test_graph_captured_step_replays_match_eager(name, L, J2, K, C, B, dtype, mode):
    say("case", name)
    w = inputs.stress_weights(K, C, 1.0, 41)
    sp = to_dev(inputs.spins_sz0(L, B, 42))
    ctx = make_ctx(L, J2, K, C, w, dtype=dtype)
    ctx.reserve(B, mode)
    dev = sp.device
    P = ctx.P
    e = torch.empty(B, dtype=torch.float64, device=dev)
    st2 = torch.empty(2, dtype=torch.float64, device=dev)
    O = torch.empty(B, P, dtype=torch.float32, device=dev)
    x = torch.empty(P, dtype=torch.float64, device=dev)
    st4 = torch.empty(4, dtype=torch.float64, device=dev)
    outs = (e, st2, O, x, st4)

    def step():
        ctx.local_energy(sp, mode=mode, out=e)
        ctx.energy_stats(e, out=st2)
        ctx.log_deriv(sp, dtype="fp32", out=O)
        ctx.sr_solve(O, e, 1e-4, 25, out=x, stats=st4)

    # eager reference (this also grows every workspace the step needs)
    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    assert torch.isfinite(ref[0]).all() and torch.isfinite(ref[3]).all()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:                     # eager work between replays
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, r in zip(outs, ref):
            assert torch.equal(a, r), f"replay {rep}: output differs from eager"
    say("  replays identical; E mean", float(ref[1][0]), "SR rel residual", float(ref[4][2]))
    assert ctx.get_error() == 0
    del g


def test_graph_captured_sampling_step_replays_match_eager():
    """Metropolis steps (cone write-back path at 16x16, K=6) captured with the
    rest of the step: with the chains reset to the same start before every
    replay, each replay reproduces the eager configurations and outputs."""
    L, J2, K, C, B, T = 16, 0.5, 6, 32, 48, 6
    w = inputs.stress_weights(K, C, 1.0, 44)
    start = to_dev(inputs.spins_sz0(L, B, 45))
    ctx = make_ctx(L, J2, K, C, w, dtype="bf16")
    rng = np.random.default_rng(46)
    rb = torch.tensor(rng.integers(0, 2 ** 31, size=(T, B)), dtype=torch.int32, device=start.device)
    ru = torch.tensor(rng.random((T, B)), device=start.device)
    sp = start.clone()
    acc = torch.zeros(B, dtype=torch.int32, device=sp.device)
    e = torch.empty(B, dtype=torch.float64, device=sp.device)
    O = torch.empty(B, ctx.P, dtype=torch.float32, device=sp.device)
    x = torch.empty(ctx.P, dtype=torch.float64, device=sp.device)
    st4 = torch.empty(4, dtype=torch.float64, device=sp.device)
    outs = (sp, acc, e, O, x, st4)

    def step():
        ctx.mcmc(sp, rb, ru, accepted=acc, mode="incremental")
        ctx.local_energy(sp, mode="incremental", out=e)
        ctx.log_deriv(sp, dtype="fp32", out=O)
        ctx.sr_solve(O, e, 1e-4, 25, out=x, stats=st4)

    def reset():
        sp.copy_(start)
        acc.zero_()

    step()                                  # grows every workspace
    reset()
    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    assert int(ref[1].sum()) > 0 and not torch.equal(ref[0], start)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        reset()
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        for t in outs[2:]:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, r in zip(outs, ref):
            assert torch.equal(a, r), f"replay {rep}: output differs from eager"
    say("  sampling step replays identical; accepted", int(ref[1].sum()))
    assert ctx.get_error() == 0
    del g
