"""Shared helpers of the GPU parity tests (imported only by tests marked gpu)."""
import sys

import numpy as np
import torch

import oracle
from paper_2204_07816_amd import inputs, nqs

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(spins):
    return torch.as_tensor(np.ascontiguousarray(spins, dtype=np.int8)).to(DEV)


def make_ctx(L, J2, K, C, w, dtype="fp64", J1=1.0, marshall=True):
    return nqs.Context(L, J1, J2, K, C, w, dtype=dtype, marshall_sign=marshall)


def oracle_item_dlog(L, K, C, w, spins, sample, bond):
    """f(S') - f(s) of one exchanged configuration, from two oracle forwards."""
    i, j, _ = oracle.bond_sites(L, int(bond))
    s = np.ascontiguousarray(spins[sample]).reshape(-1).copy()
    sp = s.copy()
    sp[i], sp[j] = s[j], s[i]
    f, _ = oracle.log_psi(L, K, C, w, np.stack([s, sp]).reshape(2, L, L))
    return f[1] - f[0]


def rel_inf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def graph_replays_equal_eager(ctx, w, start, n=3, **kw):
    """n eager VMC iterations from (w, start), then one iteration captured in a
    HIP graph and replayed n times from the same start with each iteration's
    random numbers staged: every replay must equal its eager iteration."""
    from paper_2204_07816_amd.vmc import VMC
    run = VMC(ctx, start.clone(), **kw)
    eager = [run.step() for _ in range(n)]
    w_eager, s_eager = run.weights, run.spins.clone()
    ctx.set_weights(w)
    run.spins.copy_(start)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run.stage(0)
        run.enqueue()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ctx.set_weights(w)
    run.spins.copy_(start)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run.enqueue()
    torch.cuda.synchronize()
    ctx.set_weights(w)
    run.spins.copy_(start)
    torch.cuda.synchronize()
    for it in range(n):
        run.stage(it)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st = run.stats()
        say("iteration", it, "graph", st["energy"], "eager", eager[it]["energy"])
        assert st["energy"] == eager[it]["energy"] and st["variance"] == eager[it]["variance"]
    assert np.array_equal(run.weights, w_eager)
    assert torch.equal(run.spins, s_eager)
    del g
