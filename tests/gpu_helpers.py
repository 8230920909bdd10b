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


def bf16_weights(w, K, C):
    """The network the BF16 form evaluates: the 3x3 weights of layers 2..K
    rounded to BF16 (nearest even, from the FP64 value); layer 1 and every
    bias stay as given (those run in FP32, whose rounding the bound covers)."""
    w = np.array(w, np.float64)
    off = C * 9 + C
    for _ in range(K - 1):
        seg = w[off:off + C * C * 9]
        m, e = np.frexp(seg)
        w[off:off + C * C * 9] = np.ldexp(np.round(m * 256.0), e - 8)
        off += C * C * 9 + C
    return w


# Rounding-error model of the reduced-precision forms (first order):
#   activations of layers 1..K-1 rounded with relative error <= u_act
#   (BF16, nearest even: 2^-8; split hi + lo BF16: 2^-16);
#   each FP32 accumulation of z over n = 9C + 1 <= 289 terms: worst case
#   gamma_289 = 289 * 2^-24 / (1 - 289 * 2^-24) times a = |b| + sum |W||h|,
#   probabilistic sqrt(289) * 2^-24 * a;
#   ln cosh evaluated with relative error <= eta.
# Worst case:     u_act S1_act + gamma S1_acc + eta S1_lc
# Probabilistic:  6 sqrt((u_act S2_act)^2 + (sqrt(289) 2^-24 S2_acc)^2) + eta S1_lc
#   (independent, mean-zero rounding errors; Hoeffding's inequality puts the
#   chance of exceeding it at 2 exp(-18) per value).
U32 = 2.0 ** -24
GAMMA_289 = 289 * U32 / (1 - 289 * U32)


def rounding_bound(sens, u_act, eta, extra_rel=0.0):
    """Per-item bound (the smaller of the worst-case and the probabilistic one)
    from oracle.dlog_sens rows; extra_rel adds a relative error of the weights'
    representation on every accumulation (split weights: 2^-16 twice)."""
    s1a, s2a, s1z, s1l, s2z = sens[:, 1], sens[:, 2], sens[:, 3], sens[:, 4], sens[:, 5]
    worst = 1.05 * (u_act * s1a + (GAMMA_289 + extra_rel) * s1z + eta * s1l)
    prob = 6.0 * np.sqrt((u_act * s2a) ** 2 + ((np.sqrt(289.0) * U32 + extra_rel) * s2z) ** 2) \
        + eta * s1l
    return np.minimum(worst, prob)
