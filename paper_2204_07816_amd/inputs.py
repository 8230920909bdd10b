"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: it only draws random numbers.
The paper's inputs are MCMC samples of trained networks, which do not exist
here; they are replaced by

* spin configurations drawn uniformly from the Sz = 0 sector (each sample is a
  random permutation of N/2 up and N/2 down spins); for the t-J model,
  uniform over the configurations with the given number of holes and equally
  many up and down electrons (hole doping 1/8 in the named t-J workloads),
  and
* CNN weights and biases drawn i.i.d. from N(0, sigma^2) in canonical
  parameter order (layer by layer: W_k[co][ci][ky][kx], then b_k[co]).

Both come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import numpy as np


def num_params(K: int, C: int) -> int:
    """Parameter count of K 3x3 layers with C channels (layer 1 has one input channel)."""
    return (C * 9 + C) + (K - 1) * (C * C * 9 + C)


def weights(K: int, C: int, sigma: float, seed: int) -> np.ndarray:
    """FP64 canonical weight vector, i.i.d. N(0, sigma^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, sigma, size=num_params(K, C)).astype(np.float64)


def stress_weights(K: int, C: int, gain: float, seed: int, sigma1: float = 0.5) -> np.ndarray:
    """Larger-signal weights: layer 1 ~ N(0, sigma1^2), layer k > 1 ~ N(0, gain^2/(9 C)),
    zero biases.  Used to make the connected-configuration ratios differ from 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(K):
        cin = 1 if k == 0 else C
        sd = sigma1 if k == 0 else gain / np.sqrt(9.0 * cin)
        out.append(rng.normal(0.0, sd, size=C * cin * 9))
        out.append(np.zeros(C))
    return np.concatenate(out).astype(np.float64)


def cnn1_num_params(Kb: int, C: int) -> int:
    """Parameters of the CNN1 blocks: per block a 3x3 convolution c_in -> 2C
    with bias and a 3x3 transposed convolution C -> C with bias."""
    return sum(2 * C * (1 if k == 0 else C) * 9 + 2 * C + C * C * 9 + C for k in range(Kb))


def cnn1_weights(Kb: int, C: int, sigma: float, seed: int, out_bias: float = 0.0) -> np.ndarray:
    """CNN1 parameters, i.i.d. N(0, sigma^2) in canonical order (per block
    W, a, V, v), with out_bias added to every transposed-convolution bias v
    (out_bias = 1 keeps the output neurons near 1, away from the zeros of
    their product)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.normal(0.0, sigma, cnn1_num_params(Kb, C)).astype(np.float64)
    off = 0
    for k in range(Kb):
        off += 2 * C * (1 if k == 0 else C) * 9 + 2 * C + C * C * 9
        w[off:off + C] += out_bias
        off += C
    return w


def cnn2_num_params(Kb: int, C: int) -> int:
    """Parameters of CNN2: an embedding of 3 site states into C channels, per
    block two 3x3 convolutions C -> C with biases, and a final 3x3
    convolution C -> 1 with a bias."""
    return 3 * C + Kb * (18 * C * C + 2 * C) + 9 * C + 1


def cnn2_weights(Kb: int, C: int, gain: float, seed: int, out_bias: float = 0.0) -> np.ndarray:
    """CNN2 parameters in canonical order (E; per block W, a, V, v; F, b):
    the embedding N(0, 1), every 3x3 tap N(0, gain^2 / (9C)) (fan-in scaled),
    the biases N(0, 0.1^2), and out_bias added to the final bias (out_bias
    of a few units keeps the output neurons away from the zeros of their
    product)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    taps = gain / np.sqrt(9.0 * C)
    out = [rng.normal(0.0, 1.0, 3 * C)]
    for _ in range(Kb):
        out += [rng.normal(0.0, taps, 9 * C * C), rng.normal(0.0, 0.1, C),
                rng.normal(0.0, taps, 9 * C * C), rng.normal(0.0, 0.1, C)]
    out += [rng.normal(0.0, taps, 9 * C), rng.normal(0.0, 0.1, 1) + out_bias]
    w = np.concatenate(out).astype(np.float64)
    assert w.shape[0] == cnn2_num_params(Kb, C)
    return w


def spins_sz0(L: int, B: int, seed: int) -> np.ndarray:
    """int8 [B, L, L] configurations, uniform over the Sz = 0 sector."""
    N = L * L
    assert N % 2 == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.concatenate([np.ones(N // 2, np.int8), -np.ones(N // 2, np.int8)])
    out = np.empty((B, N), np.int8)
    for b in range(B):
        out[b] = rng.permutation(base)
    return out.reshape(B, L, L)


def spins_any(L: int, B: int, seed: int) -> np.ndarray:
    """int8 [B, L, L] configurations with i.i.d. +-1 spins (any magnetisation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.where(rng.random((B, L, L)) < 0.5, 1, -1).astype(np.int8)


def spins_tj(L: int, B: int, n_holes: int, seed: int) -> np.ndarray:
    """int8 [B, L, L] t-J configurations (+1 up electron, -1 down, 0 hole),
    uniform over those with n_holes holes and equally many up and down
    electrons."""
    N = L * L
    assert 0 <= n_holes <= N and (N - n_holes) % 2 == 0
    ne = (N - n_holes) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.concatenate([np.ones(ne, np.int8), -np.ones(ne, np.int8),
                           np.zeros(n_holes, np.int8)])
    out = np.empty((B, N), np.int8)
    for b in range(B):
        out[b] = rng.permutation(base)
    return out.reshape(B, L, L)


def neel(L: int) -> np.ndarray:
    y, x = np.mgrid[0:L, 0:L]
    return np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)


def column_stripe(L: int) -> np.ndarray:
    y, x = np.mgrid[0:L, 0:L]
    return np.where(x % 2 == 0, 1, -1).astype(np.int8)


def ferro(L: int) -> np.ndarray:
    return np.ones((L, L), np.int8)


# The workloads this library is checked and measured on (J1 = 1 throughout).
# "sigma" is the weight scale; seeds follow weights_seed = 1000 + index,
# spins_seed = 2000 + index.
CONFIGS = {
    "plain4": dict(index=0, L=4, J2=0.5, K=2, C=4, sigma=0.05, B=1024),
    "cmp10": dict(index=1, L=10, J2=0.5, K=4, C=16, sigma=0.02, B=8192),
    "mixed": dict(index=2, lattices=((12, 0.0), (16, 0.5), (20, 0.55)), K=6, C=32,
                  sigma=0.02, B=4096),
    "sr24": dict(index=3, L=24, J2=0.5, K=6, C=32, sigma=0.02, B=4096),
    "full36": dict(index=4, L=36, J2=0.5, K=8, C=32, sigma=0.02, B=1024),
}


# CNN1 workload: the 10x10 J1-J2 point (J2 = 0.5) of the paper's strong
# scaling runs, 6 blocks (the paper's block count) of 16 channels; weights
# seed 1200, spins seed 2200.
CNN1_CONFIG = dict(L=10, J2=0.5, blocks=6, C=16, sigma=0.05, out_bias=1.0, B=1024)


def cnn1_config_inputs(B: int | None = None):
    """(L, J2, blocks, C, weights, spins) of the CNN1 workload."""
    cfg = CNN1_CONFIG
    nb = cfg["B"] if B is None else B
    w = cnn1_weights(cfg["blocks"], cfg["C"], cfg["sigma"], 1200, cfg["out_bias"])
    return cfg["L"], cfg["J2"], cfg["blocks"], cfg["C"], w, spins_sz0(cfg["L"], nb, 2200)


# CNN1 on 36x36 J1-J2 (J2 = 0.5), the paper's largest lattice for CNN1, same
# network and weight recipe as above; 128 configurations.
CNN1_36_CONFIG = dict(L=36, J2=0.5, blocks=6, C=16, sigma=0.05, out_bias=1.0, B=128)


def cnn1_36_config_inputs(B: int | None = None):
    """(L, J2, blocks, C, weights, spins) of the 36x36 CNN1 workload."""
    cfg = CNN1_36_CONFIG
    nb = cfg["B"] if B is None else B
    w = cnn1_weights(cfg["blocks"], cfg["C"], cfg["sigma"], 1210, cfg["out_bias"])
    return cfg["L"], cfg["J2"], cfg["blocks"], cfg["C"], w, spins_sz0(cfg["L"], nb, 2210)


# t-J workloads (t = 1, J = 0.4, hole doping 1/8, the parameters of the
# paper's t-J runs): seeds weights 1100 + index, spins 2100 + index.
TJ_CONFIGS = {
    "tj8": dict(index=0, L=8, t=1.0, J=0.4, n_holes=8, K=4, C=16, sigma=0.02, B=2048),
    "tj12": dict(index=1, L=12, t=1.0, J=0.4, n_holes=18, K=6, C=32, sigma=0.02, B=4096),
}


# CNN2 t-J workload: 12x12 (the paper's largest t-J lattice), t = 1, J = 0.4,
# hole doping 1/8, CNN2 with 6 blocks of 32 channels (P = 111,361; the
# paper's CNN2 has 113,815); weights seed 1300, configurations seed 2300.
CNN2_TJ_CONFIG = dict(L=12, t=1.0, J=0.4, n_holes=18, blocks=6, C=32, gain=1.0, out_bias=2.0,
                      B=1024)


def cnn2_tj_config_inputs(B: int | None = None):
    """(L, t, J, blocks, C, weights, configurations) of the CNN2 t-J workload."""
    cfg = CNN2_TJ_CONFIG
    nb = cfg["B"] if B is None else B
    w = cnn2_weights(cfg["blocks"], cfg["C"], cfg["gain"], 1300, cfg["out_bias"])
    s = spins_tj(cfg["L"], nb, cfg["n_holes"], 2300)
    return cfg["L"], cfg["t"], cfg["J"], cfg["blocks"], cfg["C"], w, s


def tj_config_inputs(name: str, B: int | None = None):
    """(L, t, J, K, C, weights, configurations) of a named t-J workload."""
    cfg = TJ_CONFIGS[name]
    idx = cfg["index"]
    nb = cfg["B"] if B is None else B
    w = weights(cfg["K"], cfg["C"], cfg["sigma"], 1100 + idx)
    s = spins_tj(cfg["L"], nb, cfg["n_holes"], 2100 + idx)
    return cfg["L"], cfg["t"], cfg["J"], cfg["K"], cfg["C"], w, s


def config_inputs(name: str, B: int | None = None, lattice: int = 0):
    """(L, J2, K, C, weights, spins) of a named workload; B overrides the batch."""
    cfg = CONFIGS[name]
    idx = cfg["index"]
    if "lattices" in cfg:
        L, J2 = cfg["lattices"][lattice]
        sseed = 2000 + idx + 100 * (lattice + 1)
    else:
        L, J2 = cfg["L"], cfg["J2"]
        sseed = 2000 + idx
    nb = cfg["B"] if B is None else B
    w = weights(cfg["K"], cfg["C"], cfg["sigma"], 1000 + idx)
    s = spins_sz0(L, nb, sseed)
    return L, J2, cfg["K"], cfg["C"], w, s


def mcmc_randoms(seed: int, iteration: int, steps: int, B: int):
    """Random numbers of `steps` Metropolis steps of B chains for one
    iteration of a sampling loop: (proposal integers in [0, 2^31) int64
    [steps, B], uniforms in [0, 1) FP64 [steps, B]), from the stream seeded by
    (seed, iteration)."""
    rng = np.random.Generator(np.random.PCG64([seed, iteration]))
    return rng.integers(0, 2 ** 31, size=(steps, B)), rng.random((steps, B))
