"""Pins of the oracle's Metropolis sampler (Sec. 3.2: walkers sample |psi|^2;
Sec. 5.4.1: independent chains, exchange proposals).

* Uniform amplitude (all weights zero): every antiparallel proposal is
  accepted, so the chains follow the exchanges a direct loop over the bond
  geometry (written here from x/y arithmetic) applies.
* Stationarity: chains started from uniform Sz = 0 configurations of 4x4 and
  run well past the mixing time give a mean local energy equal, within 5
  standard errors, to the exact |psi|^2-weighted mean over all 12,870 states
  (which the starting configurations miss by more than 20 standard errors).
* Sz is conserved and the random numbers decide reproducibly.
"""
import numpy as np

from oracle import ed
from paper_2204_07816_amd import inputs


def _pair(L, q, n, types):
    i = q // n
    t = types[q % n]
    x, y = i % L, i // L
    dx, dy = [(1, 0), (0, 1), (1, 1), (1, -1)][t]
    return i, ((y + dy) % L) * L + (x + dx) % L


def test_uniform_amplitude_accepts_every_exchange(orc):
    L, K, C, B, T = 6, 2, 4, 16, 25
    w = np.zeros(inputs.num_params(K, C))
    sp = inputs.spins_sz0(L, B, 3)
    rng = np.random.default_rng(4)
    rb = rng.integers(0, 2 ** 31, size=(T, B))
    ru = rng.random((T, B))
    for J2, types in ((0.5, [0, 1, 2, 3]), (0.0, [0, 1])):
        out, acc = orc.mcmc(L, 1.0, J2, K, C, w, sp, rb, ru)
        ref = sp.reshape(B, -1).copy()
        racc = np.zeros(B, np.int64)
        n = len(types)
        for t in range(T):
            for b in range(B):
                i, j = _pair(L, int(rb[t, b]) % (L * L * n), n, types)
                if ref[b, i] != ref[b, j]:
                    ref[b, i], ref[b, j] = ref[b, j], ref[b, i]
                    racc[b] += 1
        assert np.array_equal(out.reshape(B, -1), ref)
        assert np.array_equal(acc, racc)
        assert np.all(out.reshape(B, -1).sum(axis=1) == 0)      # Sz = 0 kept


def test_stationary_mean_energy_4x4(orc):
    L, K, C, J2 = 4, 2, 4, 0.5
    w = inputs.weights(K, C, 0.3, 11)
    H, basis = ed.hamiltonian(L, 1.0, J2)
    allsp = ed.basis_to_spins(basis, L * L).reshape(-1, L, L)
    la, _ = orc.log_psi(L, K, C, w, allsp)
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    e_all = orc.local_energy(L, 1.0, J2, K, C, w, allsp)
    exact = float(p @ e_all)
    B, T = 600, 600
    sp = inputs.spins_sz0(L, B, 12)
    rng = np.random.default_rng(13)
    out, acc = orc.mcmc(L, 1.0, J2, K, C, w, sp, rng.integers(0, 2 ** 31, size=(T, B)),
                        rng.random((T, B)))
    e = orc.local_energy(L, 1.0, J2, K, C, w, out)
    se = e.std(ddof=1) / np.sqrt(B)
    assert abs(e.mean() - exact) < 5 * se, (e.mean(), exact, se)
    # the starts (uniform over Sz = 0) are far from |psi|^2: without the
    # sampler the mean would miss by far more than the bar
    e0 = orc.local_energy(L, 1.0, J2, K, C, w, sp)
    assert abs(e0.mean() - exact) > 20 * se
    assert 0.02 < acc.mean() / T < 0.98
