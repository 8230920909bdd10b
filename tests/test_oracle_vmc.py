"""Pin of the oracle's VMC loop (Sec. 3.2 self-learning: sample |psi|^2,
local energies and log-derivatives, SR update): on the 4x4 Heisenberg point
(J2 = 0) the CNN energy approaches the exact ground energy from exact
diagonalisation (-11.2285), and the energy variance drops by an order of
magnitude."""
import numpy as np

from oracle import ed
from paper_2204_07816_amd import inputs


def test_vmc_converges_to_exact_ground_energy(orc):
    L, J2, K, C, B = 4, 0.0, 2, 4, 256
    H, _ = ed.hamiltonian(L, 1.0, J2)
    E0, _ = ed.lanczos_ground(H)
    w = inputs.weights(K, C, 0.05, 1)
    sp = inputs.spins_sz0(L, B, 2)
    means, variances, _, _ = orc.vmc(L, 1.0, J2, K, C, w, sp, 120, 16, 0.05, 1e-3, 100,
                                     lambda it: inputs.mcmc_randoms(5, it, 16, B))
    tail = means[-20:].mean()
    assert abs(tail - E0) < 3e-3 * abs(E0), (tail, E0)
    assert means[0] > E0 + 1.0                      # it started far away
    assert variances[-20:].mean() < 0.1 * variances[0]
