"""The VMC self-learning loop on the GPU (paper_2204_07816_amd.vmc.VMC):
Metropolis steps, local energies, log-derivatives, SR and the weight update,
all through the C ABI.

* FP64: six iterations reproduce the oracle's loop fed the same random
  numbers (energies to 1e-9, weights to 1e-7 relative, the same samples).
* Convergence on the 4x4 Heisenberg point: the FP64 loop (C = 4) and the
  BF16 loop (C = 16) reach the exact-diagonalisation ground energy
  (-11.2285) within 0.3% and 1%.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ed
from paper_2204_07816_amd import inputs
from paper_2204_07816_amd.vmc import VMC
from gpu_helpers import make_ctx, say, to_dev

pytestmark = pytest.mark.gpu


def _e0():
    H, _ = ed.hamiltonian(4, 1.0, 0.0)
    return ed.lanczos_ground(H)[0]


def test_vmc_fp64_matches_oracle():
    L, J2, K, C, B, T = 4, 0.0, 2, 4, 128, 16
    w = inputs.weights(K, C, 0.05, 1)
    sp = inputs.spins_sz0(L, B, 2)
    ctx = make_ctx(L, J2, K, C, w)
    d = to_dev(sp)
    run = VMC(ctx, w, d, steps=T, lr=0.05, diag_shift=1e-3, cg_iters=100, seed=7)
    got = [run.step()["energy"] for _ in range(6)]
    means, _, w_ref, s_ref = oracle.vmc(L, 1.0, J2, K, C, w, sp, 6, T, 0.05, 1e-3, 100,
                                        lambda it: inputs.mcmc_randoms(7, it, T, B))
    say("energies gpu", got, "oracle", means)
    np.testing.assert_allclose(got, means, rtol=1e-9)
    np.testing.assert_allclose(run.w, w_ref, rtol=1e-7, atol=1e-12)
    assert np.array_equal(d.cpu().numpy(), s_ref)
    assert ctx.get_error() == 0


@pytest.mark.parametrize("dtype,C,lr,lam,n_iter,tol", [("fp64", 4, 0.05, 1e-3, 150, 3e-3),
                                                      ("bf16", 16, 0.02, 1e-2, 80, 1e-2)])
def test_vmc_reaches_exact_ground_energy_4x4(dtype, C, lr, lam, n_iter, tol):
    L, J2, K, B = 4, 0.0, 2, 256
    E0 = _e0()
    w = inputs.weights(K, C, 0.05, 1)
    ctx = make_ctx(L, J2, K, C, w, dtype=dtype)
    run = VMC(ctx, w, to_dev(inputs.spins_sz0(L, B, 2)), steps=16, lr=lr, diag_shift=lam,
              cg_iters=100, seed=11)
    hist = [run.step() for _ in range(n_iter)]
    e = np.array([h["energy"] for h in hist])
    v = np.array([h["variance"] for h in hist])
    tail = e[-10:].mean()
    say(dtype, "first", e[0], "last 10 mean", tail, "ED", E0, "variance", v[0], "->", v[-10:].mean())
    assert abs(tail - E0) < tol * abs(E0)
    assert v[-10:].mean() < 0.2 * v[0]
    assert ctx.get_error() == 0
