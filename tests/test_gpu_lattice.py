"""GPU integer stage vs the oracle, bit-exact: connected-configuration lists
(antiparallel J1/J2 pairs in canonical bond order, Sec. 5.4.1), per-sample
counts and offsets, Marshall ratios, and the diagonal energy (Sec. 6.1)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs
from gpu_helpers import make_ctx, say, to_dev

pytestmark = pytest.mark.gpu


CASES = [
    ("4x4 J2=0.5 Sz0 B=1024", 4, 0.5, 1024, "sz0"),
    ("10x10 J2=0.5 Sz0 B=512", 10, 0.5, 512, "sz0"),
    ("12x12 J2=0 Sz0 B=64", 12, 0.0, 64, "sz0"),
    ("6x6 J2=0.55 any B=77", 6, 0.55, 77, "any"),
    ("36x36 J2=0.5 Sz0 B=12", 36, 0.5, 12, "sz0"),
    ("64x64 J2=0.5 any B=3", 64, 0.5, 3, "any"),
]


@pytest.mark.parametrize("name,L,J2,B,kind", CASES, ids=[c[0] for c in CASES])
def test_connected_bit_exact(name, L, J2, B, kind):
    say("case", name)
    sp = inputs.spins_sz0(L, B, 7) if kind == "sz0" else inputs.spins_any(L, B, 7)
    K, C = 2, 4
    ctx = make_ctx(L, J2, K, C, inputs.weights(K, C, 0.1, 1))
    counts, offs, bonds, mu, ed = ctx.connected(to_dev(sp))
    torch.cuda.synchronize()
    assert ctx.get_error() == 0
    oc, ob, om, oe = oracle.connected(L, 1.0, J2, sp)
    assert np.array_equal(counts.cpu().numpy(), oc)
    offs = offs.cpu().numpy()
    assert offs[0] == 0 and np.array_equal(np.diff(offs), oc)
    bonds = bonds.cpu().numpy()
    mu = mu.cpu().numpy()
    for s in range(B):
        assert np.array_equal(bonds[offs[s]:offs[s + 1]], ob[s])
        assert np.array_equal(mu[offs[s]:offs[s + 1]], om[s])
    if J2 in (0.0, 0.5):
        assert np.array_equal(ed.cpu().numpy(), oe)      # multiples of 1/8: exact
    else:
        np.testing.assert_allclose(ed.cpu().numpy(), oe, rtol=1e-14, atol=1e-14)


def test_special_states_and_empty_batch():
    L = 8
    ctx = make_ctx(L, 0.5, 2, 4, inputs.weights(2, 4, 0.1, 1))
    sp = np.stack([inputs.neel(L), inputs.ferro(L), inputs.column_stripe(L), -inputs.ferro(L)])
    counts, offs, bonds, mu, ed = ctx.connected(to_dev(sp))
    N = L * L
    assert counts.cpu().tolist() == [2 * N, 0, 3 * N, 0]
    np.testing.assert_array_equal(ed.cpu().numpy(), [-N / 2 + N / 4, N * 1.5 / 2, -N * 0.25, N * 1.5 / 2])
    counts, offs, bonds, mu, ed = ctx.connected(to_dev(np.zeros((0, L, L), np.int8)))
    assert offs.cpu().tolist() == [0]


def test_bad_spin_sets_sticky_error():
    L = 6
    ctx = make_ctx(L, 0.5, 2, 4, inputs.weights(2, 4, 0.1, 1))
    sp = inputs.spins_sz0(L, 4, 3)
    sp[2, 1, 1] = 0
    ctx.connected(to_dev(sp))
    assert ctx.get_error() == 5          # NQS_E_SPIN
    assert ctx.get_error() == 0          # cleared on read
