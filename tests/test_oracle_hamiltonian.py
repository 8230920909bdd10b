"""Pins of the oracle's lattice, bond list, Marshall sign and diagonal energy.

The connected-configuration rule follows Sec. 5.4.1 ("Hotspot energy
calculation": every antiparallel nearest / next-nearest pair gives one
exchanged configuration) and the Hamiltonian of Sec. 6.1, Eq. (J1J2).
Everything here is checked against closed forms or against the torus geometry
computed independently in oracle/ed.py.
"""
import numpy as np
import pytest

from oracle import ed
from paper_2204_07816_amd import inputs


@pytest.mark.parametrize("L", [4, 6, 10])
def test_bond_set_matches_geometry(orc, L):
    nn, nnn = ed.torus_pairs(L)
    got1, got2 = set(), set()
    for b in range(4 * L * L):
        i, j, cls = orc.bond_sites(L, b)
        key = (min(i, j), max(i, j))
        target = got1 if cls == 1 else got2
        assert key not in target, "bond listed twice"
        target.add(key)
    assert got1 == set(nn) and got2 == set(nnn)
    assert len(nn) == 2 * L * L and len(nnn) == 2 * L * L


@pytest.mark.parametrize("L,J2", [(4, 0.5), (6, 0.5), (10, 0.0), (8, 0.55)])
def test_closed_forms(orc, L, J2):
    N = L * L
    J1 = 1.0
    # Neel: every J1 pair antiparallel, every J2 pair parallel
    c, bonds, mus, ed_ = orc.connected(L, J1, J2, inputs.neel(L))
    assert c[0] == 2 * N
    assert np.all(np.array(bonds[0]) % 4 < 2)
    assert ed_[0] == pytest.approx(-N * J1 / 2 + N * J2 / 2, abs=1e-12)
    # column stripe: x-bonds J1 antiparallel, y-bonds parallel, both J2 antiparallel
    c, bonds, mus, ed_ = orc.connected(L, J1, J2, inputs.column_stripe(L))
    assert c[0] == N + (2 * N if J2 != 0 else 0)
    assert ed_[0] == pytest.approx(-N * J2 / 2, abs=1e-12)
    # ferromagnet: nothing connected
    c, bonds, mus, ed_ = orc.connected(L, J1, J2, inputs.ferro(L))
    assert c[0] == 0
    assert ed_[0] == pytest.approx(N * (J1 + J2) / 2, abs=1e-12)


def test_neel_4x4_worked_numbers(orc):
    c, _, _, e = orc.connected(4, 1.0, 0.5, inputs.neel(4))
    assert c[0] == 32 and e[0] == -4.0


@pytest.mark.parametrize("L,J2", [(4, 0.5), (6, 0.0), (10, 0.5)])
def test_connected_brute_force_and_marshall_ratio(orc, L, J2):
    nn, nnn = ed.torus_pairs(L)
    spins = inputs.spins_any(L, 12, seed=11)
    counts, bonds, mus, ediag = orc.connected(L, 1.0, J2, spins)
    for s in range(spins.shape[0]):
        flat = spins[s].reshape(-1)
        anti = sum(flat[i] != flat[j] for (i, j) in nn)
        if J2 != 0.0:
            anti += sum(flat[i] != flat[j] for (i, j) in nnn)
        assert counts[s] == anti
        diag = 0.25 * (sum(flat[i] * flat[j] for (i, j) in nn)
                       + J2 * sum(flat[i] * flat[j] for (i, j) in nnn))
        assert ediag[s] == pytest.approx(diag, abs=1e-12)
        # bond ids strictly increasing (canonical order)
        assert np.all(np.diff(bonds[s]) > 0)
        # Marshall ratio: exchanging an A-B (J1) pair flips the sign, A-A or B-B (J2) does not
        for b, m in zip(bonds[s], mus[s]):
            assert m == (-1 if b % 4 < 2 else 1)
        if J2 == 0.0:
            assert np.all(np.array(bonds[s]) % 4 < 2)


def test_marshall_sign_values(orc):
    L = 4
    # Neel with up spins on A: 8 up on A -> (+1)
    assert orc.marshall_sign(L, inputs.neel(L)) == 1
    assert orc.marshall_sign(L, -inputs.neel(L)) == 1      # 0 up on A
    s = inputs.neel(L).copy()
    s[0, 0] = -1                                           # 7 up on A
    assert orc.marshall_sign(L, s) == -1
    # Sz=0 and even L: sign invariant under global spin flip and translations
    sp = inputs.spins_sz0(6, 20, seed=5)
    for b in range(20):
        m = orc.marshall_sign(6, sp[b])
        assert orc.marshall_sign(6, -sp[b]) == m
        assert orc.marshall_sign(6, np.roll(sp[b], 1, axis=1)) == m
        assert orc.marshall_sign(6, np.roll(sp[b], 1, axis=0)) == m


def test_exchange_conserves_sz(orc):
    L = 6
    sp = inputs.spins_any(L, 4, seed=3)
    counts, bonds, _, _ = orc.connected(L, 1.0, 0.5, sp)
    for s in range(4):
        for b in bonds[s]:
            i, j, _ = orc.bond_sites(L, int(b))
            flat = sp[s].reshape(-1).copy()
            flat[i], flat[j] = flat[j], flat[i]
            assert flat.sum() == sp[s].sum()
