"""Pins of the oracle's t-J model [Sec. 6.1, Eq. tJ: hopping of electrons
plus J (S_i.S_j - n_i n_j / 4) on nearest-neighbour pairs, fermions encoded by
the Jordan-Wigner transformation] and of the exact diagonalisation it is
checked against.

The exact diagonalisation (oracle/ed.py) builds H from fermion creation and
annihilation operators acting on mode strings, each operator taking the sign
of the occupied modes below it; it never counts electrons between two sites.
It is pinned first, against what does not depend on it:

* a fully polarised sector is free spinless fermions on the torus: the whole
  spectrum is the set of sums of distinct band energies -2t(cos kx + cos ky),
  k = 2 pi n / L (which hard-core bosons, i.e. dropped fermion signs, miss);
* with no hole the t-J model is the Heisenberg model minus J/4 per bond
  (spectrum against the spin-operator exact diagonalisation).

The oracle is then pinned against the exact diagonalisation:

* every column <S'|H|S> of random configurations (bond list, matrix
  elements, Jordan-Wigner signs, diagonal part);
* E_loc of the exact ground state equals E_0 on every configuration of the
  sector (one hole; two up and two down electrons);
* <psi|H|psi> / <psi|psi> = sum_S psi(S)^2 E_loc(S) / sum_S psi(S)^2 for the
  CNN amplitude over a whole sector;
* hand-written hops across the periodic boundary with a known number of
  electrons in between.
"""
import numpy as np
import pytest

from oracle import ed
from paper_2204_07816_amd import inputs

T_HOP, J_EX = 1.0, 0.4        # the paper's t-J parameters


def _band(L, t):
    k = 2.0 * np.pi * np.arange(L) / L
    return np.sort((-2.0 * t * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel())


@pytest.mark.parametrize("n_el", [1, 2, 3, 15])
def test_ed_polarised_sector_is_free_fermions(n_el):
    from itertools import combinations
    L = 4
    H, basis = ed.tj_hamiltonian(L, T_HOP, J_EX, n_el, 0)
    eps = _band(L, T_HOP)
    if n_el <= 3:
        ref = np.sort([sum(c) for c in combinations(eps, n_el)])
        got = np.linalg.eigvalsh(H.toarray())
        np.testing.assert_allclose(got, ref, atol=1e-10)
    else:   # one hole: the empty band level is the top one, 4t
        e0, _ = ed.tj_ground(H)
        assert e0 == pytest.approx(eps[:n_el].sum(), abs=1e-9)
        assert e0 == pytest.approx(-4.0 * T_HOP, abs=1e-9)


def test_ed_polarised_fermion_signs_matter():
    # three fermions fill the band bottom, -4t - 2t - 2t = -8t exactly; three
    # hard-core bosons (the same hops without fermion signs) lie lower
    H, _ = ed.tj_hamiltonian(4, T_HOP, J_EX, 3, 0)
    A = H.toarray()
    assert np.linalg.eigvalsh(A)[0] == pytest.approx(-8.0 * T_HOP, abs=1e-10)
    bosons = -np.abs(A)
    np.fill_diagonal(bosons, np.diag(A))
    assert np.linalg.eigvalsh(bosons)[0] < -8.0 * T_HOP - 1.0


@pytest.mark.parametrize("n_up", [2, 3])
def test_ed_no_holes_is_heisenberg(n_up):
    L = 4
    N = L * L
    Ht, _ = ed.tj_hamiltonian(L, T_HOP, J_EX, n_up, N - n_up)
    Hh, _ = ed.hamiltonian(L, J_EX, 0.0, n_up=n_up)
    got = np.linalg.eigvalsh(Ht.toarray())
    ref = np.linalg.eigvalsh(Hh.toarray()) - J_EX * (2 * N) / 4.0
    np.testing.assert_allclose(got, ref, atol=1e-10)


def test_columns_match_ed(orc):
    L, B = 4, 40
    for n_holes in (2, 6, 10):
        sp = inputs.spins_tj(L, B, n_holes, 10 + n_holes)
        counts, bonds, mus, hs, ediag = orc.tj_connected(L, T_HOP, J_EX, sp)
        for b in range(B):
            s = sp[b].reshape(-1)
            col = ed.tj_column(L, T_HOP, J_EX, s)
            diag = col.pop(s.tobytes(), 0.0)
            assert ediag[b] == pytest.approx(diag, abs=1e-12)
            got = {}
            for bid, h in zip(bonds[b], hs[b]):
                i, j, cls = orc.bond_sites(L, int(bid))
                assert cls == 1
                s2 = s.copy()
                s2[i], s2[j] = s[j], s[i]
                got[s2.tobytes()] = h
            assert counts[b] == len(got)
            assert set(got) == set(k for k, v in col.items() if v != 0.0)
            for k, v in got.items():
                assert v == pytest.approx(col[k], abs=1e-12)


def test_marshall_ratio_of_moves(orc):
    L = 6
    sp = inputs.spins_tj(L, 20, 4, 31)
    counts, bonds, mus, hs, _ = orc.tj_connected(L, T_HOP, J_EX, sp)
    for b in range(20):
        s = sp[b].reshape(-1)
        m0 = orc.marshall_sign(L, s)
        for bid, mu in zip(bonds[b], mus[b]):
            i, j, _ = orc.bond_sites(L, int(bid))
            s2 = s.copy()
            s2[i], s2[j] = s[j], s[i]
            assert mu == orc.marshall_sign(L, s2) * m0
            # a spin exchange or an up electron moving changes the count on A by one
            up_moves = (s[i] * s[j] == -1) or (s[i] + s[j] > 0)
            assert mu == (-1 if up_moves else 1)


def test_hops_across_the_boundary(orc):
    L = 4
    s = np.zeros((L, L), np.int8)
    # row 1: hole at x = 3, electron at x = 0, electrons at x = 1, 2 in between
    s[1] = [1, -1, 1, 0]
    s[3, 3] = -1
    s[0, 3] = 1
    counts, bonds, mus, hs, ediag = orc.tj_connected(L, T_HOP, J_EX, s)
    h = dict(zip(bonds[0].tolist(), hs[0].tolist()))
    # bond (x=3, y=1) -> (0, 1): sites 7 and 4, electrons on 5, 6 between: +
    assert h[4 * 7 + 0] == pytest.approx(-T_HOP * (+1))
    # bond (x=2, y=1) -> (3, 1): neighbours in the site order: -t
    assert h[4 * 6 + 0] == pytest.approx(-T_HOP)
    # bond (x=3, y=0) -> (3, 1): sites 3 and 7, sites 4, 5, 6 hold 3 electrons: +t
    assert h[4 * 3 + 1] == pytest.approx(+T_HOP)
    # bond (x=3, y=3) -> (3, 0): sites 15 and 3 hold a down and an up electron,
    # a spin exchange: +J/2 whatever lies between
    assert h[4 * 15 + 1] == pytest.approx(J_EX / 2)
    # diagonal: antiparallel pairs (4,5), (5,6), (15,3) -> -J/2 each
    assert ediag[0] == pytest.approx(-1.5 * J_EX)


@pytest.fixture(scope="module")
def tj_sectors():
    out = {}
    for key in ((8, 7), (2, 2)):
        H, basis = ed.tj_hamiltonian(4, T_HOP, J_EX, *key)
        E0, vec = ed.tj_ground(H)
        out[key] = (H, basis, E0, vec)
    return out


@pytest.mark.parametrize("sector", [(8, 7), (2, 2)])
def test_eloc_of_exact_ground_state_is_e0(orc, tj_sectors, sector):
    H, basis, E0, vec = tj_sectors[sector]
    assert np.linalg.norm(H @ vec - E0 * vec) < 1e-8
    spins = ed.tj_modes_to_spins(basis, 16)
    keys = orc.tj_key(spins, 4)
    order = np.argsort(keys)
    big = np.abs(vec) > 1e-6 * np.abs(vec).max()
    la = np.log(np.maximum(np.abs(vec), 1e-300))
    sg = np.sign(vec).astype(np.int8)
    e = orc.tj_local_energy_table(4, T_HOP, J_EX, keys[order], la[order], sg[order],
                                  spins[big])
    np.testing.assert_allclose(e, E0, rtol=0, atol=1e-6)


@pytest.mark.parametrize("sigma", [0.05, 0.5])
def test_rayleigh_quotient_of_cnn(orc, tj_sectors, sigma):
    H, basis, E0, _ = tj_sectors[(2, 2)]
    K, C = 2, 4
    w = inputs.weights(K, C, sigma, 41)
    spins = ed.tj_modes_to_spins(basis, 16).reshape(-1, 4, 4)
    la, sg = orc.log_psi(4, K, C, w, spins)
    psi = sg * np.exp(la - la.max())
    e = orc.tj_local_energy(4, T_HOP, J_EX, K, C, w, spins)
    lhs = np.sum(psi ** 2 * e) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-11)
    assert rhs > E0


def test_check_and_conservation(orc):
    L, B, T = 6, 12, 30
    sp = inputs.spins_tj(L, B, 4, 51)
    assert orc.tj_check(L, sp)
    bad = sp.copy()
    bad[3, 2, 2] = 2
    assert not orc.tj_check(L, bad)
    K, C = 2, 4
    w = inputs.weights(K, C, 0.3, 52)
    rb, ru = inputs.mcmc_randoms(53, 0, T, B)
    out, acc = orc.tj_mcmc(L, T_HOP, J_EX, K, C, w, sp, rb, ru)
    for v in (1, -1, 0):
        assert np.array_equal((out == v).sum(axis=(1, 2)), (sp == v).sum(axis=(1, 2)))
    assert acc.sum() > 0
    out2, acc2 = orc.tj_mcmc(L, T_HOP, J_EX, K, C, w, sp, rb, ru)
    assert np.array_equal(out, out2) and np.array_equal(acc, acc2)
