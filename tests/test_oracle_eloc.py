"""Pins of the oracle's local energy (Sec. 5.4.1: E_loc(S) = sum_S' W(S')/W(S) <S'|H|S>)
and of the exact-diagonalisation support code (Sec. 6.1 Hamiltonian).

* ED ground energy of the 4x4 Heisenberg point vs the literature value
  (-11.228483, sanity only; not in the paper) and vs ARPACK.
* Marshall's theorem at J2 = 0: M(s) psi_0(s) has one sign on the whole sector.
* Exhaustive identity on 4x4: sum_s |psi|^2 E_loc / sum |psi|^2 = <psi|H|psi>/<psi|psi>
  for the CNN wave function, with H from ED (independent code), on single Sz
  sectors and over all 2^16 states.
* Zero variance: E_loc of the exact eigenvector equals E_0 on every configuration.
* Variational bound, translation and spin-flip invariance of E_loc.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import ed
from paper_2204_07816_amd import inputs


@pytest.fixture(scope="module")
def ed44():
    out = {}
    for J2 in (0.0, 0.5):
        H, basis = ed.hamiltonian(4, 1.0, J2)
        E0, vec = ed.lanczos_ground(H)
        out[J2] = (H, basis, E0, vec)
    return out


def test_ed_ground_energy(ed44):
    H, basis, E0, vec = ed44[0.0]
    assert basis.shape[0] == 12870
    assert E0 == pytest.approx(-11.228483, abs=2e-6)          # literature, 4x4 Heisenberg
    ref = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert E0 == pytest.approx(ref, rel=1e-10)
    H5, _, E05, vec5 = ed44[0.5]
    ref5 = spla.eigsh(H5, k=1, which="SA", tol=1e-14)[0][0]
    assert E05 == pytest.approx(ref5, rel=1e-10)
    # eigen-residual
    assert np.linalg.norm(H @ vec - E0 * vec) < 1e-8


def test_marshall_theorem(orc, ed44):
    H, basis, E0, vec = ed44[0.0]
    spins = ed.basis_to_spins(basis, 16).reshape(-1, 4, 4)
    m = np.array([orc.marshall_sign(4, s) for s in spins])
    prod = m * vec
    prod *= np.sign(prod[np.argmax(np.abs(prod))])
    assert np.all(prod > 0)


def _cnn_psi_on_sector(orc, L, K, C, w, basis):
    spins = ed.basis_to_spins(basis, L * L).reshape(-1, L, L)
    la, sg = orc.log_psi(L, K, C, w, spins)
    psi = sg * np.exp(la - la.max())
    return spins, psi


@pytest.mark.parametrize("J2,sigma", [(0.5, 0.05), (0.0, 0.6), (0.5, 0.8)])
def test_exhaustive_expectation_4x4(orc, J2, sigma):
    L, K, C = 4, 2, 4
    w = inputs.weights(K, C, sigma, seed=1000)
    H, basis = ed.hamiltonian(L, 1.0, J2)
    spins, psi = _cnn_psi_on_sector(orc, L, K, C, w, basis)
    eloc = orc.local_energy(L, 1.0, J2, K, C, w, spins)
    p = psi ** 2
    lhs = np.sum(p * eloc) / np.sum(p)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # variational bound
    E0 = spla.eigsh(H, k=1, which="SA", tol=1e-12)[0][0]
    assert lhs >= E0 - 1e-9


def test_exhaustive_other_sector(orc):
    """Same identity on the Sz = +1 sector (9 up spins) - H conserves Sz."""
    L, K, C = 4, 2, 4
    w = inputs.weights(K, C, 0.5, seed=5)
    H, basis = ed.hamiltonian(L, 1.0, 0.5, n_up=9)
    spins, psi = _cnn_psi_on_sector(orc, L, K, C, w, basis)
    eloc = orc.local_energy(L, 1.0, 0.5, K, C, w, spins)
    lhs = np.sum(psi ** 2 * eloc) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("J2", [0.0, 0.5])
def test_zero_variance_exact_eigenstate(orc, ed44, J2):
    H, basis, E0, vec = ed44[J2]
    N = 16
    log_tab = np.full(1 << N, -1e300)
    sign_tab = np.ones(1 << N, np.int8)
    log_tab[basis] = np.log(np.abs(vec))
    sign_tab[basis] = np.where(vec >= 0, 1, -1)
    keep = np.abs(vec) > 1e-8 * np.abs(vec).max()
    spins = ed.basis_to_spins(basis[keep], N).reshape(-1, 4, 4)
    eloc = orc.local_energy_table(4, 1.0, J2, log_tab, sign_tab, spins)
    # local energy is (H psi)(s) / psi(s) for any psi; for the eigenvector it is E_0
    # up to the eigen-residual r = H psi - E_0 psi divided by psi(s)
    hv = H @ vec
    np.testing.assert_allclose(eloc, hv[keep] / vec[keep], rtol=1e-10)
    resid = np.abs(hv - E0 * vec)[keep] / np.abs(vec[keep])
    assert np.all(np.abs(eloc - E0) <= resid + 1e-10 * abs(E0))
    assert np.median(np.abs(eloc - E0)) < 1e-7 * abs(E0)
    # the mean over |psi|^2 is E_0 to machine precision
    p = vec[keep] ** 2
    assert np.sum(p * eloc) / np.sum(p) == pytest.approx(E0, rel=1e-11)


def test_eloc_symmetries(orc):
    L, K, C = 6, 2, 4
    w = inputs.weights(K, C, 0.4, seed=77)
    sp = inputs.spins_sz0(L, 6, seed=1)
    e = orc.local_energy(L, 1.0, 0.5, K, C, w, sp)
    et = orc.local_energy(L, 1.0, 0.5, K, C, w, np.roll(sp, (1, 3), axis=(1, 2)))
    np.testing.assert_allclose(et, e, rtol=1e-12)
    w0 = w.copy()
    w0[C * 9:C * 9 + C] = 0.0
    a = orc.local_energy(L, 1.0, 0.5, K, C, w0, sp)
    b = orc.local_energy(L, 1.0, 0.5, K, C, w0, -sp)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_eloc_uniform_amplitude_reduces_to_bond_sums(orc):
    """With all weights zero, f = const, psi = M exp(const): E_loc = E_diag + sum (J/2) mu_b."""
    L, K, C = 6, 2, 3
    w = np.zeros(inputs.num_params(K, C))
    sp = inputs.spins_sz0(L, 5, seed=12)
    e = orc.local_energy(L, 1.0, 0.5, K, C, w, sp)
    counts, bonds, mus, ediag = orc.connected(L, 1.0, 0.5, sp)
    for s in range(5):
        J = np.where(np.array(bonds[s]) % 4 < 2, 1.0, 0.5)
        assert e[s] == pytest.approx(ediag[s] + np.sum(0.5 * J * mus[s]), rel=1e-13)


def test_energy_stats(orc):
    e = np.array([1.0, 2.0, 4.0, -3.0])
    m, v = orc.energy_stats(e)
    assert m == 1.0 and v == pytest.approx(np.mean((e - 1.0) ** 2))


def test_exhaustive_all_2pow16_states(orc):
    """The identity over the whole 2^16-state space of 4x4 (every Sz sector):
    H is block diagonal in Sz, so <psi|H|psi> is the sum over sectors of
    psi_s^T H_s psi_s, with one common normalisation of psi."""
    L, K, C, J2 = 4, 2, 4, 0.5
    w = inputs.weights(K, C, 0.4, seed=7)
    num = den = ph = pp = 0.0
    parts = []
    for n_up in range(17):
        H, basis = ed.hamiltonian(L, 1.0, J2, n_up=n_up)
        spins = ed.basis_to_spins(basis, L * L).reshape(-1, L, L)
        la, sg = orc.log_psi(L, K, C, w, spins)
        parts.append((H, spins, la, sg))
    lmax = max(p[2].max() for p in parts)
    n_states = 0
    for H, spins, la, sg in parts:
        psi = sg * np.exp(la - lmax)
        eloc = orc.local_energy(L, 1.0, J2, K, C, w, spins)
        num += np.sum(psi ** 2 * eloc)
        den += np.sum(psi ** 2)
        ph += psi @ (H @ psi)
        pp += psi @ psi
        n_states += spins.shape[0]
    assert n_states == 1 << 16
    assert num / den == pytest.approx(ph / pp, rel=1e-12)
