"""Pins of the oracle's CNN1 [Sec. 5.2: blocks of a 2D convolution, a 1D
max-pooling and a transposed convolution with periodic padding; output the
product of the neurons].

The block figure is missing, so the architecture is a reading (stated in
oracle/nqs_oracle.h) and is parity unpinned against the paper.  What is
pinned is that the oracle computes that reading:

* log|psi| and sign against the same network written with torch's conv2d
  (circular padding), a max over channel pairs and conv_transpose2d whose
  overhanging border is folded back onto the torus;
* O = d log|psi| / d theta against torch autograd through that network, and
  against central finite differences;
* the local energy: sum_S psi^2 E_loc / sum psi^2 = <psi|H|psi> / <psi|psi>
  over the whole 4x4 Sz = 0 sector with H from the exact diagonalisation and
  psi signed by the network;
* the parameter count against the torch network's.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import ed
from paper_2204_07816_amd import inputs


def torch_cnn1(L, Kb, C, w, spins):
    """(log|psi_net|, number of negative output neurons) per configuration."""
    w = torch.as_tensor(w, dtype=torch.float64)
    h = torch.as_tensor(np.asarray(spins, np.float64).reshape(-1, 1, L, L))
    off = 0
    for k in range(Kb):
        cin = 1 if k == 0 else C
        W = w[off:off + 2 * C * cin * 9].view(2 * C, cin, 3, 3); off += 2 * C * cin * 9
        a = w[off:off + 2 * C]; off += 2 * C
        V = w[off:off + C * C * 9].view(C, C, 3, 3); off += C * C * 9
        v = w[off:off + C]; off += C
        z = F.conv2d(F.pad(h, (1, 1, 1, 1), mode="circular"), W, a)
        m = z.view(z.shape[0], C, 2, L, L).amax(dim=2)
        full = F.conv_transpose2d(m, V)                     # (L+2) x (L+2), no padding
        u = full[:, :, 1:L + 1, 1:L + 1].clone()
        # fold the overhanging rows / columns back (periodic boundary)
        u[:, :, L - 1, :] += full[:, :, 0, 1:L + 1]
        u[:, :, 0, :] += full[:, :, L + 1, 1:L + 1]
        u[:, :, :, L - 1] += full[:, :, 1:L + 1, 0]
        u[:, :, :, 0] += full[:, :, 1:L + 1, L + 1]
        u[:, :, L - 1, L - 1] += full[:, :, 0, 0]
        u[:, :, L - 1, 0] += full[:, :, 0, L + 1]
        u[:, :, 0, L - 1] += full[:, :, L + 1, 0]
        u[:, :, 0, 0] += full[:, :, L + 1, L + 1]
        h = u + v.view(1, C, 1, 1)
    assert off == w.shape[0]
    return torch.log(torch.abs(h)).sum(dim=(1, 2, 3)), (h < 0).sum(dim=(1, 2, 3))


@pytest.mark.parametrize("L,Kb,C,sigma", [(4, 2, 4, 0.3), (6, 3, 3, 0.5), (8, 1, 2, 0.7),
                                          (5, 2, 2, 0.4)])
def test_forward_matches_torch(orc, L, Kb, C, sigma):
    w = inputs.cnn1_weights(Kb, C, sigma, 11)
    sp = inputs.spins_any(L, 24, 12)
    la, sg = orc.cnn1_log_psi(L, Kb, C, w, sp, marshall=False)
    f, neg = torch_cnn1(L, Kb, C, w, sp)
    np.testing.assert_allclose(la, f.numpy(), rtol=1e-12, atol=1e-12)
    assert np.array_equal(sg, np.where(neg.numpy() % 2 == 0, 1, -1))
    la2, sg2 = orc.cnn1_log_psi(L, Kb, C, w, sp, marshall=True)
    m = np.array([orc.marshall_sign(L, s) for s in sp])
    assert np.array_equal(la2, la) and np.array_equal(sg2, sg * m)


def test_param_count(orc):
    for Kb, C in ((1, 1), (2, 4), (6, 16), (3, 7)):
        P = orc.cnn1_num_params(Kb, C)
        assert P == inputs.cnn1_num_params(Kb, C)
        torch_count = sum((2 * C) * (1 if k == 0 else C) * 9 + 2 * C + C * C * 9 + C
                          for k in range(Kb))
        assert P == torch_count


@pytest.mark.parametrize("L,Kb,C,sigma", [(4, 2, 4, 0.3), (6, 3, 3, 0.5)])
def test_log_deriv_matches_autograd(orc, L, Kb, C, sigma):
    w = inputs.cnn1_weights(Kb, C, sigma, 21)
    sp = inputs.spins_any(L, 6, 22)
    O = orc.cnn1_log_deriv(L, Kb, C, w, sp)
    for s in range(sp.shape[0]):
        wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
        f, _ = torch_cnn1(L, Kb, C, wt, sp[s:s + 1])
        (g,) = torch.autograd.grad(f.sum(), wt)
        # 1/u at small output neurons makes entries up to ~1e4: compare at the row's scale
        g = g.numpy()
        np.testing.assert_allclose(O[s], g, rtol=1e-10, atol=1e-12 * np.abs(g).max())


def test_log_deriv_finite_differences(orc):
    L, Kb, C = 4, 2, 3
    w = inputs.cnn1_weights(Kb, C, 0.4, 31)
    sp = inputs.spins_any(L, 3, 32)
    O = orc.cnn1_log_deriv(L, Kb, C, w, sp)
    rng = np.random.default_rng(33)
    for p in rng.choice(w.shape[0], 12, replace=False):
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd = (orc.cnn1_log_psi(L, Kb, C, wp, sp)[0] - orc.cnn1_log_psi(L, Kb, C, wm, sp)[0]) / (2 * h)
        np.testing.assert_allclose(O[:, p], fd, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("J2,marshall", [(0.5, True), (0.0, False)])
def test_rayleigh_quotient_over_sector(orc, J2, marshall):
    L, Kb, C = 4, 2, 3
    H, basis = ed.hamiltonian(L, 1.0, J2)
    w = inputs.cnn1_weights(Kb, C, 0.3, 41)
    spins = ed.basis_to_spins(basis, 16).reshape(-1, 4, 4)
    la, sg = orc.cnn1_log_psi(L, Kb, C, w, spins, marshall=marshall)
    psi = sg * np.exp(la - la.max())
    e = orc.cnn1_local_energy(L, 1.0, J2, Kb, C, w, spins, marshall=marshall)
    lhs = np.sum(psi ** 2 * e) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_cnn1_mcmc_conserves_sz_and_is_reproducible(orc):
    L, Kb, C, B, T = 4, 2, 3, 16, 20
    w = inputs.cnn1_weights(Kb, C, 0.3, 51)
    sp = inputs.spins_sz0(L, B, 52)
    rb, ru = inputs.mcmc_randoms(53, 0, T, B)
    out, acc = orc.cnn1_mcmc(L, 1.0, 0.5, Kb, C, w, sp, rb, ru)
    assert np.array_equal(out.sum(axis=(1, 2)), sp.sum(axis=(1, 2)))
    assert 0 < acc.sum() < B * T
    out2, acc2 = orc.cnn1_mcmc(L, 1.0, 0.5, Kb, C, w, sp, rb, ru)
    assert np.array_equal(out, out2) and np.array_equal(acc, acc2)


@pytest.mark.parametrize("marshall", [True, False])
def test_tj_rayleigh_quotient_with_cnn1_sign(orc, marshall):
    """The t-J local energy with the signed CNN1 amplitude, summed over the
    whole 4x4 sector of two up and two down electrons, equals <psi|H|psi> /
    <psi|psi> with H from the fermion-operator exact diagonalisation."""
    L, Kb, C, t, J = 4, 2, 3, 1.0, 0.4
    H, basis = ed.tj_hamiltonian(L, t, J, 2, 2)
    w = inputs.cnn1_weights(Kb, C, 0.3, 61)
    spins = ed.tj_modes_to_spins(basis, 16).reshape(-1, 4, 4)
    la, sg = orc.cnn1_log_psi(L, Kb, C, w, spins, marshall=marshall)
    psi = sg * np.exp(la - la.max())
    e = orc.tj_cnn1_local_energy(L, t, J, Kb, C, w, spins, marshall=marshall)
    lhs = np.sum(psi ** 2 * e) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-10)
