"""Pins of the oracle's CNN2 [Sec. 5.2: CNN1's building block behind an
embedding of the site states, with the max-pooling taken at stride one and
padding done by copying the first neurons after the last; six blocks; a final
convolution down to one channel; the product of its neurons].

The block figure and the hyper-parameters are missing, so the architecture
is a reading (stated in oracle/nqs_oracle.h) and is parity unpinned against
the paper; the paper's 113,815 parameters are not reached by any natural
channel count of it (C = 32 gives 111,361).  What is pinned is that the
oracle computes that reading:

* log|psi| and sign against the same network written with torch: an
  embedding lookup, conv2d with circular padding, a max of each channel with
  the next under torch.roll, and conv_transpose2d whose overhanging border
  is folded back onto the torus, then a conv2d to one channel;
* O = d log|psi| / d theta against torch autograd through that network and
  against central finite differences;
* symmetries the reading implies and a plausible slip breaks: invariance
  under lattice translations (circular spatial padding) and under a cyclic
  shift of the pooled channels carried through W, a and V (the stride-one
  max with the first channel copied after the last; a zero-padded or
  shortened window breaks it);
* the t-J local energy: sum_S psi^2 E_loc / sum psi^2 = <psi|H|psi> /
  <psi|psi> over the whole 4x4 sector of two up and two down electrons, H
  from the fermion-operator exact diagonalisation, psi signed by the network;
* the parameter count against the torch network's.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import ed
from paper_2204_07816_amd import inputs

T_HOP, J_EX = 1.0, 0.4


def _fold(full, L):
    """conv_transpose2d's (L+2) x (L+2) output folded back onto the L x L torus."""
    u = full[:, :, 1:L + 1, 1:L + 1].clone()
    u[:, :, L - 1, :] += full[:, :, 0, 1:L + 1]
    u[:, :, 0, :] += full[:, :, L + 1, 1:L + 1]
    u[:, :, :, L - 1] += full[:, :, 1:L + 1, 0]
    u[:, :, :, 0] += full[:, :, 1:L + 1, L + 1]
    u[:, :, L - 1, L - 1] += full[:, :, 0, 0]
    u[:, :, L - 1, 0] += full[:, :, 0, L + 1]
    u[:, :, 0, L - 1] += full[:, :, L + 1, 0]
    u[:, :, 0, 0] += full[:, :, L + 1, L + 1]
    return u


def torch_cnn2(L, Kb, C, w, spins):
    """(log|psi_net|, number of negative output neurons) per configuration."""
    w = torch.as_tensor(w, dtype=torch.float64)
    s = torch.as_tensor(np.asarray(spins, np.int64).reshape(-1, L, L))
    cls = torch.where(s == 0, 0, torch.where(s > 0, 1, 2))
    off = 0
    E = w[off:off + 3 * C].view(3, C); off += 3 * C
    h = F.embedding(cls, E).permute(0, 3, 1, 2)              # [B][C][L][L]
    for _ in range(Kb):
        W = w[off:off + 9 * C * C].view(C, C, 3, 3); off += 9 * C * C
        a = w[off:off + C]; off += C
        V = w[off:off + 9 * C * C].view(C, C, 3, 3); off += 9 * C * C
        v = w[off:off + C]; off += C
        z = F.conv2d(F.pad(h, (1, 1, 1, 1), mode="circular"), W, a)
        m = torch.maximum(z, torch.roll(z, shifts=-1, dims=1))
        h = _fold(F.conv_transpose2d(m, V), L) + v.view(1, C, 1, 1)
    Fw = w[off:off + 9 * C].view(1, C, 3, 3); off += 9 * C
    b = w[off:off + 1]; off += 1
    assert off == w.shape[0]
    y = F.conv2d(F.pad(h, (1, 1, 1, 1), mode="circular"), Fw, b)
    return torch.log(torch.abs(y)).sum(dim=(1, 2, 3)), (y < 0).sum(dim=(1, 2, 3))


@pytest.mark.parametrize("L,Kb,C,gain,holes", [(4, 2, 4, 1.0, 2), (6, 3, 3, 1.5, 6),
                                               (8, 1, 2, 2.0, 8), (4, 6, 4, 1.2, 0)])
def test_forward_matches_torch(orc, L, Kb, C, gain, holes):
    w = inputs.cnn2_weights(Kb, C, gain, 11, out_bias=1.0)
    sp = inputs.spins_tj(L, 24, holes, 12)
    la, sg = orc.cnn2_log_psi(L, Kb, C, w, sp, marshall=False)
    f, neg = torch_cnn2(L, Kb, C, w, sp)
    np.testing.assert_allclose(la, f.numpy(), rtol=1e-12, atol=1e-11)
    assert np.array_equal(sg, np.where(neg.numpy() % 2 == 0, 1, -1))
    assert 0 < (neg.numpy() % 2).sum() < sp.shape[0] or Kb == 6   # both signs occur
    la2, sg2 = orc.cnn2_log_psi(L, Kb, C, w, sp, marshall=True)
    m = np.array([orc.marshall_sign(L, s) for s in sp])
    assert np.array_equal(la2, la) and np.array_equal(sg2, sg * m)


def test_param_count(orc):
    for Kb, C in ((1, 1), (2, 4), (6, 16), (6, 32), (3, 7)):
        P = orc.cnn2_num_params(Kb, C)
        assert P == inputs.cnn2_num_params(Kb, C)
        assert P == 3 * C + Kb * (2 * (9 * C * C + C)) + 9 * C + 1
    assert orc.cnn2_num_params(6, 32) == 111361


@pytest.mark.parametrize("L,Kb,C,gain", [(4, 2, 4, 1.0), (6, 3, 3, 1.5)])
def test_log_deriv_matches_autograd(orc, L, Kb, C, gain):
    w = inputs.cnn2_weights(Kb, C, gain, 21, out_bias=1.0)
    sp = inputs.spins_tj(L, 6, 4, 22)
    O = orc.cnn2_log_deriv(L, Kb, C, w, sp)
    for s in range(sp.shape[0]):
        wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
        f, _ = torch_cnn2(L, Kb, C, wt, sp[s:s + 1])
        (g,) = torch.autograd.grad(f.sum(), wt)
        g = g.numpy()
        np.testing.assert_allclose(O[s], g, rtol=1e-10, atol=1e-12 * np.abs(g).max())


def test_log_deriv_finite_differences(orc):
    L, Kb, C = 4, 2, 3
    w = inputs.cnn2_weights(Kb, C, 1.2, 31, out_bias=2.0)
    sp = inputs.spins_tj(L, 3, 2, 32)
    O = orc.cnn2_log_deriv(L, Kb, C, w, sp)
    rng = np.random.default_rng(33)
    picks = np.concatenate([np.arange(3 * C), rng.choice(w.shape[0], 16, replace=False)])
    for p in picks:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd = (orc.cnn2_log_psi(L, Kb, C, wp, sp)[0] - orc.cnn2_log_psi(L, Kb, C, wm, sp)[0]) / (2 * h)
        np.testing.assert_allclose(O[:, p], fd, rtol=1e-5, atol=1e-6)


def test_translation_invariance(orc):
    L, Kb, C = 6, 3, 4
    w = inputs.cnn2_weights(Kb, C, 1.5, 41, out_bias=1.0)
    sp = inputs.spins_tj(L, 8, 4, 42)
    la, sg = orc.cnn2_log_psi(L, Kb, C, w, sp, marshall=False)
    for dy, dx in ((1, 0), (0, 1), (2, 3)):
        la2, sg2 = orc.cnn2_log_psi(L, Kb, C, w, np.roll(sp, (dy, dx), axis=(1, 2)),
                                    marshall=False)
        np.testing.assert_allclose(la2, la, rtol=1e-13, atol=1e-12)
        assert np.array_equal(sg2, sg)


def _shift_pooled_channels(w, Kb, C, r):
    """Weights whose pre-pool channel c is the original channel (c + r) mod C
    in every block: rows of W and a, and the input channels of V."""
    w = w.copy()
    perm = (np.arange(C) + r) % C
    off = 3 * C
    for _ in range(Kb):
        W = w[off:off + 9 * C * C].reshape(C, C, 9)
        w[off:off + 9 * C * C] = W[perm].ravel()
        off += 9 * C * C
        w[off:off + C] = w[off:off + C][perm]
        off += C
        V = w[off:off + 9 * C * C].reshape(C, C, 9)
        w[off:off + 9 * C * C] = V[perm].ravel()
        off += 9 * C * C + C
    return w


def test_stride_one_pool_wraps_the_channels(orc):
    """A cyclic shift of the pooled channels leaves psi unchanged only if the
    last channel's window takes the first channel; a transposition of two
    channels (not a cyclic shift) does change it."""
    L, Kb, C = 4, 2, 5
    w = inputs.cnn2_weights(Kb, C, 1.5, 51, out_bias=1.0)
    sp = inputs.spins_tj(L, 8, 2, 52)
    la, sg = orc.cnn2_log_psi(L, Kb, C, w, sp, marshall=False)
    for r in (1, 2, 4):
        la2, sg2 = orc.cnn2_log_psi(L, Kb, C, _shift_pooled_channels(w, Kb, C, r), sp,
                                    marshall=False)
        np.testing.assert_allclose(la2, la, rtol=1e-13, atol=1e-12)
        assert np.array_equal(sg2, sg)
    wt = w.copy()
    off = 3 * C
    W = wt[off:off + 9 * C * C].reshape(C, C, 9).copy()
    W[[0, 2]] = W[[2, 0]]
    wt[off:off + 9 * C * C] = W.ravel()
    a = wt[off + 9 * C * C:off + 9 * C * C + C]
    a[[0, 2]] = a[[2, 0]]
    V0 = off + 9 * C * C + C
    V = wt[V0:V0 + 9 * C * C].reshape(C, C, 9).copy()
    V[[0, 2]] = V[[2, 0]]
    wt[V0:V0 + 9 * C * C] = V.ravel()
    la3, _ = orc.cnn2_log_psi(L, Kb, C, wt, sp, marshall=False)
    assert np.abs(la3 - la).max() > 1e-6


@pytest.mark.parametrize("marshall", [True, False])
def test_tj_rayleigh_quotient_with_cnn2_sign(orc, marshall):
    L, Kb, C = 4, 2, 3
    H, basis = ed.tj_hamiltonian(L, T_HOP, J_EX, 2, 2)
    w = inputs.cnn2_weights(Kb, C, 1.5, 61, out_bias=0.5)
    spins = ed.tj_modes_to_spins(basis, 16).reshape(-1, 4, 4)
    la, sg = orc.cnn2_log_psi(L, Kb, C, w, spins, marshall=marshall)
    assert 0 < (sg < 0).sum() < sg.shape[0]
    psi = sg * np.exp(la - la.max())
    e = orc.tj_cnn2_local_energy(L, T_HOP, J_EX, Kb, C, w, spins, marshall=marshall)
    lhs = np.sum(psi ** 2 * e) / np.sum(psi ** 2)
    rhs = psi @ (H @ psi) / (psi @ psi)
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_tj_cnn2_mcmc_conserves_and_is_reproducible(orc):
    L, Kb, C, B, T = 6, 2, 3, 12, 20
    w = inputs.cnn2_weights(Kb, C, 1.0, 71, out_bias=1.0)
    sp = inputs.spins_tj(L, B, 4, 72)
    rb, ru = inputs.mcmc_randoms(73, 0, T, B)
    out, acc = orc.tj_cnn2_mcmc(L, T_HOP, J_EX, Kb, C, w, sp, rb, ru)
    for v in (1, -1, 0):
        assert np.array_equal((out == v).sum(axis=(1, 2)), (sp == v).sum(axis=(1, 2)))
    assert 0 < acc.sum() < B * T
    out2, acc2 = orc.tj_cnn2_mcmc(L, T_HOP, J_EX, Kb, C, w, sp, rb, ru)
    assert np.array_equal(out, out2) and np.array_equal(acc, acc2)
