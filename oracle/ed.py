"""Exact diagonalisation of the spin-1/2 J1-J2 model on small tori (test support).

TEST INFRASTRUCTURE ONLY.  Builds the Hamiltonian of Sec. 6.1, Eq. (J1J2) of
arxiv 2204.07816 directly from spin operators acting on basis integers (bit i
set = spin up at site i), independently of the oracle's canonical bond
enumeration: neighbour pairs are found from torus geometry (minimum-image
displacement |dx|+|dy| = 1 for J1, |dx| = |dy| = 1 for J2), each unordered
pair counted once.  S = sigma/2, so S_i.S_j = S^z_i S^z_j + (S^+_i S^-_j + h.c.)/2.

The ground state is found by Lanczos with full reorthogonalisation; scipy's
ARPACK and dense LAPACK serve as library pins in the tests.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def torus_pairs(L: int):
    """(J1 pairs, J2 pairs): sorted lists of unordered site pairs (i < j)."""
    def disp(a, b):
        d = (b - a) % L
        return d - L if d > L // 2 else d

    nn, nnn = set(), set()
    N = L * L
    for i in range(N):
        for j in range(i + 1, N):
            dx = abs(disp(i % L, j % L))
            dy = abs(disp(i // L, j // L))
            if dx + dy == 1:
                nn.add((i, j))
            elif dx == 1 and dy == 1:
                nnn.add((i, j))
    return sorted(nn), sorted(nnn)


def sector_basis(N: int, n_up: int) -> np.ndarray:
    """All basis integers with n_up bits set, ascending."""
    states = []
    for ups in combinations(range(N), n_up):
        v = 0
        for u in ups:
            v |= 1 << u
        states.append(v)
    return np.array(sorted(states), dtype=np.int64)


def hamiltonian(L: int, J1: float, J2: float, n_up: int | None = None):
    """Sparse H on the sector with n_up up-spins (default N/2). Returns (H, basis)."""
    N = L * L
    if n_up is None:
        n_up = N // 2
    basis = sector_basis(N, n_up)
    nn, nnn = torus_pairs(L)
    pairs = [(i, j, J1) for (i, j) in nn] + [(i, j, J2) for (i, j) in nnn]
    dim = basis.shape[0]
    diag = np.zeros(dim)
    rows, cols, vals = [], [], []
    for (i, j, J) in pairs:
        if J == 0.0:
            continue
        bi = (basis >> i) & 1
        bj = (basis >> j) & 1
        szsz = np.where(bi == bj, 0.25, -0.25)
        diag += J * szsz
        anti = np.nonzero(bi != bj)[0]
        flipped = basis[anti] ^ ((1 << i) | (1 << j))
        tgt = np.searchsorted(basis, flipped)
        assert np.all(basis[tgt] == flipped)
        rows.append(tgt)
        cols.append(anti)
        vals.append(np.full(anti.shape[0], 0.5 * J))
    rows.append(np.arange(dim))
    cols.append(np.arange(dim))
    vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    return H, basis


def lanczos_ground(H, m: int = 300, seed: int = 7, tol: float = 1e-13):
    """Lowest eigenpair by Lanczos with full reorthogonalisation."""
    dim = H.shape[0]
    m = min(m, dim)
    rng = np.random.default_rng(seed)
    V = np.zeros((m + 1, dim))
    v = rng.standard_normal(dim)
    V[0] = v / np.linalg.norm(v)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    k_used = m
    prev = None
    for k in range(m):
        w = H @ V[k]
        alpha[k] = V[k] @ w
        w -= V[: k + 1].T @ (V[: k + 1] @ w)       # full reorthogonalisation
        w -= V[: k + 1].T @ (V[: k + 1] @ w)
        beta[k] = np.linalg.norm(w)
        if k >= 10 and k % 10 == 0:
            T = np.diag(alpha[: k + 1]) + np.diag(beta[:k], 1) + np.diag(beta[:k], -1)
            e0 = np.linalg.eigvalsh(T)[0]
            if prev is not None and abs(e0 - prev) < tol * abs(e0):
                k_used = k + 1
                break
            prev = e0
        if beta[k] < 1e-14:
            k_used = k + 1
            break
        V[k + 1] = w / beta[k]
    T = np.diag(alpha[:k_used]) + np.diag(beta[: k_used - 1], 1) + np.diag(beta[: k_used - 1], -1)
    evals, evecs = np.linalg.eigh(T)
    vec = V[:k_used].T @ evecs[:, 0]
    vec /= np.linalg.norm(vec)
    return float(evals[0]), vec


def basis_to_spins(basis: np.ndarray, N: int) -> np.ndarray:
    """int8 [dim, N] +-1 configurations of basis integers."""
    bits = (basis[:, None] >> np.arange(N)[None, :]) & 1
    return np.where(bits == 1, 1, -1).astype(np.int8)


def spins_to_index(spins: np.ndarray) -> np.ndarray:
    """Basis integer of each +-1 configuration (rows of [B, N])."""
    s = np.asarray(spins).reshape(spins.shape[0], -1)
    return ((s > 0).astype(np.int64) << np.arange(s.shape[1])[None, :]).sum(axis=1)
