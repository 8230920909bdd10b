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


# ----------------------------------------------------------------------------
# t-J model [Sec. 6.1, Eq. tJ] from fermion operators
# ----------------------------------------------------------------------------
# A basis state is a string of 2N mode bits, bit 2 i for an up electron on
# site i and bit 2 i + 1 for a down electron, read as the product of its
# creation operators in increasing mode order acting on the vacuum.  An
# operator on mode m then picks up (-1)^{occupied modes below m}: that is the
# whole of the fermion sign, applied one operator at a time, with no shortcut
# through site strings.  Doubly occupied sites are outside the t-J space and
# are projected out.

_EVEN = sum(1 << (2 * i) for i in range(31))


def tj_sector_basis(N: int, n_up: int, n_dn: int) -> np.ndarray:
    """Mode strings of every configuration with n_up up and n_dn down
    electrons and no doubly occupied site, ascending."""
    states = []
    for ups in combinations(range(N), n_up):
        base = sum(1 << (2 * u) for u in ups)
        rest = [k for k in range(N) if k not in ups]
        for dns in combinations(rest, n_dn):
            states.append(base + sum(1 << (2 * d + 1) for d in dns))
    return np.array(sorted(states), dtype=np.int64)


def apply_fermion_ops(ops, states: np.ndarray):
    """Apply the operator product ops = [(mode, dagger), ...] (rightmost acts
    first) to every mode string.  Returns (new strings, signs, mask of the
    strings the product does not annihilate)."""
    st = np.array(states, dtype=np.int64)
    sign = np.ones(st.shape, np.int64)
    ok = np.ones(st.shape, bool)
    for m, dagger in reversed(ops):
        occ = (st >> m) & 1
        ok &= (occ == 0) if dagger else (occ == 1)
        below = np.bitwise_count(st & ((1 << m) - 1)).astype(np.int64)
        sign *= 1 - 2 * (below & 1)
        st = st ^ (1 << m)
    return st, sign, ok


def tj_terms(L: int, t: float, J: float):
    """(coefficient, operator product) of every term of H on the nearest-
    neighbour pairs of the torus: hopping, J S^z S^z, the J/2 spin flips and
    -J n n / 4, each written with c+ / c of the two modes of a site."""
    nn, _ = torus_pairs(L)
    terms = []
    for (i, j) in nn:
        for s in (0, 1):
            terms.append((-t, [(2 * i + s, True), (2 * j + s, False)]))
            terms.append((-t, [(2 * j + s, True), (2 * i + s, False)]))
        for si in (0, 1):
            for sj in (0, 1):
                ni_nj = [(2 * i + si, True), (2 * i + si, False),
                         (2 * j + sj, True), (2 * j + sj, False)]
                terms.append((J * (0.25 if si == sj else -0.25), ni_nj))   # S^z S^z
                terms.append((-J / 4.0, ni_nj))                             # -n n / 4
        # S+_i S-_j + S-_i S+_j with S+ = c+_up c_dn, S- = c+_dn c_up
        terms.append((J / 2.0, [(2 * i, True), (2 * i + 1, False),
                                (2 * j + 1, True), (2 * j, False)]))
        terms.append((J / 2.0, [(2 * i + 1, True), (2 * i, False),
                                (2 * j, True), (2 * j + 1, False)]))
    return terms


def _tj_allowed(st: np.ndarray) -> np.ndarray:
    return (st & (st >> 1) & _EVEN) == 0


def tj_hamiltonian(L: int, t: float, J: float, n_up: int, n_dn: int):
    """Sparse t-J Hamiltonian on the (n_up, n_dn) sector. Returns (H, basis)."""
    basis = tj_sector_basis(L * L, n_up, n_dn)
    dim = basis.shape[0]
    rows, cols, vals = [], [], []
    for coef, ops in tj_terms(L, t, J):
        if coef == 0.0:
            continue
        st, sign, ok = apply_fermion_ops(ops, basis)
        ok &= _tj_allowed(st)
        src = np.nonzero(ok)[0]
        tgt = np.searchsorted(basis, st[src])
        assert np.all(basis[tgt] == st[src])
        rows.append(tgt)
        cols.append(src)
        vals.append(coef * sign[src].astype(np.float64))
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    return H, basis


def tj_column(L: int, t: float, J: float, spins: np.ndarray):
    """H |S> of one configuration (site values +1 / -1 / 0): a dict from the
    site values of S' (bytes) to <S'|H|S>, the diagonal included."""
    st0 = np.array([tj_spins_to_modes(spins.reshape(1, -1))[0]], np.int64)
    out = {}
    for coef, ops in tj_terms(L, t, J):
        if coef == 0.0:
            continue
        st, sign, ok = apply_fermion_ops(ops, st0)
        if ok[0] and _tj_allowed(st)[0]:
            key = tj_modes_to_spins(st, L * L)[0].tobytes()
            out[key] = out.get(key, 0.0) + coef * float(sign[0])
    return out


def tj_modes_to_spins(basis: np.ndarray, N: int) -> np.ndarray:
    """int8 [dim, N] site values (+1 up, -1 down, 0 hole) of mode strings."""
    up = (basis[:, None] >> (2 * np.arange(N))[None, :]) & 1
    dn = (basis[:, None] >> (2 * np.arange(N) + 1)[None, :]) & 1
    return (up - dn).astype(np.int8)


def tj_spins_to_modes(spins: np.ndarray) -> np.ndarray:
    """Mode strings of site-value rows [B, N]."""
    s = np.asarray(spins).reshape(spins.shape[0], -1).astype(np.int64)
    N = s.shape[1]
    bit = np.where(s > 0, 2 * np.arange(N), 2 * np.arange(N) + 1)
    return np.where(s != 0, np.left_shift(np.int64(1), bit), 0).sum(axis=1)


def tj_ground(H):
    """Lowest eigenpair of a t-J sector by ARPACK (large sectors)."""
    from scipy.sparse.linalg import eigsh
    v0 = np.random.default_rng(5).standard_normal(H.shape[0])
    vals, vecs = eigsh(H, k=1, which="SA", tol=1e-13, v0=v0)
    return float(vals[0]), vecs[:, 0]
