"""FP64 CPU oracle for the CNN-VMC J1-J2 hot path (arxiv 2204.07816).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and nothing here imports the GPU library.

The arithmetic lives in ``nqs_oracle.c`` (plain C, FP64); this module only
marshals numpy arrays through ctypes.  ``ed.py`` holds the exact-diagonalisation
test support (Hamiltonian built from spin operators by bit manipulation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nqs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-D_GNU_SOURCE", "-o", _LIB_PATH, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    d, i8, i32, i64 = ctypes.c_double, ctypes.c_int8, ctypes.c_int32, ctypes.c_int64
    ci = ctypes.c_int
    sig = {
        "oracle_num_params": (i64, [ci, ci]),
        "oracle_marshall_sign": (ci, [ci, P(i8)]),
        "oracle_bond_sites": (ci, [ci, ci, P(ci), P(ci)]),
        "oracle_connected": (None, [ci, d, d, P(i8), P(i32), P(i32), P(i8), P(d)]),
        "oracle_log_psi": (None, [ci, ci, ci, P(d), P(i8), i64, P(d), P(i8), ci]),
        "oracle_local_energy": (None, [ci, d, d, ci, ci, P(d), P(i8), i64, P(d), ci]),
        "oracle_local_energy_table": (None, [ci, d, d, P(d), P(i8), P(i8), i64, P(d), ci]),
        "oracle_tj_check": (ci, [ci, P(i8), i64]),
        "oracle_tj_connected": (None, [ci, d, d, P(i8), P(i32), P(i32), P(i8), P(d), P(d)]),
        "oracle_tj_local_energy": (None, [ci, d, d, ci, ci, P(d), P(i8), i64, P(d), ci]),
        "oracle_tj_local_energy_table": (None, [ci, d, d, i64, P(i64), P(d), P(i8), P(i8), i64,
                                                P(d), ci]),
        "oracle_log_deriv": (None, [ci, ci, ci, P(d), P(i8), i64, P(d), ci]),
        "oracle_cnn1_num_params": (i64, [ci, ci]),
        "oracle_cnn1_log_psi": (None, [ci, ci, ci, P(d), ci, P(i8), i64, P(d), P(i8), ci]),
        "oracle_cnn1_local_energy": (None, [ci, d, d, ci, ci, P(d), ci, P(i8), i64, P(d), ci]),
        "oracle_cnn1_log_deriv": (None, [ci, ci, ci, P(d), P(i8), i64, P(d), ci]),
        "oracle_tj_cnn1_local_energy": (None, [ci, d, d, ci, ci, P(d), ci, P(i8), i64, P(d),
                                               ci]),
        "oracle_cnn2_num_params": (i64, [ci, ci]),
        "oracle_cnn2_log_psi": (None, [ci, ci, ci, P(d), ci, P(i8), i64, P(d), P(i8), ci]),
        "oracle_cnn2_log_deriv": (None, [ci, ci, ci, P(d), P(i8), i64, P(d), ci]),
        "oracle_tj_cnn2_local_energy": (None, [ci, d, d, ci, ci, P(d), ci, P(i8), i64, P(d),
                                               ci]),
        "oracle_sens_layers": (None, [ci, ci, ci, P(d), P(i8), P(d), P(d), P(d), P(d), P(d)]),
        "oracle_dlog_sens": (None, [ci, ci, ci, P(d), P(i8), i64, P(i32), P(i32), i64, P(d),
                                    ci]),
        "oracle_energy_stats": (None, [P(d), i64, P(d)]),
        "oracle_sr_cg": (None, [P(d), P(d), i64, i64, d, ci, P(d), P(d)]),
        "oracle_sr_dense": (ci, [P(d), P(d), i64, i64, d, P(d)]),
        "oracle_sr_apply": (None, [P(d), i64, i64, d, P(d), P(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _spins(spins, L):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1, L * L)
    return s


def num_params(K: int, C: int) -> int:
    return int(_load().oracle_num_params(K, C))


def marshall_sign(L: int, spins) -> int:
    s = _spins(spins, L)[0]
    return int(_load().oracle_marshall_sign(L, _p(s, ctypes.c_int8)))


def bond_sites(L: int, b: int):
    i, j = ctypes.c_int(), ctypes.c_int()
    cls = _load().oracle_bond_sites(L, b, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value, int(cls)


def connected(L: int, J1: float, J2: float, spins):
    """Per-sample connected list: (counts[B], list of bond-id arrays, list of mu arrays, e_diag[B])."""
    s = _spins(spins, L)
    B, N = s.shape
    lib = _load()
    counts = np.zeros(B, np.int32)
    ediag = np.zeros(B, np.float64)
    bonds, mus = [], []
    bid = np.zeros(4 * N, np.int32)
    mu = np.zeros(4 * N, np.int8)
    for b in range(B):
        c = ctypes.c_int32()
        e = ctypes.c_double()
        row = np.ascontiguousarray(s[b])
        lib.oracle_connected(L, J1, J2, _p(row, ctypes.c_int8), ctypes.byref(c),
                             _p(bid, ctypes.c_int32), _p(mu, ctypes.c_int8), ctypes.byref(e))
        counts[b] = c.value
        ediag[b] = e.value
        bonds.append(bid[:c.value].copy())
        mus.append(mu[:c.value].copy())
    return counts, bonds, mus, ediag


def log_psi(L: int, K: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    la = np.zeros(B, np.float64)
    sg = np.zeros(B, np.int8)
    _load().oracle_log_psi(L, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8), B,
                           _p(la, ctypes.c_double), _p(sg, ctypes.c_int8), nthreads)
    return la, sg


def local_energy(L: int, J1: float, J2: float, K: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_local_energy(L, J1, J2, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8),
                                B, _p(e, ctypes.c_double), nthreads)
    return e


def local_energy_table(L: int, J1: float, J2: float, log_abs_tab, sign_tab, spins,
                       nthreads: int = 0):
    s = _spins(spins, L)
    la = np.ascontiguousarray(log_abs_tab, np.float64)
    sg = np.ascontiguousarray(sign_tab, np.int8)
    assert la.shape[0] == (1 << (L * L)) and sg.shape[0] == la.shape[0]
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_local_energy_table(L, J1, J2, _p(la, ctypes.c_double), _p(sg, ctypes.c_int8),
                                      _p(s, ctypes.c_int8), B, _p(e, ctypes.c_double), nthreads)
    return e


def tj_connected(L: int, t: float, J: float, spins):
    """t-J connected lists (Sec. 6.1, Eq. tJ): (counts[B], bond-id arrays,
    Marshall-ratio arrays, matrix-element arrays, e_diag[B])."""
    s = _spins(spins, L)
    B, N = s.shape
    lib = _load()
    counts = np.zeros(B, np.int32)
    ediag = np.zeros(B, np.float64)
    bonds, mus, hs = [], [], []
    bid = np.zeros(4 * N, np.int32)
    mu = np.zeros(4 * N, np.int8)
    hv = np.zeros(4 * N, np.float64)
    for b in range(B):
        c = ctypes.c_int32()
        e = ctypes.c_double()
        row = np.ascontiguousarray(s[b])
        lib.oracle_tj_connected(L, t, J, _p(row, ctypes.c_int8), ctypes.byref(c),
                                _p(bid, ctypes.c_int32), _p(mu, ctypes.c_int8),
                                _p(hv, ctypes.c_double), ctypes.byref(e))
        counts[b] = c.value
        ediag[b] = e.value
        bonds.append(bid[:c.value].copy())
        mus.append(mu[:c.value].copy())
        hs.append(hv[:c.value].copy())
    return counts, bonds, mus, hs, ediag


def tj_check(L: int, spins) -> bool:
    s = _spins(spins, L)
    return bool(_load().oracle_tj_check(L, _p(s, ctypes.c_int8), s.shape[0]))


def tj_local_energy(L: int, t: float, J: float, K: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_tj_local_energy(L, t, J, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8),
                                   B, _p(e, ctypes.c_double), nthreads)
    return e


def tj_key(spins, L: int):
    """Table keys sum_i c_i 4^i (c = 0 hole, 1 up, 2 down) of [B][N] configurations."""
    s = _spins(spins, L).astype(np.int64)
    code = np.where(s > 0, 1, np.where(s < 0, 2, 0)).astype(np.int64)
    return (code << (2 * np.arange(L * L, dtype=np.int64))).sum(axis=1)


def tj_local_energy_table(L: int, t: float, J: float, keys, log_abs_tab, sign_tab, spins,
                          nthreads: int = 0):
    s = _spins(spins, L)
    k = np.ascontiguousarray(keys, np.int64)
    assert L * L <= 31 and np.all(np.diff(k) > 0)
    la = np.ascontiguousarray(log_abs_tab, np.float64)
    sg = np.ascontiguousarray(sign_tab, np.int8)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_tj_local_energy_table(L, t, J, k.shape[0], _p(k, ctypes.c_int64),
                                         _p(la, ctypes.c_double), _p(sg, ctypes.c_int8),
                                         _p(s, ctypes.c_int8), B, _p(e, ctypes.c_double),
                                         nthreads)
    return e


def log_deriv(L: int, K: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    P = num_params(K, C)
    assert w.shape[0] == P
    O = np.zeros((B, P), np.float64)
    _load().oracle_log_deriv(L, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8), B,
                             _p(O, ctypes.c_double), nthreads)
    return O


def cnn1_num_params(Kb: int, C: int) -> int:
    return int(_load().oracle_cnn1_num_params(Kb, C))


def cnn1_log_psi(L: int, Kb: int, C: int, w, spins, marshall: bool = True, nthreads: int = 0):
    """CNN1 (Sec. 5.2, reading in nqs_oracle.h): (log|psi| [B], sign [B])."""
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    assert w.shape[0] == cnn1_num_params(Kb, C)
    B = s.shape[0]
    la = np.zeros(B, np.float64)
    sg = np.zeros(B, np.int8)
    _load().oracle_cnn1_log_psi(L, Kb, C, _p(w, ctypes.c_double), int(marshall),
                                _p(s, ctypes.c_int8), B, _p(la, ctypes.c_double),
                                _p(sg, ctypes.c_int8), nthreads)
    return la, sg


def cnn1_local_energy(L: int, J1: float, J2: float, Kb: int, C: int, w, spins,
                      marshall: bool = True, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_cnn1_local_energy(L, J1, J2, Kb, C, _p(w, ctypes.c_double), int(marshall),
                                     _p(s, ctypes.c_int8), B, _p(e, ctypes.c_double), nthreads)
    return e


def tj_cnn1_local_energy(L: int, t: float, J: float, Kb: int, C: int, w, spins,
                         marshall: bool = True, nthreads: int = 0):
    """t-J local energy (Sec. 6.1) with the CNN1 amplitude, sign included."""
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_tj_cnn1_local_energy(L, t, J, Kb, C, _p(w, ctypes.c_double), int(marshall),
                                        _p(s, ctypes.c_int8), B, _p(e, ctypes.c_double),
                                        nthreads)
    return e


def cnn1_log_deriv(L: int, Kb: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    P = cnn1_num_params(Kb, C)
    O = np.zeros((B, P), np.float64)
    _load().oracle_cnn1_log_deriv(L, Kb, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8), B,
                                  _p(O, ctypes.c_double), nthreads)
    return O


def cnn2_num_params(Kb: int, C: int) -> int:
    return int(_load().oracle_cnn2_num_params(Kb, C))


def cnn2_log_psi(L: int, Kb: int, C: int, w, spins, marshall: bool = True, nthreads: int = 0):
    """CNN2 (Sec. 5.2, reading in nqs_oracle.h): (log|psi| [B], sign [B]).
    Site values 0 (hole), +1 (up), -1 (down) select the embedding rows."""
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    assert w.shape[0] == cnn2_num_params(Kb, C)
    B = s.shape[0]
    la = np.zeros(B, np.float64)
    sg = np.zeros(B, np.int8)
    _load().oracle_cnn2_log_psi(L, Kb, C, _p(w, ctypes.c_double), int(marshall),
                                _p(s, ctypes.c_int8), B, _p(la, ctypes.c_double),
                                _p(sg, ctypes.c_int8), nthreads)
    return la, sg


def tj_cnn2_local_energy(L: int, t: float, J: float, Kb: int, C: int, w, spins,
                         marshall: bool = True, nthreads: int = 0):
    """t-J local energy (Sec. 6.1) with the CNN2 amplitude, sign included."""
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    assert w.shape[0] == cnn2_num_params(Kb, C)
    B = s.shape[0]
    e = np.zeros(B, np.float64)
    _load().oracle_tj_cnn2_local_energy(L, t, J, Kb, C, _p(w, ctypes.c_double), int(marshall),
                                        _p(s, ctypes.c_int8), B, _p(e, ctypes.c_double),
                                        nthreads)
    return e


def cnn2_log_deriv(L: int, Kb: int, C: int, w, spins, nthreads: int = 0):
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    B = s.shape[0]
    P = cnn2_num_params(Kb, C)
    assert w.shape[0] == P
    O = np.zeros((B, P), np.float64)
    _load().oracle_cnn2_log_deriv(L, Kb, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8), B,
                                  _p(O, ctypes.c_double), nthreads)
    return O


def sens_layers(L: int, K: int, C: int, w, spins):
    """Every layer of one configuration, arrays [K, C, L, L]: z, h = ln cosh z,
    a = |b| + sum |W||h_in|, g = df/dh_k, d = df/dz_k (test support)."""
    s = _spins(spins, L)[:1].copy()
    w = np.ascontiguousarray(w, np.float64)
    arrs = [np.zeros(K * C * L * L) for _ in range(5)]
    _load().oracle_sens_layers(L, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8),
                               *[_p(a, ctypes.c_double) for a in arrs])
    return {k: a.reshape(K, C, L, L) for k, a in zip("zhagd", arrs)}


def dlog_sens(L: int, K: int, C: int, w, spins, samples, bonds, nthreads: int = 0):
    """Per item (samples[m], bonds[m]): [f(S')-f(S), S1_act, S2_act, S1_acc,
    S1_lc, S2_acc] (bond < 0: the sample itself), the first-order rounding
    sensitivities of nqs_oracle.h.  Returns float64 [M, 6]."""
    s = _spins(spins, L)
    w = np.ascontiguousarray(w, np.float64)
    sm = np.ascontiguousarray(samples, np.int32)
    bd = np.ascontiguousarray(bonds, np.int32)
    M = sm.shape[0]
    out = np.zeros((M, 6))
    _load().oracle_dlog_sens(L, K, C, _p(w, ctypes.c_double), _p(s, ctypes.c_int8), s.shape[0],
                             _p(sm, ctypes.c_int32), _p(bd, ctypes.c_int32), M,
                             _p(out, ctypes.c_double), nthreads)
    return out


def energy_stats(e):
    e = np.ascontiguousarray(e, np.float64)
    st = np.zeros(2, np.float64)
    _load().oracle_energy_stats(_p(e, ctypes.c_double), e.shape[0], _p(st, ctypes.c_double))
    return float(st[0]), float(st[1])


def sr_cg(O, e, lam: float = 1e-4, n_iter: int = 100):
    O = np.ascontiguousarray(O, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    B, P = O.shape
    x = np.zeros(P, np.float64)
    st = np.zeros(2, np.float64)
    _load().oracle_sr_cg(_p(O, ctypes.c_double), _p(e, ctypes.c_double), B, P, lam, n_iter,
                         _p(x, ctypes.c_double), _p(st, ctypes.c_double))
    return x, float(st[0]), int(st[1])


def sr_dense(O, e, lam: float = 1e-4):
    O = np.ascontiguousarray(O, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    B, P = O.shape
    x = np.zeros(P, np.float64)
    rc = _load().oracle_sr_dense(_p(O, ctypes.c_double), _p(e, ctypes.c_double), B, P, lam,
                                 _p(x, ctypes.c_double))
    if rc != 0:
        raise np.linalg.LinAlgError("S + lambda I not positive definite")
    return x


def sr_apply(O, v, lam: float = 1e-4):
    O = np.ascontiguousarray(O, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    B, P = O.shape
    y = np.zeros(P, np.float64)
    _load().oracle_sr_apply(_p(O, ctypes.c_double), B, P, lam, _p(v, ctypes.c_double),
                            _p(y, ctypes.c_double))
    return y


def _metropolis(L, types, K, C, w, spins, rand_bond, rand_u, logpsi=None):
    """Metropolis steps of every chain with proposals over the bond types
    `types` (see mcmc); the pair's site values are exchanged on acceptance.
    logpsi(w, spins) -> log|psi| (default: the ln cosh CNN)."""
    if logpsi is None:
        def logpsi(w_, s_):
            return log_psi(L, K, C, w_, s_)[0]
    s = _spins(spins, L).copy()
    B, N = s.shape
    acc = np.zeros(B, np.int64)
    if not types:
        return s.reshape(B, L, L), acc
    rb = np.asarray(rand_bond, np.int64).astype(np.uint32)
    ru = np.asarray(rand_u, np.float64)
    n = len(types)
    for t in range(rb.shape[0]):
        prop = s.copy()
        pairs = []
        for b in range(B):
            q = int(rb[t, b]) % (N * n)
            i, j, _ = bond_sites(L, 4 * (q // n) + types[q % n])
            pairs.append((i, j))
            prop[b, i], prop[b, j] = s[b, j], s[b, i]
        f0 = logpsi(w, s)
        f1 = logpsi(w, prop)
        for b, (i, j) in enumerate(pairs):
            if s[b, i] != s[b, j] and ru[t, b] < np.exp(2.0 * (f1[b] - f0[b])):
                s[b] = prop[b]
                acc[b] += 1
    return s.reshape(B, L, L), acc


def mcmc(L: int, J1: float, J2: float, K: int, C: int, w, spins, rand_bond, rand_u):
    """Metropolis sampling of |psi|^2 by pair exchanges (Sec. 3.2: walkers
    sample |psi|^2; Sec. 5.4.1: independent chains whose proposals are the
    exchanged configurations).  Step t of chain b proposes the bond of
    q = rand_bond[t, b] mod (N n), n = 2 for one non-zero coupling and 4 for
    both: site q // n, type the (q mod n)-th of the types of the non-zero
    couplings (J1: 0, 1; J2: 2, 3).  A pair of different values is exchanged
    when rand_u[t, b] < exp(2 (f(S') - f(S))), f = log|psi| by two full
    forwards.  Returns (spins after the steps, accepted moves per chain)."""
    types = ([0, 1] if J1 != 0.0 else []) + ([2, 3] if J2 != 0.0 else [])
    return _metropolis(L, types, K, C, w, spins, rand_bond, rand_u)


def tj_mcmc(L: int, t: float, J: float, K: int, C: int, w, spins, rand_bond, rand_u):
    """The same sampler for the t-J model (Sec. 6.1): proposals over the
    nearest-neighbour bonds (n = 2) when t or J is non-zero; a move exchanges
    two antiparallel electrons or an electron and a hole, so the numbers of up
    electrons, down electrons and holes are conserved."""
    types = [0, 1] if (t != 0.0 or J != 0.0) else []
    return _metropolis(L, types, K, C, w, spins, rand_bond, rand_u)


def cnn1_mcmc(L: int, J1: float, J2: float, Kb: int, C: int, w, spins, rand_bond, rand_u):
    """The sampler of mcmc with the CNN1 amplitude."""
    types = ([0, 1] if J1 != 0.0 else []) + ([2, 3] if J2 != 0.0 else [])
    return _metropolis(L, types, Kb, C, w, spins, rand_bond, rand_u,
                       lambda w_, s_: cnn1_log_psi(L, Kb, C, w_, s_)[0])


def _vmc(L, sampler, eloc, K, C, w, spins, n_iter, lr, lam, cg_iters, randoms, oderiv=None,
         solve=None):
    """solve(O, e, lam, n_iter) -> (x, rel_res, it) replaces sr_cg when given
    (the same system solved with its sums taken in another order)."""
    if solve is None:
        solve = sr_cg
    w = np.array(w, np.float64)
    s = _spins(spins, L).reshape(-1, L, L).copy()
    means, variances = [], []
    for it in range(n_iter):
        rb, ru = randoms(it)
        s, _ = sampler(w, s, rb, ru)
        e = eloc(w, s)
        m, v = energy_stats(e)
        means.append(m)
        variances.append(v)
        O = oderiv(w, s) if oderiv else log_deriv(L, K, C, w, s)
        x, _, _ = solve(O, e, lam, cg_iters)
        w = w - lr * x
    return np.array(means), np.array(variances), w, s


def vmc(L: int, J1: float, J2: float, K: int, C: int, w, spins, n_iter: int, steps: int,
        lr: float, lam: float, cg_iters: int, randoms):
    """The variational Monte Carlo self-learning loop (Sec. 3.2): per
    iteration, `steps` Metropolis steps of every chain, the local energies and
    log-derivatives of the resulting samples, the SR direction by CG
    (sr_cg), and the update theta <- theta - lr * delta.  randoms(it) gives the
    iteration's (rand_bond, rand_u).  Returns (energy means per iteration,
    variances per iteration, final weights, final spins)."""
    del steps   # the step count is the leading dimension of the randoms
    return _vmc(L, lambda w, s, rb, ru: mcmc(L, J1, J2, K, C, w, s, rb, ru),
                lambda w, s: local_energy(L, J1, J2, K, C, w, s),
                K, C, w, spins, n_iter, lr, lam, cg_iters, randoms)


def tj_vmc(L: int, t: float, J: float, K: int, C: int, w, spins, n_iter: int, lr: float,
           lam: float, cg_iters: int, randoms, solve=None):
    """The same loop for the t-J model (tj_mcmc, tj_local_energy)."""
    return _vmc(L, lambda w, s, rb, ru: tj_mcmc(L, t, J, K, C, w, s, rb, ru),
                lambda w, s: tj_local_energy(L, t, J, K, C, w, s),
                K, C, w, spins, n_iter, lr, lam, cg_iters, randoms, solve=solve)


def cnn1_vmc(L: int, J1: float, J2: float, Kb: int, C: int, w, spins, n_iter: int, lr: float,
             lam: float, cg_iters: int, randoms, marshall: bool = True):
    """The loop of vmc with the CNN1 amplitude (cnn1_mcmc, cnn1_local_energy,
    cnn1_log_deriv)."""
    return _vmc(L, lambda w, s, rb, ru: cnn1_mcmc(L, J1, J2, Kb, C, w, s, rb, ru),
                lambda w, s: cnn1_local_energy(L, J1, J2, Kb, C, w, s, marshall=marshall),
                Kb, C, w, spins, n_iter, lr, lam, cg_iters, randoms,
                oderiv=lambda w, s: cnn1_log_deriv(L, Kb, C, w, s))


def tj_cnn2_mcmc(L: int, t: float, J: float, Kb: int, C: int, w, spins, rand_bond, rand_u):
    """The t-J sampler (tj_mcmc) with the CNN2 amplitude."""
    types = [0, 1] if (t != 0.0 or J != 0.0) else []
    return _metropolis(L, types, Kb, C, w, spins, rand_bond, rand_u,
                       lambda w_, s_: cnn2_log_psi(L, Kb, C, w_, s_)[0])


def tj_cnn1_mcmc(L: int, t: float, J: float, Kb: int, C: int, w, spins, rand_bond, rand_u):
    """The t-J sampler (tj_mcmc) with the CNN1 amplitude."""
    types = [0, 1] if (t != 0.0 or J != 0.0) else []
    return _metropolis(L, types, Kb, C, w, spins, rand_bond, rand_u,
                       lambda w_, s_: cnn1_log_psi(L, Kb, C, w_, s_)[0])
