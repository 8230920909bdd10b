"""Shared helpers of the GPU parity tests (imported only by tests marked gpu)."""
import sys

import numpy as np
import torch

import oracle
from paper_2204_07816_amd import inputs, nqs

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(spins):
    return torch.as_tensor(np.ascontiguousarray(spins, dtype=np.int8)).to(DEV)


def make_ctx(L, J2, K, C, w, dtype="fp64", J1=1.0, marshall=True):
    return nqs.Context(L, J1, J2, K, C, w, dtype=dtype, marshall_sign=marshall)


def oracle_item_dlog(L, K, C, w, spins, sample, bond):
    """f(S') - f(s) of one exchanged configuration, from two oracle forwards."""
    i, j, _ = oracle.bond_sites(L, int(bond))
    s = np.ascontiguousarray(spins[sample]).reshape(-1).copy()
    sp = s.copy()
    sp[i], sp[j] = s[j], s[i]
    f, _ = oracle.log_psi(L, K, C, w, np.stack([s, sp]).reshape(2, L, L))
    return f[1] - f[0]


def rel_inf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
