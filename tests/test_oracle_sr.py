"""Pins of the oracle's stochastic-reconfiguration solve (Sec. 3.2 and Sec. 5.4.1
"Distributed SR computation"; the paper forms S explicitly and factorises it, the
oracle's CG converges to the same solution).  Library pins: numpy dense algebra."""
import numpy as np
import pytest

from paper_2204_07816_amd import inputs


def dense_system(O, e, lam):
    Ob = O - O.mean(axis=0)
    S = Ob.T @ Ob / O.shape[0] + lam * np.eye(O.shape[1])
    F = Ob.T @ (e - e.mean()) / O.shape[0]
    return S, F


@pytest.fixture(scope="module")
def sr44(orc):
    L, K, C = 4, 2, 4
    w = inputs.weights(K, C, 0.05, seed=1000)
    sp = inputs.spins_sz0(L, 256, seed=2000)
    O = orc.log_deriv(L, K, C, w, sp)
    e = orc.local_energy(L, 1.0, 0.5, K, C, w, sp)
    return O, e


def test_sr_apply_matches_dense(orc, sr44):
    O, e = sr44
    rng = np.random.default_rng(0)
    v = rng.standard_normal(O.shape[1])
    S, _ = dense_system(O, e, 1e-4)
    np.testing.assert_allclose(orc.sr_apply(O, v, 1e-4), S @ v, rtol=1e-11, atol=1e-14)


def test_sr_dense_cholesky_matches_numpy(orc, sr44):
    O, e = sr44
    S, F = dense_system(O, e, 1e-3)
    x = orc.sr_dense(O, e, 1e-3)
    ref = np.linalg.solve(S, F)
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-12 * np.abs(ref).max())


def test_sr_cg_converges_to_dense(orc, sr44):
    O, e = sr44
    lam = 1e-2
    S, F = dense_system(O, e, lam)
    x, rel, it = orc.sr_cg(O, e, lam, n_iter=2000)
    ref = np.linalg.solve(S, F)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_sr_cg_fixed_iterations_and_error_monotone(orc):
    """CG runs exactly n_iter steps, and the A-norm of its error decreases monotonically."""
    L, K, C = 4, 2, 4
    w = inputs.weights(K, C, 0.6, seed=3)
    sp = inputs.spins_sz0(L, 300, seed=4)
    O = orc.log_deriv(L, K, C, w, sp)
    e = orc.local_energy(L, 1.0, 0.5, K, C, w, sp)
    lam = 1e-4
    S, F = dense_system(O, e, lam)
    ref = np.linalg.solve(S, F)
    errs = []
    for n in (1, 2, 4, 8, 16, 32):
        x, rel, it = orc.sr_cg(O, e, lam, n_iter=n)
        assert it == n
        d = x - ref
        errs.append(d @ S @ d)
        # the recursive residual tracks the true residual before convergence
        true_rel = np.linalg.norm(F - S @ x) / np.linalg.norm(F)
        assert rel == pytest.approx(true_rel, rel=1e-6)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_sr_cg_small_system_exact():
    """CG in exact arithmetic solves an n x n SPD system in n steps: 2x2 by hand."""
    import oracle
    # columns have zero mean, so Obar = O and S = O^T O / 4 = diag(0.5, 2);
    # F = O^T (e - mean e) / 4 = (0.5, 2); with lambda = 0.5, x = F / diag(S + lambda)
    O = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 2.0], [0.0, -2.0]])
    e = np.array([2.0, 0.0, 5.0, 1.0])
    x, rel, it = oracle.sr_cg(O, e, 0.5, n_iter=2)
    S = np.diag([0.5, 2.0]) + 0.5 * np.eye(2)
    F = O.T @ (e - e.mean()) / 4
    np.testing.assert_allclose(F, [0.5, 2.0])
    np.testing.assert_allclose(x, [0.5, 0.8], rtol=1e-14)
    assert it <= 2
