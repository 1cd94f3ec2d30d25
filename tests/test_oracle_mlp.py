"""Pins of the oracle's learned-preconditioner reference (CPU).

* MLP backward against central finite differences of the forward;
* the loss gradient through a stale-factor solve against finite differences;
* the preconditioner D K_s^{-1} D is SPD for arbitrary parameters;
* Adam against its closed form on a one-parameter quadratic;
* PCG with M^{-1} = K^{-1} converges in one step (exact preconditioner).
"""
import numpy as np
import scipy.sparse as sp

from oracle import mlp


def rand_features(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, mlp.F)) * 0.5
    f[:, 7] = 1.0
    return f


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1) + 0.05 * rng.standard_normal(mlp.NPARAM)
    f = rand_features(9, 2)
    g_o = rng.standard_normal(9)
    o, cache = mlp.forward(theta, f)
    g = mlp.backward(theta, f, cache, g_o)
    idx = rng.choice(mlp.NPARAM, 40, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, mlp.H * mlp.F]])
    for i in idx:
        e = np.zeros(mlp.NPARAM); e[i] = 1e-6
        fd = (g_o @ mlp.forward(theta + e, f)[0] - g_o @ mlp.forward(theta - e, f)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_gradient_through_stale_solve():
    rng = np.random.default_rng(3)
    n = 12
    A = rng.standard_normal((n, n))
    Ks = A @ A.T + n * np.eye(n)
    Kn = Ks + np.diag(rng.random(n) * 5)
    b = rng.standard_normal(n)
    x = np.linalg.solve(Kn, b)
    solve = lambda v: np.linalg.solve(Ks, v)
    theta = mlp.init_params(4) + 0.1 * rng.standard_normal(mlp.NPARAM)
    f = rand_features(n, 5)
    L, g = mlp.loss_and_grad(theta, f, b, x, solve)
    for i in rng.choice(mlp.NPARAM, 30, replace=False):
        e = np.zeros(mlp.NPARAM); e[i] = 1e-6
        Lp, _ = mlp.loss_and_grad(theta + e, f, b, x, solve)
        Lm, _ = mlp.loss_and_grad(theta - e, f, b, x, solve)
        fd = (Lp - Lm) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_preconditioner_is_spd_for_any_parameters():
    rng = np.random.default_rng(6)
    n = 10
    A = rng.standard_normal((n, n))
    Ks = A @ A.T + np.eye(n)
    for s in range(5):
        theta = rng.standard_normal(mlp.NPARAM) * 0.3
        D = mlp.diag_of(mlp.forward(theta, rand_features(n, s))[0])
        M = np.diag(D) @ np.linalg.inv(Ks) @ np.diag(D)
        assert np.linalg.eigvalsh((M + M.T) / 2).min() > 0
        for _ in range(5):
            v = rng.standard_normal(n)
            assert v @ M @ v > 0


def test_adam_closed_form():
    theta, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    g = np.array([0.5])
    t1, m1, v1 = mlp.adam(theta, g, m, v, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> update = lr * g / (|g| + eps)
    assert np.allclose(t1, 1.0 - 0.1 * 0.5 / (0.5 + 1e-8))
    assert np.allclose(m1, 0.05) and np.allclose(v1, 0.00025)


def test_pcg_exact_preconditioner_one_step():
    rng = np.random.default_rng(7)
    n = 15
    A = rng.standard_normal((n, n))
    K = A @ A.T + np.eye(n)
    b = rng.standard_normal(n)
    Kinv = np.linalg.inv(K)
    x, it, ok = mlp.pcg(lambda v: K @ v, b, lambda r: Kinv @ r, np.zeros(n),
                        lambda x: np.abs(K @ x - b).max() < 1e-10, 10)
    assert ok and it == 1


def test_features_definition_on_tiny_data():
    """Features of a 3-variable system computed by hand."""
    n = 3
    w_ptr = np.array([0, 1, 3, 4]); w_idx = np.array([0, 0, 1, 2]); w_val = np.array([2.0, 0.5, 3.0, 1.0])
    J = sp.csr_matrix(np.array([[1.0, 0.0, 2.0], [0.0, 0.0, 1.0]]))
    sx_new, sx_old = np.array([1e2, 1.0, 1e-2]), np.array([1.0, 1.0, 1.0])
    d_new, d_old = np.array([1e4, 10.0]), np.array([1.0, 1.0])
    f = mlp.features(n, w_ptr, w_idx, w_val, J, sx_new, d_new, sx_old, d_old)
    kn = np.array([2 + 1e2 + 1e4, 3 + 1.0, 1 + 1e-2 + 4e4 + 10.0])
    ko = np.array([2 + 1 + 1, 3 + 1, 1 + 1 + 4 + 1])
    assert np.allclose(f[:, 0], np.log10(sx_new) / 8)
    assert np.allclose(f[:, 1], np.log10(sx_new / sx_old) / 8)
    assert np.allclose(f[:, 2], np.log10(kn) / 8)
    assert np.allclose(f[:, 3], np.log10(kn / ko) / 8)
    assert np.allclose(f[:, 4], [4 / 8, 0.0, 4 / 8])
    assert np.allclose(f[:, 5], [4 / 8, 0.0, 4 / 8])
    assert np.allclose(f[:, 6], [4 / 8, 0.0, 1 / 8])
    assert np.all(f[:, 7] == 1.0)
