"""Pins of the oracle's learned-preconditioner reference (CPU).

* MLP backward against central finite differences of the forward;
* the loss gradient through a stale-factor solve against finite differences;
* the preconditioner D K_s^{-1} D is SPD for arbitrary parameters;
* Adam against its closed form on a one-parameter quadratic;
* PCG with M^{-1} = K^{-1} converges in one step (exact preconditioner).
"""
import numpy as np
import pytest
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


def _pcg_iterate(K, b, Minv, k):
    """x_k of the oracle's PCG from x0 = 0 (its stopping test is called once
    on x0 and once per iteration; it stops after the k-th)."""
    calls = [0]

    def stop(_x):
        calls[0] += 1
        return calls[0] > k
    x, it, ok = mlp.pcg(lambda v: K @ v, b, lambda r: Minv @ r, np.zeros(len(b)), stop, 50)
    assert it == k and ok
    return x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pcg_iterates_are_krylov_projections(seed):
    """CG optimality (Hestenes & Stiefel 1952): with K SPD and the SPD
    preconditioner M^{-1}, the k-th iterate from x0 = 0 minimises the K-norm
    of the error over the Krylov space span{M^{-1}b, (M^{-1}K)M^{-1}b, ...,
    (M^{-1}K)^{k-1}M^{-1}b}, i.e. x_k = V (V^T K V)^{-1} V^T b for any basis V
    of that space.  A wrong beta, a wrong direction update p = z + beta p, a
    residual update with the wrong sign or an unpreconditioned inner product
    all leave that space or lose the optimality from the second step on."""
    rng = np.random.default_rng(100 + seed)
    n = 30
    A = rng.standard_normal((n, n))
    K = A @ A.T / n + np.diag(10.0 ** rng.uniform(-1, 1, n))
    B = rng.standard_normal((n, n))
    Minv = B @ B.T / n + np.diag(rng.uniform(0.5, 2.0, n))   # SPD, far from K^{-1}
    b = rng.standard_normal(n)
    z0 = Minv @ b
    for k in range(1, 6):
        cols = [z0]
        for _ in range(k - 1):
            cols.append(Minv @ (K @ cols[-1]))
        V, _ = np.linalg.qr(np.array(cols).T)
        x_ref = V @ np.linalg.solve(V.T @ K @ V, V.T @ b)
        x = _pcg_iterate(K, b, Minv, k)
        assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref), k


def test_pcg_counts_match_eigenvalue_clusters():
    """Exact arithmetic: CG ends after as many steps as M^{-1}K has distinct
    eigenvalues; with M^{-1} = K^{-1} times a matrix with 3 distinct
    eigenvalues the oracle's PCG reaches 1e-12 in exactly 3 steps."""
    rng = np.random.default_rng(9)
    n = 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    K = Q @ np.diag(rng.uniform(1, 5, n)) @ Q.T
    C = np.diag(np.repeat([1.0, 3.0, 7.0], n // 3))
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    # M^{-1} K is similar to C: M^{-1} = K^{-1/2} U C U^T K^{-1/2}
    w, E = np.linalg.eigh(K)
    Kmh = E @ np.diag(w ** -0.5) @ E.T
    Minv = Kmh @ U @ C @ U.T @ Kmh
    b = rng.standard_normal(n)
    x, it, ok = mlp.pcg(lambda v: K @ v, b, lambda r: Minv @ r, np.zeros(n),
                        lambda x: np.linalg.norm(K @ x - b) <= 1e-12 * np.linalg.norm(b), 20)
    assert ok and it == 3


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
