"""Pins of the oracle's element model against closed forms and invariants (CPU only)."""
import numpy as np
import pytest

from oracle import fem

RNG = np.random.default_rng(1234)


def _rand_elems(d, ne=7, strain=0.2):
    X = RNG.standard_normal((ne, d + 1, d))
    # fix orientation
    D = np.swapaxes(X[:, 1:] - X[:, :1], 1, 2)
    neg = np.linalg.det(D) < 0
    idx = np.flatnonzero(neg)
    X[idx[:, None], [d - 1, d]] = X[idx[:, None], [d, d - 1]]
    x = X + strain * RNG.standard_normal(X.shape)
    Dx = np.swapaxes(x[:, 1:] - x[:, :1], 1, 2)
    bad = np.linalg.det(Dx) / np.linalg.det(np.swapaxes(X[:, 1:] - X[:, :1], 1, 2)) < 0.3
    x[bad] = X[bad] + 0.01 * RNG.standard_normal(X[bad].shape)  # keep J well above 0
    mu = 1e6 * np.exp(0.3 * RNG.standard_normal(ne)) / 2.6
    lam = 2.0 * mu
    return x, X, mu, lam


def _linear_elastic_stiffness(X, mu, lam):
    """Textbook small-strain element stiffness V0 B^T D B (Voigt, engineering shear)."""
    ne, nv, d = X.shape
    out = np.empty((ne, nv * d, nv * d))
    for e in range(ne):
        Dm = (X[e, 1:] - X[e, :1]).T
        V0 = np.linalg.det(Dm) / (2.0 if d == 2 else 6.0)
        Ginv = np.linalg.inv(Dm)  # row k = grad of shape function k+1
        grads = np.vstack([-Ginv.sum(0), Ginv])
        if d == 2:
            B = np.zeros((3, nv * d))
            for a in range(nv):
                gx, gy = grads[a]
                B[:, 2 * a:2 * a + 2] = [[gx, 0], [0, gy], [gy, gx]]
            Dmat = np.array([[lam[e] + 2 * mu[e], lam[e], 0], [lam[e], lam[e] + 2 * mu[e], 0], [0, 0, mu[e]]])
        else:
            B = np.zeros((6, nv * d))
            for a in range(nv):
                gx, gy, gz = grads[a]
                B[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz],
                                         [gy, gx, 0], [0, gz, gy], [gz, 0, gx]]
            Dmat = np.zeros((6, 6))
            Dmat[:3, :3] = lam[e]
            Dmat[np.arange(3), np.arange(3)] += 2 * mu[e]
            Dmat[3:, 3:] = mu[e] * np.eye(3)
        out[e] = V0 * B.T @ Dmat @ B
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_rest_state_is_stress_free(d):
    _, X, mu, lam = _rand_elems(d)
    assert np.allclose(fem.element_energy(X, X, mu, lam), 0.0, atol=1e-9)
    g = fem.element_gradient(X, X, mu, lam)
    assert np.max(np.abs(g)) < 1e-8 * np.max(mu)


@pytest.mark.parametrize("d", [2, 3])
def test_tangent_at_rest_is_linear_elasticity(d):
    _, X, mu, lam = _rand_elems(d)
    H = fem.element_hessian(X, X, mu, lam)
    K = _linear_elastic_stiffness(X, mu, lam)
    assert np.max(np.abs(H - K)) <= 1e-10 * np.max(np.abs(K))


@pytest.mark.parametrize("d", [2, 3])
def test_frame_invariance(d):
    x, X, mu, lam = _rand_elems(d)
    Q, _ = np.linalg.qr(RNG.standard_normal((d, d)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    xr = x @ Q.T + RNG.standard_normal(d)
    e0 = fem.element_energy(x, X, mu, lam)
    e1 = fem.element_energy(xr, X, mu, lam)
    assert np.allclose(e0, e1, rtol=1e-11, atol=0)
    g0 = fem.element_gradient(x, X, mu, lam)
    g1 = fem.element_gradient(xr, X, mu, lam)
    assert np.allclose(g0 @ Q.T, g1, rtol=1e-9, atol=1e-9 * np.abs(g0).max())


@pytest.mark.parametrize("d", [2, 3])
def test_element_forces_balance(d):
    x, X, mu, lam = _rand_elems(d)
    g = fem.element_gradient(x, X, mu, lam)
    assert np.max(np.abs(g.sum(axis=1))) <= 1e-9 * np.abs(g).max()


@pytest.mark.parametrize("d", [2, 3])
def test_gradient_matches_central_differences_of_energy(d):
    x, X, mu, lam = _rand_elems(d)
    g = fem.element_gradient(x, X, mu, lam)
    h = 1e-6
    for a in range(d + 1):
        for c in range(d):
            xp = x.copy(); xp[:, a, c] += h
            xm = x.copy(); xm[:, a, c] -= h
            fd = (fem.element_energy(xp, X, mu, lam) - fem.element_energy(xm, X, mu, lam)) / (2 * h)
            assert np.allclose(fd, g[:, a, c], rtol=1e-6, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("d", [2, 3])
def test_hessian_matches_differences_of_gradient_and_is_symmetric(d):
    x, X, mu, lam = _rand_elems(d)
    H = fem.element_hessian(x, X, mu, lam)
    ne, n, _ = H.shape
    assert np.max(np.abs(H - np.swapaxes(H, 1, 2))) <= 1e-9 * np.abs(H).max()
    h = 1e-6
    for k in range(n):
        xp = x.copy(); xp[:, k // d, k % d] += h
        xm = x.copy(); xm[:, k // d, k % d] -= h
        fd = (fem.element_gradient(xp, X, mu, lam) - fem.element_gradient(xm, X, mu, lam)).reshape(ne, n) / (2 * h)
        assert np.allclose(fd, H[:, :, k], rtol=1e-5, atol=1e-6 * np.abs(H).max())


@pytest.mark.parametrize("d", [2, 3])
def test_log_modulus_jacobian_equals_gradient(d):
    x, X, mu, lam = _rand_elems(d)
    kp = fem.element_dgrad_dlogE(x, X, mu, lam)
    g = fem.element_gradient(x, X, mu, lam).reshape(x.shape[0], -1)
    assert np.allclose(kp, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


@pytest.mark.parametrize("d", [2, 3])
def test_rest_position_jacobian_matches_differences(d):
    x, X, mu, lam = _rand_elems(d)
    M = fem.element_dgrad_drest(x, X, mu, lam)
    ne, n, _ = M.shape
    h = 1e-6
    for k in range(n):
        Xp = X.copy(); Xp[:, k // d, k % d] += h
        Xm = X.copy(); Xm[:, k // d, k % d] -= h
        fd = (fem.element_gradient(x, Xp, mu, lam) - fem.element_gradient(x, Xm, mu, lam)).reshape(ne, n) / (2 * h)
        assert np.allclose(fd, M[:, :, k], rtol=1e-5, atol=1e-6 * np.abs(M).max())
    # moving rest and deformed configurations together rigidly leaves the forces unchanged
    # => sum over the two Jacobians applied to a common translation vanishes
    H = fem.element_hessian(x, X, mu, lam)
    t = np.tile(RNG.standard_normal(d), d + 1)
    assert np.max(np.abs(M @ t)) <= 1e-8 * np.abs(M).max()
    assert np.max(np.abs(H @ t)) <= 1e-8 * np.abs(H).max()
