"""Pins of the full-rank VI oracle (oracle/vi_fullrank.py): the reparameterised
ELBO and its gradient equal the closed forms for a Gaussian target when the
draws have exactly zero mean and identity second moment; Adam's first step;
whole fits whose family contains the target recover its mean and covariance
(in log space through the Jacobian term as well); the draws are normal."""
import math

import numpy as np
import pytest

from oracle import hmc as oh
from oracle import vi_fullrank as vf


def _whitened(rng, S, n):
    """S x n draws with mean exactly 0 and (1/S) X^T X = I (to rounding)."""
    X = rng.standard_normal((S, n))
    X -= X.mean(axis=0)
    C = X.T @ X / S
    w, V = np.linalg.eigh(C)
    return X @ (V @ np.diag(w ** -0.5) @ V.T)


def _gauss_target(m, A):
    return lambda th: (-0.5 * (th - m) @ A @ (th - m), -A @ (th - m))


def test_elbo_gradient_closed_form_for_gaussian_target():
    rng = np.random.default_rng(5)
    n = 4
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    m = rng.standard_normal(n)
    r = vf.Restart(rng.standard_normal(n), 0.3, [oh.AFFINE] * n, [0.0] * n, [1.0] * n)
    r.omega = rng.uniform(-1.5, 0.5, n)
    r.lam = np.tril(rng.standard_normal((n, n)) * 0.2, -1)
    L = r.cholesky()
    eps = _whitened(rng, 64, n)
    elbo, g = r.elbo_grad(eps, _gauss_target(m, A))
    d = r.mu - m
    exact = (-0.5 * (d @ A @ d + np.trace(L.T @ A @ L)) + np.sum(np.log(np.diag(L)))
             + 0.5 * n * math.log(2 * math.pi * math.e))
    assert abs(elbo - exact) <= 1e-11 * max(1.0, abs(exact))
    assert np.allclose(g["mu"], -A @ d, rtol=1e-11, atol=1e-11)
    AL = A @ L
    assert np.allclose(g["lam"], np.tril(-AL, -1), rtol=1e-10, atol=1e-11)
    sig = 1.0 / (1.0 + np.exp(-r.omega))
    assert np.allclose(g["omega"], (-np.diag(AL) + 1.0 / np.diag(L)) * sig, rtol=1e-10,
                       atol=1e-11)


def test_adam_first_step_is_lr_times_sign():
    r = vf.Restart([0.5, -0.2], 0.1, [oh.AFFINE] * 2, [0.0] * 2, [1.0] * 2)
    mu0, om0 = r.mu.copy(), r.omega.copy()
    g = {"mu": np.array([3.0, -1e-3]), "omega": np.array([-2.0, 5.0]),
         "lam": np.array([[0.0, 0.0], [0.7, 0.0]])}
    lam0 = r.lam.copy()
    r.adam_step(g, lr=0.05)
    # bias-corrected moments at t = 1 are g and g^2
    assert np.allclose(r.mu - mu0, 0.05 * g["mu"] / (np.abs(g["mu"]) + 1e-8), rtol=1e-12)
    assert np.allclose(r.omega - om0, 0.05 * g["omega"] / (np.abs(g["omega"]) + 1e-8),
                       rtol=1e-12)
    assert r.lam[1, 0] - lam0[1, 0] == pytest.approx(0.05 * 0.7 / (0.7 + 1e-8), rel=1e-12)
    assert r.lam[0, 1] == 0.0


def _fit(r, target, S, iters, lr, seed):
    rng = np.random.default_rng(seed)
    for _ in range(iters):
        _, g = r.elbo_grad(rng.standard_normal((S, r.n)), target)
        r.adam_step(g, lr)
    return r


def test_fit_recovers_a_correlated_gaussian():
    m = np.array([1.0, -2.0])
    Sig = np.array([[0.5, 0.3], [0.3, 0.4]])
    A = np.linalg.inv(Sig)
    r = vf.Restart([0.0, 0.0], 0.1, [oh.AFFINE] * 2, [0.0] * 2, [1.0] * 2)
    _fit(r, _gauss_target(m, A), 32, 1500, 0.05, 11)
    _fit(r, _gauss_target(m, A), 256, 300, 0.005, 12)
    L = r.cholesky()
    assert np.allclose(r.mu, m, atol=0.05)
    assert np.allclose(L @ L.T, Sig, atol=0.05)


def test_fit_in_log_space_needs_the_jacobian():
    # ln theta ~ N(0.3, 0.5^2): the surrogate in z = ln theta is exact
    mlog, s = 0.3, 0.5

    def tgt(th):
        lt = math.log(th[0])
        return (-(lt - mlog) ** 2 / (2 * s * s) - lt,
                np.array([(-(lt - mlog) / (s * s) - 1.0) / th[0]]))

    r = vf.Restart([0.0], 0.1, [oh.LOG], [0.0], [1.0])
    _fit(r, tgt, 32, 1500, 0.05, 21)
    _fit(r, tgt, 256, 300, 0.005, 22)
    # without the Jacobian the mean would settle at mlog - s^2 = 0.05
    assert abs(r.mu[0] - mlog) < 0.04
    assert abs(r.cholesky()[0, 0] - s) < 0.04


def test_draws_are_standard_normal():
    from scipy import stats
    z = np.concatenate([vf.draws(3, it, 7, 2000) for it in range(4)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # a different purpose than the HMC momentum draws of the same counter
    assert not np.array_equal(vf.draws(3, 0, 7, 8), oh.momentum_normals(3, 0, 7, 8))


def test_inverse_softplus():
    for s in (1e-3, 0.1, 1.0, 20.0):
        assert vf.softplus(vf.inverse_softplus(s)) == pytest.approx(s, rel=1e-13)
