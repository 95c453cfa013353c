"""Pins of the integrator oracle (oracle/integrators.py) on analytic targets:
the exact leapfrog map of the harmonic oscillator, time reversibility, the
O(dt^2) energy error, and the reparameterised ELBO gradient of a Gaussian
log-likelihood in closed form."""
import numpy as np
import pytest

from oracle import integrators as oi


def test_leapfrog_harmonic_exact_map():
    # logL = -x^2/2: one leapfrog step is the linear map A below (Sec. 2.3
    # equations composed by hand for U = x^2/2, M = 1)
    dt, n = 0.1, 37
    A = np.array([[1 - dt * dt / 2, dt], [-dt * (1 - dt * dt / 4), 1 - dt * dt / 2]])
    x0 = np.array([0.7, -1.3])
    r0 = np.array([0.2, 0.5])
    x, r, _ = oi.leapfrog(x0, r0, lambda t: -t, dt, n)
    ref = np.linalg.matrix_power(A, n) @ np.vstack([x0, r0])
    assert np.allclose(x, ref[0], rtol=1e-13, atol=1e-14)
    assert np.allclose(r, ref[1], rtol=1e-13, atol=1e-14)


def test_leapfrog_reversible_and_energy_order():
    grad = lambda t: -t - 0.3 * t ** 3  # logL = -t^2/2 - 0.075 t^4
    U = lambda t: np.sum(t * t / 2 + 0.075 * t ** 4)
    x0 = np.array([0.9, -0.4, 1.1])
    r0 = np.array([0.3, 0.8, -0.5])
    x, r, _ = oi.leapfrog(x0, r0, grad, 0.05, 40)
    xb, rb, _ = oi.leapfrog(x, -r, grad, 0.05, 40)
    assert np.allclose(xb, x0, atol=1e-12) and np.allclose(-rb, r0, atol=1e-12)
    errs = []
    for dt in (0.02, 0.01):
        x, r, _ = oi.leapfrog(x0, r0, grad, dt, int(round(0.4 / dt)))
        errs.append(abs(U(x) + r @ r / 2 - U(x0) - r0 @ r0 / 2))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_leapfrog_frozen_entries():
    x0 = np.array([1.0, 2.0])
    x, r, _ = oi.leapfrog(x0, np.array([1.0, 1.0]), lambda t: -t, 0.1, 5,
                          inv_mass=np.array([1.0, 0.0]))
    assert x[1] == 2.0 and x[0] != 1.0


def test_vi_gradient_gaussian_target_closed_form():
    rng = np.random.default_rng(3)
    P, S = 5, 7
    mu = rng.normal(size=P)
    omega = rng.normal(size=P)
    mask = np.array([1, 1, 0, 1, 1])
    eps = rng.normal(size=(S, P))
    f = lambda th: (-0.5 * th @ th, -th)
    elbo, gmu, gom, ll = oi.vi_elbo_grad(mu, omega, mask, eps, f)
    s = np.log1p(np.exp(omega))
    sp = 1 / (1 + np.exp(-omega))
    th = np.where(mask != 0, mu + s * eps, mu)
    m = mask != 0
    assert np.allclose(gmu[m], -th.mean(axis=0)[m], rtol=1e-14, atol=1e-15)
    assert np.allclose(gom[m], (-(th * eps)).mean(axis=0)[m] * sp[m] + sp[m] / s[m], rtol=1e-13)
    assert gmu[2] == 0 and gom[2] == 0
    assert np.isclose(elbo, np.mean(-0.5 * np.sum(th * th, axis=1)) + np.sum(np.log(s[m])))


def test_vi_zero_noise_is_the_plain_gradient():
    mu = np.array([0.3, -1.2])
    f = lambda th: (-np.sum(np.cos(th)), np.sin(th))
    _, gmu, _, _ = oi.vi_elbo_grad(mu, np.zeros(2), np.ones(2), np.zeros((4, 2)), f)
    assert np.allclose(gmu, np.sin(mu), rtol=1e-15)


def test_softplus_sigmoid_stable():
    w = np.array([-800.0, -30.0, 0.0, 30.0, 800.0])
    assert np.all(np.isfinite(oi.softplus(w))) and np.all(np.isfinite(oi.sigmoid(w)))
    assert oi.softplus(np.array([800.0]))[0] == 800.0
    assert np.isclose(oi.softplus(np.array([0.0]))[0], np.log(2.0))
