"""Plain NumPy oracle for the integrator steps around the gradient.

TEST INFRASTRUCTURE ONLY (same rule as the rest of oracle/).

* leapfrog: Sec. 2.3, leapfrog equations, for U = -logL with a diagonal mass:
      r_half  = r + dt/2 * grad logL(theta)
      theta'  = theta + dt * M^-1 r_half
      r'      = r_half + dt/2 * grad logL(theta')
  Entries with inverse mass 0 never move.
* vi_elbo_grad: Sec. 2.4, Monte-Carlo estimate of the loss and of its gradient
  with the reparameterisation theta_i = mu + s(omega) eps_i, s = softplus,
  for a mean-field Gaussian q with flat priors:
      ELBO ~ mean_i logL(theta_i) + sum_p ln s(omega_p)   (+ const)
      dELBO/dmu    = mean_i g_i
      dELBO/domega = mean_i g_i * eps_i * s'(omega) + s'(omega)/s(omega)
  Only entries with mask != 0 are variational.
Both take the gradient (and logL) as a callable, so they are pinned on
analytic targets (harmonic potential, Gaussian logL) in the tests.
"""
from __future__ import annotations

import numpy as np


def softplus(w):
    w = np.asarray(w, float)
    return np.where(w > 0, w + np.log1p(np.exp(-np.abs(w))), np.log1p(np.exp(np.minimum(w, 0))))


def sigmoid(w):
    w = np.asarray(w, float)
    return np.where(w >= 0, 1.0 / (1.0 + np.exp(-np.abs(w))),
                    np.exp(np.minimum(w, 0)) / (1.0 + np.exp(np.minimum(w, 0))))


def leapfrog(theta, r, grad_logL, dt, n_steps, inv_mass=None, g0=None):
    """n_steps leapfrog steps; returns (theta, r, g at theta)."""
    theta = np.array(theta, float, copy=True)
    r = np.array(r, float, copy=True)
    im = np.ones_like(theta) if inv_mass is None else np.asarray(inv_mass, float)
    g = grad_logL(theta) if g0 is None else np.array(g0, float)
    for _ in range(n_steps):
        r = r + 0.5 * dt * g
        theta = theta + dt * im * r
        g = grad_logL(theta)
        r = r + 0.5 * dt * g
    return theta, r, g


def vi_elbo_grad(mu, omega, mask, eps, logL_and_grad):
    """eps: (S, P) draws; logL_and_grad(theta) -> (logL, g) for one sample."""
    mu = np.asarray(mu, float)
    omega = np.asarray(omega, float)
    mask = np.asarray(mask) != 0
    eps = np.asarray(eps, float)
    s = softplus(omega)
    S = eps.shape[0]
    ll = np.empty(S)
    G = np.empty_like(eps)
    for i in range(S):
        th = np.where(mask, mu + s * eps[i], mu)
        ll[i], G[i] = logL_and_grad(th)
    sp = sigmoid(omega)
    gmu = np.where(mask, G.mean(axis=0), 0.0)
    gom = np.where(mask, (G * eps).mean(axis=0) * sp + sp / s, 0.0)
    elbo = ll.mean() + np.sum(np.log(s[mask]))
    return elbo, gmu, gom, ll
