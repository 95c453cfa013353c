"""Plain NumPy oracle of the full-rank Gaussian variational fit (Sec. 2.4 VI,
Sec. 4.2: a multivariate normal surrogate in unconstrained space, initial
covariance sigma_0^2 I with sigma_0 = 0.1, ELBO maximised with Adam,
independent restarts, the best ELBO kept).

TEST INFRASTRUCTURE ONLY (same rule as the rest of oracle/).

Per restart, with z = mu + L eps, eps ~ N(0, I), theta = theta(z) (the
transforms of oracle/hmc.py) and flat priors in theta:
    ELBO = E_q[ logL(theta(z)) + sum_p ln|dtheta_p/dz_p| ] + sum_i ln L_ii
           + (n/2) ln(2 pi e)                (the Gaussian entropy)
L is lower triangular with L_ii = softplus(omega_i) and free entries
lambda_ij below the diagonal.  The Monte-Carlo estimate over S draws and its
reparameterisation gradient (h_s = the z-gradient of the log target at z_s):
    dELBO/dmu_i       = mean_s h_si
    dELBO/dlambda_ij  = mean_s h_si eps_sj                       (i > j)
    dELBO/domega_i    = (mean_s h_si eps_si + 1 / L_ii) sigmoid(omega_i)
Adam (Kingma and Ba 2015, Algorithm 1) ascends the ELBO:
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
    x <- x + lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
Readings: the paper names the family, sigma_0, the optimiser, its learning
rate and the restart count; the Cholesky parameterisation (softplus
diagonal), the number of draws per step and Adam's b1 = 0.9, b2 = 0.999,
eps = 1e-8 (the library defaults) are choices made here.
Draws: Philox4x64-10 as in oracle/hmc.py, key (seed, 0), counter
(iteration, restart * S + s, entry // 4, purpose 2), Box-Muller normal
entry % 4 of each block; entries are the variational coordinates in order.
"""
from __future__ import annotations

import math

import numpy as np

from . import hmc as _h

PURPOSE_VI = 2


def draws(seed, iteration, item, n):
    """n standard normals for one (restart, sample) item."""
    out = np.empty(n)
    for e in range(n):
        u = [_h.open_uniform(v) for v in _h.philox4x64((iteration, item, e // 4, PURPOSE_VI),
                                                       (seed, 0))]
        j = e % 4
        u0, u1 = u[2 * (j // 2)], u[2 * (j // 2) + 1]
        rad = math.sqrt(-2.0 * math.log(u0))
        ang = 2.0 * math.pi * u1
        out[e] = rad * (math.cos(ang) if j % 2 == 0 else math.sin(ang))
    return out


def softplus(w):
    return w + math.log1p(math.exp(-w)) if w > 0 else math.log1p(math.exp(w))


def sigmoid(w):
    return 1.0 / (1.0 + math.exp(-w)) if w >= 0 else math.exp(w) / (1.0 + math.exp(w))


def inverse_softplus(s):
    return s + math.log(-math.expm1(-s))


class Restart:
    """Variational parameters of one restart over n coordinates (the moving
    entries), with the transform of each."""

    def __init__(self, mu, sigma0, kind, a, b):
        self.n = len(mu)
        self.mu = np.array(mu, float)
        self.omega = np.full(self.n, inverse_softplus(sigma0))
        self.lam = np.zeros((self.n, self.n))  # strictly lower part used
        self.kind = np.asarray(kind, np.int64)
        self.a = np.asarray(a, float)
        self.b = np.asarray(b, float)
        self.adam_t = 0
        self.m = {k: np.zeros_like(v) for k, v in self.params().items()}
        self.v = {k: np.zeros_like(v) for k, v in self.params().items()}

    def params(self):
        return {"mu": self.mu, "omega": self.omega, "lam": self.lam}

    def cholesky(self):
        L = np.tril(self.lam, -1)
        L[np.diag_indices(self.n)] = [softplus(w) for w in self.omega]
        return L

    def elbo_grad(self, eps, target):
        """MC ELBO and its gradient from the draws eps (S, n); target(theta)
        -> (logL, dlogL/dtheta) over the n coordinates."""
        L = self.cholesky()
        S = eps.shape[0]
        H = np.empty_like(eps)
        f = np.empty(S)
        for s in range(S):
            z = self.mu + L @ eps[s]
            th = np.empty(self.n)
            dt = np.empty(self.n)
            lj = 0.0
            dlj = np.empty(self.n)
            for p in range(self.n):
                th[p], dt[p], l, dlj[p] = _h.transform(self.kind[p], self.a[p], self.b[p], z[p])
                lj += l
            ll, g = target(th)
            f[s] = ll + lj
            H[s] = g * dt + dlj
        diag = np.diag(L)
        gmu = H.mean(axis=0)
        G = (H.T @ eps) / S           # G_ij = mean_s h_si eps_sj
        glam = np.tril(G, -1)
        gom = (np.diag(G) + 1.0 / diag) * np.array([sigmoid(w) for w in self.omega])
        elbo = f.mean() + np.sum(np.log(diag)) + 0.5 * self.n * math.log(2 * math.pi * math.e)
        return elbo, {"mu": gmu, "omega": gom, "lam": glam}

    def adam_step(self, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.adam_t += 1
        t = self.adam_t
        for k, x in self.params().items():
            g = grads[k]
            self.m[k] = b1 * self.m[k] + (1 - b1) * g
            self.v[k] = b2 * self.v[k] + (1 - b2) * g * g
            mh = self.m[k] / (1 - b1 ** t)
            vh = self.v[k] / (1 - b2 ** t)
            x += lr * mh / (np.sqrt(vh) + eps)
        self.lam = np.tril(self.lam, -1)
