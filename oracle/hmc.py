"""Plain NumPy oracle of one Hamiltonian Monte Carlo transition per chain, with
its warm-up adaptation.

TEST INFRASTRUCTURE ONLY (same rule as the rest of oracle/).

What one transition of one chain computes (Sec. 2.3):
  * momentum r ~ N(0, M), M = diag(1 / inv_mass), drawn afresh;
  * L leapfrog steps (the Sec. 2.3 leapfrog equations) of step dt in the
    sampler's unconstrained coordinates z, for the potential
        U(z) = -logL(theta(z)) - sum_p ln |dtheta_p/dz_p|
    (flat priors; the second term is the change of variables);
  * the Metropolis-Hastings step: accept (z', r') with probability
        alpha = min{1, exp(H(z, r) - H(z', r'))},  H = U + r^T M^-1 r / 2,
    else keep z.
Sec. 2.3 (practitioners) motivates the coordinates: pre-scaling (an affine
map), sampling positive quantities in log space, and hard bounds; each entry
has one of
    FIXED   theta = its given value, never moved
    AFFINE  theta = a + b z
    LOG     theta = a + b exp(z)                  (b > 0: theta > a)
    LOGIT   theta = a + (b - a) sigmoid(z)        (a < theta < b)
Readings where the paper stops short (samplers are taken from a library):
  * divergence: a transition whose energy error H' - H exceeds max_error, or
    is not a number, is divergent and rejected (alpha = 0);
  * warm-up: the diagonal inverse mass is estimated from a window of
    post-transition positions by Welford's running variance, regularised
    toward 1e-3 as (n/(n+5)) var + 1e-3 (5/(n+5)); the step size follows the
    dual-averaging scheme of Hoffman and Gelman (JMLR 15, 2014, Sec. 3.2.1)
    with gamma = 0.05, t0 = 10, kappa = 0.75, mu = ln(10 dt_0).
Random numbers: the counter-based generator Philox4x64-10 (Salmon, Moraes,
Dror and Shaw, SC'11), written out here from its definition; key
(seed, 0); counter (iteration, chain, block, purpose).  Momentum entry e
takes Box-Muller normal e mod 4 of block e div 4 (purpose 0); the accept
uniform is output 0 of block 0, purpose 1.  A 64-bit output x maps to the
open interval as ((x >> 11) + 1/2) 2^-53.
"""
from __future__ import annotations

import math

import numpy as np

FIXED, AFFINE, LOG, LOGIT = 0, 1, 2, 3

_MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (SC'11, Table 2)
_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4x64(counter, key, rounds=10):
    """Philox4x64-R bijection of a 4 x 64-bit counter under a 2 x 64-bit key:
    each round multiplies words 0 and 2 by the round constants, swaps in the
    high halves XOR-ed with the other words and the key, and bumps the key."""
    x0, x1, x2, x3 = (int(v) & _MASK64 for v in counter)
    k0, k1 = (int(v) & _MASK64 for v in key)
    for _ in range(rounds):
        p0 = _PHILOX_M[0] * x0
        p1 = _PHILOX_M[1] * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & _MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & _MASK64)
        k0 = (k0 + _PHILOX_W[0]) & _MASK64
        k1 = (k1 + _PHILOX_W[1]) & _MASK64
    return [x0, x1, x2, x3]


def open_uniform(x):
    """(0, 1) double from a 64-bit integer: the top 53 bits, centred."""
    return ((int(x) >> 11) + 0.5) * 2.0 ** -53


def momentum_normals(seed, iteration, chain, n):
    """n standard normals of one chain's momentum draw (Box-Muller on
    consecutive uniform pairs of each block)."""
    out = np.empty(n)
    for e in range(n):
        u = [open_uniform(v) for v in philox4x64((iteration, chain, e // 4, 0), (seed, 0))]
        j = e % 4
        u0, u1 = u[2 * (j // 2)], u[2 * (j // 2) + 1]
        rad = math.sqrt(-2.0 * math.log(u0))
        ang = 2.0 * math.pi * u1
        out[e] = rad * (math.cos(ang) if j % 2 == 0 else math.sin(ang))
    return out


def accept_uniform(seed, iteration, chain):
    return open_uniform(philox4x64((iteration, chain, 0, 1), (seed, 0))[0])


def _exp(x):
    """exp that overflows to inf (a runaway trajectory must reach the
    divergence rule, not raise)."""
    return math.exp(x) if x < 709.0 else math.inf


def _sigmoid(z):
    return 1.0 / (1.0 + math.exp(-z)) if z >= 0 else math.exp(z) / (1.0 + math.exp(z))


def _softplus(z):
    return z + math.log1p(math.exp(-z)) if z > 0 else math.log1p(math.exp(z))


def transform(kind, a, b, z):
    """(theta, dtheta/dz, ln|dtheta/dz|, d ln|dtheta/dz| / dz) of one entry."""
    if kind == AFFINE:
        return a + b * z, b, math.log(abs(b)), 0.0
    if kind == LOG:
        ez = _exp(z)
        return a + b * ez, b * ez, math.log(b) + z, 1.0
    if kind == LOGIT:
        s = _sigmoid(z)
        w = b - a
        return a + w * s, w * s * (1.0 - s), math.log(w) - _softplus(-z) - _softplus(z), 1.0 - 2.0 * s
    raise ValueError("FIXED entries have no transform")


def inverse_transform(kind, a, b, theta):
    if kind == AFFINE:
        return (theta - a) / b
    if kind == LOG:
        return math.log((theta - a) / b)
    if kind == LOGIT:
        f = (theta - a) / (b - a)
        return math.log(f) - math.log1p(-f)
    raise ValueError("FIXED entries have no transform")


class Chain:
    """One chain.  Entries are the sampler's coordinates in a fixed order;
    `target(theta)` returns (logL, dlogL/dtheta) over all entries (the values
    of FIXED entries are passed through unchanged)."""

    def __init__(self, target, theta, kind, a, b, inv_mass, step, chain_id=0, seed=0):
        self.target = target
        self.kind = np.asarray(kind, np.int64)
        self.a = np.asarray(a, float)
        self.b = np.asarray(b, float)
        self.theta = np.array(theta, float)
        self.moving = self.kind != FIXED
        self.z = np.zeros_like(self.theta)
        for p in np.flatnonzero(self.moving):
            self.z[p] = inverse_transform(self.kind[p], self.a[p], self.b[p], self.theta[p])
        self.inv_mass = np.array(inv_mass, float)
        self.step = float(step)
        self.chain_id = int(chain_id)
        self.seed = int(seed)
        self.iteration = 0
        self.n_accept = 0
        self.n_divergent = 0
        self.accept_prob = 0.0
        self.energy_error = 0.0
        # warm-up state
        self.w_n = 0
        self.w_mean = np.zeros_like(self.theta)
        self.w_m2 = np.zeros_like(self.theta)
        self.da_restart()
        self.set_position(self.z)

    # -- potential and its gradient in z --------------------------------
    def set_position(self, z):
        """theta = theta(z) on moving entries; logL, its gradient and U."""
        self.z = np.array(z, float)
        self.dtdz = np.zeros_like(self.z)
        logj = 0.0
        self.dlogj = np.zeros_like(self.z)
        for p in np.flatnonzero(self.moving):
            t, d, lj, dlj = transform(self.kind[p], self.a[p], self.b[p], self.z[p])
            self.theta[p] = t
            self.dtdz[p] = d
            logj += lj
            self.dlogj[p] = dlj
        self.logL, self.g = self.target(self.theta)
        self.U = -self.logL - logj

    def grad_U(self):
        """dU/dz = -(dlogL/dtheta dtheta/dz + d ln|dtheta/dz| / dz) on moving
        entries, 0 elsewhere."""
        return np.where(self.moving, -(self.g * self.dtdz + self.dlogj), 0.0)

    # -- one transition (Sec. 2.3) ----------------------------------------
    def transition(self, n_leapfrog, max_error=1000.0, adapt_mass=False, adapt_step=False,
                   target_accept=0.8):
        live = self.moving & (self.inv_mass > 0)
        xi = momentum_normals(self.seed, self.iteration, self.chain_id, self.z.size)
        r = np.where(live, xi * np.sqrt(1.0 / np.where(live, self.inv_mass, 1.0)), 0.0)
        H0 = self.U + 0.5 * np.sum(self.inv_mass[live] * r[live] ** 2)
        saved = (self.z.copy(), self.theta.copy(), self.logL, self.g.copy(), self.U,
                 self.dtdz.copy(), self.dlogj.copy())
        dt = self.step
        im = np.where(live, self.inv_mass, 0.0)
        for _ in range(n_leapfrog):
            r = r - 0.5 * dt * self.grad_U()
            self.set_position(self.z + dt * im * r)
            r = r - 0.5 * dt * self.grad_U()
        H1 = self.U + 0.5 * np.sum(self.inv_mass[live] * r[live] ** 2)
        delta = H1 - H0
        divergent = not (delta <= max_error)
        alpha = 0.0 if divergent else min(1.0, _exp(-delta))
        u = accept_uniform(self.seed, self.iteration, self.chain_id)
        accept = u < alpha
        if not accept:
            (self.z, self.theta, self.logL, self.g, self.U, self.dtdz, self.dlogj) = saved
        self.accept_prob = alpha
        self.energy_error = delta
        self.n_accept += int(accept)
        self.n_divergent += int(divergent)
        self.iteration += 1
        if adapt_mass:
            self.welford_push(self.z)
        if adapt_step:
            self.da_update(alpha, target_accept)
        return accept

    # -- warm-up ----------------------------------------------------------
    def welford_push(self, x):
        self.w_n += 1
        d = x - self.w_mean
        self.w_mean = self.w_mean + d / self.w_n
        self.w_m2 = self.w_m2 + d * (x - self.w_mean)

    def mass_window_end(self):
        """inv_mass = regularised sample variance of the window (moving
        entries, windows of at least 2 positions); the window restarts."""
        n = self.w_n
        if n >= 2:
            var = self.w_m2 / (n - 1)
            reg = (n / (n + 5.0)) * var + 1e-3 * (5.0 / (n + 5.0))
            self.inv_mass = np.where(self.moving, reg, self.inv_mass)
        self.w_n = 0
        self.w_mean = np.zeros_like(self.w_mean)
        self.w_m2 = np.zeros_like(self.w_m2)

    def da_restart(self):
        self.da_mu = math.log(10.0 * self.step)
        self.da_log_bar = 0.0
        self.da_hbar = 0.0
        self.da_t = 0

    def da_update(self, alpha, target_accept, gamma=0.05, t0=10.0, kappa=0.75):
        self.da_t += 1
        t = self.da_t
        w = 1.0 / (t + t0)
        self.da_hbar = (1.0 - w) * self.da_hbar + w * (target_accept - alpha)
        log_eps = self.da_mu - math.sqrt(t) / gamma * self.da_hbar
        eta = t ** (-kappa)
        self.da_log_bar = eta * log_eps + (1.0 - eta) * self.da_log_bar
        self.step = math.exp(log_eps)

    def da_final(self):
        self.step = math.exp(self.da_log_bar)
