"""Pins of the HMC-transition oracle (oracle/hmc.py): its Philox4x64-10
against NumPy's Philox bit generator, the normal draws and the transforms
against their definitions, the energy error against the exact leapfrog map of
the harmonic oscillator, and the stationary distributions of whole chains on
analytic targets (Gaussian, log-normal in log space, Beta through the logit),
which a wrong accept rule, kinetic energy or Jacobian term would shift."""
import math

import numpy as np
import pytest

from oracle import hmc


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((0x123456789ABCDEF0, 0x0FEDCBA987654321), (5, 7, 11, 13)),
    ((2 ** 64 - 1, 1), (2 ** 64 - 1, 3, 0, 9)),   # carry into the second word
])
def test_philox_matches_numpy_bit_generator(key, ctr):
    # NumPy's Philox (4x64, 10 rounds) increments its counter before each
    # block, so its first block is the bijection of counter + 1
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
    raw = [int(v) for v in bg.random_raw(8)]
    c = list(ctr)
    for blk in range(2):
        c[0] += 1
        k = 0
        while c[k] == 2 ** 64:
            c[k] = 0
            c[k + 1] += 1
            k += 1
        assert hmc.philox4x64(c, key) == raw[4 * blk:4 * blk + 4]


def test_open_uniform_range():
    assert hmc.open_uniform(0) == 2.0 ** -54
    assert hmc.open_uniform(2 ** 64 - 1) == 1.0 - 2.0 ** -54
    assert hmc.open_uniform(1 << 63) == 0.5 + 2.0 ** -54


def test_momentum_normals_are_standard_normal():
    from scipy import stats
    z = np.concatenate([hmc.momentum_normals(7, it, 3, 2000) for it in range(5)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the pairs of one block are independent: no correlation between cos and sin halves
    x = hmc.momentum_normals(11, 0, 0, 4 * 4000).reshape(-1, 4)
    assert abs(np.corrcoef(x[:, 0], x[:, 1])[0, 1]) < 5 / math.sqrt(4000)


@pytest.mark.parametrize("kind,a,b,z", [
    (hmc.AFFINE, 3.0, 1e-6, 0.7), (hmc.AFFINE, -2.0, 50.0, -1.3),
    (hmc.LOG, 0.0, 1.0, 0.4), (hmc.LOG, 5.0, 2e-7, -2.2),
    (hmc.LOGIT, 0.0, 1.0, 0.3), (hmc.LOGIT, -1e-6, 7e-6, -3.1), (hmc.LOGIT, 10.0, 300.0, 4.0),
])
def test_transform_derivatives_and_inverse(kind, a, b, z):
    t, d, lj, dlj = hmc.transform(kind, a, b, z)
    h = 1e-5
    fd = (hmc.transform(kind, a, b, z + h)[0] - hmc.transform(kind, a, b, z - h)[0]) / (2 * h)
    # relative error of the difference: truncation plus the rounding of theta
    rel = 1e-8 + 4e-16 * (abs(t) + abs(a)) / (h * abs(d))
    assert abs(d - fd) <= rel * abs(d)
    assert abs(lj - math.log(abs(fd))) <= 2 * rel
    fd_lj = (hmc.transform(kind, a, b, z + h)[2] - hmc.transform(kind, a, b, z - h)[2]) / (2 * h)
    assert abs(dlj - fd_lj) <= 1e-7
    # the inverse recovers z up to the rounding of theta, divided by the slope
    assert abs(hmc.inverse_transform(kind, a, b, t) - z) <= 1e-12 + 4e-16 * (abs(t) + abs(a)) / abs(d)
    if kind == hmc.LOGIT:
        assert a < t < b
    if kind == hmc.LOG:
        assert t > a


def test_energy_error_is_that_of_the_exact_leapfrog_map():
    # logL = -z^2/2, M = 1, one leapfrog step of dt: the linear map A
    dt = 0.9
    A = np.array([[1 - dt * dt / 2, dt], [-dt * (1 - dt * dt / 4), 1 - dt * dt / 2]])
    ch = hmc.Chain(lambda th: (-0.5 * th[0] ** 2, np.array([-th[0]])), [0.8], [hmc.AFFINE],
                   [0.0], [1.0], [1.0], dt, chain_id=2, seed=99)
    r0 = hmc.momentum_normals(99, 0, 2, 1)[0]
    z1, r1 = A @ np.array([0.8, r0])
    delta = 0.5 * (z1 * z1 + r1 * r1) - 0.5 * (0.8 ** 2 + r0 * r0)
    accepted = ch.transition(1)
    assert abs(ch.energy_error - delta) <= 1e-14
    alpha = min(1.0, math.exp(-delta))
    assert ch.accept_prob == pytest.approx(alpha, rel=1e-14)
    assert accepted == (hmc.accept_uniform(99, 0, 2) < alpha)
    assert ch.z[0] == pytest.approx(z1 if accepted else 0.8, rel=1e-14)


def _run(ch, n, L, **kw):
    zs = np.empty((n, ch.z.size))
    th = np.empty((n, ch.z.size))
    for i in range(n):
        ch.transition(L, **kw)
        zs[i] = ch.z
        th[i] = ch.theta
    return zs, th


def test_gaussian_target_stationary_moments():
    mu = np.array([1.5, -4.0])
    sd = np.array([1.0, 3.0])
    tgt = lambda th: (-0.5 * np.sum(((th - mu) / sd) ** 2), -(th - mu) / sd ** 2)
    ch = hmc.Chain(tgt, [0.0, 0.0], [hmc.AFFINE] * 2, [0.0, 0.0], [1.0, 1.0], [1.0, 9.0], 0.35,
                   seed=5)
    _run(ch, 200, 8)
    _, th = _run(ch, 3000, 8)
    n = th.shape[0]
    assert np.all(np.abs(th.mean(0) - mu) < 6 * sd / math.sqrt(n / 2))
    assert np.all(np.abs(th.var(0) / sd ** 2 - 1) < 6 * math.sqrt(2.0 / (n / 2)))
    assert ch.n_accept > 0.7 * ch.iteration


def test_lognormal_target_in_log_space_needs_the_jacobian():
    # ln theta ~ N(0.5, 0.4^2): logL(theta) = -(ln theta - 0.5)^2 / 0.32 - ln theta
    m, s = 0.5, 0.4
    def tgt(th):
        lt = math.log(th[0])
        return -(lt - m) ** 2 / (2 * s * s) - lt, np.array([(-(lt - m) / (s * s) - 1.0) / th[0]])
    ch = hmc.Chain(tgt, [1.0], [hmc.LOG], [0.0], [1.0], [s * s], 0.5, seed=17)
    _run(ch, 200, 6)
    zs, th = _run(ch, 3000, 6)
    n = zs.shape[0]
    assert np.all(th > 0)
    # without the Jacobian term the z mean would sit at m - s^2 = 0.34
    assert abs(zs.mean() - m) < 6 * s / math.sqrt(n / 2)
    assert abs(zs.var() / (s * s) - 1) < 6 * math.sqrt(2.0 / (n / 2))


def test_beta_target_through_the_logit():
    # Beta(2, 3) on (0, 1): logL = ln theta + 2 ln(1 - theta); mean 0.4, var 0.04
    tgt = lambda th: (math.log(th[0]) + 2 * math.log1p(-th[0]),
                      np.array([1 / th[0] - 2 / (1 - th[0])]))
    ch = hmc.Chain(tgt, [0.5], [hmc.LOGIT], [0.0], [1.0], [1.0], 0.9, seed=23)
    _run(ch, 200, 5)
    _, th = _run(ch, 4000, 5)
    n = th.shape[0]
    assert np.all((th > 0) & (th < 1))
    assert abs(th.mean() - 0.4) < 6 * 0.2 / math.sqrt(n / 3)
    assert abs(th.var() - 0.04) < 0.006


def test_fixed_entries_and_divergence():
    tgt = lambda th: (-0.5 * (th[0] ** 2 + th[1] ** 2), -th.copy())
    ch = hmc.Chain(tgt, [0.3, 2.0], [hmc.AFFINE, hmc.FIXED], [0.0, 0.0], [1.0, 1.0], [1.0, 1.0],
                   60.0, seed=3)
    z0 = ch.z.copy()
    ch.transition(20, max_error=1000.0)
    # a step far beyond the stability limit 2 blows the energy up
    assert ch.n_divergent == 1 and ch.accept_prob == 0.0 and ch.n_accept == 0
    assert np.array_equal(ch.z, z0) and ch.theta[1] == 2.0
    ch.step = 0.2
    _run(ch, 50, 5)
    assert ch.theta[1] == 2.0 and ch.n_accept > 40


def test_welford_window_and_mass_adaptation():
    sd = np.array([0.1, 10.0])
    tgt = lambda th: (-0.5 * np.sum((th / sd) ** 2), -th / sd ** 2)
    ch = hmc.Chain(tgt, [0.0, 0.0], [hmc.AFFINE] * 2, [0.0, 0.0], [1.0, 1.0], [1.0, 1.0], 0.05,
                   seed=41)
    zs, _ = _run(ch, 300, 10, adapt_mass=True, adapt_step=True)
    assert ch.w_n == 300
    assert np.allclose(ch.w_mean, zs.mean(0), rtol=1e-12, atol=1e-15)
    assert np.allclose(ch.w_m2 / (ch.w_n - 1), zs.var(0, ddof=1), rtol=1e-10)
    ch.mass_window_end()
    assert ch.w_n == 0
    # a first window from a poor metric: the right order of magnitude
    assert np.all(np.abs(np.log10(ch.inv_mass / sd ** 2)) < 1.0)
    ch.da_restart()
    _run(ch, 600, 10, adapt_mass=True, adapt_step=True)
    ch.mass_window_end()
    assert np.all(np.abs(ch.inv_mass / sd ** 2 - 1) < 0.35)


def test_dual_averaging_reaches_the_target_acceptance():
    # one leapfrog step on a Gaussian: the acceptance falls monotonically with
    # the step (longer trajectories on a Gaussian resonate, so the acceptance
    # is not monotone there)
    tgt = lambda th: (-0.5 * np.sum(th ** 2), -th)
    ch = hmc.Chain(tgt, [0.5, -0.5, 0.1], [hmc.AFFINE] * 3, [0.0] * 3, [1.0] * 3, [1.0] * 3,
                   0.01, seed=77)
    _run(ch, 600, 1, adapt_step=True, target_accept=0.8)
    ch.da_final()
    assert 0.5 < ch.step < 1.5
    acc = []
    for _ in range(1000):
        ch.transition(1)
        acc.append(ch.accept_prob)
    assert abs(np.mean(acc) - 0.8) < 0.05
