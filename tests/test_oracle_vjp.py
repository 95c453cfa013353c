"""Pins of the oracle's vector-Jacobian product of R_hat and of its batched
entry point (paper Sec. 2.1 AD figure, Sec. 3 gradient listing).

The VJP referee is checked against three things other than itself:
  * the chain rule of the likelihood: with the seed ghat_i = dlogL/dR_hat_i =
    -(R_hat_i - R_i) / e_i^2, sum_i ghat_i dR_hat_i/dtheta is dlogL/dtheta,
    which the pinned loglik gradient gives (its own pins: Richardson
    differences, closed forms, invariances);
  * Richardson central differences of the pinned model curve for a one-hot
    seed (no complex step on that side);
  * the definition of the smeared curve: for a one-hot seed the row gradient
    is scale times the weighted sum of dR/dtheta at the point's quadrature
    nodes (the pinned unsmeared Jacobian and the pinned rule), and the
    instrument pair is (R_sm,i, 1).
The batch entry point must reproduce the per-item calls bitwise, with one or
several threads.
"""
import numpy as np
import pytest

from test_oracle_pins import rand_stack

UNITS = np.array([1.0, 1e-6, 1e-6, 1.0])


def _scaled(g):
    return np.asarray(g) * UNITS


def _data(orc, rows, Q, dqq, scale, bkg, seed=5):
    Rm = orc.model_curve(rows, scale, bkg, Q, dqq)
    rng = np.random.default_rng(seed)
    e = 0.03 * Rm
    return Rm * 1.02 + e * rng.standard_normal(Q.size), e


@pytest.mark.parametrize("L,dqq", [(0, 0.0), (2, 0.0), (5, 0.05), (9, 0.03)])
def test_vjp_with_likelihood_seed_is_the_loglik_gradient(orc, L, dqq):
    rng = np.random.default_rng(700 + L)
    rows = rand_stack(rng, L)
    Q = np.geomspace(0.006, 0.3, 37)
    sc, bk = 0.97, 1.3e-7
    Robs, e = _data(orc, rows, Q, dqq, sc, bk)
    Rhat = orc.model_curve(rows, sc, bk, Q, dqq)
    ghat = -(Rhat - Robs) / (e * e)
    g, gi = orc.model_vjp_cs(rows, sc, bk, Q, dqq, ghat)
    _, gl, gil = orc.loglik_grad_cs(rows, sc, bk, Q, Robs, e, dqq)
    a, b = _scaled(g), _scaled(gl)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    big = np.abs(b) >= 1e-3 * np.max(np.abs(b))
    assert np.max(np.abs(a[big] - b[big]) / np.abs(b[big])) <= 1e-10
    assert np.max(np.abs(gi - gil) / np.abs(gil)) <= 1e-12
    # entries the model does not read get exactly 0
    assert g[0, 0] == 0 and g[0, 2] == 0 and g[0, 3] == 0 and g[-1, 0] == 0


def _richardson_model(orc, rows, sc, bk, Q, dqq, i, p, h):
    def f(x):
        r = rows.copy()
        r.flat[p] = x
        return orc.model_curve(r, sc, bk, Q, dqq)[i]
    x0 = rows.flat[p]
    return (8.0 * (f(x0 + h) - f(x0 - h)) - (f(x0 + 2 * h) - f(x0 - 2 * h))) / (12.0 * h)


@pytest.mark.parametrize("dqq", [0.0, 0.05])
def test_one_hot_vjp_matches_finite_differences(orc, dqq):
    rng = np.random.default_rng(711)
    L = 3
    rows = rand_stack(rng, L)
    rows[1:, 2] = rng.uniform(2e-8, 5e-8, L + 1)  # FD steps stay off the |rho_im| kink
    Q = np.geomspace(0.008, 0.25, 23)
    sc, bk = 1.05, 2e-7
    for i in (3, 11, 19):
        seed = np.zeros(Q.size)
        seed[i] = 1.0
        g, gi = orc.model_vjp_cs(rows, sc, bk, Q, dqq, seed)
        ref = np.zeros_like(rows)
        for p in range(rows.size):
            if g.flat[p] == 0.0:
                continue
            h = 1e-4 * UNITS[p % 4]
            ref.flat[p] = _richardson_model(orc, rows, sc, bk, Q, dqq, i, p, h)
        a, b = _scaled(g), _scaled(ref)
        assert np.max(np.abs(a - b)) <= 1e-7 * np.max(np.abs(b)), i
        # the instrument pair: dR_hat_i/dscale = R_sm,i, dR_hat_i/dbkg = 1
        Rsm = orc.smeared(rows, Q, dqq)[i]
        assert abs(gi[0] - Rsm) <= 1e-14 * Rsm and gi[1] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("dqq", [0.0, 0.05])
def test_one_hot_vjp_is_the_weighted_node_jacobian(orc, dqq):
    rng = np.random.default_rng(712)
    L = 4
    rows = rand_stack(rng, L)
    Q = np.geomspace(0.006, 0.3, 15)
    sc, bk = 0.9, 1e-7
    t, w = orc.smear_rule(dqq)
    nodes = orc.smear_nodes(Q, dqq)
    for i in (0, 7, 14):
        seed = np.zeros(Q.size)
        seed[i] = 1.0
        g, _ = orc.model_vjp_cs(rows, sc, bk, Q, dqq, seed)
        J = orc.reflectivity_jac_cs(rows, nodes[i])  # (K, L+2, 4)
        ref = sc * np.tensordot(w, J, axes=(0, 0))
        a, b = _scaled(g), _scaled(ref)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b)), i


def test_vjp_is_linear_in_the_seed(orc):
    rng = np.random.default_rng(713)
    rows = rand_stack(rng, 3)
    Q = np.geomspace(0.006, 0.3, 19)
    s1, s2 = rng.standard_normal(Q.size), rng.standard_normal(Q.size)
    g1, i1 = orc.model_vjp_cs(rows, 1.0, 1e-7, Q, 0.05, s1)
    g2, i2 = orc.model_vjp_cs(rows, 1.0, 1e-7, Q, 0.05, s2)
    g3, i3 = orc.model_vjp_cs(rows, 1.0, 1e-7, Q, 0.05, 2.0 * s1 - 0.5 * s2)
    ref = _scaled(2.0 * g1 - 0.5 * g2)
    assert np.max(np.abs(_scaled(g3) - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(i3 - (2.0 * i1 - 0.5 * i2))) <= 1e-12 * np.max(np.abs(i3))


def _ragged(rng, n_items=9):
    Ls = [0, 1, 3, 7, 2, 12, 5, 1, 4][:n_items]
    nqs = [13, 0, 29, 7]
    dqqs = [0.05, 0.0, 0.02, 0.08]
    q_off = np.concatenate([[0], np.cumsum(nqs)]).astype(np.int64)
    Q = np.concatenate([np.geomspace(0.007, 0.3, n) for n in nqs])
    dsi = np.array([b % len(nqs) for b in range(n_items)], np.int32)
    stacks = [rand_stack(rng, L) for L in Ls]
    row_off = np.concatenate([[0], np.cumsum([s.shape[0] for s in stacks])]).astype(np.int64)
    layers = np.vstack(stacks)
    scale = rng.uniform(0.9, 1.1, n_items)
    bkg = rng.uniform(0.5e-7, 1.5e-7, n_items)
    Robs = np.empty_like(Q)
    Rerr = np.empty_like(Q)
    for s in range(len(nqs)):
        sl = slice(q_off[s], q_off[s + 1])
        Rm = 10.0 ** rng.uniform(-7, 0, nqs[s])
        Rerr[sl] = 0.03 * Rm
        Robs[sl] = Rm
    return q_off, Q, Robs, Rerr, np.array(dqqs), dsi, row_off, layers, scale, bkg


@pytest.mark.parametrize("nthreads", [1, 4])
def test_batch_entry_point_equals_per_item_calls_bitwise(orc, nthreads):
    rng = np.random.default_rng(714)
    q_off, Q, Robs, Rerr, dqq, dsi, row_off, layers, scale, bkg = _ragged(rng)
    ll, g, gi = orc.loglik_grad_batch(q_off, Q, Robs, Rerr, dqq, dsi, row_off, layers, scale,
                                      bkg, want_grad=True, nthreads=nthreads)
    llf, _, _ = orc.loglik_grad_batch(q_off, Q, Robs, Rerr, dqq, dsi, row_off, layers, scale,
                                      bkg, want_grad=False, nthreads=nthreads)
    g = g.reshape(-1, 4)
    for b in range(dsi.size):
        s = dsi[b]
        sl = slice(q_off[s], q_off[s + 1])
        rows = layers[row_off[b]:row_off[b + 1]]
        llo, go, gio = orc.loglik_grad_cs(rows, scale[b], bkg[b], Q[sl], Robs[sl], Rerr[sl],
                                          dqq[s])
        lv = orc.loglik(rows, scale[b], bkg[b], Q[sl], Robs[sl], Rerr[sl], dqq[s])
        assert ll[b] == llo and llf[b] == lv
        assert np.array_equal(g[row_off[b]:row_off[b + 1]], go)
        assert np.array_equal(gi[b], gio)


def test_batch_entry_point_rejects_a_bad_dataset_index(orc):
    rng = np.random.default_rng(715)
    q_off, Q, Robs, Rerr, dqq, dsi, row_off, layers, scale, bkg = _ragged(rng, 3)
    dsi = dsi.copy()
    dsi[1] = 9
    with pytest.raises(ValueError):
        orc.loglik_grad_batch(q_off, Q, Robs, Rerr, dqq, dsi, row_off, layers, scale, bkg)
