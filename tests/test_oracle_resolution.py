"""Pins of the oracle's resolution functions: per-point widths (Sec. 3
pointwise Gaussian smearing, Sec. 4.1 per-point FWHM) and the derivative of
logL with respect to a free relative width dQ/Q (Sec. 4.2, the smearing size
inferred as a parameter)."""
import numpy as np
import pytest

import oracle as orc
from paper_2509_06924_amd import inputs

FWHM = 2.3548200450309493


def _case(seed, L=3, nq=60, dqq=0.05):
    rng = np.random.default_rng(seed)
    rows = inputs.draw_stack(rng, L)
    Q = inputs.log_grid(0.008, 0.3, nq)
    Robs, err = inputs.synthetic_curve(Q, rng)
    return rows, Q, Robs, err, dqq


def test_pointwise_widths_equal_to_relative_width_reproduce_it():
    rows, Q, Robs, err, dqq = _case(1)
    dQ = dqq * Q  # the same product the relative width forms
    a = orc.model_curve(rows, 1.02, 1e-7, Q, dqq)
    b = orc.model_curve_res(rows, 1.02, 1e-7, Q, dqq, dQ)
    c = orc.model_curve_res(rows, 1.02, 1e-7, Q, dqq)
    # the same node positions: bit-identical within the resolution path ...
    assert np.array_equal(b, c)
    # ... and the plain path's curve to rounding (bicomplex vs complex division)
    assert np.allclose(a, c, rtol=1e-13, atol=0)


def test_pointwise_widths_change_the_curve_and_zero_width_is_unsmeared():
    rows, Q, Robs, err, dqq = _case(2)
    dQ = np.linspace(0.02, 0.08, Q.size) * Q
    a = orc.model_curve_res(rows, 1.0, 0.0, Q, dqq, dQ)
    assert np.max(np.abs(a / orc.model_curve(rows, 1.0, 0.0, Q, dqq) - 1)) > 1e-3
    z = orc.model_curve_res(rows, 1.0, 0.0, Q, dqq, np.zeros_like(Q))
    # all 17 nodes at Q and normalised weights: the unsmeared R to rounding
    assert np.allclose(z, orc.reflectivity(rows, Q), rtol=1e-14, atol=0)


def test_dR_dq_single_interface_closed_form():
    """R = ((k0 - k1)/(k0 + k1))^2 above the edge, sigma = 0: dR/dq by the
    chain rule with dk1/dk0 = k0/k1 and dk0/dq = 1/2."""
    rho = 2.07e-6
    rows = np.array([[0, 0.0, 0, 0], [0, rho, 0.0, 0.0]])
    q = np.linspace(0.02, 0.3, 40)
    k0 = q / 2
    a = 4 * np.pi * rho
    k1 = np.sqrt(k0 * k0 - a)
    r = (k0 - k1) / (k0 + k1)
    dk1 = k0 / k1
    dr = ((1 - dk1) * (k0 + k1) - (k0 - k1) * (1 + dk1)) / (k0 + k1) ** 2
    ref = 2 * r * dr * 0.5
    got = orc.reflectivity_dq_cs(rows, q)
    assert np.allclose(got, ref, rtol=1e-9, atol=0)


@pytest.mark.parametrize("seed,L,dqq", [(3, 2, 0.05), (4, 5, 0.02), (5, 9, 0.08)])
def test_width_derivative_complex_step_vs_richardson(seed, L, dqq):
    rows, Q, Robs, err, _ = _case(seed, L=L, dqq=dqq)
    _, _, _, gcs = orc.loglik_grad_res_cs(rows, 1.0, 1e-7, Q, Robs, err, dqq)
    gfd = orc.loglik_res_fd(rows, 1.0, 1e-7, Q, Robs, err, dqq, rel_step=1e-3)
    assert abs(gcs - gfd) <= 1e-6 * abs(gcs)


def test_width_derivative_assembled_from_node_slopes():
    """dlogL/d(dQ/Q) = sum_i ghat_i scale sum_k w_k R'(q_ik) Q_i t_k / FWHM,
    with R' from the complex step through q at each node."""
    rows, Q, Robs, err, dqq = _case(6, L=4, nq=30)
    scale, bkg = 0.97, 1e-7
    Rhat = orc.model_curve(rows, scale, bkg, Q, dqq)
    ghat = -(Rhat - Robs) / err ** 2
    K = 17
    t = np.empty(K)
    w = np.empty(K)
    orc.lib().orc_smear_rule(orc._D(dqq), orc._p(t), orc._p(w))
    nodes = orc.smear_nodes(Q, dqq).reshape(Q.size, K)
    slope = orc.reflectivity_dq_cs(rows, nodes.ravel()).reshape(Q.size, K)
    ref = np.sum(ghat * scale * np.sum(w * slope * (Q[:, None] * t / FWHM), axis=1))
    _, _, _, g = orc.loglik_grad_res_cs(rows, scale, bkg, Q, Robs, err, dqq)
    assert abs(g - ref) <= 1e-10 * abs(ref)


def test_width_derivative_vanishes_at_zero_width():
    """The rule is symmetric (sum w_k t_k = 0), so d/ds sum_k w_k R(Q + s t_k)
    is 0 at s = 0 and O(s) near it."""
    rows, Q, Robs, err, _ = _case(7, L=3)
    g = [orc.loglik_grad_res_cs(rows, 1.0, 1e-7, Q, Robs, err, d)[3] for d in (1e-5, 2e-5)]
    assert abs(g[1] / g[0] - 2.0) < 1e-3
    _, _, _, g0 = orc.loglik_grad_res_cs(rows, 1.0, 1e-7, Q, Robs, err, 0.0)
    assert g0 == 0.0


def test_pointwise_width_gradient_rows_match_relative_when_equal():
    rows, Q, Robs, err, dqq = _case(8, L=3)
    a = orc.loglik_grad_cs(rows, 1.0, 1e-7, Q, Robs, err, dqq)
    b = orc.loglik_grad_res_cs(rows, 1.0, 1e-7, Q, Robs, err, dqq, dqq * Q)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(a[0])
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=0) and b[3] == 0.0
