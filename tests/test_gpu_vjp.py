"""Vector-Jacobian product of R_hat (nr_reflectivity_vjp) against the oracle's
complex-step VJP, its autograd function, and the EDGE_SINGULAR status."""
import numpy as np
import pytest

from nr_check import G_TOL, INST_UNITS, R_TOL, ROW_UNITS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def nr(torch_cuda):
    import paper_2509_06924_amd as nr
    return nr


@pytest.mark.parametrize("seed", [0, 1])
def test_reflectivity_vjp_matches_oracle(nr, orc, torch_cuda, seed):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(300 + seed)
    batch = inputs.random_batch(rng, n_items=8, L_choices=[0, 1, 3, 6, 11, 17],
                                nq_choices=[1, 40, 70, 130], dqq_choices=[0.0, 0.05],
                                n_datasets=4)
    prob = nr.Problem.from_batch(batch)
    off = prob.out_off
    v = rng.standard_normal(int(off[-1]))
    dot, g_rows, g_inst = (t.cpu().numpy() for t in prob.reflectivity_vjp(v))
    assert np.all(prob.item_status.cpu().numpy() == 0)
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, _, _, dqq = batch.data_of(b)
        vb = v[off[b]:off[b + 1]]
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        # dot: each R_hat within R_TOL relative
        assert abs(dot[b] - vb @ Ro) <= R_TOL * (np.abs(vb) @ np.abs(Ro)) + 1e-300
        go, gio = orc.model_vjp_cs(rows, batch.scale[b], batch.bkg[b], Q, dqq, vb)
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        a = np.concatenate([(g_rows[r0:r1] * ROW_UNITS).ravel(), g_inst[b] * INST_UNITS])
        o = np.concatenate([(go * ROW_UNITS).ravel(), gio * INST_UNITS])
        scale = np.max(np.abs(o))
        assert np.max(np.abs(a - o)) <= G_TOL * scale, f"item {b}"


def test_reflectivity_autograd(nr, torch_cuda):
    torch = torch_cuda
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(310)
    batch = inputs.random_batch(rng, n_items=3, L_choices=[2, 5], nq_choices=[60],
                                dqq_choices=[0.05], n_datasets=2)
    prob = nr.Problem.from_batch(batch)
    layers = prob.layers.clone().requires_grad_(True)
    scale = prob.scale.clone().requires_grad_(True)
    bkg = prob.bkg.clone().requires_grad_(True)
    R = nr.NRReflectivity.apply(layers, scale, bkg, prob)
    assert torch.equal(R, prob.reflectivity())
    w = torch.linspace(-1.0, 2.0, R.numel(), dtype=torch.float64, device=R.device)
    (R * w).sum().backward()
    _, g_rows, g_inst = prob.reflectivity_vjp(w)
    assert torch.equal(layers.grad, g_rows)
    assert torch.equal(scale.grad, g_inst[:, 0]) and torch.equal(bkg.grad, g_inst[:, 1])


def _edge_rho(Q):
    """A rho_1 (fronting rho 0) with fl(4 pi rho_1) == fl(fl(Q/4) Q): the
    kernel's kz0^2 - 4 pi (rho_1 - rho_0) is then exactly 0 at q = Q."""
    four_pi = 12.566370614359172
    kz0sq = (0.25 * Q) * Q
    rho = kz0sq / four_pi
    for _ in range(64):
        a = four_pi * rho
        if a == kz0sq:
            return rho
        rho = np.nextafter(rho, np.inf if a < kz0sq else -np.inf)
    return None


def test_edge_singular_flag(nr, torch_cuda):
    from paper_2509_06924_amd import inputs
    Qs = [0.02 + 1e-6 * k for k in range(200)]
    found = [(q, _edge_rho(q)) for q in Qs]
    Q, rho = next((q, r) for q, r in found if r is not None)
    rows_edge = np.array([[0, 0.0, 0, 0], [50.0, rho, 0.0, 3.0], [0, 2.07e-6, 1e-9, 4.0]])
    rows_ok = rows_edge.copy()
    rows_ok[1, 1] = 3.0e-6
    Qv = np.array([0.015, Q, 0.03])
    R = np.array([0.5, 0.3, 0.01])
    batch = inputs._pack("edge", [(Qv, R, 0.03 * R, 0.0)],
                         [(0, rows_edge, 1.0, 1e-7), (0, rows_ok, 1.0, 1e-7)], {})
    prob = nr.Problem.from_batch(batch)
    prob.loglik()
    assert np.all(prob.item_status.cpu().numpy() == 0)  # value calls do not look
    prob.loglik_grad()
    st = prob.item_status.cpu().numpy()
    assert st[0] & nr.NR_ITEM_EDGE_SINGULAR
    assert st[1] == 0
