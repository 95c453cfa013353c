"""Parity of the HIP path (through the C ABI) with the CPU oracle.

R_hat element by element, logL per item and the gradient per item, on seeded
synthetic inputs: small ragged batches that cross bucket and tile boundaries
(empty datasets, 1 point, 63/64/65 points, 0..40 layers, smeared and not),
the single-film workload in full, and the 4096-draw workload at full size on
sampled items.
"""
import numpy as np
import pytest

from nr_check import check_grad, check_logL, check_R, logL_bound

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


def _run_all(nr, batch, options=None):
    prob = nr.Problem.from_batch(batch, options=options)
    Rhat = prob.reflectivity().cpu().numpy()
    ll = prob.loglik().cpu().numpy()
    llg, g_rows, g_inst = prob.loglik_grad()
    status = prob.item_status.cpu().numpy()
    return prob, Rhat, ll, llg.cpu().numpy(), g_rows.cpu().numpy(), g_inst.cpu().numpy(), status


def _check_items(orc, batch, items, Rhat, ll, llg, g_rows, g_inst, out_off, grad=True):
    for b in items:
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        check_R(Rhat[out_off[b]:out_off[b + 1]], Ro, what=f"R_hat item {b}")
        llo = orc.loglik(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        bound = logL_bound(Ro, Robs, Rerr)
        check_logL(ll[b], llo, bound, what=f"logL item {b}")
        check_logL(llg[b], llo, bound, what=f"logL(grad call) item {b}")
        if grad:
            _, go, gio = orc.loglik_grad_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
            r0, r1 = batch.row_off[b], batch.row_off[b + 1]
            check_grad(g_rows[r0:r1], g_inst[b], go, gio, what=f"grad item {b}")


def test_single_film_workload(nr, orc):
    from paper_2509_06924_amd import inputs
    batch = inputs.c1_single_film()
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch)
    assert st[0] == 0
    _check_items(orc, batch, [0], Rhat, ll, llg, g_rows, g_inst, prob.out_off)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ragged_small_batches(nr, orc, seed):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(1000 + seed)
    batch = inputs.random_batch(rng, n_items=14, L_choices=[0, 1, 2, 3, 5, 8, 10, 11, 12],
                                nq_choices=[0, 1, 17, 63, 64, 65, 130],
                                dqq_choices=[0.0, 0.02, 0.05, 0.08], n_datasets=7)
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch)
    assert np.all(st == 0)
    _check_items(orc, batch, range(batch.n_items), Rhat, ll, llg, g_rows, g_inst, prob.out_off)


def test_deep_stacks(nr, orc):
    """Every layer-count bucket up to the maximum, small Q sets."""
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(77)
    batch = inputs.random_batch(rng, n_items=10, L_choices=[13, 16, 17, 20, 24, 31, 32, 39, 40],
                                nq_choices=[5, 64, 70], dqq_choices=[0.0, 0.05], n_datasets=4)
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch)
    assert np.all(st == 0)
    _check_items(orc, batch, range(batch.n_items), Rhat, ll, llg, g_rows, g_inst, prob.out_off)


def test_empty_dataset_items(nr):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(5)
    batch = inputs.random_batch(rng, n_items=3, L_choices=[2], nq_choices=[0],
                                dqq_choices=[0.05], n_datasets=1)
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch)
    assert Rhat.size == 0
    assert np.all(ll == 0.0) and np.all(llg == 0.0)
    assert np.all(g_rows == 0.0) and np.all(g_inst == 0.0)


def test_batched_workload_full_size_sampled(nr, orc, tmp_path):
    """4096 draws x 10 layers x 400 Q, 17-node smearing, at full size, with the
    default schedule and with the one the autotuner picks (the benchmark's);
    items sampled across the batch are checked against the oracle."""
    from paper_2509_06924_amd import autotune, inputs
    batch = inputs.c2_batched()
    tuned = autotune.tune(batch, cache=str(tmp_path / "tune.json"), reps=3)
    for options in (None, tuned):
        prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch, options)
        assert np.all(st == 0)
        assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g_rows))
        _check_items(orc, batch, [0, 1, 1234, 2047, 4095], Rhat, ll, llg, g_rows, g_inst,
                     prob.out_off)


@pytest.mark.parametrize("n_items", [1, 5, 40])
def test_small_smeared_plans(nr, orc, n_items):
    """Draws of the 10-layer, 400-point, 5 % dQ/Q workload in plans small
    enough that every point group is split over node groups (17, 17 and 6
    groups for 1, 5 and 40 items); the last draw against the oracle."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c2_batched(n_items=n_items)
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run_all(nr, batch)
    assert np.all(st == 0)
    _check_items(orc, batch, [n_items - 1], Rhat, ll, llg, g_rows, g_inst, prob.out_off)


def test_deterministic(nr, torch_cuda):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(9)
    batch = inputs.random_batch(rng, n_items=20, L_choices=[3, 10, 25], nq_choices=[100, 300],
                                dqq_choices=[0.05], n_datasets=4)
    prob = nr.Problem.from_batch(batch)
    a = [t.cpu().numpy().copy() for t in prob.loglik_grad()]
    b = [t.cpu().numpy().copy() for t in prob.loglik_grad()]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_item_status_flags(nr, torch_cuda):
    torch = torch_cuda
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(11)
    batch = inputs.random_batch(rng, n_items=3, L_choices=[2], nq_choices=[40],
                                dqq_choices=[0.05], n_datasets=3)
    batch.dataset_of_item[:] = [0, 1, 2]
    Q = batch.Q.copy()
    Q[batch.q_off[1] + 3] = -0.01          # dataset 1: a negative Q
    Rerr = batch.Rerr.copy()
    Rerr[batch.q_off[2] + 5] = 0.0         # dataset 2: a zero error bar
    plan = nr.Plan(batch.q_off, batch.dq_over_q, batch.dataset_of_item, batch.row_off)
    prob = nr.Problem(plan, Q, batch.Robs, Rerr, batch.layers, batch.scale, batch.bkg)
    ll, g, gi = prob.loglik_grad()
    st = prob.item_status.cpu().numpy()
    ll = ll.cpu().numpy()
    assert st[0] == 0 and np.isfinite(ll[0])
    assert st[1] & nr.NR_ITEM_BAD_Q and np.isnan(ll[1])
    assert st[2] & nr.NR_ITEM_BAD_ERR and np.isnan(ll[2])


def test_autograd_function(nr, torch_cuda):
    torch = torch_cuda
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(12)
    batch = inputs.random_batch(rng, n_items=4, L_choices=[1, 4], nq_choices=[50],
                                dqq_choices=[0.05], n_datasets=2)
    prob = nr.Problem.from_batch(batch)
    layers = prob.layers.clone().requires_grad_(True)
    scale = prob.scale.clone().requires_grad_(True)
    bkg = prob.bkg.clone().requires_grad_(True)
    ll = nr.NRLogLik.apply(layers, scale, bkg, prob)
    w = torch.arange(1, 5, dtype=torch.float64, device="cuda")
    (ll * w).sum().backward()
    _, g_rows, g_inst = prob.loglik_grad()
    row_w = w[prob.row_item].unsqueeze(1)
    assert torch.equal(layers.grad, g_rows * row_w)
    assert torch.equal(scale.grad, g_inst[:, 0] * w)
    assert torch.equal(bkg.grad, g_inst[:, 1] * w)
