"""The README's Python examples run as written (GPU): the batch workflow,
a stack from the paper's parameter dictionary, the autograd function and the
autotuner."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_quick_start(torch_cuda):
    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import inputs
    batch = inputs.c2_batched(n_items=8)
    prob = nr.Problem.from_batch(batch)
    logL, g_rows, g_inst = prob.loglik_grad()
    R = prob.reflectivity()
    assert logL.shape == (8,) and g_rows.shape == prob.layers.shape and g_inst.shape == (8, 2)
    assert R.numel() == int(prob.out_off[-1])


def test_own_data_and_autograd(torch_cuda, orc):
    torch = torch_cuda
    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import inputs
    rows = nr.pack_theta({"thick": [120.0, 40.0], "SLD": [0.0, 3.5, 1.2, 2.07],
                          "rough": [3.0, 5.0, 2.0]}, sld_unit=1e-6)
    Q = inputs.log_grid(0.01, 0.25, 90)
    rng = np.random.default_rng(5)
    Robs, err = inputs.synthetic_curve(Q, rng)
    plan = nr.Plan(q_off=[0, Q.size], dq_over_q=[0.05], dataset_of_item=[0], row_off=[0, 4])
    prob = nr.Problem(plan, Q, Robs, err, rows, [1.0], [1e-7])
    layers = prob.layers.clone().requires_grad_(True)
    scale = prob.scale.clone().requires_grad_(True)
    bkg = prob.bkg.clone().requires_grad_(True)
    logL = nr.NRLogLik.apply(layers, scale, bkg, prob)
    logL.sum().backward()
    llo, go, gio = orc.loglik_grad_cs(rows, 1.0, 1e-7, Q, Robs, err, 0.05)
    assert abs(float(logL.detach()[0]) - llo) <= 1e-9 * abs(llo)
    units = np.array([1.0, 1e-6, 1e-6, 1.0])
    g = layers.grad.cpu().numpy()
    assert np.max(np.abs((g - go) * units)) <= 1e-8 * np.max(np.abs(go * units))


def test_autotune_options(torch_cuda, tmp_path):
    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import autotune, inputs
    batch = inputs.c2_batched(n_items=256)
    opts = autotune.tune(batch, cache=str(tmp_path / "t.json"), reps=2)
    prob = nr.Problem.from_batch(batch, options=opts)
    logL, _, _ = prob.loglik_grad()
    assert bool(torch_cuda.isfinite(logL).all())
