"""nr_loglik_grad_noalloc, the gradient call for callers that cannot allocate:
it must give exactly what nr_loglik_grad gives with a caller workspace, on
two calls in a row (the second with a smaller batch, so that stale scratch
contents of the first would show), and refuse a plan whose workspace exceeds
its fixed scratch before enqueuing anything."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_noalloc(nr, prob):
    import torch
    from paper_2509_06924_amd import _native
    n = prob.plan.n_items
    f = dict(dtype=torch.float64, device=prob.device)
    out = (torch.full((n,), float("nan"), **f), torch.full_like(prob.layers, float("nan")),
           torch.full((n, 2), float("nan"), **f))
    v = prob.values()
    stream = torch.cuda.current_stream()
    rc = _native.lib().nr_loglik_grad_noalloc(
        prob.plan.handle, ctypes.byref(v), ctypes.c_void_p(out[0].data_ptr()),
        ctypes.c_void_p(out[1].data_ptr()), ctypes.c_void_p(out[2].data_ptr()),
        ctypes.c_void_p(stream.cuda_stream))
    assert rc == _native.NR_OK, _native.status_string(rc)
    torch.cuda.synchronize()
    return out


def test_noalloc_equals_the_workspace_call_on_two_calls_in_a_row():
    import torch

    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import inputs
    torch.cuda.set_device(0)
    rng = np.random.default_rng(2509)
    big = inputs.random_batch(rng, n_items=48, L_choices=[0, 1, 4, 10, 17, 33, 40, 77],
                              nq_choices=[0, 9, 64, 130, 333], dqq_choices=[0.0, 0.05],
                              n_datasets=5)
    small = inputs.random_batch(rng, n_items=3, L_choices=[2, 6], nq_choices=[11, 70],
                                dqq_choices=[0.03], n_datasets=2)
    for name, batch in (("first, 48 items", big), ("second, 3 items", small)):
        print("no-alloc call:", name, flush=True)
        prob = nr.Problem.from_batch(batch, device="cuda:0")
        ref = prob.loglik_grad()
        torch.cuda.synchronize()
        got = _call_noalloc(nr, prob)
        for a, b, what in zip(got, ref, ("logL", "g_rows", "g_inst")):
            assert torch.equal(a, b), (name, what)
        prob.plan.close()


def test_noalloc_refuses_a_plan_beyond_its_scratch():
    import torch

    import paper_2509_06924_amd as nr
    from paper_2509_06924_amd import _native
    torch.cuda.set_device(0)
    # 1700 items of 2047 layers: 3.5e6 rows, 280 MB of per-row constants alone
    n_items, rows = 1700, 2049
    plan = nr.Plan(np.array([0, 4], np.int64), np.array([0.05]),
                   np.zeros(n_items, np.int32),
                   np.arange(n_items + 1, dtype=np.int64) * rows)
    assert plan.workspace_size(nr.NR_OP_LOGLIK_GRAD) > _native.NR_NOALLOC_SCRATCH_BYTES
    f = dict(dtype=torch.float64, device="cuda:0")
    q = torch.tensor([0.01, 0.02, 0.05, 0.1], **f)
    layers = torch.zeros(n_items * rows, 4, **f)
    scale = torch.ones(n_items, **f)
    bkg = torch.zeros(n_items, **f)
    v = nr._values(q, q, q, layers, scale, bkg)
    logL = torch.empty(n_items, **f)
    g_inst = torch.empty(n_items, 2, **f)
    rc = _native.lib().nr_loglik_grad_noalloc(
        plan.handle, ctypes.byref(v), ctypes.c_void_p(logL.data_ptr()),
        ctypes.c_void_p(layers.data_ptr()), ctypes.c_void_p(g_inst.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _native.NR_ESCRATCH
    assert "NR_NOALLOC_SCRATCH_BYTES" in _native.status_string(rc)
    plan.close()
