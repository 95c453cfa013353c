"""The side_stream plan option: the gradient's small tail and split launches on
a second stream give bitwise the results of the one-stream schedule, in eager
calls and in a captured leapfrog graph replayed between eager work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

UNITS = np.array([1.0, 1e-6, 1e-6, 1.0])


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


def _tail_batch(seed):
    """84-point grids leave 20-point tails: unsmeared items of one depth pack
    three to a wave (a packed launch), smeared ones of up to 10 layers split
    over three node groups (a split launch); 128-point items have full units
    only."""
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(seed)
    datasets = []
    for nq, dqq in ((84, 0.0), (84, 0.05), (128, 0.03)):
        Q = inputs.log_grid(0.005, 0.35, nq)
        Robs, err = inputs.synthetic_curve(Q, rng)
        datasets.append((Q, Robs, err, dqq))
    items = []
    for ds, L in [(0, 3)] * 6 + [(1, 3)] * 3 + [(1, 8)] * 3 + [(2, 12)] * 2 + [(0, 20)] * 4:
        items.append((ds, inputs.draw_stack(rng, L), rng.uniform(0.9, 1.1),
                      rng.uniform(0.5e-7, 1.5e-7)))
    return inputs._pack("tails", datasets, items, {})


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_side_stream_results_bitwise_equal(nr, torch_cuda, precision):
    torch = torch_cuda
    batch = _tail_batch(900)
    prec = nr.NR_F32 if precision == "f32" else nr.NR_F64
    p0 = nr.Problem.from_batch(batch, precision=prec, options={"side_stream": 0})
    p1 = nr.Problem.from_batch(batch, precision=prec, options={"side_stream": 1})
    for rep in range(3):
        a = p0.loglik_grad()
        b = p1.loglik_grad()
        ar = p0.loglik_grad_res()
        br = p1.loglik_grad_res()
        torch.cuda.synchronize()
        for x, y in zip(list(a) + list(ar), list(b) + list(br)):
            assert torch.equal(x, y), f"call {rep}"
    assert np.all(p1.item_status.cpu().numpy() == 0)


def test_side_stream_leapfrog_graph_replays_equal_eager(nr, torch_cuda):
    torch = torch_cuda
    batch = _tail_batch(901)
    rng = np.random.default_rng(7)
    mom_rows = rng.standard_normal(batch.layers.shape) / UNITS
    mom_inst = rng.standard_normal((batch.n_items, 2)) / np.array([1.0, 1e-7])
    im_rows = np.tile(UNITS ** 2, (batch.layers.shape[0], 1))
    im_inst = np.tile(np.array([1.0, 1e-14]), (batch.n_items, 1))
    prob_e = nr.Problem.from_batch(batch, options={"side_stream": 0})
    prob_g = nr.Problem.from_batch(batch, options={"side_stream": 1})
    st_e = nr.HmcState(prob_e, mom_rows, mom_inst, im_rows, im_inst)
    st_g = nr.HmcState(prob_g, mom_rows, mom_inst, im_rows, im_inst)
    # a step small enough that the trajectory stays finite over the replays
    dt = 1e-5
    graph = nr.LeapfrogGraph(prob_g, st_g, dt, 3)
    for rep in range(3):
        prob_e.leapfrog(st_e, dt, 3)
        graph.launch()
        torch.cuda.synchronize()
        assert bool(torch.isfinite(st_g.logL).all()), f"replay {rep}: trajectory left the model"
        for a, b in [(st_e.layers, st_g.layers), (st_e.mom_rows, st_g.mom_rows),
                     (st_e.mom_inst, st_g.mom_inst), (st_e.g_rows, st_g.g_rows),
                     (st_e.logL, st_g.logL), (st_e.scale, st_g.scale)]:
            assert torch.equal(a.view(torch.int64), b.view(torch.int64)), \
                f"replay {rep} differs from eager"
        # the program's own eager work between replays, on both plans
        _ = (st_e.layers * 2.0).sum().item()
        _ = prob_g.loglik_grad()
    graph.close()


def test_side_stream_calls_from_two_host_threads(nr, torch_cuda):
    """Two host threads call nr_loglik_grad on one plan, each with its own
    stream, workspace and outputs: the plan's side stream and its fork ...
    join sequence are shared, and every result equals a one-thread call."""
    import threading
    torch = torch_cuda
    from paper_2509_06924_amd import NR_OP_LOGLIK_GRAD, nr_loglik_grad
    batch = _tail_batch(902)
    prob = nr.Problem.from_batch(batch, options={"side_stream": 1})
    ref = prob.loglik_grad()
    torch.cuda.synchronize()
    n_words = max(1, (prob.plan.workspace_size(NR_OP_LOGLIK_GRAD) + 7) // 8)
    vals = prob.values()
    n_calls = 12
    results, errors = {}, []

    def worker(tid):
        try:
            s = torch.cuda.Stream()
            ws = torch.empty(n_words, dtype=torch.float64, device=prob.device)
            outs = [tuple(torch.empty_like(t) for t in ref) for _ in range(n_calls)]
            for o in outs:
                nr_loglik_grad(prob.plan, vals, o[0], o[1], o[2], ws, stream=s)
            s.synchronize()
            results[tid] = outs
        except Exception as exc:  # reported below, on the test's thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for tid, outs in results.items():
        for k, o in enumerate(outs):
            for a, b in zip(o, ref):
                assert torch.equal(a, b), f"thread {tid} call {k}"
