"""Every schedule the plan options select computes the same thing: each
alternative is checked against the oracle like the default schedule, and the
autotuner's choice (and its JSON cache) round-trips."""
import numpy as np
import pytest

from nr_check import check_grad, check_logL, check_R, logL_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_06924_amd as nr
    return nr


def _batch(seed):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(seed)
    return inputs.random_batch(rng, n_items=12, L_choices=[0, 1, 2, 3, 4, 5, 7, 9, 10, 13],
                               nq_choices=[1, 30, 64, 100], dqq_choices=[0.0, 0.05],
                               n_datasets=5)


def _check_against_oracle(nr, orc, batch, options):
    prob = nr.Problem.from_batch(batch, options=options)
    Rhat = prob.reflectivity().cpu().numpy()
    ll, g_rows, g_inst = prob.loglik_grad()
    ll, g_rows, g_inst = ll.cpu().numpy(), g_rows.cpu().numpy(), g_inst.cpu().numpy()
    off = prob.out_off
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        check_R(Rhat[off[b]:off[b + 1]], Ro, what=f"R item {b}")
        llo = orc.loglik(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        check_logL(ll[b], llo, logL_bound(Ro, Robs, Rerr), what=f"logL item {b}")
        _, go, gio = orc.loglik_grad_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        check_grad(g_rows[r0:r1], g_inst[b], go, gio, what=f"grad item {b} {options}")


@pytest.mark.parametrize("options", [
    {"grad_variant": {str(k): 2 for k in (1, 2, 4, 6, 8, 10)}},   # recompute everywhere
    {"pack_tails": 0},
    {"xcd_run": 1},
    {"xcd_run": 3, "pack_tails": 0},
    {"split_tails": 0},
    {"split_tails": 1},
    {"split_tails": 2, "pack_tails": 0,
     "grad_variant": {str(k): 2 for k in (1, 2, 4, 6, 8, 10)}},
    {"side_stream": 0},
    {"side_stream": 0, "split_tails": 0, "pack_tails": 0},
    {"split_tails": 3},   # no small-plan split
    {"split_tails": 4},   # the small-plan split only
    {"node_groups": 2},   # (sample, Q) tilings: 32, 16, 8 and 3 points per wave
    {"node_groups": 4},
    {"node_groups": 8, "side_stream": 0},
    {"node_groups": 17, "pack_tails": 0},
])
def test_schedules_match_oracle(nr, orc, options):
    _check_against_oracle(nr, orc, _batch(501), options)


@pytest.mark.parametrize("groups", [2, 4])
def test_node_group_tilings_of_a_large_plan(nr, orc, groups):
    """A plan large enough that the library's rules keep 64 points per wave
    (4096 draws of 10 layers x 400 points), tiled with node groups instead:
    sampled draws against the oracle."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c2_batched()
    prob = nr.Problem.from_batch(batch, options={"node_groups": groups})
    Rhat = prob.reflectivity().cpu().numpy()
    ll, g_rows, g_inst = (t.cpu().numpy() for t in prob.loglik_grad())
    assert np.all(prob.item_status.cpu().numpy() == 0)
    for b in (0, 2049, 4095):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        check_R(Rhat[prob.out_off[b]:prob.out_off[b + 1]], Ro, what=f"R item {b}")
        llo, go, gio = orc.loglik_grad_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        check_logL(ll[b], llo, logL_bound(Ro, Robs, Rerr), what=f"logL item {b}")
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        check_grad(g_rows[r0:r1], g_inst[b], go, gio, what=f"grad item {b}, {groups} groups")


def test_autotune_choice_and_cache(nr, orc, tmp_path):
    from paper_2509_06924_amd import autotune, inputs
    batch = inputs.c2_batched(n_items=512, L=6)
    cache = str(tmp_path / "tune.json")
    opts = autotune.tune(batch, cache=cache, reps=2)
    assert set(opts) == {"grad_variant", "xcd_run", "pack_tails", "split_tails", "side_stream",
                         "node_groups"}
    assert autotune.tune(batch, cache=cache) == opts  # served from the cache
    p_def = nr.Problem.from_batch(batch)
    p_tun = nr.Problem.from_batch(batch, options=opts)
    a = [t.cpu().numpy() for t in p_def.loglik_grad()]
    b = [t.cpu().numpy() for t in p_tun.loglik_grad()]
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=0)
    units = np.array([1.0, 1e-6, 1e-6, 1.0])
    scale = np.max(np.abs(a[1] * units))
    assert np.max(np.abs((a[1] - b[1]) * units)) <= 1e-10 * scale
    # and the tuned schedule still matches the oracle on a few items
    _check_against_oracle(nr, orc, batch.subset(np.arange(3)), opts)


def test_native_autotune_entry_point(nr):
    """nr_autotune through the C ABI: valid options that build a plan, and
    the defaults' and the winner's timings."""
    import ctypes
    from paper_2509_06924_amd import _native as n, autotune, inputs
    batch = inputs.c2_batched(n_items=256, L=4)
    prob = nr.Problem.from_batch(batch)
    o = n.PlanOptions()
    ms = (ctypes.c_double * 2)()
    import torch
    st = n.lib().nr_autotune(ctypes.byref(prob.plan.desc), ctypes.byref(prob.values()), 2,
                             ctypes.byref(o), ctypes.cast(ms, ctypes.c_void_p),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == n.NR_OK
    assert ms[0] > 0 and ms[1] > 0 and ms[0] <= ms[1] * 1.0001
    opts = autotune.options_to_dict(o)
    nr.Problem.from_batch(batch, options=opts).loglik_grad()
    assert n.lib().nr_autotune(None, ctypes.byref(prob.values()), 2, ctypes.byref(o), None,
                               None) == n.NR_EINVAL
