"""Deep stacks (more than NR_MAX_LAYERS layers) through the C-ABI: the value
kernels and the parallel-in-layers scan gradient against the oracle, at depths
that put one level per lane, leave lanes empty, fill every lane, and give
several levels per lane; mixed with shallow items in one plan; the resolution
derivative; the microsliced-layer identities on the device."""
import numpy as np
import pytest

from nr_check import G_TOL, INST_UNITS, ROW_UNITS, check_grad, check_logL, check_R, logL_bound

pytestmark = pytest.mark.gpu

RES_UNIT = 1e-2


@pytest.fixture(scope="module")
def nr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_06924_amd as nr
    return nr


def _profile(rng, L, dz=3.0):
    from test_oracle_deep import smooth_profile
    return smooth_profile(rng, L, dz)


def _batch(rng, depths, nq, dqq, extra_shallow=0):
    from paper_2509_06924_amd import inputs
    datasets = []
    Q = inputs.log_grid(0.008, 0.25, nq)
    Robs, err = inputs.synthetic_curve(Q, rng)
    datasets.append((Q, Robs, err, dqq))
    items = [(0, _profile(rng, L), float(rng.uniform(0.9, 1.1)), 1e-7) for L in depths]
    for _ in range(extra_shallow):
        items.append((0, inputs.draw_stack(rng, int(rng.integers(1, 12))), 1.0, 1e-7))
    return inputs._pack("deep", datasets, items, {})


def _check_items(nr, orc, batch, prob, with_res=False):
    Rhat = prob.reflectivity().cpu().numpy()
    ll_v = prob.loglik().cpu().numpy()
    if with_res:
        ll, g_rows, g_inst, g_res = (t.cpu().numpy() for t in prob.loglik_grad_res())
    else:
        ll, g_rows, g_inst = (t.cpu().numpy() for t in prob.loglik_grad())
    assert np.all(prob.item_status.cpu().numpy() == 0)
    off = prob.out_off
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        # against 50-digit values the kernels' R is within 6e-14 up to 2047
        # slabs (test_deep_R_against_fifty_digit_parratt) and the oracle's
        # within 8e-12 (its Fresnel difference kz_j - kz_{j+1} cancels between
        # near-equal slices), so the shallow stacks' tolerance holds here
        check_R(Rhat[off[b]:off[b + 1]], Ro, what=f"R item {b}")
        bound = logL_bound(Ro, Robs, Rerr)
        llo_v = orc.loglik(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        check_logL(ll_v[b], llo_v, bound, what=f"logL item {b}")
        if with_res:
            llo, go, gio, gro = orc.loglik_grad_res_cs(rows, batch.scale[b], batch.bkg[b], Q,
                                                       Robs, Rerr, dqq)
            a = np.concatenate([(g_rows[batch.row_off[b]:batch.row_off[b + 1]] * ROW_UNITS)
                                .ravel(), g_inst[b] * INST_UNITS, [g_res[b] * RES_UNIT]])
            o = np.concatenate([(go * ROW_UNITS).ravel(), gio * INST_UNITS, [gro * RES_UNIT]])
            assert np.max(np.abs(a - o)) <= G_TOL * np.max(np.abs(o)), f"item {b}"
        else:
            llo, go, gio = orc.loglik_grad_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr,
                                              dqq)
            check_grad(g_rows[batch.row_off[b]:batch.row_off[b + 1]], g_inst[b], go, gio,
                       what=f"grad item {b} (L = {rows.shape[0] - 2})")
        check_logL(ll[b], llo, bound, what=f"logL (grad call) item {b}")


# 41: one level per lane, 22 lanes empty; 63: every lane one level;
# 64: two levels in lane 0 ... ; 100, 127, 300: several levels per lane
@pytest.mark.parametrize("depths", [[41, 63], [64, 100], [127, 300]])
def test_deep_items_match_oracle(nr, orc, depths):
    rng = np.random.default_rng(800 + depths[0])
    batch = _batch(rng, depths, nq=9, dqq=0.0)
    _check_items(nr, orc, batch, nr.Problem.from_batch(batch))


# 600 slabs: two waves per data point; 1500 slabs: four; with a shallower
# deep item in the same plan, each class in a launch of its own
@pytest.mark.parametrize("depths", [[600], [45, 1500], [1100, 700, 300]])
def test_multi_wave_points_match_oracle(nr, orc, depths):
    rng = np.random.default_rng(860 + depths[0])
    batch = _batch(rng, depths, nq=3, dqq=0.0)
    _check_items(nr, orc, batch, nr.Problem.from_batch(batch))


def test_multi_wave_smeared_with_resolution_gradient(nr, orc):
    rng = np.random.default_rng(870)
    batch = _batch(rng, [600], nq=1, dqq=0.04, extra_shallow=1)
    _check_items(nr, orc, batch, nr.Problem.from_batch(batch), with_res=True)


def test_deep_smeared_with_resolution_gradient_and_shallow_items(nr, orc):
    rng = np.random.default_rng(820)
    batch = _batch(rng, [45, 90], nq=5, dqq=0.04, extra_shallow=3)
    _check_items(nr, orc, batch, nr.Problem.from_batch(batch), with_res=True)


def test_deep_items_in_fp32_plan(nr, orc):
    """An FP32 plan: deep gradients are FP64 (the value kernels are FP32)."""
    rng = np.random.default_rng(830)
    batch = _batch(rng, [70], nq=7, dqq=0.0)
    prob = nr.Problem.from_batch(batch, precision=nr.NR_F32)
    _, g_rows, g_inst = (t.cpu().numpy() for t in prob.loglik_grad())
    rows = batch.rows_of(0)
    Q, Robs, Rerr, dqq = batch.data_of(0)
    _, go, gio = orc.loglik_grad_cs(rows, batch.scale[0], batch.bkg[0], Q, Robs, Rerr, dqq)
    check_grad(g_rows, g_inst[0], go, gio, what="fp32 plan, deep item")


def test_microsliced_layer_identities_on_device(nr, orc):
    from test_oracle_deep import _sliced
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(840)
    Q = inputs.log_grid(0.01, 0.25, 20)
    R = orc.model_curve(_sliced(1), 1.0, 1e-7, Q, 0.03)
    Robs = R * (1 + 0.05 * rng.standard_normal(Q.size))
    Rerr = 0.03 * Robs
    n = 200
    batch = inputs._pack("sliced", [(Q, Robs, Rerr, 0.03)],
                         [(0, _sliced(1), 1.0, 1e-7), (0, _sliced(n), 1.0, 1e-7)], {})
    prob = nr.Problem.from_batch(batch)
    ll, g, _ = (t.cpu().numpy() for t in prob.loglik_grad())
    # measured on MI355X: 2e-15, 4e-13 and 2e-13 (1e-14, 1.2e-12 and 7e-13
    # at 1000 slices)
    assert abs(ll[1] - ll[0]) <= 1e-10 * abs(ll[0])
    g1 = g[0:3]
    gn = g[3:3 + n + 2]
    assert np.allclose(gn[1:n + 1, 0], g1[1, 0], rtol=1e-10, atol=0)
    assert abs(np.sum(gn[1:n + 1, 1]) - g1[1, 1]) <= 1e-10 * abs(g1[1, 1])


def _golden_deep():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "deep_parratt50.json")
    return json.load(open(path))["cases"]


@pytest.mark.parametrize("case", range(5))
def test_deep_R_against_fifty_digit_parratt(nr, case):
    """Microsliced profiles of 300..2047 slabs against the 50-digit Parratt
    values of tests/golden/deep_parratt50.json: the value kernel (R_hat) and
    the scan kernel (its R, read out as the vector-Jacobian product with a
    unit seed, one single-point item per Q so that nothing is summed)."""
    from paper_2509_06924_amd import inputs
    c = _golden_deep()[case]
    rows = inputs.microsliced_stack(np.random.default_rng(c["seed"]), c["L"], c["dz"])
    q, ref = np.array(c["q"]), np.array(c["R"])
    datasets = [(np.array([qi]), np.array([1.0]), np.array([1.0]), 0.0) for qi in q]
    items = [(i, rows, 1.0, 0.0) for i in range(q.size)]
    prob = nr.Problem.from_batch(inputs._pack("golden_deep", datasets, items, {}))
    Rv = prob.reflectivity().cpu().numpy()
    dot = prob.reflectivity_vjp(np.ones(q.size))[0].cpu().numpy()
    check_R(Rv, ref, what=f"value kernel, {c['L']} slabs")
    check_R(dot, ref, what=f"scan kernel, {c['L']} slabs")


def test_depth_limit(nr):
    import ctypes
    from paper_2509_06924_amd import _native as n
    for rows, ok in ((n.NR_MAX_DEEP_LAYERS + 2, True), (n.NR_MAX_DEEP_LAYERS + 3, False)):
        q_off = np.array([0, 3], np.int64)
        dqq = np.array([0.0])
        dsi = np.array([0], np.int32)
        row_off = np.array([0, rows], np.int64)
        d = n.BatchDesc(1, q_off.ctypes.data, dqq.ctypes.data, 1, dsi.ctypes.data,
                        row_off.ctypes.data, 0)
        h = ctypes.c_void_p()
        st = n.lib().nr_plan_create(ctypes.byref(d), ctypes.byref(h))
        assert (st == n.NR_OK) == ok
        if h.value:
            n.lib().nr_plan_destroy(h)
