"""Resolution as data and as a parameter (Sec. 3 pointwise Gaussian smearing;
Sec. 4.1 per-point FWHM; Sec. 4.2 the smearing size inferred): per-point widths
and per-item dQ/Q through the C-ABI against the oracle, and the derivative
g_res = dlogL/d(dQ/Q) of nr_loglik_grad_res against the oracle's complex step
through the node positions."""
import numpy as np
import pytest

from nr_check import G_TOL, INST_UNITS, ROW_UNITS, check_grad, check_logL, check_R, logL_bound

pytestmark = pytest.mark.gpu

# natural unit of dQ/Q for the gradient scale: a 1% change of the width
RES_UNIT = 1e-2


@pytest.fixture(scope="module")
def nr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_06924_amd as nr
    return nr


def _batch(seed, n_items=10, L_choices=(0, 1, 3, 6, 10, 13, 17, 26)):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(seed)
    return inputs.random_batch(rng, n_items=n_items, L_choices=list(L_choices),
                               nq_choices=[1, 40, 70, 130], dqq_choices=[0.0, 0.03, 0.08],
                               n_datasets=5)


def _point_widths(batch, seed):
    """Per-point FWHMs around (dQ/Q) Q, varying point to point (0 on
    unsmeared datasets, where they are not read)."""
    rng = np.random.default_rng(seed)
    dq = np.zeros_like(batch.Q)
    for s in range(batch.dq_over_q.size):
        a, e = int(batch.q_off[s]), int(batch.q_off[s + 1])
        dq[a:e] = batch.dq_over_q[s] * batch.Q[a:e] * rng.uniform(0.5, 1.5, e - a)
    return dq


@pytest.mark.parametrize("seed", [0, 1])
def test_pointwise_widths_match_oracle(nr, orc, seed):
    batch = _batch(700 + seed)
    dq = _point_widths(batch, 710 + seed)
    prob = nr.Problem.from_batch(batch).set_resolution(dq=dq)
    Rhat = prob.reflectivity().cpu().numpy()
    ll = prob.loglik().cpu().numpy()
    llg, g_rows, g_inst, g_res = (t.cpu().numpy() for t in prob.loglik_grad_res())
    assert np.all(prob.item_status.cpu().numpy() == 0)
    off = prob.out_off
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        s = int(batch.dataset_of_item[b])
        dQ = dq[batch.q_off[s]:batch.q_off[s + 1]]
        Ro = orc.model_curve_res(rows, batch.scale[b], batch.bkg[b], Q, dqq, dQ)
        check_R(Rhat[off[b]:off[b + 1]], Ro, what=f"R item {b}")
        llo, go, gio, gro = orc.loglik_grad_res_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs,
                                                   Rerr, dqq, dQ)
        bound = logL_bound(Ro, Robs, Rerr)
        check_logL(ll[b], llo, bound, what=f"logL item {b}")
        check_logL(llg[b], llo, bound, what=f"logL (grad call) item {b}")
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        check_grad(g_rows[r0:r1], g_inst[b], go, gio, what=f"grad item {b}")
        # fixed per-point widths are data: no width derivative
        assert gro == 0.0 and g_res[b] == 0.0


@pytest.mark.parametrize("seed", [0, 1])
def test_resolution_gradient_matches_oracle(nr, orc, seed):
    batch = _batch(720 + seed)
    prob = nr.Problem.from_batch(batch)
    ll, g_rows, g_inst, g_res = (t.cpu().numpy() for t in prob.loglik_grad_res())
    assert np.all(prob.item_status.cpu().numpy() == 0)
    smeared = 0
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        llo, go, gio, gro = orc.loglik_grad_res_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs,
                                                   Rerr, dqq)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        check_logL(ll[b], llo, logL_bound(Ro, Robs, Rerr), what=f"logL item {b}")
        # the width derivative joins the gradient vector in its natural unit
        a = np.concatenate([(g_rows[batch.row_off[b]:batch.row_off[b + 1]] * ROW_UNITS).ravel(),
                            g_inst[b] * INST_UNITS, [g_res[b] * RES_UNIT]])
        o = np.concatenate([(go * ROW_UNITS).ravel(), gio * INST_UNITS, [gro * RES_UNIT]])
        scale = np.max(np.abs(o))
        assert np.max(np.abs(a - o)) <= G_TOL * scale, f"item {b}"
        if dqq > 0.0:
            smeared += 1
            assert abs(g_res[b] - gro) <= G_TOL * max(abs(gro), 1e-3 * scale / RES_UNIT), \
                f"g_res item {b}: {g_res[b]!r} vs {gro!r}"
        else:
            assert g_res[b] == 0.0 and gro == 0.0
    assert smeared > 0


def test_resolution_form_leaves_other_outputs_unchanged(nr):
    """The resolution-derivative form is the recompute form plus one more
    accumulator: with the recompute form selected everywhere, logL and the
    parameter gradient are those of nr_loglik_grad.  Bitwise where the two
    forms run the same schedule.  The plain full units of 6 to 10 layers are
    software-pipelined and the resolution form's are not; the compiler then
    fuses a few products into FMAs differently, so items in those buckets
    agree to rounding."""
    batch = _batch(730, n_items=16)
    opts = {"grad_variant": {str(k): nr._n.NR_VARIANT_RECOMPUTE for k in nr.bucket_lmax()}}
    prob = nr.Problem.from_batch(batch, options=opts)
    llg_a, rows_a, inst_a = (t.cpu().numpy() for t in prob.loglik_grad())
    llg_b, rows_b, inst_b = (t.cpu().numpy() for t in prob.loglik_grad_res()[:3])
    L = np.diff(batch.row_off) - 2
    buckets = np.array(sorted(nr.bucket_lmax()))
    depth = buckets[np.searchsorted(buckets, L)]
    piped = (depth >= 6) & (depth <= 10)
    assert piped.any() and (~piped).any()
    row_item = np.repeat(np.arange(batch.n_items), np.diff(batch.row_off))
    for x, y, sel in ((llg_a, llg_b, piped), (inst_a, inst_b, piped),
                      (rows_a, rows_b, piped[row_item])):
        assert np.array_equal(x[~sel], y[~sel])
    for b in np.flatnonzero(piped):
        assert abs(llg_a[b] - llg_b[b]) <= 1e-12 * abs(llg_b[b])
        ga = np.concatenate([rows_a[batch.row_off[b]:batch.row_off[b + 1]].ravel(), inst_a[b]])
        gb = np.concatenate([rows_b[batch.row_off[b]:batch.row_off[b + 1]].ravel(), inst_b[b]])
        assert np.max(np.abs(ga - gb)) <= 1e-11 * np.max(np.abs(gb)), f"item {b}"


def test_item_dqq_override(nr, orc):
    batch = _batch(740)
    base = nr.Problem.from_batch(batch)
    ref = [t.cpu().numpy() for t in base.loglik_grad_res()]
    same = batch.dq_over_q[batch.dataset_of_item]
    # the dataset's own value per item: bitwise the same results
    prob = nr.Problem.from_batch(batch).set_resolution(dqq_item=same)
    got = [t.cpu().numpy() for t in prob.loglik_grad_res()]
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)
    # other values: the oracle at each item's dQ/Q (smeared datasets only)
    rng = np.random.default_rng(741)
    dqq_item = np.where(same > 0, rng.uniform(0.01, 0.1, same.size), 0.0)
    prob.set_resolution(dqq_item=dqq_item)
    Rhat = prob.reflectivity().cpu().numpy()
    ll, g_rows, g_inst, g_res = (t.cpu().numpy() for t in prob.loglik_grad_res())
    off = prob.out_off
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, _ = batch.data_of(b)
        d = float(dqq_item[b])
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, d)
        check_R(Rhat[off[b]:off[b + 1]], Ro, what=f"R item {b}")
        llo, go, gio, gro = orc.loglik_grad_res_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs,
                                                   Rerr, d)
        check_logL(ll[b], llo, logL_bound(Ro, Robs, Rerr), what=f"logL item {b}")
        a = np.concatenate([(g_rows[batch.row_off[b]:batch.row_off[b + 1]] * ROW_UNITS).ravel(),
                            g_inst[b] * INST_UNITS, [g_res[b] * RES_UNIT]])
        o = np.concatenate([(go * ROW_UNITS).ravel(), gio * INST_UNITS, [gro * RES_UNIT]])
        assert np.max(np.abs(a - o)) <= G_TOL * np.max(np.abs(o)), f"item {b}"


def test_resolution_gradient_fp32(nr, orc):
    """FP32 variant: the width derivative within the FP32 gradient ceiling."""
    batch = _batch(750, L_choices=(2, 5, 9))
    prob = nr.Problem.from_batch(batch, precision=nr.NR_F32)
    _, _, _, g_res = (t.cpu().numpy() for t in prob.loglik_grad_res())
    for b in range(batch.n_items):
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        _, go, gio, gro = orc.loglik_grad_res_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs,
                                                 Rerr, dqq)
        o = np.concatenate([(go * ROW_UNITS).ravel(), gio * INST_UNITS, [gro * RES_UNIT]])
        if dqq > 0.0:
            err = abs(g_res[b] - gro) * RES_UNIT / np.max(np.abs(o))
            print(f"FP32 g_res item {b}: {err:.2e} of the gradient scale")
            assert err <= 1e-2, f"item {b}"
        else:
            assert g_res[b] == 0.0


def test_resolution_argument_checks(nr):
    batch = _batch(760, n_items=3)
    prob = nr.Problem.from_batch(batch)
    with pytest.raises(ValueError):
        prob.set_resolution(dq=np.ones(batch.Q.size + 1))
    with pytest.raises(ValueError):
        prob.set_resolution(dqq_item=np.ones(batch.n_items + 1))
