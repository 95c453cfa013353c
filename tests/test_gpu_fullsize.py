"""Parity at the full sizes of the benchmarked workloads, in the launch
configuration the benchmark times (default plans: two streams, packed, split
and lone tail units): items sampled across each batch are checked against
the oracle one by one (R_hat element by element, logL, the gradient), and
properties that hold at any size are checked on every item (finite values,
clean status, equal logL from the value and gradient calls)."""
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


def _run(nr, batch, precision=None):
    prob = nr.Problem.from_batch(batch, precision=precision or nr.NR_F64)
    Rhat = prob.reflectivity().cpu().numpy()
    ll = prob.loglik().cpu().numpy()
    llg, g_rows, g_inst = (t.cpu().numpy() for t in prob.loglik_grad())
    return prob, Rhat, ll, llg, g_rows, g_inst, prob.item_status.cpu().numpy()


def _check_all_items(batch, ll, llg, g_rows, st):
    assert np.all(st == 0)
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(llg)) and np.all(np.isfinite(g_rows))
    # the value kernels and the gradient kernels sum in different orders
    assert np.allclose(ll, llg, rtol=1e-9, atol=1e-6)


def _check_items(orc, batch, items, prob, Rhat, ll, llg, g_rows, g_inst, grad_items):
    off = prob.out_off
    for b in items:
        rows = batch.rows_of(b)
        Q, Robs, Rerr, dqq = batch.data_of(b)
        Ro = orc.model_curve(rows, batch.scale[b], batch.bkg[b], Q, dqq)
        check_R(Rhat[off[b]:off[b + 1]], Ro, what=f"R_hat item {b}")
        llo = orc.loglik(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
        bound = logL_bound(Ro, Robs, Rerr)
        check_logL(ll[b], llo, bound, what=f"logL item {b}")
        check_logL(llg[b], llo, bound, what=f"logL (grad call) item {b}")
        if b in grad_items:
            _, go, gio = orc.loglik_grad_cs(rows, batch.scale[b], batch.bkg[b], Q, Robs, Rerr, dqq)
            r0, r1 = batch.row_off[b], batch.row_off[b + 1]
            check_grad(g_rows[r0:r1], g_inst[b], go, gio, what=f"grad item {b}")


def _first(cond):
    idx = np.nonzero(cond)[0]
    assert idx.size, "no item of the sampled kind"
    return int(idx[0])


def test_ragged_16384_items_sampled(nr, orc):
    """16384 items, L 2..40, nQ 100..1000, dQ/Q 2-8 %: the deepest and the
    shallowest bucket, a middle bucket of each wave class, items whose
    trailing partial group is a lone, a split and a packed tail unit, and a
    deep item with close to 1000 points (15 full units and a tail)."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c4_ragged()
    L = np.diff(batch.row_off) - 2
    nq = np.diff(batch.q_off)[batch.dataset_of_item]
    tail = nq % 64
    small = nq < 200
    picks = {
        "L40": _first((L == 40) & small),
        "L2": _first((L == 2) & small),
        "L14": _first((L == 14) & small),
        "L25": _first((L == 25) & small),
        "lone tail": _first((L <= 10) & (tail >= 48) & small),
        "split tail": _first((L <= 10) & (tail >= 12) & (tail <= 32) & small),
        "packed deep tail": _first((L >= 29) & (tail > 0) & (tail < 48) & small),
        # most of the batch's work sits in deep items with many points
        "L>=36, nQ>=900": _first((L >= 36) & (nq >= 900)),
    }
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run(nr, batch)
    _check_all_items(batch, ll, llg, g_rows, st)
    items = sorted(set(picks.values()))
    _check_items(orc, batch, items, prob, Rhat, ll, llg, g_rows, g_inst, set(items))


def test_cofit_3072_items_sampled(nr, orc):
    """1024 draws x 3 contrasts x 12 layers, nQ 250 / 300 / 350: one item of
    each contrast (a lone tail unit; a 44-point tail that no other fits
    beside, run as a full unit; a split tail unit)."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c3_cofit()
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run(nr, batch)
    _check_all_items(batch, ll, llg, g_rows, st)
    items = [int(np.nonzero(batch.dataset_of_item == s)[0][-1]) for s in range(3)]
    _check_items(orc, batch, items, prob, Rhat, ll, llg, g_rows, g_inst, set(items))


def test_vi_8192_samples_sampled(nr, orc):
    """8192 samples x 20 layers x 1000 Q, 5 % dQ/Q: R_hat and logL of three
    samples, the gradient of one."""
    from paper_2509_06924_amd import inputs
    batch = inputs.c5_vi()
    prob, Rhat, ll, llg, g_rows, g_inst, st = _run(nr, batch)
    _check_all_items(batch, ll, llg, g_rows, st)
    _check_items(orc, batch, [0, 4095, 8191], prob, Rhat, ll, llg, g_rows, g_inst, {8191})
