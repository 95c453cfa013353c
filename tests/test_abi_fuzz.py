"""Property tests of the host-side validation of nr_plan_create and
nr_plan_create_ex over ragged batch structures: layer counts 0..2047, point
counts 0..1000, empty datasets, and one corruption at a time.  A valid
description is never rejected as invalid (without a GPU the call then fails
at the device query with NR_EHIP; with one it builds a plan, which is
destroyed again); every corrupted description is rejected with NR_EINVAL
before the device is touched, and no plan handle is returned."""
import ctypes
import os

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

from paper_2509_06924_amd import _native as n  # noqa: E402

if not os.path.exists(n.LIB_PATH):
    pytest.skip("libnr.so not built", allow_module_level=True)

INT32_MAX = 2**31 - 1


@st.composite
def batches(draw):
    nd = draw(st.integers(0, 6))
    nqs = draw(st.lists(st.integers(0, 1000), min_size=nd, max_size=nd))
    dqq = draw(st.lists(st.one_of(st.just(0.0), st.floats(1e-4, 0.12)), min_size=nd,
                        max_size=nd))
    ni = draw(st.integers(0, 12)) if nd > 0 else 0
    Ls = draw(st.lists(st.one_of(st.integers(0, 40), st.integers(41, n.NR_MAX_DEEP_LAYERS)),
                       min_size=ni, max_size=ni))
    dsi = draw(st.lists(st.integers(0, max(nd - 1, 0)), min_size=ni, max_size=ni))
    prec = draw(st.sampled_from([n.NR_F64, n.NR_F32]))
    return {"q_off": np.concatenate([[0], np.cumsum(nqs)]).astype(np.int64),
            "dqq": np.array(dqq, np.float64),
            "row_off": np.concatenate([[0], np.cumsum([L + 2 for L in Ls])]).astype(np.int64),
            "dsi": np.array(dsi, np.int32), "prec": prec}


def _desc(b):
    keep = [np.ascontiguousarray(b["q_off"], np.int64), np.ascontiguousarray(b["dqq"], np.float64),
            np.ascontiguousarray(b["dsi"], np.int32), np.ascontiguousarray(b["row_off"], np.int64)]
    ptr = [ctypes.c_void_p(k.ctypes.data) if k.size else None for k in keep]
    d = n.BatchDesc(int(keep[1].size), ptr[0], ptr[1], int(keep[2].size), ptr[2], ptr[3],
                    b["prec"])
    # the offsets arrays are never empty (one entry more than their count)
    d.q_off = ctypes.c_void_p(keep[0].ctypes.data)
    d.row_off = ctypes.c_void_p(keep[3].ctypes.data)
    return d, keep


def _create(d, opts=None):
    L = n.lib()
    h = ctypes.c_void_p()
    if opts is None:
        rc = L.nr_plan_create(ctypes.byref(d), ctypes.byref(h))
    else:
        rc = L.nr_plan_create_ex(ctypes.byref(d), ctypes.byref(opts), ctypes.byref(h))
    if h.value:
        L.nr_plan_destroy(h)
    return rc, h.value


SETTINGS = settings(max_examples=150, deadline=None,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(batches())
def test_valid_descriptions_pass_validation(b):
    d, keep = _desc(b)
    rc, h = _create(d)
    assert rc in (n.NR_OK, n.NR_EHIP), rc
    if rc != n.NR_OK:
        assert not h


CORRUPTIONS = ["q_off_start", "q_off_decreasing", "dqq_negative", "dqq_nan", "dqq_inf",
               "rows_too_few", "rows_too_many", "dataset_negative", "dataset_too_large",
               "precision", "n_items_negative", "n_datasets_negative", "dataset_too_long",
               "row_off_start", "null_q_off", "null_row_off"]


@SETTINGS
@given(batches(), st.sampled_from(CORRUPTIONS), st.integers(0, 2**16))
def test_corrupted_descriptions_are_rejected(b, what, pick):
    nd, ni = b["dqq"].size, b["dsi"].size
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in b.items()}
    if what == "q_off_start":
        b["q_off"] = b["q_off"] + 1
    elif what == "q_off_decreasing":
        if nd == 0:
            return
        s = pick % nd
        b["q_off"][s + 1] = b["q_off"][s] - 1 - pick % 7
    elif what in ("dqq_negative", "dqq_nan", "dqq_inf"):
        if nd == 0:
            return
        b["dqq"][pick % nd] = {"dqq_negative": -1e-3, "dqq_nan": np.nan,
                               "dqq_inf": np.inf}[what]
    elif what in ("rows_too_few", "rows_too_many"):
        if ni == 0:
            return
        rows = np.diff(b["row_off"])
        rows[pick % ni] = (pick % 2) if what == "rows_too_few" else n.NR_MAX_DEEP_LAYERS + 3
        b["row_off"] = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    elif what in ("dataset_negative", "dataset_too_large"):
        if ni == 0:
            return
        b["dsi"][pick % ni] = -1 - pick % 3 if what == "dataset_negative" else nd + pick % 3
    elif what == "precision":
        b["prec"] = 2 + pick % 5
    elif what == "dataset_too_long":
        if nd == 0:
            return
        s = pick % nd
        b["q_off"][s + 1:] += INT32_MAX + 1
    elif what == "row_off_start":
        b["row_off"] = b["row_off"] + 2
    d, keep = _desc(b)
    if what == "n_items_negative":
        d.n_items = -1 - pick % 4
    elif what == "n_datasets_negative":
        d.n_datasets = -1 - pick % 4
    elif what == "null_q_off":
        d.q_off = None
    elif what == "null_row_off":
        d.row_off = None
    rc, h = _create(d)
    assert rc == n.NR_EINVAL, (what, rc)
    assert not h


OPTION_CORRUPTIONS = ["xcd_run_low", "xcd_run_high", "pack_tails", "split_tails", "side_stream",
                      "variant_unknown", "store_too_deep", "node_groups_one", "node_groups_high",
                      "node_groups_negative"]


@SETTINGS
@given(batches(), st.sampled_from(OPTION_CORRUPTIONS), st.integers(0, 2**16))
def test_corrupted_options_are_rejected(b, what, pick):
    L = n.lib()
    d, keep = _desc(b)
    o = n.PlanOptions()
    assert L.nr_plan_options_default(ctypes.byref(o)) == n.NR_OK
    assert _create(d, o)[0] in (n.NR_OK, n.NR_EHIP)
    if what == "xcd_run_low":
        o.xcd_run = -(pick % 5)
    elif what == "xcd_run_high":
        o.xcd_run = 65 + pick % 100
    elif what == "pack_tails":
        o.pack_tails = 2 + pick % 5
    elif what == "split_tails":
        o.split_tails = 8 << (pick % 4)
    elif what == "side_stream":
        o.side_stream = -1 - pick % 3
    elif what == "variant_unknown":
        o.grad_variant[pick % n.NR_NUM_BUCKETS] = 3 + pick % 4
    elif what == "node_groups_one":
        o.node_groups = 1
    elif what == "node_groups_high":
        o.node_groups = 18 + pick % 50
    elif what == "node_groups_negative":
        o.node_groups = -1 - pick % 5
    elif what == "store_too_deep":
        smax = L.nr_store_max_layers(b["prec"])
        deep = [k for k in range(n.NR_NUM_BUCKETS) if L.nr_bucket_lmax(k) > smax]
        o.grad_variant[deep[pick % len(deep)]] = n.NR_VARIANT_STORE
    rc, h = _create(d, o)
    assert rc == n.NR_EINVAL, (what, rc)
    assert not h
