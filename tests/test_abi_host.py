"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/nr.h declares, and rejects invalid batch descriptions
before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2509_06924_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libnr.so not built")
    return _native, _native.lib()


def test_header_declares_exactly_the_exported_api():
    from paper_2509_06924_amd import _native
    text = open(os.path.join(ROOT, "include", "nr.h")).read()
    declared = set(re.findall(r"^\s*(?:nr_status|int32_t|const char\*)\s+(nr_\w+)\s*\(", text, re.M))
    assert declared == set(_native.EXPORTS)


def test_library_exports_every_declared_symbol():
    n, L = _lib()
    for name in n.EXPORTS:
        assert hasattr(L, name), name
    assert L.nr_version() == 2


def test_status_strings():
    n, L = _lib()
    for s in range(0, 6):
        assert isinstance(n.status_string(s), str) and n.status_string(s)


def _desc(n, q_off, dqq, dsi, row_off, precision=0):
    keep = [np.ascontiguousarray(q_off, np.int64), np.ascontiguousarray(dqq, np.float64),
            np.ascontiguousarray(dsi, np.int32), np.ascontiguousarray(row_off, np.int64)]
    d = n.BatchDesc(len(dqq), ctypes.c_void_p(keep[0].ctypes.data),
                    ctypes.c_void_p(keep[1].ctypes.data) if len(dqq) else None, len(dsi),
                    ctypes.c_void_p(keep[2].ctypes.data) if len(dsi) else None,
                    ctypes.c_void_p(keep[3].ctypes.data), precision)
    return d, keep


@pytest.mark.parametrize("case", [
    "null", "neg_items", "bad_precision", "q_off_start", "q_off_decreasing", "neg_dqq",
    "nan_dqq", "too_few_rows", "too_many_layers", "bad_dataset"])
def test_invalid_descriptions_rejected(case):
    n, L = _lib()
    q_off, dqq, dsi, row_off, prec = [0, 10, 20], [0.05, 0.0], [0, 1], [0, 4, 7], 0
    if case == "null":
        h = ctypes.c_void_p()
        assert L.nr_plan_create(None, ctypes.byref(h)) == n.NR_EINVAL
        return
    if case == "neg_items":
        d, keep = _desc(n, q_off, dqq, dsi, row_off)
        d.n_items = -1
    else:
        if case == "bad_precision":
            prec = 7
        elif case == "q_off_start":
            q_off = [1, 10, 20]
        elif case == "q_off_decreasing":
            q_off = [0, 10, 5]
        elif case == "neg_dqq":
            dqq = [-0.01, 0.0]
        elif case == "nan_dqq":
            dqq = [float("nan"), 0.0]
        elif case == "too_few_rows":
            row_off = [0, 1, 4]
        elif case == "too_many_layers":
            row_off = [0, 4, 4 + n.NR_MAX_DEEP_LAYERS + 3]
        elif case == "bad_dataset":
            dsi = [0, 2]
        d, keep = _desc(n, q_off, dqq, dsi, row_off, prec)
    h = ctypes.c_void_p()
    assert L.nr_plan_create(ctypes.byref(d), ctypes.byref(h)) == n.NR_EINVAL
    assert not h.value


def test_null_plan_calls_rejected():
    n, L = _lib()
    sz = ctypes.c_size_t()
    assert L.nr_workspace_size(None, 0, ctypes.byref(sz)) == n.NR_EINVAL
    v = n.Values()
    assert L.nr_loglik(None, ctypes.byref(v), None, None, 0, None) == n.NR_EINVAL
    assert L.nr_loglik_grad(None, ctypes.byref(v), None, None, None, None, 0, None) == n.NR_EINVAL
    assert L.nr_reflectivity(None, ctypes.byref(v), None, None, 0, None) == n.NR_EINVAL
    assert L.nr_loglik_grad_res(None, ctypes.byref(v), None, None, None, None, None, 0,
                                None) == n.NR_EINVAL
    assert L.nr_plan_destroy(None) == n.NR_OK
    # the drivers around the gradient
    h = ctypes.c_void_p()
    cfg = n.HmcConfig(5, 1000.0, 1, 0.8)
    assert L.nr_hmc_create(None, ctypes.byref(cfg), ctypes.byref(h)) == n.NR_EINVAL
    assert not h.value
    ch = n.HmcChains()
    assert L.nr_hmc_init(None, ctypes.byref(v), ctypes.byref(ch), 1, None, 0, None) == n.NR_EINVAL
    assert L.nr_hmc_transition(None, ctypes.byref(v), ctypes.byref(ch), 0, None, 0,
                               None) == n.NR_EINVAL
    assert L.nr_hmc_adapt(None, ctypes.byref(ch), 1, None) == n.NR_EINVAL
    assert L.nr_hmc_destroy(None) == n.NR_OK
    mcfg = n.MvnConfig(2, 3, 0.05, 0.9, 0.999, 1e-8, 0)
    assert L.nr_vi_mvn_create(None, ctypes.byref(mcfg), ctypes.byref(h)) == n.NR_EINVAL
    prm = n.MvnParams()
    assert L.nr_vi_mvn_step(None, ctypes.byref(v), ctypes.byref(prm), 1, None, 0,
                            None) == n.NR_EINVAL
    assert L.nr_vi_mvn_destroy(None) == n.NR_OK
    g = ctypes.c_void_p()
    assert L.nr_hmc_graph_create(None, ctypes.byref(v), ctypes.byref(ch), 0, 1, None, 0,
                                 ctypes.byref(g)) == n.NR_EINVAL
    assert L.nr_vi_mvn_graph_create(None, ctypes.byref(v), ctypes.byref(prm), 1, None, 0,
                                    ctypes.byref(g)) == n.NR_EINVAL
    assert not g.value


def test_paper_parameter_dict_packs_to_rows():
    """The Sec. 3 parameter dict (shapes only: n = 2 layers) maps to rows."""
    import json
    from paper_2509_06924_amd import pack_theta
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_theta_example.json")))
    rows = pack_theta(g["theta"], sld_unit=1e-6)
    n = len(g["theta"]["thick"])
    assert rows.shape == (n + 2, 4)
    assert np.array_equal(rows[1:n + 1, 0], g["theta"]["thick"])
    assert np.allclose(rows[:, 1], np.array(g["theta"]["SLD"]) * 1e-6)
    assert np.array_equal(rows[1:, 3], g["theta"]["rough"])
    assert rows[0, 0] == 0 and rows[-1, 0] == 0 and rows[0, 3] == 0


def test_bucket_table_and_store_limits():
    n, L = _lib()
    lm = [L.nr_bucket_lmax(k) for k in range(n.NR_NUM_BUCKETS)]
    assert lm == sorted(lm) and lm[-1] == n.NR_MAX_LAYERS and lm[0] >= 1
    assert L.nr_bucket_lmax(-1) == -1 and L.nr_bucket_lmax(n.NR_NUM_BUCKETS) == -1
    for prec in (n.NR_F64, n.NR_F32):
        assert L.nr_store_max_layers(prec) in lm
    assert L.nr_store_max_layers(7) == -1


def test_plan_options_defaults_and_dict():
    n, L = _lib()
    from paper_2509_06924_amd import plan_options
    o = plan_options()
    assert list(o.grad_variant) == [n.NR_VARIANT_AUTO] * n.NR_NUM_BUCKETS
    assert o.xcd_run == 8 and o.pack_tails == 1 and o.split_tails == 7 and o.side_stream == 1
    o = plan_options({"grad_variant": {"10": n.NR_VARIANT_RECOMPUTE}, "xcd_run": 4,
                      "pack_tails": 0, "side_stream": 0})
    k10 = [L.nr_bucket_lmax(k) for k in range(n.NR_NUM_BUCKETS)].index(10)
    assert o.grad_variant[k10] == n.NR_VARIANT_RECOMPUTE and o.xcd_run == 4 and o.pack_tails == 0
    assert o.side_stream == 0


@pytest.mark.parametrize("case", ["xcd_zero", "xcd_big", "pack_two", "split_two", "side_two",
                                  "side_negative", "variant_unknown", "store_too_deep_f64",
                                  "store_too_deep_f32"])
def test_invalid_plan_options_rejected(case):
    n, L = _lib()
    from paper_2509_06924_amd import plan_options
    o = plan_options()
    prec = n.NR_F64
    deep = n.NR_NUM_BUCKETS - 1
    if case == "xcd_zero":
        o.xcd_run = 0
    elif case == "xcd_big":
        o.xcd_run = 65
    elif case == "pack_two":
        o.pack_tails = 2
    elif case == "split_two":
        o.split_tails = 8
    elif case == "side_two":
        o.side_stream = 2
    elif case == "side_negative":
        o.side_stream = -1
    elif case == "variant_unknown":
        o.grad_variant[0] = 9
    elif case == "store_too_deep_f64":
        o.grad_variant[deep] = n.NR_VARIANT_STORE
    else:
        prec = n.NR_F32
        o.grad_variant[deep] = n.NR_VARIANT_STORE
    d, keep = _desc(n, [0, 10, 20], [0.05, 0.0], [0, 1], [0, 4, 7], prec)
    h = ctypes.c_void_p()
    assert L.nr_plan_create_ex(ctypes.byref(d), ctypes.byref(o), ctypes.byref(h)) == n.NR_EINVAL
    assert not h.value


def test_autotune_structure_key_classes():
    """Batches of the same shape class share a key; depth mix, size class and
    precision separate them."""
    _lib()
    from paper_2509_06924_amd import autotune, inputs
    a = inputs.c2_batched(n_items=256)
    b = inputs.c2_batched(n_items=256, seed_offset=9)
    c = inputs.c2_batched(n_items=256, L=20)
    k = lambda x, p=0: autotune.structure_key(x.q_off, x.row_off, x.dataset_of_item, p, "dev")
    assert k(a) == k(b)
    assert k(a) != k(c) and k(a) != k(a, 1)
    assert k(a) != k(inputs.c2_batched(n_items=1024))


def test_binding_shares_torchs_hip_runtime():
    """Loading the library before torch is touched must still leave one HIP
    runtime in the process, torch's (a second runtime would make torch's
    streams invalid in the library and, loaded first, hide the GPU from
    torch)."""
    import subprocess
    import sys
    code = ("import paper_2509_06924_amd as nr\n"
            "nr._n.lib()\n"
            "import torch, os\n"
            "rt = sorted(set(l.split()[-1] for l in open('/proc/self/maps') if 'amdhip64' in l))\n"
            "print(len(rt), os.path.dirname(rt[0]) == os.path.dirname(torch.__file__) + '/lib')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["1", "True"], r.stdout


def test_quadrature_rule_is_bitwise_the_oracles():
    """The kernel side builds its 17-point rule with its own Newton iteration
    on the host; node offsets and weights must be the oracle's doubles
    exactly (the smearing step of the model, Sec. 3 / Sec. 4.1)."""
    import oracle
    n, L = _lib()
    t, w = n.smearing_rule()
    to, wo = oracle.smear_rule(0.05)
    assert np.array_equal(np.array(t), to)
    assert np.array_equal(np.array(w), wo)
    assert L.nr_smearing_rule(None, None) == n.NR_EINVAL
