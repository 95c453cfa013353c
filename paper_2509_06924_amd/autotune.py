"""Autotuner of the plan schedule for one batch structure.

The library offers equivalent schedules of the same computation
(`nr_plan_options` in include/nr.h): per layer-count bucket, the store or the
recompute form of the gradient kernel; the length of the runs of work units
given to one XCD; packing of the trailing partial point groups, or a wave of
their own with the lanes split over smearing-node groups.  Which is
fastest depends on the batch (depth mix, points per item, number of items)
and the precision.  `tune` runs the library's autotuner (nr_autotune: a
coordinate search timing nr_loglik_grad on the caller's own data with HIP
events) and returns the fastest options; results are cached as JSON keyed by
the batch's structure class, so the search runs once per class.

    opts = autotune.tune(batch, precision=NR_F64)
    prob = Problem.from_batch(batch, options=opts)
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import _native as _n
from . import Problem, bucket_lmax



def default_cache_path():
    return os.environ.get("NR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2509_06924_amd",
                                       "autotune.json"))


def structure_key(q_off, row_off, dataset_of_item, precision, device_name=""):
    """Class of a batch structure: precision, the layer-count buckets present
    (with their share of the work rounded to tenths), points per item and
    number of items on a log2 scale, and the device."""
    q_off = np.asarray(q_off, np.int64)
    row_off = np.asarray(row_off, np.int64)
    dsi = np.asarray(dataset_of_item, np.int64)
    n = dsi.size
    L = np.diff(row_off) - 2
    nq = np.diff(q_off)[dsi] if n else np.zeros(0, np.int64)
    lm = np.array(bucket_lmax())
    b = np.searchsorted(lm, L) if n else np.zeros(0, np.int64)
    # items deeper than the last bucket (the scan kernel) count as their depth
    depth = np.where(b < lm.size, lm[np.minimum(b, lm.size - 1)], L) if n else np.zeros(0)
    work = (depth + 1) * nq if n else np.zeros(0)
    tot = float(work.sum()) or 1.0
    shares = {(int(lm[k]) if k < lm.size else "deep"): round(float(work[b == k].sum()) / tot, 1)
              for k in np.unique(b)}
    mean_nq = float(nq.mean()) if n else 0.0
    return json.dumps({
        "precision": int(precision),
        "buckets": {str(k): v for k, v in sorted(shares.items(), key=lambda kv: str(kv[0]))
                    if v > 0},
        "log2_points_per_item": int(round(math.log2(mean_nq))) if mean_nq > 0 else 0,
        "log2_items": int(round(math.log2(n))) if n > 0 else 0,
        "device": device_name,
        "library": int(_n.lib().nr_version()),
    }, sort_keys=True)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def options_to_dict(o):
    """nr_plan_options as the dict Plan / Problem.from_batch take."""
    lm = bucket_lmax()
    gv = {str(lm[k]): int(o.grad_variant[k]) for k in range(_n.NR_NUM_BUCKETS)
          if o.grad_variant[k] != _n.NR_VARIANT_AUTO}
    return {"grad_variant": gv, "xcd_run": int(o.xcd_run), "pack_tails": int(o.pack_tails),
            "split_tails": int(o.split_tails), "side_stream": int(o.side_stream),
            "node_groups": int(o.node_groups)}


def tune(batch, precision=_n.NR_F64, device="cuda", cache=None, reps=7, verbose=False,
         use_cache=True):
    """Fastest plan options for `batch` (an inputs.Batch or anything with the
    same fields), as a dict for Plan / Problem.from_batch.  The search itself
    is the library's nr_autotune on the batch's data; results are cached per
    structure class."""
    import ctypes

    import torch
    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    key = structure_key(batch.q_off, batch.row_off, batch.dataset_of_item, precision,
                        torch.cuda.get_device_name(dev))
    path = cache or default_cache_path()
    table = _load(path) if use_cache else {}
    if key in table:
        return table[key]["options"]

    prob = Problem.from_batch(batch, device=dev, precision=precision)
    plan = prob.plan
    o = _n.PlanOptions()
    ms = (ctypes.c_double * 2)()
    stream = torch.cuda.current_stream(dev)
    _n.check(_n.lib().nr_autotune(ctypes.byref(plan.desc), ctypes.byref(prob.values()), int(reps),
                                  ctypes.byref(o), ctypes.cast(ms, ctypes.c_void_p),
                                  ctypes.c_void_p(stream.cuda_stream)))
    best = options_to_dict(o)
    record = {"options": best, "ms": float(ms[0]), "default_ms": float(ms[1])}
    if use_cache:
        table[key] = record
        _save(path, table)
    if verbose:
        print(f"autotune best {best}: {ms[0]:.3f} ms (default {ms[1]:.3f} ms)")
    return best
